"""Python access to the plain serial C oracle (nasch_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use it; the library under test never imports it.  It shares no
code with the HIP path.  `build()` compiles the C file with gcc; everything
else is argument marshalling through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nasch_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

EMPTY = 0xFF

u8p = ctypes.POINTER(ctypes.c_uint8)
u32p = ctypes.POINTER(ctypes.c_uint32)
i32p = ctypes.POINTER(ctypes.c_int32)
u64p = ctypes.POINTER(ctypes.c_uint64)
U32, U64, I32, DBL = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double


def build() -> str:
    """Compile the oracle (gcc -O2, OpenMP for the all-core twin)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    sig = {
        "oracle_philox4x32_10": (None, [u32p, u32p, u32p]),
        "oracle_rand32": (U32, [U64, U32, U32, U32]),
        "oracle_threshold": (U32, [DBL]),
        "oracle_place": (U64, [U64, U64, U32, U64]),
        "oracle_place_inverse": (U64, [U64, U64, U32, U64]),
        "oracle_initial_velocity": (U32, [U32, U32, U32, U32, U64]),
        "oracle_init_grid": (None, [U64, U64, U32, U32, U32, U64, u8p]),
        "oracle_init_window": (None, [U64, U64, U32, U32, U32, U64, U64, U64, u8p]),
        "oracle_step_grid": (U64, [U64, U32, U32, U64, U32, U32, u8p, u8p, I32]),
        "oracle_run_grid": (I32, [U64, U32, DBL, U64, U32, U64, U64, u8p, u64p, I32]),
        "oracle_step_agent": (U64, [U64, U64, U32, U32, U64, U32, U32, i32p, u8p, i32p, u8p]),
        "oracle_run_agent": (I32, [U64, U64, U32, DBL, U64, U32, U64, U64, i32p, u8p, u64p]),
        "oracle_grid_to_agent": (U64, [U64, u8p, i32p, u8p]),
        "oracle_mlcg_seed": (U32, [U64]),
        "oracle_mlcg_next": (U32, [U32]),
        "oracle_mlcg_threshold": (U32, [DBL]),
        "oracle_run_agent_mlcg": (I32, [U64, U64, U32, DBL, u32p, U64, i32p, u8p, u64p]),
        "oracle_advance_segment": (I32, [U64, U32, DBL, U64, U32, U64, U64, U64, U64, u8p,
                                         u8p]),
        "oracle_window_from_init": (I32, [U64, U64, U32, DBL, U64, U32, U32, U64, U64, U64,
                                          u8p]),
        "oracle_gate_threshold": (U64, [DBL]),
        "oracle_gate_words": (None, [U64, U32, U32, u32p, u32p]),
        "oracle_step_open": (U64, [U64, U64, U64, U32, U32, U64, U64, U64, U32, U32, u8p, u8p,
                                   u64p, u64p]),
        "oracle_run_open": (I32, [U64, U64, U64, U32, DBL, DBL, DBL, U64, U32, U64, U64, u8p,
                                  u64p, u64p, u64p]),
        "oracle_open_window_from_init": (I32, [U64, U64, U32, DBL, DBL, DBL, U64, U32, U32,
                                               U64, U64, U64, u8p]),
        "oracle_num_threads_available": (I32, []),
        "oracle_fnv1a64": (U64, [u8p, U64, U64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray, t):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


# --------------------------------------------------------------------------- PRNG
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    _load().oracle_philox4x32_10(_ptr(c, u32p), _ptr(k, u32p), _ptr(out, u32p))
    return out


def rand32(seed: int, replica: int, t: int, x: int) -> int:
    return int(_load().oracle_rand32(seed, replica, t, x))


def threshold(p: float) -> int:
    return int(_load().oracle_threshold(float(p)))


# --------------------------------------------------------------------------- init
def place(i: int, L: int, replica: int, seed: int) -> int:
    return int(_load().oracle_place(i, L, replica, seed))


def place_inverse(y: int, L: int, replica: int, seed: int) -> int:
    return int(_load().oracle_place_inverse(y, L, replica, seed))


def initial_velocity(x: int, vmax: int, init_v: int, replica: int, seed: int) -> int:
    return int(_load().oracle_initial_velocity(x, vmax, init_v, replica, seed))


def init_grid(L, N, vmax, seed, replica=0, init_v=0) -> np.ndarray:
    g = np.empty(L, np.uint8)
    _load().oracle_init_grid(L, N, vmax, init_v, replica, seed, _ptr(g, u8p))
    return g


def init_window(L, N, vmax, seed, a, w, replica=0, init_v=0) -> np.ndarray:
    out = np.empty(w, np.uint8)
    _load().oracle_init_window(L, N, vmax, init_v, replica, seed, a, w, _ptr(out, u8p))
    return out


# --------------------------------------------------------------------------- steps
def step_grid(g: np.ndarray, vmax: int, p: float, seed: int, t: int, replica=0, nthreads=1):
    """One step; returns (new grid, F(t))."""
    g = np.ascontiguousarray(g, dtype=np.uint8)
    out = np.empty_like(g)
    f = _load().oracle_step_grid(g.size, vmax, threshold(p), seed, replica, t, _ptr(g, u8p),
                                 _ptr(out, u8p), nthreads)
    return out, int(f)


def run_grid(g: np.ndarray, vmax: int, p: float, seed: int, T: int, t0=0, replica=0,
             nthreads=1):
    """T steps from t0; returns (final grid, flux[T] as uint64)."""
    g = np.array(g, dtype=np.uint8, copy=True, order="C")
    flux = np.zeros(max(T, 1), np.uint64)
    rc = _load().oracle_run_grid(g.size, vmax, float(p), seed, replica, t0, T, _ptr(g, u8p),
                                 _ptr(flux, u64p), nthreads)
    if rc:
        raise MemoryError("oracle_run_grid")
    return g, flux[:T]


def step_agent(L, x, v, vmax, p, seed, t, replica=0):
    x = np.ascontiguousarray(x, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.uint8)
    xo, vo = np.empty_like(x), np.empty_like(v)
    f = _load().oracle_step_agent(L, x.size, vmax, threshold(p), seed, replica, t,
                                  _ptr(x, i32p), _ptr(v, u8p), _ptr(xo, i32p), _ptr(vo, u8p))
    return xo, vo, int(f)


def run_agent(L, x, v, vmax, p, seed, T, t0=0, replica=0):
    x = np.array(x, dtype=np.int32, copy=True, order="C")
    v = np.array(v, dtype=np.uint8, copy=True, order="C")
    flux = np.zeros(max(T, 1), np.uint64)
    rc = _load().oracle_run_agent(L, x.size, vmax, float(p), seed, replica, t0, T,
                                  _ptr(x, i32p), _ptr(v, u8p), _ptr(flux, u64p))
    if rc:
        raise MemoryError("oracle_run_agent")
    return x, v, flux[:T]


def mlcg_seed(seed: int) -> int:
    return int(_load().oracle_mlcg_seed(seed))


def mlcg_next(x: int) -> int:
    return int(_load().oracle_mlcg_next(x))


def mlcg_threshold(p: float) -> int:
    return int(_load().oracle_mlcg_threshold(float(p)))


def run_agent_mlcg(L, x, v, vmax, p, seed, T, t0=0, state0=None):
    """T steps with the shared minstd stream, starting at step t0 (the stream
    is first advanced serially past the t0 * N draws of the earlier steps).
    With state0 given, the stream starts from that generator state instead
    and seed and t0 are not used: a caller that jumps far into the stream
    passes the state it computed.  Returns (x, v, flux[T])."""
    x = np.array(x, dtype=np.int32, copy=True, order="C")
    v = np.array(v, dtype=np.uint8, copy=True, order="C")
    lib = _load()
    if state0 is not None:
        st = ctypes.c_uint32(int(state0))
    else:
        st = ctypes.c_uint32(lib.oracle_mlcg_seed(seed))
        for _ in range(t0 * x.size):
            st.value = lib.oracle_mlcg_next(st.value)
    flux = np.zeros(max(T, 1), np.uint64)
    rc = lib.oracle_run_agent_mlcg(L, x.size, vmax, float(p), ctypes.byref(st), T,
                                   _ptr(x, i32p), _ptr(v, u8p), _ptr(flux, u64p))
    if rc:
        raise MemoryError("oracle_run_agent_mlcg")
    return x, v, flux[:T]


def grid_to_agent(g: np.ndarray):
    g = np.ascontiguousarray(g, dtype=np.uint8)
    x = np.empty(g.size, np.int32)
    v = np.empty(g.size, np.uint8)
    n = _load().oracle_grid_to_agent(g.size, _ptr(g, u8p), _ptr(x, i32p), _ptr(v, u8p))
    return x[:n].copy(), v[:n].copy()


def agent_to_grid(L, x, v) -> np.ndarray:
    g = np.full(L, EMPTY, np.uint8)
    g[np.asarray(x, dtype=np.int64)] = np.asarray(v, dtype=np.uint8)
    return g


def advance_segment(L, seg, vmax, p, seed, t0, T, a, w, replica=0):
    seg = np.array(seg, dtype=np.uint8, copy=True, order="C")
    assert seg.size == w + 2 * T * vmax
    out = np.empty(w, np.uint8)
    rc = _load().oracle_advance_segment(L, vmax, float(p), seed, replica, t0, T, a, w,
                                        _ptr(seg, u8p), _ptr(out, u8p))
    if rc:
        raise MemoryError("oracle_advance_segment")
    return out


def window_from_init(L, N, vmax, p, seed, T, a, w, replica=0, init_v=0) -> np.ndarray:
    """Cells [a, a+w) mod L after T steps from the initial state (light cone)."""
    out = np.empty(w, np.uint8)
    rc = _load().oracle_window_from_init(L, N, vmax, float(p), seed, replica, init_v, T, a, w,
                                         _ptr(out, u8p))
    if rc:
        raise MemoryError("oracle_window_from_init")
    return out


# --------------------------------------------------------------------------- open road
def gate_threshold(a: float) -> int:
    return int(_load().oracle_gate_threshold(float(a)))


def gate_words(seed: int, t: int, replica=0):
    """(entry word, exit word) of the gate draw of step t."""
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _load().oracle_gate_words(seed, replica, t, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def step_open(g, vmax, p, alpha, beta, seed, t, replica=0, L=None, lo=0):
    """One step of cells [lo, lo + len(g)) of an open road of L cells (default:
    the whole road).  Returns (new cells, F(t), entered, left)."""
    g = np.ascontiguousarray(g, dtype=np.uint8)
    L = g.size if L is None else L
    out = np.empty_like(g)
    e, l = ctypes.c_uint64(), ctypes.c_uint64()
    f = _load().oracle_step_open(L, lo, g.size, vmax, threshold(p), gate_threshold(alpha),
                                 gate_threshold(beta), seed, replica, t, _ptr(g, u8p),
                                 _ptr(out, u8p), ctypes.byref(e), ctypes.byref(l))
    return out, int(f), e.value, l.value


def run_open(g, vmax, p, alpha, beta, seed, T, t0=0, replica=0, L=None, lo=0):
    """T steps of an open road (or of cells [lo, lo + len(g)) of one of L
    cells) from step t0.  Returns (cells, flux[T], entered[T], left[T])."""
    g = np.array(g, dtype=np.uint8, copy=True, order="C")
    L = g.size if L is None else L
    flux = np.zeros(max(T, 1), np.uint64)
    ent = np.zeros(max(T, 1), np.uint64)
    lft = np.zeros(max(T, 1), np.uint64)
    rc = _load().oracle_run_open(L, lo, g.size, vmax, float(p), float(alpha), float(beta), seed,
                                 replica, t0, T, _ptr(g, u8p), _ptr(flux, u64p),
                                 _ptr(ent, u64p), _ptr(lft, u64p))
    if rc:
        raise MemoryError("oracle_run_open")
    return g, flux[:T], ent[:T], lft[:T]


def open_window_from_init(L, N, vmax, p, alpha, beta, seed, T, a, w, replica=0, init_v=0):
    """Cells [a, a+w) of an open road after T steps from its initial state."""
    out = np.empty(w, np.uint8)
    rc = _load().oracle_open_window_from_init(L, N, vmax, float(p), float(alpha), float(beta),
                                              seed, replica, init_v, T, a, w, _ptr(out, u8p))
    if rc:
        raise MemoryError("oracle_open_window_from_init")
    return out


FNV64_OFFSET = 14695981039346656037


def fnv1a64(data, h: int = FNV64_OFFSET) -> int:
    """64-bit FNV-1a of the bytes of `data` (any C-contiguous numpy array, in
    its in-memory little-endian layout), continuing from running hash h."""
    a = np.ascontiguousarray(data)
    b = a.view(np.uint8).reshape(-1) if a.size else np.zeros(0, np.uint8)
    return int(_load().oracle_fnv1a64(_ptr(b, u8p), b.size, h))


def num_threads_available() -> int:
    return int(_load().oracle_num_threads_available())
