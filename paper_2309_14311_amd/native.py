"""ctypes binding of libnasch (include/nasch.h): same names, argument marshalling only.

Every step of the simulation runs in the HIP library; this module only converts
Python values and numpy buffers to the C ABI.  There is no fallback: if the
library is missing or fails to load, `load()` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnasch.so")
_lib = None

NASCH_OK, NASCH_EINVAL, NASCH_ENOMEM, NASCH_EDEVICE = 0, -1, -2, -3
NASCH_ERANGE, NASCH_ESTATE, NASCH_EBUSY, NASCH_ENOTFOUND = -4, -5, -6, -7
REP = {"grid": 0, "agent": 1}
KERNEL = {"auto": 0, "onestep": 1, "kstep": 2}
RNG = {"keyed": 0, "stream": 1}
BOUNDARY = {"ring": 0, "open": 1}
EMPTY = 0xFF

u8p = ctypes.POINTER(ctypes.c_uint8)
i32p = ctypes.POINTER(ctypes.c_int32)
u32p = ctypes.POINTER(ctypes.c_uint32)
u64p = ctypes.POINTER(ctypes.c_uint64)
f64p = ctypes.POINTER(ctypes.c_double)
vpp = ctypes.POINTER(ctypes.c_void_p)
U32, U64, I32, DBL, VP = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p


class Opts(ctypes.Structure):
    _fields_ = [("replica", U32), ("rep", U32), ("init_v", U32), ("kernel", U32), ("k", U32),
                ("q", U32), ("use_graph", U32), ("rng", U32), ("stream", VP),
                ("boundary", U32), ("reserved", U32), ("alpha", DBL), ("beta", DBL)]


class Info(ctypes.Structure):
    _fields_ = [("L", U64), ("N", U64), ("t", U64), ("vmax", U32), ("thr", U32),
                ("replica", U32), ("rep", U32), ("init_v", U32), ("kernel", U32), ("k", U32),
                ("q", U32), ("seed", U64), ("device_bytes", U64)]


class Replica(ctypes.Structure):
    _fields_ = [("L", U64), ("N", U64), ("vmax", U32), ("init_v", U32), ("p", DBL),
                ("seed", U64), ("replica", U32), ("reserved", U32), ("warmup", U64),
                ("boundary", U32), ("reserved2", U32), ("alpha", DBL), ("beta", DBL)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("stream", VP), ("k", U32), ("q", U32), ("use_graph", U32), ("keep_log", U32),
                ("log_steps", U64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", U64), ("max_slots", U32), ("k", U32), ("q", U32),
                ("reserved", U32), ("stream", VP)]


class Request(ctypes.Structure):
    _fields_ = [("L", U64), ("N", U64), ("vmax", U32), ("init_v", U32), ("p", DBL),
                ("seed", U64), ("replica", U32), ("reserved", U32), ("T", U64),
                ("flux_out", u64p), ("grid_out", u8p)]


class Ini(ctypes.Structure):
    _fields_ = [("L", U64), ("T", U64), ("N", U64), ("p", DBL), ("vmax", U32),
                ("reserved", U32), ("seed", U64), ("per", U64),
                ("outputprefix", ctypes.c_char * 256)]


class Result(ctypes.Structure):
    _fields_ = [("id", U64), ("status", ctypes.c_int32), ("reserved", U32), ("flux_sum", U64),
                ("t_submit", DBL), ("t_admit", DBL), ("t_done", DBL)]


_SIGS = {
    "nasch_default_opts": (None, [ctypes.POINTER(Opts)]),
    "nasch_init": (I32, [vpp, U64, U64, U32, DBL, U64, ctypes.POINTER(Opts)]),
    "nasch_step_n": (I32, [VP, U64]),
    "nasch_reserve_log": (I32, [VP, U64]),
    "nasch_timed_step_n": (I32, [VP, U64, f64p]),
    "nasch_flux": (I32, [VP, U64, U64, u64p]),
    "nasch_snapshot": (I32, [VP, u8p, u64p]),
    "nasch_snapshot_range": (I32, [VP, U64, U64, u8p]),
    "nasch_agent_state": (I32, [VP, i32p, u8p]),
    "nasch_restore": (I32, [VP, u8p, U64]),
    "nasch_restore_agent": (I32, [VP, i32p, u8p, U64]),
    "nasch_set_tuning": (I32, [VP, U32, U32, U32]),
    "nasch_autotune": (I32, [VP]),
    "nasch_get_info": (I32, [VP, ctypes.POINTER(Info)]),
    "nasch_last_device_error": (I32, [VP]),
    "nasch_thread_last_device_error": (I32, []),
    "nasch_free": (None, [VP]),
    "nasch_strerror": (ctypes.c_char_p, [I32]),
    "nasch_batch_default_opts": (None, [ctypes.POINTER(BatchOpts)]),
    "nasch_batch_init": (I32, [vpp, ctypes.POINTER(Replica), U32, ctypes.POINTER(BatchOpts)]),
    "nasch_batch_reset": (I32, [VP]),
    "nasch_batch_step_n": (I32, [VP, U64]),
    "nasch_batch_timed_step_n": (I32, [VP, U64, f64p]),
    "nasch_batch_flux_sums": (I32, [VP, u64p]),
    "nasch_batch_flux": (I32, [VP, U32, U64, U64, u64p]),
    "nasch_batch_snapshot": (I32, [VP, U32, u8p, u64p]),
    "nasch_batch_snapshot_all": (I32, [VP, u8p, u64p]),
    "nasch_batch_restore": (I32, [VP, u8p, U64]),
    "nasch_batch_autotune": (I32, [VP, u32p, u32p]),
    "nasch_batch_set_tuning": (I32, [VP, U32, U32]),
    "nasch_batch_last_device_error": (I32, [VP]),
    "nasch_batch_free": (None, [VP]),
    "nasch_server_default_opts": (None, [ctypes.POINTER(ServerOpts)]),
    "nasch_server_create": (I32, [vpp, ctypes.POINTER(ServerOpts)]),
    "nasch_server_submit": (I32, [VP, ctypes.POINTER(Request), u64p]),
    "nasch_server_poll": (I32, [VP, ctypes.POINTER(Result), U32, u32p, U32]),
    "nasch_server_cancel": (I32, [VP, U64]),
    "nasch_server_stats": (I32, [VP, u64p, u64p, u64p, u64p, u64p]),
    "nasch_server_now": (DBL, [VP]),
    "nasch_server_health": (I32, [VP, ctypes.POINTER(ctypes.c_double), u64p]),
    "nasch_server_destroy": (None, [VP]),
    "nasch_ini_read": (I32, [ctypes.c_char_p, ctypes.POINTER(Ini)]),
    "nasch_writer_open": (I32, [vpp, ctypes.c_char_p, U64]),
    "nasch_writer_frame": (I32, [VP, VP]),
    "nasch_writer_frame_host": (I32, [VP, u8p, U64]),
    "nasch_writer_close": (I32, [VP]),
    "nasch_grid_step_device": (I32, [VP, VP, U64, U32, DBL, U64, U32, U64, VP, VP]),
    "nasch_grid_step_device_noalloc": (I32, [VP, VP, U64, U32, DBL, U64, U32, U64, VP, VP]),
}

SYMBOLS = tuple(_SIGS)


class NaschError(RuntimeError):
    def __init__(self, code: int, where: str, device_error: int = 0):
        msg = f"{where}: {strerror(code)} ({code})"
        if device_error:
            msg += f", hipError {device_error}"
        super().__init__(msg)
        self.code = code
        self.device_error = device_error


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnasch.so.  torch is imported first so that the library binds to the
    HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnasch.so not built ({path}); run python -m paper_2309_14311_amd.build")
    import torch  # noqa: F401  (shares its libamdhip64 with the library)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    if _lib is None:
        return {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "HIP device error",
                -4: "step counter would reach 2^32", -5: "invalid state for this call",
                -6: "busy", -7: "not found"}.get(code, "unknown status")
    return _lib.nasch_strerror(code).decode()


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


def _u8(a):
    return a.ctypes.data_as(u8p)


def _u64(a):
    return a.ctypes.data_as(u64p)


class Sim:
    """One ring (nasch_init ... nasch_free)."""

    def __init__(self, L, N, vmax, p, seed, *, replica=0, rep="grid", init_v=0, kernel="auto",
                 k=0, q=0, use_graph=False, stream=None, rng="keyed", boundary="ring",
                 alpha=0.0, beta=0.0):
        lib = load()
        o = Opts()
        lib.nasch_default_opts(ctypes.byref(o))
        o.replica, o.rep, o.init_v, o.rng = replica, REP[rep], int(init_v), RNG[rng]
        o.boundary, o.alpha, o.beta = BOUNDARY[boundary], float(alpha), float(beta)
        o.kernel, o.k, o.q, o.use_graph = KERNEL[kernel], k, q, int(bool(use_graph))
        o.stream = _stream_ptr(stream)
        h = VP()
        rc = lib.nasch_init(ctypes.byref(h), L, N, vmax, float(p), seed, ctypes.byref(o))
        if rc:
            raise NaschError(rc, "nasch_init", lib.nasch_thread_last_device_error())
        self._h = h
        self.L, self.N, self.vmax, self.p, self.seed = L, N, vmax, p, seed
        self.replica, self.rep = replica, rep
        self.boundary, self.alpha, self.beta = boundary, alpha, beta

    def _check(self, rc, where):
        if rc:
            raise NaschError(rc, where, _lib.nasch_last_device_error(self._h))

    def step(self, T: int):
        self._check(_lib.nasch_step_n(self._h, T), "nasch_step_n")

    def reserve_log(self, steps: int):
        self._check(_lib.nasch_reserve_log(self._h, steps), "nasch_reserve_log")

    def timed_step(self, T: int) -> float:
        ms = ctypes.c_double()
        self._check(_lib.nasch_timed_step_n(self._h, T, ctypes.byref(ms)), "nasch_timed_step_n")
        return ms.value

    def flux(self, t0: int, count: int) -> np.ndarray:
        out = np.zeros(count, np.uint64)
        self._check(_lib.nasch_flux(self._h, t0, count, _u64(out)), "nasch_flux")
        return out

    def snapshot(self):
        out = np.empty(self.L, np.uint8)
        t = ctypes.c_uint64()
        self._check(_lib.nasch_snapshot(self._h, _u8(out), ctypes.byref(t)), "nasch_snapshot")
        return out, t.value

    def snapshot_range(self, start: int, length: int) -> np.ndarray:
        out = np.empty(length, np.uint8)
        self._check(_lib.nasch_snapshot_range(self._h, start, length, _u8(out)),
                    "nasch_snapshot_range")
        return out

    def agent_state(self):
        x = np.empty(self.N, np.int32)
        v = np.empty(self.N, np.uint8)
        self._check(_lib.nasch_agent_state(self._h, x.ctypes.data_as(i32p), _u8(v)),
                    "nasch_agent_state")
        return x, v

    def restore(self, grid: np.ndarray, t: int):
        g = np.ascontiguousarray(grid, dtype=np.uint8)
        self._check(_lib.nasch_restore(self._h, _u8(g), t), "nasch_restore")

    def restore_agent(self, x: np.ndarray, v: np.ndarray, t: int):
        xa = np.ascontiguousarray(x, dtype=np.int32)
        va = np.ascontiguousarray(v, dtype=np.uint8)
        self._check(_lib.nasch_restore_agent(self._h, xa.ctypes.data_as(i32p), _u8(va), t),
                    "nasch_restore_agent")

    def set_tuning(self, kernel="kstep", k=0, q=0):
        self._check(_lib.nasch_set_tuning(self._h, KERNEL[kernel], k, q), "nasch_set_tuning")

    def autotune(self):
        self._check(_lib.nasch_autotune(self._h), "nasch_autotune")

    def info(self) -> dict:
        i = Info()
        self._check(_lib.nasch_get_info(self._h, ctypes.byref(i)), "nasch_get_info")
        return {f: getattr(i, f) for f, _ in Info._fields_}

    @property
    def t(self) -> int:
        return self.info()["t"]

    def close(self):
        if getattr(self, "_h", None):
            _lib.nasch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many replicas advanced together (nasch_batch_*)."""

    def __init__(self, replicas, *, k=0, q=0, use_graph=False, keep_log=False, log_steps=0,
                 stream=None):
        lib = load()
        arr = (Replica * len(replicas))()
        for i, r in enumerate(replicas):
            arr[i].L, arr[i].N, arr[i].vmax = r["L"], r["N"], r["vmax"]
            arr[i].init_v, arr[i].p, arr[i].seed = int(r.get("init_v", 0)), float(r["p"]), r["seed"]
            arr[i].replica, arr[i].warmup = r.get("replica", 0), r.get("warmup", 0)
            arr[i].boundary = BOUNDARY[r.get("boundary", "ring")]
            arr[i].alpha, arr[i].beta = float(r.get("alpha", 0.0)), float(r.get("beta", 0.0))
        o = BatchOpts()
        lib.nasch_batch_default_opts(ctypes.byref(o))
        o.stream, o.k, o.q = _stream_ptr(stream), k, q
        o.use_graph, o.keep_log, o.log_steps = int(bool(use_graph)), int(bool(keep_log)), log_steps
        h = VP()
        rc = lib.nasch_batch_init(ctypes.byref(h), arr, len(replicas), ctypes.byref(o))
        if rc:
            raise NaschError(rc, "nasch_batch_init", lib.nasch_thread_last_device_error())
        self._h = h
        self.replicas = list(replicas)
        self.R = len(replicas)

    def _check(self, rc, where):
        if rc:
            raise NaschError(rc, where, _lib.nasch_batch_last_device_error(self._h))

    def reset(self):
        self._check(_lib.nasch_batch_reset(self._h), "nasch_batch_reset")

    def step(self, T):
        self._check(_lib.nasch_batch_step_n(self._h, T), "nasch_batch_step_n")

    def timed_step(self, T) -> float:
        ms = ctypes.c_double()
        self._check(_lib.nasch_batch_timed_step_n(self._h, T, ctypes.byref(ms)),
                    "nasch_batch_timed_step_n")
        return ms.value

    def flux_sums(self) -> np.ndarray:
        out = np.zeros(self.R, np.uint64)
        self._check(_lib.nasch_batch_flux_sums(self._h, _u64(out)), "nasch_batch_flux_sums")
        return out

    def flux(self, r, t0, count) -> np.ndarray:
        out = np.zeros(count, np.uint64)
        self._check(_lib.nasch_batch_flux(self._h, r, t0, count, _u64(out)), "nasch_batch_flux")
        return out

    def snapshot(self, r):
        out = np.empty(self.replicas[r]["L"], np.uint8)
        t = ctypes.c_uint64()
        self._check(_lib.nasch_batch_snapshot(self._h, r, _u8(out), ctypes.byref(t)),
                    "nasch_batch_snapshot")
        return out, t.value

    def snapshot_all(self):
        """Every replica's grid back to back (replica order) and the step count."""
        out = np.empty(sum(r["L"] for r in self.replicas), np.uint8)
        t = ctypes.c_uint64()
        self._check(_lib.nasch_batch_snapshot_all(self._h, _u8(out), ctypes.byref(t)),
                    "nasch_batch_snapshot_all")
        return out, t.value

    def restore(self, grids, t):
        """Set every replica's grid (back to back, as snapshot_all returns them) and
        the step count."""
        g = np.ascontiguousarray(grids, dtype=np.uint8)
        if g.size != sum(r["L"] for r in self.replicas):
            raise ValueError("grids must hold every replica's L cells back to back")
        self._check(_lib.nasch_batch_restore(self._h, _u8(g), t), "nasch_batch_restore")

    def autotune(self):
        k, q = ctypes.c_uint32(), ctypes.c_uint32()
        self._check(_lib.nasch_batch_autotune(self._h, ctypes.byref(k), ctypes.byref(q)),
                    "nasch_batch_autotune")
        return k.value, q.value

    def set_tuning(self, k=0, q=0):
        self._check(_lib.nasch_batch_set_tuning(self._h, k, q), "nasch_batch_set_tuning")

    def close(self):
        if getattr(self, "_h", None):
            _lib.nasch_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (nasch_server_*)."""

    def __init__(self, *, hbm_budget=0, max_slots=0, k=0, q=0, stream=None):
        lib = load()
        o = ServerOpts()
        lib.nasch_server_default_opts(ctypes.byref(o))
        o.hbm_budget, o.max_slots, o.k, o.q = hbm_budget, max_slots, k, q
        o.stream = _stream_ptr(stream)
        h = VP()
        rc = lib.nasch_server_create(ctypes.byref(h), ctypes.byref(o))
        if rc:
            raise NaschError(rc, "nasch_server_create", lib.nasch_thread_last_device_error())
        self._h = h
        self._bufs = {}

    def submit(self, L, N, vmax, p, seed, T, *, replica=0, init_v=0, want_flux=True,
               want_grid=False) -> int:
        r = Request()
        r.L, r.N, r.vmax, r.init_v, r.p, r.seed = L, N, vmax, int(init_v), float(p), seed
        r.replica, r.T = replica, T
        flux = np.zeros(T, np.uint64) if want_flux else None
        grid = np.empty(L, np.uint8) if want_grid else None
        r.flux_out = _u64(flux) if flux is not None else None
        r.grid_out = _u8(grid) if grid is not None else None
        rid = ctypes.c_uint64()
        rc = _lib.nasch_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if rc:
            raise NaschError(rc, "nasch_server_submit")
        self._bufs[rid.value] = (flux, grid)
        return rid.value

    def poll(self, max_results=256, wait_ms=0):
        out = (Result * max_results)()
        n = ctypes.c_uint32()
        rc = _lib.nasch_server_poll(self._h, out, max_results, ctypes.byref(n), wait_ms)
        if rc:
            raise NaschError(rc, "nasch_server_poll")
        res = []
        for i in range(n.value):
            r = out[i]
            flux, grid = self._bufs.pop(r.id, (None, None))
            res.append({"id": r.id, "status": r.status, "flux_sum": r.flux_sum,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "flux": flux, "grid": grid})
        return res

    def cancel(self, rid):
        rc = _lib.nasch_server_cancel(self._h, rid)
        if rc:
            raise NaschError(rc, "nasch_server_cancel")

    def stats(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(5)]
        rc = _lib.nasch_server_stats(self._h, *[ctypes.byref(x) for x in v])
        if rc:
            raise NaschError(rc, "nasch_server_stats")
        return dict(zip(["pending", "running", "done", "bytes_in_use", "launches"],
                        [x.value for x in v]))

    def now(self) -> float:
        return _lib.nasch_server_now(self._h)

    def health(self) -> dict:
        """Seconds since the scheduling thread last made progress (0 when idle)
        and the requests queued or running: a watchdog's view."""
        since, live = ctypes.c_double(), ctypes.c_uint64()
        rc = _lib.nasch_server_health(self._h, ctypes.byref(since), ctypes.byref(live))
        if rc:
            raise NaschError(rc, "nasch_server_health")
        return {"since_progress_s": since.value, "live": live.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.nasch_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ini_read(path: str) -> dict:
    """Parse a starter-code parameter file (nasch_ini_read)."""
    lib = load()
    ini = Ini()
    rc = lib.nasch_ini_read(os.fsencode(path), ctypes.byref(ini))
    if rc:
        raise NaschError(rc, f"nasch_ini_read({path})")
    d = {f: getattr(ini, f) for f, _ in Ini._fields_ if f not in ("reserved",)}
    d["outputprefix"] = ini.outputprefix.decode()
    return d


class Writer:
    """<prefix>-dens/velo/time.npy output (nasch_writer_*)."""

    def __init__(self, prefix: str, L: int):
        lib = load()
        h = VP()
        rc = lib.nasch_writer_open(ctypes.byref(h), os.fsencode(prefix), L)
        if rc:
            raise NaschError(rc, "nasch_writer_open")
        self._h = h
        self.L = L

    def frame(self, sim: "Sim"):
        rc = _lib.nasch_writer_frame(self._h, sim._h)
        if rc:
            raise NaschError(rc, "nasch_writer_frame")

    def frame_host(self, grid: np.ndarray, t: int):
        g = np.ascontiguousarray(grid, dtype=np.uint8)
        assert g.size == self.L
        rc = _lib.nasch_writer_frame_host(self._h, _u8(g), t)
        if rc:
            raise NaschError(rc, "nasch_writer_frame_host")

    def close(self):
        if getattr(self, "_h", None):
            rc = _lib.nasch_writer_close(self._h)
            self._h = None
            if rc:
                raise NaschError(rc, "nasch_writer_close")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- device buffers
def _dptr(x) -> int | None:
    """A device address: an int, or a tensor's data pointer (None for None)."""
    if x is None:
        return None
    return x if isinstance(x, int) else x.data_ptr()


def grid_step_device(d_in, d_out, L, vmax, p, seed, t, *, d_flux=None, replica=0, stream=None):
    """nasch_grid_step_device: step t of the road in device buffer d_in into
    d_out (device addresses or torch uint8 tensors); F(t) into d_flux (a device
    uint64, optional).  Asynchronous on `stream`."""
    lib = load()
    rc = lib.nasch_grid_step_device(_dptr(d_in), _dptr(d_out), L, vmax, p, seed, replica, t,
                                    _dptr(d_flux), _stream_ptr(stream))
    if rc:
        raise NaschError(rc, "nasch_grid_step_device", lib.nasch_thread_last_device_error())


def grid_step_device_noalloc(d_in, d_out, L, vmax, p, seed, t, *, d_flux=None, replica=0,
                             stream=None):
    """nasch_grid_step_device_noalloc: grid_step_device with no allocation (the
    flux partials live in the library's static device scratch)."""
    lib = load()
    rc = lib.nasch_grid_step_device_noalloc(_dptr(d_in), _dptr(d_out), L, vmax, p, seed,
                                            replica, t, _dptr(d_flux), _stream_ptr(stream))
    if rc:
        raise NaschError(rc, "nasch_grid_step_device_noalloc",
                         lib.nasch_thread_last_device_error())


# --------------------------------------------------------------------------- measurement
PROBE_PATH = os.path.join(_PKG, "libnasch_probe.so")
PROBE_KINDS = {"bitop3": 0, "alignbit": 1, "bcnt": 2, "mul_lo": 3, "mul_hi": 4, "mad_u64": 5,
               "dpp": 6, "add": 7, "xor": 8, "shift": 9, "lshl_or": 10, "perm": 11,
               "mul_u24": 12, "add_u64": 13, "min": 14, "sub": 15, "cndmask": 16, "and_or": 17,
               "bfi": 18, "or": 19, "and": 20, "add3": 21}
_probe = None


class ProbeResult(ctypes.Structure):
    _fields_ = [("ms", DBL), ("wave_instructions", DBL), ("lane_ops_per_s", DBL),
                ("sclk_hz", DBL)]


def load_probe(path: str = PROBE_PATH) -> ctypes.CDLL:
    """Load libnasch_probe.so (include/nasch_probe.h), after torch's HIP runtime."""
    global _probe
    if _probe is not None:
        return _probe
    if not os.path.exists(path):
        raise RuntimeError(f"libnasch_probe.so not built ({path}); run python -m "
                           "paper_2309_14311_amd.build")
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    lib.nasch_probe_valu.restype = I32
    lib.nasch_probe_valu.argtypes = [U32, U32, U32, ctypes.POINTER(ProbeResult)]
    _probe = lib
    return lib


def probe_valu(kind: str, blocks: int, iters: int) -> dict:
    """nasch_probe_valu: sustained issue rate of one vector-ALU instruction kind."""
    r = ProbeResult()
    rc = load_probe().nasch_probe_valu(PROBE_KINDS[kind], blocks, iters, ctypes.byref(r))
    if rc:
        raise RuntimeError(f"nasch_probe_valu({kind}): status {rc}")
    return {"ms": r.ms, "wave_instructions": r.wave_instructions,
            "lane_ops_per_s": r.lane_ops_per_s, "sclk_hz": r.sclk_hz}
