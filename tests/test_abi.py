"""CPU checks of the C ABI: the library loads and exports every entry point that
include/nasch.h declares, the binding covers them all, and the struct layouts
of the binding match the header.  No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nasch.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(nasch_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("nasch_init", "nasch_step_n", "nasch_flux", "nasch_snapshot", "nasch_restore",
              "nasch_free", "nasch_strerror", "nasch_batch_init", "nasch_batch_step_n",
              "nasch_batch_flux_sums", "nasch_server_create", "nasch_server_submit",
              "nasch_server_poll", "nasch_server_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2309_14311_amd import native
    lib = native.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(native.SYMBOLS)


def test_exports_are_plain_c_symbols():
    from paper_2309_14311_amd import native
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in _declared():
        assert n in exported, n


def _c_sizeof(struct: str) -> int:
    src = f'#include "nasch.h"\n#include <stdio.h>\nint main(void){{printf("%zu", sizeof({struct}));return 0;}}\n'
    exe = os.path.join(ROOT, "_build", f"sizeof_{struct}")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), "-o", exe, "-"],
                   input=src, text=True, check=True)
    return int(subprocess.run([exe], capture_output=True, text=True, check=True).stdout)


@pytest.mark.parametrize("cname,pyname", [("nasch_opts", "Opts"), ("nasch_info", "Info"),
                                          ("nasch_replica", "Replica"),
                                          ("nasch_batch_opts", "BatchOpts"),
                                          ("nasch_server_opts", "ServerOpts"),
                                          ("nasch_request", "Request"),
                                          ("nasch_result", "Result")])
def test_struct_layouts_match_header(cname, pyname):
    from paper_2309_14311_amd import native
    assert ctypes.sizeof(getattr(native, pyname)) == _c_sizeof(cname)


def test_strerror_and_missing_library(tmp_path):
    from paper_2309_14311_amd import native
    native.load()
    assert native.strerror(-1) == "invalid argument"
    assert native.strerror(0) == "ok"
    # a missing library is an error, never a fallback
    native_mod = native
    saved = native_mod._lib
    try:
        native_mod._lib = None
        with pytest.raises(RuntimeError):
            native_mod.load(str(tmp_path / "nope.so"))
    finally:
        native_mod._lib = saved


def test_open_road_options_are_checked_before_any_device_call():
    """nasch_init rejects a bad boundary, an open agent road and gate
    probabilities outside [0, 1] (NaN included) with NASCH_EINVAL; the checks
    come before any HIP call, so they run without a GPU."""
    from paper_2309_14311_amd import native
    lib = native.load()
    o = native.Opts()
    lib.nasch_default_opts(ctypes.byref(o))
    assert (o.boundary, o.reserved, o.alpha, o.beta) == (0, 0, 0.0, 0.0)
    nan = float("nan")
    for boundary, rep, alpha, beta, reserved in [(2, 0, 0.5, 0.5, 0), (1, 1, 0.5, 0.5, 0),
                                                 (1, 0, 1.5, 0.5, 0), (1, 0, 0.5, -0.1, 0),
                                                 (1, 0, nan, 0.5, 0), (1, 0, 0.5, nan, 0),
                                                 (1, 0, 0.5, 0.5, 7)]:
        o.boundary, o.rep, o.alpha, o.beta, o.reserved = boundary, rep, alpha, beta, reserved
        h = ctypes.c_void_p(1)
        assert lib.nasch_init(ctypes.byref(h), 100, 10, 5, 0.1, 1, ctypes.byref(o)) == -1
        assert not h.value


def test_probe_library_exports_its_header():
    """libnasch_probe.so (the vector-ALU throughput probe) exports what
    include/nasch_probe.h declares, and the binding's result struct matches."""
    from paper_2309_14311_amd import native
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "nasch_probe.h")).read(),
                  flags=re.S)
    names = set(re.findall(r"\b(nasch_[a-z_]+)\s*\(", text))
    assert names == {"nasch_probe_valu"}
    lib = native.load_probe()
    for n in names:
        assert hasattr(lib, n)
    src = ('#include "nasch_probe.h"\n#include <stdio.h>\n'
           'int main(void){printf("%zu", sizeof(nasch_probe_result));return 0;}\n')
    exe = os.path.join(ROOT, "_build", "sizeof_probe")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), "-o", exe, "-"],
                   input=src, text=True, check=True)
    size = int(subprocess.run([exe], capture_output=True, text=True, check=True).stdout)
    assert size == ctypes.sizeof(native.ProbeResult)
