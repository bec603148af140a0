"""CPU tests of the starter-code style I/O: the parameter-file parser and the
.npy writer (frames given from the host, read back with numpy)."""
import os

import numpy as np
import pytest

from paper_2309_14311_amd import NaschError, Writer, ini_read

EMPTY = 0xFF

# the example values of the Handout's parameter-file description
EXAMPLE_INI = """# parameter file
L = 500
T = 500
N = 300
p = 0.2        ; probability of slowing down
vmax = 2
seed = 13
outputprefix = "traffic"
per = 10
"""


def test_ini_read_handout_example(tmp_path):
    f = tmp_path / "example.ini"
    f.write_text(EXAMPLE_INI)
    d = ini_read(str(f))
    assert (d["L"], d["T"], d["N"], d["vmax"], d["seed"], d["per"]) == (500, 500, 300, 2, 13, 10)
    assert d["p"] == 0.2 and d["outputprefix"] == "traffic"


@pytest.mark.parametrize("bad", ["L = 500\nT = 5\n",                       # missing keys
                                 EXAMPLE_INI.replace("N = 300", "N = 600"),  # N > L
                                 EXAMPLE_INI.replace("p = 0.2", "p = 1.5"),
                                 EXAMPLE_INI.replace("vmax = 2", "vmax = two"),
                                 EXAMPLE_INI + "garbage line\n"])
def test_ini_read_rejects(tmp_path, bad):
    f = tmp_path / "bad.ini"
    f.write_text(bad)
    with pytest.raises(NaschError):
        ini_read(str(f))
    with pytest.raises(NaschError):
        ini_read(str(tmp_path / "missing.ini"))


def test_writer_npy_files(tmp_path):
    L = 37
    rng = np.random.default_rng(0)
    frames = []
    prefix = str(tmp_path / "out")
    w = Writer(prefix, L)
    for t in (0, 10, 20, 30):
        g = np.where(rng.random(L) < 0.3, rng.integers(0, 6, L), EMPTY).astype(np.uint8)
        frames.append((t, g))
        w.frame_host(g, t)
    w.close()
    dens = np.load(prefix + "-dens.npy")
    velo = np.load(prefix + "-velo.npy")
    time = np.load(prefix + "-time.npy")
    assert dens.shape == velo.shape == (4, L) and dens.dtype == velo.dtype == np.uint8
    assert time.dtype == np.int64 and list(time) == [0, 10, 20, 30]
    for i, (t, g) in enumerate(frames):
        assert np.array_equal(dens[i], (g != EMPTY).astype(np.uint8))
        assert np.array_equal(velo[i], np.where(g != EMPTY, g, 0))
    assert os.path.getsize(prefix + "-dens.npy") == 128 + 4 * L
