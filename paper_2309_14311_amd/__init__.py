"""MI355X (gfx950) implementation of the Nagel-Schreckenberg traffic-model time step.

The simulation runs in libnasch.so (hand-written HIP); `native` is its ctypes
binding.  Build with `paper_2309_14311_amd.build.build()`.
"""
from .native import (Batch, NaschError, Server, Sim, Writer, ini_read, load, LIB_PATH,  # noqa: F401
                     SYMBOLS)

__all__ = ["Sim", "Batch", "Server", "Writer", "ini_read", "NaschError", "load", "LIB_PATH",
           "SYMBOLS"]
