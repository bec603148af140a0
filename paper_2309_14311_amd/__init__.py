"""MI355X (gfx950) implementation of the Nagel-Schreckenberg traffic-model time step.

The simulation runs in libnasch.so (hand-written HIP); `native` is its ctypes
binding.  Build with `paper_2309_14311_amd.build.build()`.
"""
from .native import (Batch, NaschError, Server, Sim, load, LIB_PATH, SYMBOLS)  # noqa: F401

__all__ = ["Sim", "Batch", "Server", "NaschError", "load", "LIB_PATH", "SYMBOLS"]
