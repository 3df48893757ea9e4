"""Exact triangle counting over a degree-ordered oriented graph on AMD MI355X.

The computation lives in ``libtc.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/tc.h``); :mod:`paper_1406_5687_amd.tc` is its ctypes binding.
"""
from .tc import (COST_DEGREE, COST_NEW, COST_ONE, COST_PRIOR, Graph, TcError, build_oriented, count,  # noqa: F401
                 count_batch, load)

__all__ = ["build_oriented", "count", "count_batch", "Graph", "TcError", "load", "COST_ONE", "COST_DEGREE",
           "COST_PRIOR", "COST_NEW"]
