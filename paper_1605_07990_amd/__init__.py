"""Stop-and-Stare influence maximization (SSA, D-SSA) on AMD MI355X.

The method runs in the HIP library ``libim.so`` (sources in ``csrc/``, C-ABI
in ``include/im.h``); ``binding`` marshals arguments to it. There is no CPU
path: without the built library the binding raises ImportError.
"""
from .binding import (IM_IC, IM_LT, Context, Graph, ImError, Pool, Stats, derived_key,  # noqa: F401
                      load_library)

__all__ = ["IM_IC", "IM_LT", "Context", "Graph", "ImError", "Pool", "Stats", "derived_key", "load_library"]
