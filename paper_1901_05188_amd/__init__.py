"""MI355X GenEO-preconditioned CG (Butler et al., arXiv 1901.05188) behind a C ABI.

The compute path is libgenpcg.so (HIP, gfx950); :mod:`.binding` only marshals
arguments.  Build it with ``python -m paper_1901_05188_amd.build_lib`` or
``__graft_entry__.build()``.
"""
from .binding import (Problem, Preconditioner, Server, solve, footprint, resident_bytes, profile_enable, profile_read, trim_memory,
                      lib, GenPCGError, EXPORTS, LIB_PATH)

__all__ = ["Problem", "Preconditioner", "Server", "solve", "footprint", "resident_bytes", "profile_enable", "profile_read", "trim_memory",
           "lib", "GenPCGError", "EXPORTS", "LIB_PATH"]
