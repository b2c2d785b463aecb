"""MI355X (gfx950) contig generation: the five steps of the paper's Algorithm 2
(branch removal, connected components, LPT partitioning, induced subgraphs,
local assembly) as hand-written HIP kernels behind the C ABI of include/cg.h.

`cg` is the ctypes binding of that ABI.
"""
from . import cg  # noqa: F401

__all__ = ["cg"]
