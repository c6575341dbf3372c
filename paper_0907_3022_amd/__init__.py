"""chebtd: Chebyshev time propagation of quantum states on AMD MI355X.

Implements the Chebyshev expansion of the time-evolution operator of Fehske
et al., arXiv:0907.3022 (Sect. 2.2) as hand-written HIP kernels for gfx950
behind the C ABI of include/chebtd.h; this package is its Python binding.
"""
from ._lib import (ADJ_REVERSE, ADJ_SQRTM, ADJ_STEP, ARMCHAIR, GRAPH, KEEP_CHECKPOINTS, NO_CHECK,
                   NO_PERSISTENT, SCHED_DEEP, SCHED_LEVELS, SCHED_PAIRS, SCHED_PERSISTENT, SINGLE_ORDER, ZIGZAG,
                   ChebError)
from ._lib import lib as load_library
from .api import Context, holstein_csr_host, holstein_occupations, region_sum_noalloc

__all__ = [
    "Context", "ChebError", "load_library", "holstein_csr_host", "holstein_occupations", "region_sum_noalloc",
    "ZIGZAG", "ARMCHAIR", "KEEP_CHECKPOINTS", "NO_CHECK", "GRAPH", "NO_PERSISTENT", "SINGLE_ORDER",
    "SCHED_LEVELS", "SCHED_PERSISTENT", "SCHED_PAIRS", "SCHED_DEEP", "ADJ_STEP", "ADJ_SQRTM", "ADJ_REVERSE",
]


def __getattr__(name):
    # torch is imported only when the autograd wrapper is used
    if name in ("ChebPropagate", "Propagator"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
