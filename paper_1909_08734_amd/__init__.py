"""MI355X (gfx950) Schwarz-preconditioned GMRES for the closest point method.

The solver lives in the HIP/C++ shared library ``libcpm.so`` (C ABI in
``include/cpm.h``); this package is its thin Python binding.
"""

from .binding import (  # noqa: F401
    Context, CpmError, SolveInfo, lib, selftest_tile, set_workspace_cache, workspace_cache, EXPORTED,
    OK, ENOTCONV, EINVAL, ESTATE, ENOMEM, ESINGULAR, EDEVICE, ECALLBACK,
    RAS, ORAS, FP64, FP32, PART_OCTANT, PART_RCB, PART_GRAPH, PART_ALIGN, PRECOND_TILINGS, MULTI_TILINGS,
    TIMER_PRECOND, TIMER_EXTEND, TIMER_STENCIL, TIMER_LU_GEMM, TIMER_KRYLOV, TIMER_UPDATE, PHASES,
)
