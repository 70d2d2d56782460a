"""MI355X (gfx950) s-step PCG with Chebyshev basis and FGS Gram solves.

The solver and its kernels live in the HIP library libsspcg.so (C ABI in
include/sspcg.h).  Importing this package loads that library and fails if it
has not been built (python paper_2603_09790_amd/build.py); there is no CPU
fallback.
"""
from ._lib import (ERR_ARG, ERR_BREAKDOWN, ERR_HIP, ERR_NONFINITE, ERR_UNSUPPORTED,
                   ERR_WORKSPACE, EXPORTS, LIB_PATH, MAX_S, NOT_CONVERGED, OK, SSPCGError, lib)
from .solver import (Matrix, block_update_gram, csr_value_grad, diffusion7_assemble,
                     diffusion7_theta_grad, fgs, gram_rect, interval, leading_dim, mpk, pcg,
                     solve, spmv, stream_triad, xr_update)
from .autograd import DiffusionSolve, SparseSolve

lib()   # load now: a missing library is an import error, never a silent fallback
