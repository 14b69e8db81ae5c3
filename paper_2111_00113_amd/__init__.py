"""Sketched GMRES (sGMRES) for AMD MI355X (gfx950).

Nakatsukasa & Tropp, "Fast & accurate randomized algorithms for linear systems
and eigenvalue problems" (arXiv:2111.00113), Algorithm 1 with restarting, as
hand-written HIP kernels behind a C ABI (include/sgmres.h).  This package is the
Python binding; the library is loaded lazily on first use.
"""

from .sgmres import (  # noqa: F401
    DeviceCSR,
    Plan,
    SGMRESError,
    OK,
    NOT_CONVERGED,
    FLAG_BREAKDOWN,
    FLAG_KAPPA_TRUNC,
    BASIS_ARNOLDI,
    BASIS_CHEBYSHEV,
    PREC_FP64,
    PREC_FP32,
    PREC_BF16_BASIS,
    PATH_ARNOLDI_3BAR,
    PATH_ARNOLDI_HALO,
    PATH_CHEBYSHEV,
    PATH_PART_SPLIT,
    PATH_STREAM,
    PATH_MULTI,
    LIB_PATH,
    lib,
    sgmres_solve,
    sgmres_solve_transposed,
    sgmres_solve_batched,
    sgmres_sketch_pattern,
    sgmres_sketch_apply,
    sgmres_sketch_apply_noalloc,
    sgmres_residual,
    sgmres_arnoldi_cycle,
    sgmres_chebyshev_cycle,
    sgmres_chebyshev_box,
    hessenberg_eigenvalues,
    sgmres_sketched_lsq,
    sgmres_basis_combine,
    sgmres_csr_transpose,
    sgmres_csr_outer_grad,
    sgmres_release_workspace,
    sgmres_version,
)
from .autograd import SGMRESSolve, sgmres_solve_diff  # noqa: F401,E402
