"""MI355X (gfx950) solvers for reversed-gradient EPI susceptibility-artifact correction on the
face-staggered grid (Macdonald & Ruthotto): GN-PCG with the block-Jacobi preconditioner and
ADMM with the line-separable SQP b-step and the DCT z-step, as HIP kernels behind the C ABI
of include/epi.h. This package is the thin Python binding over libepi.so."""
from .epi import (  # noqa: F401
    Problem, Batch, Server, EpiError, lib, to_canonical, from_canonical, gn_default_opts, admm_default_opts,
    restrict_cells, prolong_faces, solve_multilevel_admm, solve_multilevel_gnpcg, RHO_MODES,
    ML_RESTARTS, PRECOND,
    EPI_OK, EPI_EINVAL, EPI_ENOMEM, EPI_EINFEASIBLE, EPI_ENUMERIC, EPI_EHIP, EPI_ENOTSUP, EPI_EBUSY,
)
