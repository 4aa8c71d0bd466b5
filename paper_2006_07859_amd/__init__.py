"""MI355X (gfx950) hot path of "Repulsive Curves": tangent-point energy and
differential, the fractional Sobolev operator, projected Sobolev gradient,
line-search step and Barnes-Hut far field, behind the C ABI of librcurves.so.

The Python side is a thin ctypes binding (:mod:`._lib`); all computation runs
in the HIP kernels of ``csrc/``.
"""

from ._lib import (  # noqa: F401
    RC_C_BARYCENTER,
    RC_C_EDGE_LENGTH,
    RC_SURFACE_SPHERE,
    RC_SURFACE_TORUS,
    RC_C_TOTAL_LENGTH,
    RC_F32,
    RC_F64,
    RC_SOLVE_DENSE,
    RC_SOLVE_PCG_JACOBI,
    RC_SOLVE_PCG_LEARNED,
    RC_SOLVE_PCG_MG,
    RC_SOLVE_MG_FMG,
    Batch,
    Context,
    Mlp,
    RcError,
    default_batch_opts,
    default_ls_opts,
    default_solve_opts,
    load,
    mlp_n_params,
)
