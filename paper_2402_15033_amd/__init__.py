"""MI355X-native s-step GMRES with two-stage block orthogonalization.

The numerical work runs in the HIP library ``libtsgmres.so`` (hand-written gfx950
kernels behind the C ABI of ``include/tsgmres.h``).  This package is the thin Python
binding: it marshals torch device tensors into pointers and calls the library.
PyTorch supplies device memory and streams only.

    import paper_2402_15033_amd as tsg
    A = tsg.CSRMatrix(row_ptr, col, val)              # device tensors (int32, int32, float64)
    x, info = tsg.solve(A, b, m=60, s=5, tol=1e-10)   # two-stage s-step GMRES
    Q, R = tsg.orthogonalize(X, s=5)                  # two-stage block orthogonalization
    srv = tsg.Server(arena_bytes)                      # continuous batching of many solves

There is no CPU fallback: if the library is missing, every call raises.
"""
from .binding import (  # noqa: F401
    ORTHO,
    BASIS,
    PRECISION,
    TSGError,
    CSRMatrix,
    SolveInfo,
    library_path,
    load_library,
    solve,
    solve_workspace_bytes,
    orthogonalize,
    block_pip,
    precond_apply,
    ritz_newton,
    spmv,
    Server,
)
