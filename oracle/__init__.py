"""FP64 CPU oracle for s-step GMRES with two-stage block orthogonalization.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import or run anything in
this package.  The GPU library never calls it, and it shares no code with the
GPU library: the only common dependency is the ``workloads`` package, which
builds seeded inputs and holds none of the method's arithmetic.

Reference: I. Yamazaki, A. J. Higgins, E. G. Boman, D. B. Szyld,
"Two-Stage Block Orthogonalization to Improve Performance of s-step GMRES"
(arXiv:2402.15033).  Citations below name the paper's sections, equations and
figures.  The paper's pseudocode figures are not reproduced; every routine is
restated from the prose, equations and captions that define it.

Layout:
  dense.py      -- upper Cholesky factor, Givens least squares, Householder QR
                   reference, orthogonality / representation errors
  sparse.py     -- CSR sparse matrix-vector product, Gershgorin interval
  blockortho.py -- CholQR, CholQR2, BCGS, BCGS2+CholQR2, BCGS-PIP, BCGS-PIP2,
                   two-stage block orthogonalization of a tall-skinny block
  gmres.py      -- standard GMRES(m) with MGS or CGS2, and s-step GMRES(m)
                   with one-stage (BCGS2+CholQR2, BCGS-PIP2) or two-stage
                   block orthogonalization, optionally right-preconditioned
  ritz.py       -- Newton basis from Leja-ordered Ritz values
  precond.py    -- multicolor Gauss-Seidel preconditioner

Every routine is pinned by tests under ``tests/`` (``-m "not gpu"``) against
closed forms, library routines (LAPACK via numpy) and invariants the paper
states; pins are listed in each routine's docstring.
"""
from . import dense, sparse, blockortho, gmres, ritz, precond  # noqa: F401
