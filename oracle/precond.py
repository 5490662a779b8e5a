"""Multicolor Gauss-Seidel preconditioner of right-preconditioned s-step GMRES
(test infrastructure only).

The paper's last experiment (Sec. VI, Fig. 13) runs s-step GMRES with a local
Gauss-Seidel preconditioner -- block Jacobi with Gauss-Seidel inside each block,
applied on the GPU as a multicolor Gauss-Seidel sweep.  One GPU holds the whole
operator here, so the local block is the whole matrix.  Right preconditioning keeps
the residual GMRES minimizes equal to the true one: the Krylov space is that of
A M^{-1}, and the cycle's update is x += M^{-1} (Q y).

* ``priority``   -- the hashed priority of row i: the i-th output of the SplitMix64
                    generator seeded with 0 (Steele, Lea and Flood's generator, with
                    Vigna's published constants), ties broken by the row index.
* ``coloring``   -- distance-1 coloring of the (structurally symmetric) pattern,
                    greedy in decreasing priority: each row takes the smallest color
                    that none of its higher-priority neighbours holds.  This equals
                    the result of Jones and Plassmann's parallel rounds with the same
                    priorities, which is what a GPU computes.
* ``mcgs_apply`` -- z = M^{-1} w, M = D + L_c: the diagonal and the entries a_ij
                    whose column has a lower color than the row.  One forward
                    Gauss-Seidel sweep from z = 0 over the colors in increasing order;
                    rows of one color do not couple, so each color is one parallel
                    step.

Reading (the paper gives no preconditioner details beyond the citations): one sweep
per application, colors from the hashed priorities above, and the basis interval
[0, 2] for the preconditioned operator (for a convergent Gauss-Seidel splitting the
eigenvalues of A M^{-1} = I - (I - A M^{-1}) lie in the disc |z - 1| < 1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

PRECOND_INTERVAL = (0.0, 2.0)


def splitmix64(state: np.ndarray) -> np.ndarray:
    """SplitMix64's output function of the (already advanced) state, uint64 arithmetic."""
    z = np.asarray(state, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def priority(n: int) -> np.ndarray:
    """Priority of rows 0..n-1: output i of SplitMix64 seeded with 0 (state (i+1) gamma)."""
    with np.errstate(over="ignore"):
        st = (np.arange(1, n + 1, dtype=np.uint64) * _GAMMA).astype(np.uint64)
    return splitmix64(st)


def _neighbours(A):
    M = sp.csr_matrix((np.ones_like(A.val), A.col, A.row_ptr), shape=(A.n, A.n))
    S = (M + M.T).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    return S


def coloring(A) -> np.ndarray:
    """Greedy coloring in decreasing (priority, index) order; int32 colors."""
    n = A.n
    pr = priority(n)
    order = np.argsort(pr, kind="stable")[::-1]  # decreasing priority, equal: higher index first
    S = _neighbours(A)
    colors = np.full(n, -1, dtype=np.int64)
    for i in order:
        nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
        taken = set(int(c) for c in colors[nb] if c >= 0)
        c = 0
        while c in taken:
            c += 1
        colors[i] = c
    return colors.astype(np.int32)


def mcgs_apply(A, colors: np.ndarray, w: np.ndarray) -> np.ndarray:
    """z = (D + L_c)^{-1} w by one forward multicolor Gauss-Seidel sweep from z = 0."""
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    d = M.diagonal()
    off = (M - sp.diags(d)).tocsr()
    z = np.zeros(A.n)
    w = np.asarray(w, dtype=np.float64)
    for c in range(int(colors.max()) + 1 if len(colors) else 0):
        rows = np.nonzero(colors == c)[0]
        z[rows] = (w[rows] - off[rows] @ z) / d[rows]
    return z


class MulticolorGS:
    """The preconditioner object the solvers take: apply(w) = M^{-1} w."""

    def __init__(self, A):
        self.A = A
        self.colors = coloring(A)
        self.ncolors = int(self.colors.max()) + 1

    def apply(self, w: np.ndarray) -> np.ndarray:
        return mcgs_apply(self.A, self.colors, w)
