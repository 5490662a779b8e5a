"""Small dense FP64 operations of the oracle (test infrastructure only).

* ``chol_upper``   -- Chol(G) of Fig. 3's caption: the upper-triangular factor R
                      with R^T R = G and a positive diagonal.
* ``givens_lsq``   -- min_y || g - H y ||_2 for an upper Hessenberg H by Givens
                      rotations (the projected least-squares problem of GMRES,
                      Sec. I/III).
* ``householder_qr`` -- LAPACK Householder QR with the sign fixed so that
                      diag(R) > 0 (the unique thin QR named in Fig. 1's caption).
* ``orth_error`` / ``repr_error`` -- ||I - Q^T Q||_F and ||X - QR||_F/||X||_F.
"""
from __future__ import annotations

import numpy as np


class CholeskyBreakdown(ArithmeticError):
    """Raised when a Gram matrix is not numerically positive definite (CholQR fails)."""


# Relative pivot threshold used where a Gram matrix is formed by subtraction (the
# block Pythagorean Gram of BCGS-PIP) and for the stage-2 Gram of a pre-processed,
# nearly orthonormal basis: a pivot d_j = R_jj^2 at or below PIVOT_TOL * ref_jj
# (ref = diagonal of the raw Gram matrix) is rounding noise, i.e. the new column is
# numerically in the span of the earlier ones.  The paper leaves this case open; the
# threshold is our reading.  It sits above the noise of a k+s <= 61 column reduction
# over a few million rows in FP64 and far below the pivots of the bases the solver
# builds.  The stand-alone block orthogonalization routines keep LAPACK's rule
# (tol = 0: fail only if not SPD); the GMRES cycles pass PIVOT_TOL.
PIVOT_TOL = 1e-12

# Relative pivot threshold of two-stage stage 1's one-reduction pass (BCGS-PIP, Fig. 4a)
# below which the panel takes the explicit second pass instead.  Sec. IV-C: the Pythagorean
# Gram G_W - P^T P keeps its accuracy only while kappa([Q, W])^2 eps stays well below 1; a
# pivot near PIVOT_TOL is then at the rounding level of the subtraction.  On the s-step
# bases this happens: the monomial basis at s = 10 (2D Laplacian, 64^2) has relative pivots
# of 5e-12..1.5e-9 whose Pythagorean values differ from the explicitly projected ones by up
# to 2e-9, so a test at PIVOT_TOL is decided by rounding and two correct implementations
# take the second pass on different panels.  Below PIP_TOL (kappa above ~1e4, kappa^2 eps
# above ~1e-8) the explicit pass is taken; that decision has four decades of margin over
# the Pythagorean pivots' rounding while they are still this large, and the bases of s <= 5
# (relative pivots >= 2e-6 measured on 64^2 .. 512^2 Laplacians, 3D Laplacians and
# convection-diffusion) never reach it.  Our reading; the paper does not treat the case.
PIP_TOL = 1e-8


def chol_upper(G: np.ndarray, ref_diag=None, tol: float = 0.0) -> np.ndarray:
    """Upper Cholesky factor R (R^T R = G, diag(R) > 0); library primitive: LAPACK potrf.

    Raises CholeskyBreakdown (with attribute ``index``, the first failing pivot) when G is
    not positive definite or a pivot R_jj^2 <= tol * ref_diag[j] (ref_diag defaults to
    diag(G)).
    """
    G = np.asarray(G, dtype=np.float64)
    Gs = 0.5 * (G + G.T)
    ref = np.diag(Gs).copy() if ref_diag is None else np.asarray(ref_diag, dtype=np.float64)
    try:
        L = np.linalg.cholesky(Gs)
    except np.linalg.LinAlgError as exc:  # not SPD in floating point
        # locate the first failing pivot on the leading blocks
        idx = 0
        for j in range(1, Gs.shape[0] + 1):
            try:
                np.linalg.cholesky(Gs[:j, :j])
            except np.linalg.LinAlgError:
                idx = j - 1
                break
        err = CholeskyBreakdown(str(exc))
        err.index = idx
        raise err from exc
    d = np.diag(L) ** 2
    bad = np.nonzero(~np.isfinite(d) | (d <= tol * ref))[0]
    if bad.size:
        err = CholeskyBreakdown("pivot below the relative threshold")
        err.index = int(bad[0])
        raise err
    return L.T.copy()


def solve_upper(R: np.ndarray, B: np.ndarray) -> np.ndarray:
    """R^{-1} B for upper-triangular R (back substitution, plain loops over columns of R)."""
    R = np.asarray(R, dtype=np.float64)
    X = np.array(B, dtype=np.float64, copy=True)
    k = R.shape[0]
    for i in range(k - 1, -1, -1):
        if i + 1 < k:
            X[i] -= R[i, i + 1:] @ X[i + 1:]
        X[i] /= R[i, i]
    return X


def right_solve_upper(M: np.ndarray, R: np.ndarray) -> np.ndarray:
    """M R^{-1} for upper-triangular R (forward substitution over the columns of R)."""
    M = np.asarray(M, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    X = np.array(M, dtype=np.float64, copy=True)
    k = R.shape[0]
    for j in range(k):
        if j > 0:
            X[..., j] -= X[..., :j] @ R[:j, j]
        X[..., j] /= R[j, j]
    return X


class GivensState:
    """Incremental Givens QR of an upper Hessenberg matrix, column by column.

    After ``add_column`` has been called for columns 0..k-1, ``residual()`` is
    |g_k|, the GMRES residual-norm estimate for the k-dimensional subspace, and
    ``solve(k)`` returns the least-squares coefficients y (length k).
    """

    def __init__(self, g0: float, kmax: int):
        self.R = np.zeros((kmax + 1, kmax))
        self.c = np.zeros(kmax)
        self.s = np.zeros(kmax)
        self.g = np.zeros(kmax + 1)
        self.g[0] = g0
        self.k = 0

    def add_column(self, h: np.ndarray) -> None:
        """h has length k+2 (entries 0..k+1 of column k of the Hessenberg matrix)."""
        k = self.k
        col = np.array(h[: k + 2], dtype=np.float64)
        for i in range(k):  # apply previous rotations
            a, b = col[i], col[i + 1]
            col[i] = self.c[i] * a + self.s[i] * b
            col[i + 1] = -self.s[i] * a + self.c[i] * b
        a, b = col[k], col[k + 1]
        rho = np.hypot(a, b)
        if rho == 0.0:
            c, s = 1.0, 0.0
        else:
            c, s = a / rho, b / rho
        self.c[k], self.s[k] = c, s
        col[k] = rho
        col[k + 1] = 0.0
        self.R[: k + 2, k] = col
        gk = self.g[k]
        self.g[k] = c * gk
        self.g[k + 1] = -s * gk
        self.k = k + 1

    def residual(self) -> float:
        return abs(self.g[self.k])

    def solve(self, k: int | None = None) -> np.ndarray:
        k = self.k if k is None else k
        return solve_upper(self.R[:k, :k], self.g[:k])


def givens_lsq(H: np.ndarray, g0: float):
    """argmin_y || g0 e_1 - H y || for (k+1) x k upper Hessenberg H.  Returns (y, residual)."""
    k = H.shape[1]
    st = GivensState(g0, k)
    for j in range(k):
        st.add_column(H[: j + 2, j])
    return st.solve(k), st.residual()


def householder_qr(X: np.ndarray):
    """Thin QR by LAPACK (Householder), signs fixed so diag(R) > 0."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def orth_error(Q: np.ndarray) -> float:
    k = Q.shape[1]
    return float(np.linalg.norm(np.eye(k) - Q.T @ Q, "fro"))


def orth_error_2(Q: np.ndarray) -> float:
    k = Q.shape[1]
    E = np.eye(k) - Q.T @ Q
    return float(np.max(np.abs(np.linalg.eigvalsh(0.5 * (E + E.T)))))


def repr_error(X: np.ndarray, Q: np.ndarray, R: np.ndarray) -> float:
    return float(np.linalg.norm(X - Q @ R, "fro") / np.linalg.norm(X, "fro"))


def cond2(X: np.ndarray) -> float:
    sv = np.linalg.svd(np.asarray(X, dtype=np.float64), compute_uv=False)
    return float(sv[0] / sv[-1]) if sv[-1] > 0 else np.inf
