"""Seeded generators for the synthetic workloads.

Operators (CSR, int32 indices, float64 values, sorted column indices,
lexicographic unknown ordering with x fastest):

* ``laplace2d(N)``  -- unscaled 5-point Dirichlet Laplacian on an N x N grid
  (diagonal 4, off-diagonals -1), the paper's 2D model problem
  (Sec. VII, Tables 2-3).
* ``laplace3d(N)``  -- unscaled 7-point Dirichlet Laplacian on N^3
  (diagonal 6, off-diagonals -1), the 3D model problem of Table 4.
* ``convdiff2d(N, pe, theta)`` -- -Lap(u) + beta . grad(u) on the unit square,
  Dirichlet, h = 1/(N+1), first-order upwind convection, multiplied by h^2;
  beta = pe * (cos theta, sin theta).  Per axis with velocity component c the
  three-point row is  [-1 - h*max(c,0),  2 + h*|c|,  -1 + h*min(c,0)].
  (Not in the paper; a nonsymmetric stand-in for its SuiteSparse inputs.)

* ``variable_width(n, seed, far, symmetric)`` -- random diagonally dominant operator
  whose rows hold 1 .. 20 nonzeros: rows 64 j .. 64 j + 63 have at most 1 + (j mod 20)
  (reached by the first of them), so consecutive 64-row slices of a packed layout take
  every width from 1 to 20.  Off-diagonal columns lie within 60 of the row
  (``far=False``) or anywhere (``far=True``); ``symmetric=True`` symmetrizes the pattern
  (row lengths then vary further).  Off-diagonal values U(-1, 1); the diagonal is the
  row's absolute off-diagonal sum plus 1.  (A test operator, not a paper workload.)

Dense test blocks for the block orthogonalization experiments (Sec. VI):

* ``gaussian_block``  -- i.i.d. N(0,1) entries (well conditioned).
* ``logscaled_block`` -- X diag(logspace) Y^T with random orthonormal X, Y
  (the "Logscaled" matrix of Fig. 6).
* ``glued_block``     -- panels of s columns whose own condition number is
  about kappa_p while the condition number of the first j panels grows like
  2^(j-1) kappa_p (our construction of the "glued" matrix of Figs. 7-8; the
  paper does not print its recipe).

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _assemble(n: int, cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> CSR:
    """cols/vals/mask have shape (n, w) with columns already sorted per row."""
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 index range")
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col, val)


def _stencil_2d(N: int, west, east, south, north, diag) -> CSR:
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    i = idx % N
    j = idx // N
    cols = np.stack([idx - N, idx - 1, idx, idx + 1, idx + N], axis=1)
    vals = np.empty((n, 5), dtype=np.float64)
    vals[:, 0] = south
    vals[:, 1] = west
    vals[:, 2] = diag
    vals[:, 3] = east
    vals[:, 4] = north
    mask = np.stack([j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1], axis=1)
    return _assemble(n, cols, vals, mask)


def laplace2d(N: int) -> CSR:
    return _stencil_2d(N, -1.0, -1.0, -1.0, -1.0, 4.0)


def laplace3d(N: int) -> CSR:
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    i = idx % N
    j = (idx // N) % N
    k = idx // (N * N)
    NN = N * N
    cols = np.stack([idx - NN, idx - N, idx - 1, idx, idx + 1, idx + N, idx + NN], axis=1)
    vals = np.full((n, 7), -1.0)
    vals[:, 3] = 6.0
    mask = np.stack([k > 0, j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1, k < N - 1], axis=1)
    return _assemble(n, cols, vals, mask)


def convdiff2d(N: int, pe: float, theta: float) -> CSR:
    h = 1.0 / (N + 1)
    bx = pe * np.cos(theta)
    by = pe * np.sin(theta)
    west = -1.0 - h * max(bx, 0.0)
    east = -1.0 + h * min(bx, 0.0)
    south = -1.0 - h * max(by, 0.0)
    north = -1.0 + h * min(by, 0.0)
    diag = 4.0 + h * (abs(bx) + abs(by))
    return _stencil_2d(N, west, east, south, north, diag)


def variable_width(n: int, seed: int, far: bool = False, symmetric: bool = False) -> CSR:
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        w = 1 + (i // 64) % 20
        L = w if i % 64 == 0 else int(rng.integers(1, w + 1))
        if L > 1:
            if far:
                pool = rng.choice(n - 1, size=L - 1, replace=False)
                c = np.where(pool >= i, pool + 1, pool)  # skip the diagonal
            else:
                lo, hi = max(0, i - 60), min(n - 1, i + 60)
                pool = np.array([j for j in range(lo, hi + 1) if j != i])
                c = rng.choice(pool, size=min(L - 1, pool.size), replace=False)
            rows.append(np.full(c.size, i))
            cols.append(c)
    r = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
    off = sp.csr_matrix((rng.uniform(-1.0, 1.0, r.size), (r, c)), shape=(n, n))
    if symmetric:
        off = off + off.T
    off = off.tocsr()
    off.sum_duplicates()
    M = (off + sp.diags(np.asarray(abs(off).sum(axis=1)).ravel() + 1.0)).tocsr()
    M.sort_indices()
    return CSR(n=n, row_ptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32),
               val=M.data.astype(np.float64))


def convdiff_params(seed: int, pe_lo: float = 10.0, pe_hi: float = 100.0):
    """(Peclet number, flow angle) drawn from the seed: Pe ~ U[pe_lo, pe_hi], theta ~ U[0, 2pi)."""
    rng = np.random.default_rng(seed)
    pe = float(rng.uniform(pe_lo, pe_hi))
    theta = float(rng.uniform(0.0, 2.0 * np.pi))
    return pe, theta


def uniform_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def rhs_from_solution(A: CSR, x: np.ndarray) -> np.ndarray:
    """b = A x, formed once in float64 by scipy and handed to every solver as data."""
    return np.asarray(A.to_scipy() @ x, dtype=np.float64)


def make_problem(kind: str, N: int, seed: int = 0, rhs: str = "solution",
                 pe_range=(10.0, 100.0)):
    """Build one synthetic linear system.

    kind: 'laplace2d' | 'laplace3d' | 'convdiff2d'.
    rhs:  'solution' -> x_true ~ U(-1,1), b = A x_true;  'uniform' -> b ~ U(-1,1).
    Returns dict(A=CSR, b=..., x_true=... or None, meta=...).
    """
    meta = {"kind": kind, "N": N, "seed": seed}
    if kind == "laplace2d":
        A = laplace2d(N)
    elif kind == "laplace3d":
        A = laplace3d(N)
    elif kind == "convdiff2d":
        pe, theta = convdiff_params(seed + 7919, *pe_range)
        meta.update(pe=pe, theta=theta)
        A = convdiff2d(N, pe, theta)
    else:
        raise ValueError(kind)
    if rhs == "solution":
        x_true = uniform_vector(A.n, seed)
        b = rhs_from_solution(A, x_true)
    elif rhs == "uniform":
        x_true = None
        b = uniform_vector(A.n, seed)
    else:
        raise ValueError(rhs)
    return {"A": A, "b": b, "x_true": x_true, "meta": meta}


# ---------------------------------------------------------------- closed forms
def laplace_eigpair_2d(N: int, a: int, c: int):
    """Eigenpair (lambda, u) of laplace2d(N) for sine mode (a, c), 1 <= a, c <= N."""
    t = np.pi / (N + 1)
    p = np.arange(1, N + 1)
    ux = np.sin(a * p * t)
    uy = np.sin(c * p * t)
    u = np.outer(uy, ux).reshape(-1)  # index = (px-1) + N*(py-1)
    lam = 4.0 - 2.0 * np.cos(a * t) - 2.0 * np.cos(c * t)
    return lam, u


def laplace_eigpair_3d(N: int, a: int, c: int, d: int):
    t = np.pi / (N + 1)
    p = np.arange(1, N + 1)
    ux, uy, uz = np.sin(a * p * t), np.sin(c * p * t), np.sin(d * p * t)
    u = (uz[:, None, None] * uy[None, :, None] * ux[None, None, :]).reshape(-1)
    lam = 6.0 - 2.0 * (np.cos(a * t) + np.cos(c * t) + np.cos(d * t))
    return lam, u


def laplace_extreme_eigs(N: int, dim: int):
    """(lambda_min, lambda_max) of the unscaled Dirichlet Laplacian (SPD)."""
    lmin = 4.0 * dim * np.sin(np.pi / (2.0 * (N + 1))) ** 2
    return lmin, 4.0 * dim - lmin


# ---------------------------------------------------------------- dense blocks
def gaussian_block(n: int, k: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n x k i.i.d. N(0,1), returned column-major (Fortran order)."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, k), dtype=dtype, order="F")
    for c in range(k):
        X[:, c] = rng.standard_normal(n)
    return X


def _random_orthonormal(rng, n: int, k: int) -> np.ndarray:
    Z = rng.standard_normal((n, k))
    Qz, Rz = np.linalg.qr(Z)
    return Qz * np.sign(np.diag(Rz))


def logscaled_block(n: int, k: int, kappa: float, seed: int) -> np.ndarray:
    """X diag(logspace(0, -log10 kappa, k)) Y^T with random orthonormal X (n x k), Y (k x k)."""
    rng = np.random.default_rng(seed)
    X = _random_orthonormal(rng, n, k)
    Y = _random_orthonormal(rng, k, k)
    sig = np.logspace(0.0, -np.log10(kappa), k)
    return np.asfortranarray((X * sig) @ Y.T)


def glued_block(n: int, npanels: int, s: int, kappa_p: float, seed: int, alpha: float = 0.1,
                lead: bool = True) -> np.ndarray:
    """Glued test matrix V = X K S, returned column-major.

    X (n x M) has random orthonormal columns.  K is block upper triangular with random
    orthogonal diagonal blocks and off-diagonal blocks alpha * G_ij / ||G_ij||_2 (G_ij
    Gaussian): a well-conditioned coupling of every panel to all earlier ones.
    S = blockdiag(c_j diag(logspace(0, -log10 kappa_p, s)) W_j^T) with c_j = 2^(1-j) and
    random orthogonal W_j.  An optional lead column (``lead=True``, scale 1, width 1)
    comes first so that the panels line up with a basis whose first column stands alone.
    Panel j then has a condition number of about kappa_p and the first j panels one of
    about 2^(j-1) kappa_p.
    """
    rng = np.random.default_rng(seed)
    widths = ([1] if lead else []) + [s] * npanels
    scales = ([1.0] if lead else []) + [2.0 ** (-j) for j in range(npanels)]
    offs = np.concatenate([[0], np.cumsum(widths)]).astype(int)
    M = int(offs[-1])
    X = _random_orthonormal(rng, n, M)
    K = np.zeros((M, M))
    S = np.zeros((M, M))
    sig = np.logspace(0.0, -np.log10(kappa_p), s)
    for b, w in enumerate(widths):
        o = offs[b]
        if w == 1:
            K[o, o] = 1.0
            S[o, o] = scales[b]
        else:
            K[o:o + w, o:o + w] = _random_orthonormal(rng, w, w)
            S[o:o + w, o:o + w] = scales[b] * (sig[:, None] * _random_orthonormal(rng, w, w).T)
        for bi in range(b):
            G = rng.standard_normal((widths[bi], w))
            K[offs[bi]:offs[bi + 1], o:o + w] = alpha * G / np.linalg.norm(G, 2)
    return np.asfortranarray(X @ (K @ S))


def nearly_dependent_panel(n: int, k: int, s: int, delta: float, seed: int):
    """(Q, V): Q n x k orthonormal and V = Q C + delta Z, C Gaussian, Z n x s orthonormal and
    orthogonal to Q.  [Q, V] has a condition number of about 1/delta while V - Q Q^T V =
    delta Z is perfectly conditioned; delta = 0 makes every column of V lie in span(Q)."""
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((n, k + s)))
    Q, Z = X[:, :k], X[:, k:]
    C = rng.standard_normal((k, s))
    return np.asfortranarray(Q), np.asfortranarray(Q @ C + delta * Z)


def ill_conditioned_panel(n: int, k: int, s: int, kappa: float, seed: int):
    """(Q, V): Q n x k orthonormal and V = Q C + Z D, Z n x s orthonormal and orthogonal to
    Q, D upper triangular with unit diagonal but D[s-1, s-1] = 1/kappa: the last column of
    V - Q Q^T V = Z D lies within 1/kappa of the span of the others (numerically full rank,
    relative Cholesky pivot ~ kappa^-2)."""
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((n, k + s)))
    Q, Z = X[:, :k], X[:, k:]
    D = np.triu(rng.standard_normal((s, s)), 1) + np.eye(s)
    D[s - 1, s - 1] = 1.0 / kappa
    return np.asfortranarray(Q), np.asfortranarray(Q @ rng.standard_normal((k, s)) + Z @ D)
