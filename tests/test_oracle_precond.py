"""Pins for the oracle's multicolor Gauss-Seidel preconditioner and the right-
preconditioned solvers.

* Priorities: the first outputs of SplitMix64 seeded with 0 are the generator's
  published ones.
* Coloring: valid (no two neighbours share a color), at most max degree + 1 colors,
  and equal to an independent simulation of Jones and Plassmann's parallel rounds
  with the same priorities.
* Sweep: z solves (D + L_c) z = w, checked against the explicitly assembled lower
  triangular matrix in color order (scipy's triangular solve); with the red-black
  coloring of the 2D Laplacian it is the textbook red-black Gauss-Seidel sweep.
* Splitting: for the SPD Laplacian the eigenvalues of A M^{-1} lie in |z - 1| < 1 (the
  basis interval [0, 2] of the reading).
* Solvers: one preconditioned cycle of every variant equals x0 + M^{-1} times the
  minimizer over K(A M^{-1}, r) (LAPACK least squares on an explicit M^{-1}); the
  solves converge to the dense-LU solution in fewer iterations than unpreconditioned.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import dense as D
from oracle import gmres as G
from oracle import precond as PC
from oracle import sparse as S


def test_splitmix64_published_outputs():
    p = PC.priority(3)
    assert [int(v) for v in p] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _sym_pattern(A):
    M = sp.csr_matrix((np.ones_like(A.val), A.col, A.row_ptr), shape=(A.n, A.n))
    S_ = ((M + M.T) != 0).tocsr()
    S_.setdiag(False)
    S_.eliminate_zeros()
    return S_


def _jp_rounds(A):
    """Jones-Plassmann: in each round every uncolored row whose (priority, index) beats all
    its uncolored neighbours takes the smallest color none of its colored neighbours has
    (neighbour colors as they stood at the start of the round)."""
    n = A.n
    pr = [int(v) for v in PC.priority(n)]
    Sg = _sym_pattern(A)
    colors = [-1] * n
    while any(c < 0 for c in colors):
        old = list(colors)
        for i in range(n):
            if old[i] >= 0:
                continue
            nb = Sg.indices[Sg.indptr[i]:Sg.indptr[i + 1]]
            if any(old[j] < 0 and (pr[j], j) > (pr[i], i) for j in nb):
                continue
            taken = {old[j] for j in nb if old[j] >= 0}
            c = 0
            while c in taken:
                c += 1
            colors[i] = c
    return np.array(colors, dtype=np.int32)


@pytest.mark.parametrize("kind,N", [("laplace2d", 20), ("laplace3d", 7), ("convdiff2d", 17)])
def test_coloring_valid_and_equal_to_jp_rounds(kind, N):
    A = W.make_problem(kind, N, seed=1)["A"]
    col = PC.coloring(A)
    Sg = _sym_pattern(A).tocoo()
    assert np.all(col[Sg.row] != col[Sg.col])
    maxdeg = int(np.max(np.diff(_sym_pattern(A).indptr)))
    assert col.max() + 1 <= maxdeg + 1
    assert np.array_equal(col, _jp_rounds(A))


@pytest.mark.parametrize("kind,N", [("laplace2d", 24), ("convdiff2d", 21)])
def test_sweep_solves_the_colored_triangular_system(kind, N):
    pr = W.make_problem(kind, N, seed=2)
    A = pr["A"]
    col = PC.coloring(A)
    w = np.random.default_rng(3).uniform(-1, 1, A.n)
    z = PC.mcgs_apply(A, col, w)
    M = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n)).tocoo()
    keep = (M.row == M.col) | (col[M.col] < col[M.row])
    Lc = sp.csr_matrix((M.data[keep], (M.row[keep], M.col[keep])), shape=M.shape)
    perm = np.argsort(col, kind="stable")  # color order: Lc becomes lower triangular
    Lp = Lc[perm][:, perm].tocsr()
    assert sp.triu(Lp, 1).nnz == 0
    zp = spla.spsolve_triangular(Lp, w[perm], lower=True)
    ref = np.empty_like(zp)
    ref[perm] = zp
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_red_black_sweep_on_the_laplacian():
    N = 16
    A = W.laplace2d(N)
    rb = np.array([(i // N + i % N) % 2 for i in range(A.n)], dtype=np.int32)  # red = 0
    w = np.random.default_rng(4).uniform(-1, 1, A.n)
    z = PC.mcgs_apply(A, rb, w)
    ref = np.zeros(A.n)
    for color in (0, 1):
        for p in range(N):
            for q in range(N):
                if (p + q) % 2 != color:
                    continue
                s = w[p * N + q]
                for dp, dq in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                    if 0 <= p + dp < N and 0 <= q + dq < N:
                        s += ref[(p + dp) * N + q + dq]  # off-diagonal entries are -1
                ref[p * N + q] = s / 4.0
    assert np.max(np.abs(z - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_preconditioned_spectrum_in_the_unit_disc_around_one():
    A = W.laplace2d(12)
    P = PC.MulticolorGS(A)
    Ad = S.as_scipy(A).toarray()
    Minv = np.column_stack([P.apply(e) for e in np.eye(A.n)])
    ev = np.linalg.eigvals(Ad @ Minv)
    assert np.max(np.abs(ev - 1.0)) < 1.0
    lo, hi = PC.PRECOND_INTERVAL
    assert lo <= ev.real.min() and ev.real.max() <= hi


def _prec_krylov_min(A, P, r, m):
    """x-update M^{-1} V c minimizing ||r - A M^{-1} V c|| over K_m(A M^{-1}, r), with an
    explicit dense M^{-1} and LAPACK least squares."""
    Ad = S.as_scipy(A).toarray()
    Minv = np.column_stack([P.apply(e) for e in np.eye(A.n)])
    Op = Ad @ Minv
    K = np.zeros((A.n, m))
    v = r / np.linalg.norm(r)
    for j in range(m):
        K[:, j] = v
        v = Op @ v
        v /= np.linalg.norm(v)
    Qk, _ = D.householder_qr(K)
    c = np.linalg.lstsq(Op @ Qk, r, rcond=None)[0]
    return Minv @ (Qk @ c)


def test_preconditioned_cycle_is_the_krylov_minimizer():
    pr = W.make_problem("convdiff2d", 14, seed=5)
    A, b = pr["A"], pr["b"]
    P = PC.MulticolorGS(A)
    m = 10
    ref = _prec_krylov_min(A, P, b, m)
    runs = {
        "mgs": G.gmres(A, b, m=m, tol=1e-14, max_iters=m, precond=P),
        "cgs2": G.gmres(A, b, m=m, tol=1e-14, max_iters=m, ortho="cgs2", precond=P),
    }
    for ortho in ("two_stage", "bcgs_pip2", "bcgs2_cholqr2"):
        runs[ortho] = G.sstep_gmres(A, b, m=m, s=5, tol=1e-14, max_iters=m, ortho=ortho, precond=P)
    for name, out in runs.items():
        assert out["cycles"] == 1, name
        assert np.linalg.norm(out["x"] - ref) <= 1e-8 * np.linalg.norm(ref), name


@pytest.mark.parametrize("kind,N", [("laplace2d", 32), ("convdiff2d", 24)])
def test_preconditioned_solves_converge_faster(kind, N):
    pr = W.make_problem(kind, N, seed=6)
    A, b = pr["A"], pr["b"]
    P = PC.MulticolorGS(A)
    x_lu, M = G.dense_solve(A, b)
    kap = np.linalg.cond(M)
    plain = G.sstep_gmres(A, b, m=60, s=5, tol=1e-10)
    for kw in (dict(ortho="two_stage"), dict(ortho="bcgs_pip2"), dict(ortho="two_stage", s_hat=20),
               dict(ortho="two_stage", basis="leja", s=10)):
        kw = dict(dict(s=5), **kw)
        out = G.sstep_gmres(A, b, m=60, tol=1e-10, precond=P, **kw)
        assert out["converged"], kw
        assert np.linalg.norm(out["x"] - x_lu) / np.linalg.norm(x_lu) <= 2 * 1e-10 * kap, kw
        assert out["iters"] < plain["iters"], kw
