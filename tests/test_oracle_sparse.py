"""Pins for the generated operators and the oracle's SpMV / Gershgorin interval.

Pinned against closed forms (Dirichlet Laplacian eigenpairs), Kronecker-product
constructions written independently with numpy, and a dense eigen-solver.
"""
import numpy as np
import pytest

import workloads as W
from oracle import sparse as S


@pytest.mark.parametrize("N,modes", [(12, [(1, 1), (3, 7), (12, 12), (5, 2)]), (31, [(1, 2), (30, 4)])])
def test_spmv_laplace2d_eigenvectors(N, modes):
    A = W.laplace2d(N)
    for a, c in modes:
        lam, u = W.laplace_eigpair_2d(N, a, c)
        r = S.spmv(A, u) - lam * u
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(u) * 8


@pytest.mark.parametrize("N,modes", [(6, [(1, 1, 1), (2, 5, 3), (6, 6, 6)]), (9, [(1, 4, 9)])])
def test_spmv_laplace3d_eigenvectors(N, modes):
    A = W.laplace3d(N)
    for a, c, d in modes:
        lam, u = W.laplace_eigpair_3d(N, a, c, d)
        r = S.spmv(A, u) - lam * u
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(u) * 12


def test_spmv_plain_matches_library_product():
    A = W.convdiff2d(9, 37.0, 1.1)
    x = W.uniform_vector(A.n, 3)
    assert np.allclose(S.spmv_plain(A, x), S.spmv(A, x), rtol=0, atol=1e-14)


def _tridiag(N, lo, d, up):
    return np.diag(np.full(N, d)) + np.diag(np.full(N - 1, lo), -1) + np.diag(np.full(N - 1, up), 1)


def test_convdiff_matches_kronecker_construction():
    N, pe, th = 7, 64.0, 2.3
    h = 1.0 / (N + 1)
    bx, by = pe * np.cos(th), pe * np.sin(th)
    # 1D upwind operators per axis (h^2-scaled): -u'' + b u'
    Tx = _tridiag(N, -1 - h * max(bx, 0), 2 + h * abs(bx), -1 + h * min(bx, 0))
    Ty = _tridiag(N, -1 - h * max(by, 0), 2 + h * abs(by), -1 + h * min(by, 0))
    I = np.eye(N)
    M = np.kron(I, Tx) + np.kron(Ty, I)  # x fastest
    A = W.convdiff2d(N, pe, th)
    assert np.allclose(A.to_scipy().toarray(), M, rtol=0, atol=1e-15)


def test_laplace_nnz_and_spectrum_closed_forms():
    for N in (4, 9, 16):
        assert W.laplace2d(N).nnz == 5 * N * N - 4 * N
        assert W.laplace3d(N).nnz == 7 * N ** 3 - 6 * N ** 2
    for N, dim in ((10, 2), (5, 3)):
        A = W.laplace2d(N) if dim == 2 else W.laplace3d(N)
        ev = np.linalg.eigvalsh(A.to_scipy().toarray())
        lmin, lmax = W.laplace_extreme_eigs(N, dim)
        assert abs(ev[0] - lmin) < 1e-12 and abs(ev[-1] - lmax) < 1e-12
    # the 64^2 and 2048^2 condition numbers used by the solution-error gate
    lmin, lmax = W.laplace_extreme_eigs(64, 2)
    assert abs(lmax / lmin - 1.711661e3) / 1.711661e3 < 1e-6
    lmin, lmax = W.laplace_extreme_eigs(2048, 2)
    assert abs(lmax / lmin - 1.701547e6) / 1.701547e6 < 1e-6


def test_gershgorin_interval():
    assert S.gershgorin(W.laplace2d(8)) == (0.0, 8.0)
    assert S.gershgorin(W.laplace3d(5)) == (0.0, 12.0)
    A = W.convdiff2d(8, 80.0, 0.4)
    lo, hi = S.gershgorin(A)
    ev = np.linalg.eigvals(A.to_scipy().toarray())
    assert lo - 1e-12 <= ev.real.min() and ev.real.max() <= hi + 1e-12


def test_basis_params():
    A = W.laplace2d(8)
    th, sg = S.basis_params(A, 5, "monomial")
    assert np.all(th == 0) and np.all(sg == 8.0)
    th, sg = S.basis_params(A, 5, "shifted")
    assert np.all(th == 4.0) and np.all(sg == 4.0)


def test_generators_are_seeded():
    a = W.make_problem("convdiff2d", 16, seed=5)
    b = W.make_problem("convdiff2d", 16, seed=5)
    c = W.make_problem("convdiff2d", 16, seed=6)
    assert np.array_equal(a["b"], b["b"]) and np.array_equal(a["A"].val, b["A"].val)
    assert not np.array_equal(a["b"], c["b"])
    assert 10.0 <= a["meta"]["pe"] <= 100.0
    A = a["A"]
    assert A.row_ptr.dtype == np.int32 and A.col.dtype == np.int32
    # sorted column indices per row, M-matrix sign pattern
    for i in range(A.n):
        cols = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    off = A.col != np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert np.all(A.val[off] < 0) and np.all(A.val[~off] > 0)
