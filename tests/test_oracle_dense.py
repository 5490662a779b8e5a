"""Pins for the oracle's small dense routines against LAPACK (numpy) and their definitions."""
import numpy as np
import pytest

from oracle import dense as D


def test_chol_upper_definition():
    rng = np.random.default_rng(0)
    for k in (1, 5, 10, 61):
        Z = rng.standard_normal((3 * k + 5, k))
        G = Z.T @ Z
        R = D.chol_upper(G)
        assert np.allclose(np.triu(R), R)
        assert np.all(np.diag(R) > 0)
        assert np.linalg.norm(R.T @ R - G) <= 1e-13 * np.linalg.norm(G)


def test_chol_upper_breakdown():
    G = np.array([[1.0, 2.0], [2.0, 1.0]])
    with pytest.raises(D.CholeskyBreakdown):
        D.chol_upper(G)


def test_triangular_solves():
    rng = np.random.default_rng(1)
    R = np.triu(rng.standard_normal((7, 7))) + 5 * np.eye(7)
    B = rng.standard_normal((7, 3))
    assert np.allclose(D.solve_upper(R, B), np.linalg.solve(R, B), rtol=1e-13, atol=1e-13)
    M = rng.standard_normal((4, 7))
    assert np.allclose(D.right_solve_upper(M, R), M @ np.linalg.inv(R), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("k", [1, 2, 5, 30, 60])
def test_givens_lsq_matches_lapack_lstsq(k):
    rng = np.random.default_rng(k)
    H = np.triu(rng.standard_normal((k + 1, k)), -1)
    H[:k, :k] += 4.0 * np.eye(k)  # keep it well conditioned so the comparison is tight
    g0 = 3.7
    y, res = D.givens_lsq(H, g0)
    rhs = np.zeros(k + 1)
    rhs[0] = g0
    y_ref = np.linalg.lstsq(H, rhs, rcond=None)[0]
    assert np.allclose(y, y_ref, rtol=1e-10, atol=1e-12)
    assert abs(res - np.linalg.norm(rhs - H @ y_ref)) <= 1e-12 * g0


def test_givens_incremental_residuals_are_the_lsq_residuals():
    rng = np.random.default_rng(7)
    k = 12
    H = np.triu(rng.standard_normal((k + 1, k)), -1)
    st = D.GivensState(1.0, k)
    prev = 1.0
    for j in range(k):
        st.add_column(H[: j + 2, j])
        rhs = np.zeros(j + 2)
        rhs[0] = 1.0
        y = np.linalg.lstsq(H[: j + 2, : j + 1], rhs, rcond=None)[0]
        ref = np.linalg.norm(rhs - H[: j + 2, : j + 1] @ y)
        assert abs(st.residual() - ref) <= 1e-12
        assert st.residual() <= prev + 1e-15  # minimal residual is non-increasing
        prev = st.residual()


def test_householder_reference():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((500, 9))
    Q, R = D.householder_qr(X)
    assert np.all(np.diag(R) > 0)
    assert D.orth_error(Q) < 1e-14
    assert D.repr_error(X, Q, R) < 1e-15
