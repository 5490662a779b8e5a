"""Pins for the oracle's block orthogonalization schemes.

* QR uniqueness: every scheme reproduces LAPACK's Householder QR (diag(R) > 0),
  the BlkOrth contract of Fig. 1's caption.
* O(eps) orthogonality and representation error on well-conditioned blocks
  (Sec. IV-B/IV-C, Thms. 1-3).
* CholQR error growth ~ kappa^2 eps and the bound of Eqs. (1)-(3) on the
  log-scaled 10^5 x 5 matrix of Fig. 6; CholQR2 stays O(eps).
* Thm. 1: kappa after the first CholQR < sqrt(3) whenever c1 kappa^2 < 1/2.
* Fig. 8 / Thm. 3: two-stage on a glued matrix (m, s_hat, s) = (180, 60, 5) with
  panel condition numbers 1e7 reaches O(eps) orthogonality, and stage 1 leaves
  the big panel with an O(1) condition number.
* The block Pythagorean identity behind BCGS-PIP (Sec. IV-C).
"""
import numpy as np
import pytest

import workloads as W
from oracle import blockortho as BO
from oracle import dense as D

EPS = np.finfo(np.float64).eps
SCHEMES = ["two_stage", "bcgs_pip2", "bcgs2_cholqr2"]


@pytest.fixture(scope="module")
def gauss_block():
    return W.gaussian_block(20000, 61, seed=11)


@pytest.mark.parametrize("algo", SCHEMES + ["cholqr2"])
@pytest.mark.parametrize("s", [5, 10])
def test_qr_matches_householder(gauss_block, algo, s):
    X = gauss_block
    Q, R = BO.orthogonalize(X, s, algo)
    Qh, Rh = D.householder_qr(X)
    kap = D.cond2(X)
    assert np.allclose(np.triu(R), R, atol=0)
    assert np.linalg.norm(R - Rh) / np.linalg.norm(Rh) <= 50 * kap * EPS
    assert np.linalg.norm(Q - Qh) / np.sqrt(Q.shape[1]) <= 50 * kap * EPS


@pytest.mark.parametrize("algo", SCHEMES)
@pytest.mark.parametrize("s", [5, 10])
def test_orthogonality_and_representation(gauss_block, algo, s):
    X = gauss_block
    Q, R = BO.orthogonalize(X, s, algo)
    assert D.orth_error(Q) <= 1e-13
    assert D.repr_error(X, Q, R) <= 1e-14


def test_short_last_panel_and_small_k():
    X = W.gaussian_block(3000, 14, seed=4)  # 1 + 5 + 5 + 3
    for algo in SCHEMES:
        Q, R = BO.orthogonalize(X, 5, algo)
        assert D.orth_error(Q) <= 1e-14 and D.repr_error(X, Q, R) <= 1e-15
    X1 = W.gaussian_block(100, 1, seed=4)
    Q, R = BO.orthogonalize(X1, 5, "two_stage")
    assert abs(R[0, 0] - np.linalg.norm(X1)) < 1e-13 and D.orth_error(Q) < 1e-15


def test_two_stage_shat_equivalences(gauss_block):
    X = gauss_block[:, :31]
    Qa, Ra = BO.two_stage(X, 5, 30)
    Qb, Rb = BO.two_stage(X, 5, 10)
    Qc, Rc = BO.two_stage(X, 5, 5)
    for Q, R in ((Qb, Rb), (Qc, Rc)):
        assert np.linalg.norm(R - Ra) <= 1e-12 * np.linalg.norm(Ra)
        assert np.linalg.norm(Q - Qa) <= 1e-12 * np.sqrt(31)


def test_pip_pythagorean_identity():
    rng = np.random.default_rng(3)
    Q, _ = D.householder_qr(rng.standard_normal((4000, 12)))
    V = rng.standard_normal((4000, 5))
    Qn, P, R = BO.bcgs_pip(Q, V)
    Y = V - Q @ P
    # Y^T Y = V^T V - P^T P when Q is orthonormal
    assert np.linalg.norm(Y.T @ Y - (V.T @ V - P.T @ P)) <= 1e-10 * np.linalg.norm(V.T @ V)
    assert np.linalg.norm(V - Q @ P - Qn @ R) <= 1e-13 * np.linalg.norm(V)
    assert np.linalg.norm(Q.T @ Qn) <= 1e-13


@pytest.fixture(scope="module")
def logscaled_sweep():
    n, s = 100000, 5
    out = {}
    for kap in (1e0, 1e2, 1e4, 1e6, 1e7, 1e8):
        rows = []
        for seed in range(10):
            V = W.logscaled_block(n, s, kap, seed)
            try:
                Q1, _ = BO.cholqr(V)
                Q2, R2 = BO.cholqr2(V)
            except D.CholeskyBreakdown:  # expected only beyond eps^(-1/2) (Sec. II)
                rows.append((np.nan,) * 4)
                continue
            rows.append((D.orth_error_2(Q1), D.cond2(Q1), D.orth_error_2(Q2), D.repr_error(V, Q2, R2)))
        out[kap] = np.array(rows)
    return n, s, out


def test_cholqr_error_bound_eq3(logscaled_sweep):
    n, s, out = logscaled_sweep
    c1 = 5.0 * (n * s + s * (s + 1)) * EPS  # Eq. (3)
    for kap, rows in out.items():
        if c1 * kap ** 2 < 0.5:  # assumption Eq. (1)
            assert np.all(rows[:, 0] <= c1 * kap ** 2)       # bound Eq. (2)
            assert np.all(rows[:, 1] < np.sqrt(3.0))          # Thm. 1


def test_cholqr_error_grows_like_kappa_squared(logscaled_sweep):
    _, _, out = logscaled_sweep
    e4 = out[1e4][:, 0].mean()
    e6 = out[1e6][:, 0].mean()
    ratio = e6 / e4
    assert 1e4 / 30 <= ratio <= 1e4 * 30  # slope 2 in log-log (Fig. 6)
    assert out[1e0][:, 0].max() <= 10 * EPS


def test_cholqr2_is_order_eps_up_to_1e7(logscaled_sweep):
    _, _, out = logscaled_sweep
    # no breakdown below eps^(-1/2) ~ 6.7e7
    for kap in (1e0, 1e2, 1e4, 1e6, 1e7):
        assert not np.isnan(out[kap]).any()
    for kap in (1e0, 1e2, 1e4, 1e6, 1e7):
        assert out[kap][:, 2].max() <= 20 * EPS
        assert out[kap][:, 3].max() <= 10 * EPS


@pytest.fixture(scope="module")
def glued():
    # (m, s_hat, s) = (180, 60, 5) and panel condition 1e7 as in Fig. 8; n reduced to 2e4
    return W.glued_block(20000, 36, 5, 1e7, seed=0)


def test_glued_matrix_conditioning(glued):
    V = glued
    for j in (1, 2, 4, 8):
        c0 = 1 + (j - 1) * 5
        kp = D.cond2(V[:, c0:c0 + 5])
        kc = D.cond2(V[:, 1:c0 + 5])
        assert 0.5e7 < kp < 2e7
        assert 0.5 * 2 ** (j - 1) * 1e7 < kc < 2 * 2 ** (j - 1) * 1e7


def test_two_stage_on_glued_matrix(glued):
    V = glued
    Q, R, (Y1, _) = BO.two_stage(V, 5, 60, return_stage1=True)
    assert D.orth_error(Q) <= 1e-13
    assert D.repr_error(V, Q, R) <= 1e-15
    # Thm. 3 / Eq. (10): after stage 1 the first big panel is O(1)-conditioned
    assert D.cond2(Y1[:, :61]) < 1.5
    # one CholQR over everything at the end (s_hat = m) also reaches O(eps)
    Q2, R2 = BO.two_stage(V, 5, 180)
    assert D.orth_error(Q2) <= 1e-13


def test_bcgs_pip2_on_glued_matrix(glued):
    Q, R = BO.orthogonalize(glued, 5, "bcgs_pip2")
    assert D.orth_error(Q) <= 1e-13 and D.repr_error(glued, Q, R) <= 1e-15


def _nearly_dependent_panel(n, k, s, delta, seed):
    return W.nearly_dependent_panel(n, k, s, delta, seed)


def test_pip_explicit_second_pass_where_pip_fails():
    """PIP's Gram G_V - P^T P cancels to rounding once kappa([Q, V]) ~ eps^-1/2 (Sec. IV-C);
    the explicit second pass still yields the thin QR of [Q, V]: orthogonal to O(eps),
    V = Q P + Qnew R to O(eps), R equal to the Householder factor's trailing block."""
    n, k, s = 4000, 9, 5
    Q, V = _nearly_dependent_panel(n, k, s, 1e-7, seed=11)
    with pytest.raises(D.CholeskyBreakdown):
        BO.bcgs_pip(Q, V, 1e-12)
    Qn, P, R, used = BO.bcgs_pip_explicit(Q, V, 1e-12)
    assert used
    Qf = np.hstack([Q, Qn])
    assert D.orth_error(Qf) <= 1e-13
    assert np.linalg.norm(V - Q @ P - Qn @ R) / np.linalg.norm(V) <= 1e-15
    _, Rh = D.householder_qr(np.hstack([Q, V]))
    Rb = Rh[k:, k:]
    assert np.linalg.norm(R - Rb) / np.linalg.norm(Rb) <= 1e-8  # O(eps kappa), kappa ~ 1e7
    # a well-conditioned panel takes the one-pass path and gives PIP's result
    Q2, V2 = _nearly_dependent_panel(n, k, s, 1.0, seed=12)
    Qa, Pa, Ra = BO.bcgs_pip(Q2, V2, 1e-12)
    Qb, Pb, Rb2, used2 = BO.bcgs_pip_explicit(Q2, V2, 1e-12)
    assert not used2 and np.array_equal(Qa, Qb) and np.array_equal(Ra, Rb2)


def test_pip_explicit_second_pass_rejects_dependent_columns():
    """A column that is in span(Q) up to rounding fails the second pass's tol^2 test
    (its pivot is at the rounding level of V) instead of being normalized noise."""
    n, k, s = 4000, 9, 5
    Q, V = _nearly_dependent_panel(n, k, s, 0.0, seed=13)
    with pytest.raises(D.CholeskyBreakdown) as e:
        BO.bcgs_pip_explicit(Q, V, 1e-12)
    assert e.value.index == 0
    # one dependent column in the middle of an otherwise healthy panel
    Q, V = _nearly_dependent_panel(n, k, s, 1e-3, seed=14)
    V[:, 2] = Q @ np.arange(1.0, k + 1.0)
    with pytest.raises(D.CholeskyBreakdown) as e:
        BO.bcgs_pip_explicit(Q, V, 1e-12)
    assert e.value.index == 2


def _ill_conditioned_panel(n, k, s, kappa, seed):
    return W.ill_conditioned_panel(n, k, s, kappa, seed)


def test_shifted_pass_where_the_second_pass_fails():
    """A relative pivot of 1e-18: the explicit second pass fails its pivot test;
    the shifted Cholesky QR pass and one more BCGS-PIP pass still give the thin QR of
    [Q, V]: orthogonal to O(eps kappa(Z)^2) with kappa(Z) ~ (mu / sigma_min^2)^(1/2),
    V = Q P + Qnew R to rounding, R equal to the Householder factor's trailing block to
    O(eps kappa(Y))."""
    n, k, s = 4000, 9, 6
    Q, V = _ill_conditioned_panel(n, k, s, 1e9, seed=21)
    with pytest.raises(D.CholeskyBreakdown):
        BO.bcgs_pip_explicit(Q, V, 1e-12)
    Qn, P, R, passes = BO.bcgs_pip_explicit(Q, V, 1e-12, shifted=True)
    assert passes == 2
    Qf = np.hstack([Q, Qn])
    assert D.orth_error(Qf) <= 1e-10
    assert np.linalg.norm(V - Q @ P - Qn @ R) / np.linalg.norm(V) <= 1e-15
    _, Rh = D.householder_qr(np.hstack([Q, V]))
    assert np.linalg.norm(P - Rh[:k, k:]) / np.linalg.norm(Rh[:k, k:]) <= 1e-12
    assert np.linalg.norm(R - Rh[k:, k:]) / np.linalg.norm(Rh[k:, k:]) <= 1e-6
    # a panel the second pass handles never reaches the shifted pass
    Q2, V2 = _nearly_dependent_panel(n, k, 5, 1e-7, seed=11)
    assert BO.bcgs_pip_explicit(Q2, V2, 1e-12, shifted=True)[3] == 1


def test_shifted_pass_still_rejects_dependent_columns():
    n, k, s = 4000, 9, 5
    Q, V = _nearly_dependent_panel(n, k, s, 0.0, seed=13)
    with pytest.raises(D.CholeskyBreakdown) as e:
        BO.bcgs_pip_explicit(Q, V, 1e-12, shifted=True)
    assert e.value.index == 0
    Q, V = _nearly_dependent_panel(n, k, s, 1e-3, seed=14)
    V[:, 2] = Q @ np.arange(1.0, k + 1.0)
    with pytest.raises(D.CholeskyBreakdown) as e:
        BO.bcgs_pip_explicit(Q, V, 1e-12, shifted=True)
    assert e.value.index == 2


def test_pip_trigger_threshold_takes_the_explicit_pass_before_pip_loses_digits():
    """Stage 1's trigger (dense.PIP_TOL): a panel whose Pythagorean pivots are ~1e-10
    relative (kappa([Q, V]) ~ 1e5) is accepted by PIP at PIVOT_TOL but loses orthogonality
    O(eps kappa^2) there (Sec. IV-C); at PIP_TOL it takes the explicit pass and gets the thin
    QR of [Q, V] to O(eps): orthogonality at rounding, R equal to the Householder factor."""
    n, k, s = 4000, 9, 5
    Q, V = _nearly_dependent_panel(n, k, s, 1e-5, seed=31)
    Qa, Pa, Ra, pa = BO.bcgs_pip_explicit(Q, V, D.PIVOT_TOL, pip_tol=D.PIVOT_TOL)
    Qb, Pb, Rb, pb = BO.bcgs_pip_explicit(Q, V, D.PIVOT_TOL, pip_tol=D.PIP_TOL)
    assert pa == 0 and pb == 1
    ea, eb = D.orth_error(np.hstack([Q, Qa])), D.orth_error(np.hstack([Q, Qb]))
    assert ea > 1e-9 and eb <= 1e-14, (ea, eb)
    _, Rh = D.householder_qr(np.hstack([Q, V]))
    assert np.linalg.norm(Rb - Rh[k:, k:]) / np.linalg.norm(Rh[k:, k:]) <= 1e-9
    assert np.linalg.norm(V - Q @ Pb - Qb @ Rb) / np.linalg.norm(V) <= 1e-15
    # the s <= 5 bases stay far above the trigger: a well-conditioned panel is PIP's
    Q2, V2 = _nearly_dependent_panel(n, k, s, 1e-2, seed=32)
    assert BO.bcgs_pip_explicit(Q2, V2, D.PIVOT_TOL, pip_tol=D.PIP_TOL)[3] == 0
