"""Pins for the oracle's Newton basis from Leja-ordered Ritz values.

* Leja ordering: hand-worked orderings of small real and complex sets; on random
  conjugate-closed sets every chosen point maximizes the product of distances (direct
  products, not the oracle's log sums) and conjugate pairs are adjacent.
* Capacity: the Leja estimate approaches the logarithmic capacity of an interval,
  (b - a) / 4, and of a circle, its radius.
* Ritz values: a symmetric tridiagonal matrix against scipy's tridiagonal eigensolver;
  a Hessenberg matrix built by similarity from known eigenvalues (complex pairs).
* Real form: the Newton steps with tau reproduce prod (A - z I) w / sigma^s computed in
  complex arithmetic; the matrix-powers relation A W = [w0, W] B holds with B(i-1, i) =
  -tau_i.
* Solver: after the first cycle the Hessenberg of a Newton-basis cycle equals Arnoldi's
  (MGS) from the same start vector; the solve converges; the panels of the Newton basis
  are far better conditioned than the shifted basis at s = 15.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import gmres as G
from oracle import ritz as Z
from oracle import sparse as S


def test_leja_real_hand_worked():
    # 4 has the largest modulus; 0 is farthest from 4; then |z-4||z| is 3, 3.75, 3 for
    # 1, 2.5, 3; then |z-4||z||z-2.5| is 4.5 for 1 and 1.5 for 3.
    zl, second = Z.leja_order([0.0, 1.0, 2.5, 3.0, 4.0])
    assert np.array_equal(zl.real, [4.0, 0.0, 2.5, 1.0, 3.0])
    assert not second.any()


def test_leja_complex_hand_worked():
    # |3| = 3 > |2i| = 2: 3 first; |z - 3| is sqrt(13) for +-2i, 4 for -1, 2 for 1 -> -1;
    # |z - 3||z + 1| is sqrt(65) for +-2i and 4 for 1 -> the pair, +2i first; then 1.
    zl, second = Z.leja_order([2j, -2j, 1.0, -1.0, 3.0])
    assert np.allclose(zl, [3.0, -1.0, 2j, -2j, 1.0], atol=0)
    assert list(second) == [False, False, False, True, False]


def _random_conj_closed(rng, n_real, n_pairs):
    pts = list(rng.uniform(-2, 6, n_real))
    for _ in range(n_pairs):
        z = complex(rng.uniform(-2, 6), rng.uniform(0.1, 3))
        pts += [z, z.conjugate()]
    rng.shuffle(pts)
    return np.array(pts, dtype=np.complex128)


@pytest.mark.parametrize("seed", range(5))
def test_leja_greedy_property_brute_force(seed):
    rng = np.random.default_rng(seed)
    z = _random_conj_closed(rng, 7, 5)
    zl, second = Z.leja_order(z)
    assert sorted(zl.tolist(), key=lambda c: (c.real, c.imag)) == sorted(z.tolist(), key=lambda c: (c.real, c.imag))
    assert abs(zl[0]) == np.max(np.abs(z))
    k = 1
    while k < len(zl):
        if second[k]:
            assert zl[k] == np.conj(zl[k - 1]) and zl[k - 1].imag != 0.0
            k += 1
            continue
        rest = zl[k:]
        prods = [np.prod(np.abs(w - zl[:k])) for w in rest]
        assert np.prod(np.abs(zl[k] - zl[:k])) >= max(prods) * (1 - 1e-12)
        if zl[k].imag != 0.0:
            assert k + 1 < len(zl) and second[k + 1]
        k += 1


def test_capacity_interval_and_circle():
    a, b = 0.5, 8.5
    t = np.cos(np.pi * (np.arange(400) + 0.5) / 400)  # Chebyshev points of [-1, 1]
    zl, _ = Z.leja_order(0.5 * (a + b) + 0.5 * (b - a) * t)
    assert abs(Z.capacity(zl) - (b - a) / 4) <= 0.05 * (b - a) / 4
    r = 3.0
    zl, _ = Z.leja_order(1.0 + r * np.exp(2j * np.pi * (np.arange(301) + 0.25) / 301))
    assert abs(Z.capacity(zl) - r) <= 0.05 * r


def test_ritz_values_symmetric_tridiagonal():
    rng = np.random.default_rng(3)
    d, e = rng.uniform(1, 5, 30), rng.uniform(0.1, 1, 29)
    H = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ref = sla.eigh_tridiagonal(d, e, eigvals_only=True)
    got = np.sort(Z.ritz_values(H).real)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(Z.ritz_values(H).imag)) == 0.0


def test_ritz_values_known_complex_spectrum():
    rng = np.random.default_rng(4)
    lam = [2.0, -1.0, 0.5]
    pairs = [(1.0, 2.0), (3.0, 0.5)]
    blocks = [np.array([[x]]) for x in lam] + [np.array([[a, b], [-b, a]]) for a, b in pairs]
    D0 = sla.block_diag(*blocks)
    X = rng.standard_normal(D0.shape) + 4 * np.eye(D0.shape[0])
    H = sla.hessenberg(X @ D0 @ np.linalg.inv(X))
    want = sorted(lam + [complex(a, s * b) for a, b in pairs for s in (1, -1)], key=lambda c: (c.real, c.imag))
    got = sorted(Z.ritz_values(H).tolist(), key=lambda c: (c.real, c.imag))
    assert np.max(np.abs(np.array(got) - np.array(want))) <= 1e-10


def _dense_csr(M):
    n = M.shape[0]
    rows, cols = np.nonzero(M)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return W.CSR(n, np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32), M[rows, cols].astype(np.float64))


def test_real_form_equals_complex_newton_product():
    rng = np.random.default_rng(5)
    n = 40
    M = rng.standard_normal((n, n)) / np.sqrt(n) + np.diag(rng.uniform(1, 3, n))
    A = _dense_csr(M)
    z = np.array([3.0, 1 + 1.5j, 1 - 1.5j, 0.5, 2 + 0.7j, 2 - 0.7j])
    second = np.array([False, False, True, False, False, True])
    sig = 1.7
    theta, tau, sigma = Z.newton_params(z, second, 6, sig)
    w0 = rng.standard_normal(n)
    Wr, B = G.mpk(S.Operator(A), w0, theta, sigma, tau)
    v = w0.astype(np.complex128)
    for i, zi in enumerate(z):
        v = (M @ v - zi * v) / sig
        if i in (0, 3) or second[i]:  # after a real point or a completed pair: real again
            assert np.max(np.abs(v.imag)) <= 1e-13 * np.max(np.abs(v))
            assert np.allclose(Wr[:, i], v.real, rtol=0, atol=1e-13 * np.max(np.abs(v)))
    # A [w0 .. w5] = [w0 .. w6] B, with B(i-1, i) = -tau_i
    V = np.column_stack([w0, Wr])
    assert np.linalg.norm(M @ V[:, :6] - V @ B) <= 1e-13 * np.linalg.norm(M) * np.linalg.norm(V)
    assert B[1, 2] == -tau[2] and tau[2] == pytest.approx(1.5 ** 2 / sig)


def test_pair_split_at_position_s_uses_the_real_part():
    z = np.array([4.0, 1 + 1j, 1 - 1j])
    second = np.array([False, False, True])
    theta, tau, sigma = Z.newton_params(z, second, 2, 2.0)
    assert list(theta) == [4.0, 1.0] and list(tau) == [0.0, 0.0]


@pytest.fixture(scope="module")
def convdiff_leja():
    pr = W.make_problem("convdiff2d", 32, seed=4)
    A, b = pr["A"], pr["b"]
    one = G.sstep_gmres(A, b, m=60, s=5, tol=1e-30, max_iters=60, basis="leja")
    two = G.sstep_gmres(A, b, m=60, s=5, tol=1e-30, max_iters=120, basis="leja", record=True)
    return A, b, one, two


def test_leja_switches_after_first_cycle_with_complex_shifts(convdiff_leja):
    A, b, one, two = convdiff_leja
    lo, hi = S.gershgorin(A)
    sh = G.sstep_gmres(A, b, m=60, s=5, tol=1e-30, max_iters=60, basis="shifted")
    assert np.array_equal(one["x"], sh["x"])  # cycle 1 runs with the shifted basis
    assert two["basis_switched_after"] == 1
    assert np.any(two["tau"] > 0)  # this spectrum gives complex Ritz values
    assert not np.array_equal(two["theta"], np.full(5, 0.5 * (lo + hi)))


def test_newton_cycle_hessenberg_equals_arnoldi(convdiff_leja):
    A, b, one, two = convdiff_leja
    rec = two["records"][1]
    arn = G.gmres(A, b, x0=one["x"], ortho="mgs", m=60, tol=1e-30, max_iters=60, record=True)["records"][0]
    H, H_arn = rec["H"], arn["H"]
    assert np.linalg.norm(H - H_arn) / np.linalg.norm(H_arn) <= 1e-9
    for ortho in ("bcgs_pip2", "bcgs2_cholqr2"):  # each from its own first-cycle iterate
        x1 = G.sstep_gmres(A, b, m=60, s=5, tol=1e-30, max_iters=60, basis="leja", ortho=ortho)["x"]
        o = G.sstep_gmres(A, b, m=60, s=5, tol=1e-30, max_iters=120, basis="leja", ortho=ortho, record=True)
        ref = G.gmres(A, b, x0=x1, ortho="mgs", m=60, tol=1e-30, max_iters=60, record=True)["records"][0]["H"]
        assert np.linalg.norm(o["records"][1]["H"] - ref) / np.linalg.norm(ref) <= 1e-9, ortho


@pytest.mark.parametrize("s_hat", [None, 20])
def test_leja_solve_converges(s_hat):
    pr = W.make_problem("convdiff2d", 24, seed=1)
    x_lu, M = G.dense_solve(pr["A"], pr["b"])
    out = G.sstep_gmres(pr["A"], pr["b"], m=60, s=10, tol=1e-10, basis="leja", s_hat=s_hat)
    assert out["converged"] and out["relres"] <= 1e-10
    kap = np.linalg.cond(M)
    assert np.linalg.norm(out["x"] - x_lu) / np.linalg.norm(x_lu) <= 2 * 1e-10 * kap


def test_newton_panels_better_conditioned_at_s15():
    pr = W.make_problem("laplace2d", 64, seed=0)
    A, b = pr["A"], pr["b"]
    op = S.Operator(A)
    one = G.sstep_gmres(A, b, m=60, s=15, tol=1e-30, max_iters=60, basis="leja")
    two = G.sstep_gmres(A, b, m=60, s=15, tol=1e-30, max_iters=120, basis="leja")
    r = b - S.spmv(op, one["x"])
    w0 = r / np.linalg.norm(r)
    Wn, _ = G.mpk(op, w0, two["theta"], two["sigma"], two["tau"])
    th, sg = S.basis_params(op, 15, "shifted")
    Ws, _ = G.mpk(op, w0, th, sg)
    k_newton = np.linalg.cond(np.column_stack([w0, Wn]))
    k_shift = np.linalg.cond(np.column_stack([w0, Ws]))
    assert k_newton * 50 <= k_shift
