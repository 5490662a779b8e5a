"""GPU parity of the Newton basis from Leja-ordered Ritz values (basis = 'leja').

* The device routine (tsg_ritz_newton: Francis double-shift QR for the Ritz values, Leja
  ordering, real-form parameters) against the oracle (LAPACK eigenvalues, the oracle's
  Leja ordering) on Hessenberg matrices of real solves, known spectra and random ones:
  the same ordered Ritz values (imaginary parts up to the order inside a conjugate pair)
  and theta, tau, sigma to 1e-10 relative.
* Whole solves with the Leja-Ritz basis against the oracle: the cycle that switches to
  the Newton basis, the iteration count, and x to 1e-10 relative; complex Ritz values
  (convection-diffusion), s = 10 and 15, one- and two-stage, big panels s_hat < m, and
  the mixed-precision form.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import workloads as W
from oracle import gmres as G
from oracle import ritz as Z
from oracle import sparse as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def tsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2402_15033_amd as m
    m.load_library()
    return m


def hessenberg_cases():
    """(name, H, s, lo, hi): Hessenberg matrices of first restart cycles, a known
    spectrum, a random matrix with complex eigenvalues, a symmetric tridiagonal one."""
    out = []
    for kind, N, s in (("laplace2d", 32, 10), ("convdiff2d", 32, 10), ("convdiff2d", 48, 16)):
        pr = W.make_problem(kind, N, seed=0)
        rec = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-30, max_iters=60, record=True,
                            basis="shifted")["records"][0]
        lo, hi = S.gershgorin(pr["A"])
        out.append((f"{kind}{N}", rec["H"][:60, :60].copy(), s, lo, hi))
    rng = np.random.default_rng(7)
    X = rng.standard_normal((40, 40)) + 3 * np.eye(40)
    Dg = np.diag(rng.uniform(0.1, 8.0, 40))
    out.append(("known40", sla.hessenberg(X @ Dg @ np.linalg.inv(X)), 10, 0.0, 8.0))
    out.append(("random63", np.triu(rng.standard_normal((63, 63)), -1), 5, -3.0, 3.0))
    d, e = rng.uniform(1, 5, 40), rng.uniform(0.1, 1, 39)
    out.append(("tridiag40", np.diag(d) + np.diag(e, 1) + np.diag(e, -1), 16, 0.0, 6.0))
    return out


def test_ritz_newton_matches_oracle(tsg):
    for name, H, s, lo, hi in hessenberg_cases():
        _say("case ritz", name, H.shape[0], s)
        k = H.shape[0]
        Hd = torch.from_numpy(np.ascontiguousarray(H.T)).cuda().T  # column-major (stride (1, k))
        got = tsg.ritz_newton(Hd, s, lo, hi)
        zl, second = Z.leja_order(Z.ritz_values(H))
        th, ta, sg = Z.leja_ritz_params(H, s, lo, hi)
        z = got["ritz"].numpy()
        scale = max(1.0, float(np.max(np.abs(zl))))
        assert np.max(np.abs(z.real - zl.real)) <= 1e-10 * scale, name
        assert np.max(np.abs(np.abs(z.imag) - np.abs(zl.imag))) <= 1e-10 * scale, name
        for g, r in ((got["theta"], th), (got["tau"], ta), (got["sigma"], sg)):
            assert np.max(np.abs(g.cpu().numpy() - r)) <= 1e-10 * scale, name


LEJA_CASES = [("two_stage", "convdiff2d", 64, 5, 0), ("bcgs_pip2", "convdiff2d", 64, 5, 0),
              ("bcgs2_cholqr2", "laplace2d", 48, 10, 0), ("two_stage", "laplace2d", 64, 15, 0),
              ("two_stage", "convdiff2d", 93, 10, 20)]


@pytest.mark.parametrize("ortho,kind,N,s,s_hat", LEJA_CASES)
def test_solve_leja_matches_oracle(tsg, ortho, kind, N, s, s_hat):
    _say("case solve leja", ortho, kind, N, s, s_hat)
    pr = W.make_problem(kind, N, seed=1)
    A = tsg.CSRMatrix.from_host(pr["A"])
    b = torch.as_tensor(pr["b"], device="cuda")
    x, info = tsg.solve(A, b, m=60, s=s, tol=1e-10, ortho=ortho, basis="leja", s_hat=s_hat)
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=s, tol=1e-10, ortho=ortho, basis="leja", s_hat=s_hat or None)
    xg = x.cpu().numpy()
    _say(f"  iters gpu {info.iters} oracle {ref['iters']}; newton from cycle {info.newton_from_cycle}")
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert info.converged and relres <= 1e-10
    assert info.newton_from_cycle == ref["basis_switched_after"]
    assert info.iters == ref["iters"] and info.cycles == ref["cycles"]
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


def test_solve_leja_mixed_precision(tsg):
    """FP32 basis with the Leja-Ritz Newton basis (Ritz values and shifts in FP64)."""
    _say("case solve leja fp32_ir")
    pr = W.make_problem("convdiff2d", 96, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"])
    b = torch.as_tensor(pr["b"], device="cuda")
    x, info = tsg.solve(A, b, m=60, s=10, tol=1e-10, basis="leja", precision="fp32_ir")
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=10, tol=1e-10, basis="leja")
    xg = x.cpu().numpy()
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    _say(f"  iters {info.iters} (fp64 oracle {ref['iters']}), newton from {info.newton_from_cycle}")
    assert info.converged and relres <= 1e-10
    assert info.newton_from_cycle == 1
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-7


def test_leja_graph_replay_matches_eager(tsg):
    """The Ritz kernel is part of the captured cycle: replays and direct launches agree."""
    _say("case leja graph vs eager")
    pr = W.make_problem("convdiff2d", 64, seed=1)
    A = tsg.CSRMatrix.from_host(pr["A"])
    b = torch.as_tensor(pr["b"], device="cuda")
    xs = []
    for graph in (True, False):
        x, info = tsg.solve(A, b, m=60, s=5, tol=1e-10, basis="leja", graph=graph)
        assert info.newton_from_cycle == 1
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
