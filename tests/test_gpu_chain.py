"""One stage-1 panel through the solver's fallback chain on the GPU (tsg_block_pip: the
solver's own reductions, updates, tails and gates) against the oracle's BCGS-PIP with the
explicit second pass and the shifted Cholesky QR pass (`blockortho.bcgs_pip_explicit`),
element by element, on panels whose pivots are decided with a wide margin:

* a healthy panel (PIP alone), and PIP's trigger at a relative pivot ~1e-10 (taken at the
  solver's 1e-8, not at 1e-12);
* a nearly dependent panel, delta = 1e-7 (kappa([Q, V]) ~ 1e7: PIP's pivots cancel to
  ~1e-14, the explicit pass's are O(1));
* an ill-conditioned panel, kappa = 1e9 (the explicit pass's last relative pivot ~1e-18:
  the shifted pass; without it, a breakdown at that column);
* columns in span(Q) (every column, and one in the middle): a breakdown at the same column.

Tolerances: the same pass on both sides; P, R and Qnew within 1e-12 kappa (relative, the
panel's conditioning times the rounding of the reductions); the GPU's own result orthogonal
to the level the chain guarantees and V = Q P + Qnew R to rounding."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import blockortho as BO
from oracle import dense as D

pytestmark = pytest.mark.gpu

PIP_TOL, PIVOT_TOL = 1e-8, 1e-12


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def tsg():
    import paper_2402_15033_amd as m

    m.load_library()
    return m


def _gpu(tsg, Q, V, chain, pip_tol=PIP_TOL):
    k, s = Q.shape[1], V.shape[1]
    X = np.hstack([Q, V])
    Xt = torch.as_tensor(np.ascontiguousarray(X.T), device="cuda")
    out = tsg.block_pip(Xt, k, s, pip_tol=pip_tol, pivot_tol=PIVOT_TOL, chain=chain)
    torch.cuda.synchronize()
    Xr = Xt.cpu().numpy().T
    return out, Xr[:, k:], out["P"].cpu().numpy(), out["R"].cpu().numpy()


def _oracle(Q, V, chain, pip_tol=PIP_TOL):
    if chain == 0:
        Qn, P, R = BO.bcgs_pip(Q, V, pip_tol)
        return Qn, P, R, 0
    return BO.bcgs_pip_explicit(Q, V, PIVOT_TOL, shifted=chain == 2, pip_tol=pip_tol)


def _compare(tsg, Q, V, chain, kappa, passes, pip_tol=PIP_TOL, orth=1e-13):
    out, Qn, P, R = _gpu(tsg, Q, V, chain, pip_tol)
    Qo, Po, Ro, po = _oracle(Q, V, chain, pip_tol)
    k, s = Q.shape[1], V.shape[1]
    eP = np.linalg.norm(P - Po) / np.linalg.norm(Po) if k else 0.0
    eR = np.linalg.norm(R - Ro) / np.linalg.norm(Ro)
    eQ = np.linalg.norm(Qn - Qo) / np.sqrt(s)
    _say(f"  passes gpu {out['passes']} oracle {po}; |P-Po| {eP:.1e} |R-Ro| {eR:.1e} |Q-Qo| {eQ:.1e}")
    assert out["status"] == 0 and out["passes"] == po == passes
    tol = 1e-12 * kappa
    assert eP <= tol and eR <= tol and eQ <= tol
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) > 0)
    # as orthogonal as the chain makes it (PIP alone on an ill-conditioned panel: O(eps kappa^2),
    # as far from orthogonal as the oracle's own result)
    assert D.orth_error(np.hstack([Q, Qn])) <= max(orth, 10 * D.orth_error(np.hstack([Q, Qo])))
    assert np.linalg.norm(V - Q @ P - Qn @ R) / np.linalg.norm(V) <= 1e-14


@pytest.mark.parametrize("n", [4000, 100003])
def test_chain_healthy_panel_is_pip(tsg, n):
    _say("case chain healthy", n)
    Q, V = W.nearly_dependent_panel(n, 9, 5, 1.0, seed=12)
    _compare(tsg, Q, V, 2, 1.0, 0)
    _compare(tsg, Q, V, 0, 1.0, 0)


def test_chain_first_panel_without_q(tsg):
    _say("case chain k = 0")
    V = W.gaussian_block(30011, 6, seed=3)
    _compare(tsg, np.zeros((30011, 0)), V, 2, 1.0, 0)


@pytest.mark.parametrize("n", [4000, 100003])
def test_chain_trigger_threshold(tsg, n):
    """Relative PIP pivots ~1e-10: the explicit pass at the solver's trigger of 1e-8, PIP's
    own result at 1e-12 (there its orthogonality is only O(eps kappa^2) ~ 1e-6)."""
    _say("case chain trigger", n)
    Q, V = W.nearly_dependent_panel(n, 9, 5, 1e-5, seed=31)
    _compare(tsg, Q, V, 2, 1e5, 1)
    # PIP's own factors carry O(eps kappa^2) errors
    _compare(tsg, Q, V, 1, 1e10, 0, pip_tol=PIVOT_TOL)


@pytest.mark.parametrize("n,k,s", [(4000, 9, 5), (100003, 50, 10), (20000, 9, 16)])
def test_chain_explicit_second_pass(tsg, n, k, s):
    _say("case chain second pass", n, k, s)
    Q, V = W.nearly_dependent_panel(n, k, s, 1e-7, seed=11)
    _compare(tsg, Q, V, 2, 1e7, 1)
    _compare(tsg, Q, V, 1, 1e7, 1)


@pytest.mark.parametrize("n", [4000, 100003])
def test_chain_shifted_pass(tsg, n):
    _say("case chain shifted", n)
    Q, V = W.ill_conditioned_panel(n, 9, 6, 1e9, seed=21)
    _compare(tsg, Q, V, 2, 1e9, 2, orth=1e-10)
    # without the shifted pass the explicit pass fails at the last column on both sides
    out, _, _, _ = _gpu(tsg, Q, V, 1)
    with pytest.raises(D.CholeskyBreakdown) as e:
        _oracle(Q, V, 1)
    assert out["status"] == 2 and out["fail_col"] == e.value.index == 5


@pytest.mark.parametrize("chain", [1, 2])
def test_chain_rejects_columns_in_span_q(tsg, chain):
    _say("case chain dependent", chain)
    n, k, s = 4000, 9, 5
    Q, V = W.nearly_dependent_panel(n, k, s, 0.0, seed=13)
    out, _, _, _ = _gpu(tsg, Q, V, chain)
    with pytest.raises(D.CholeskyBreakdown) as e:
        _oracle(Q, V, chain)
    assert out["status"] == 2 and out["fail_col"] == e.value.index == 0
    Q, V = W.nearly_dependent_panel(n, k, s, 1e-3, seed=14)
    V[:, 2] = Q @ np.arange(1.0, k + 1.0)
    out, _, _, _ = _gpu(tsg, Q, V, chain)
    with pytest.raises(D.CholeskyBreakdown) as e:
        _oracle(Q, V, chain)
    assert out["status"] == 2 and out["fail_col"] == e.value.index == 2
