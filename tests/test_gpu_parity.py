"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64):
* SpMV: per-entry relative 4 eps (CSR order on both sides; the GPU contracts to FMA).
* Block orthogonalization with the same scheme: ||R_gpu - R_oracle|| / ||R|| <= 1e-12 and
  ||Q_gpu - Q_oracle|| <= 1e-12 sqrt(k) on well-conditioned blocks (rounding of the reductions
  differs: per-lane, per-wave and per-block partial sums against BLAS); O(eps) orthogonality.
* Solves (A-19 gates): explicit relative residual <= tol recomputed by the oracle's SpMV;
  the same iteration count as the oracle's run of the same variant; relative difference of the
  iterates <= 1e-10 where both ran the same cycles; error against x_true <= 2 tol kappa_2(A).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import blockortho as BO
from oracle import dense as D
from oracle import gmres as G
from oracle import sparse as S

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def tsg():
    import paper_2402_15033_amd as m

    m.load_library()
    return m


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


# ------------------------------------------------------------------------- SpMV
@pytest.mark.parametrize("kind,N", [("laplace2d", 37), ("laplace3d", 11), ("convdiff2d", 45)])
def test_spmv_and_gershgorin(tsg, kind, N):
    _say("case spmv", kind, N)
    pr = W.make_problem(kind, N, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x = W.uniform_vector(pr["A"].n, 9)
    y = tsg.spmv(A, _dev(x)).cpu().numpy()
    yr = S.spmv(pr["A"], x)
    scale = np.abs(pr["A"].to_scipy()) @ np.abs(x)
    assert np.all(np.abs(y - yr) <= 4 * EPS * scale + 1e-300)
    lo, hi = A.gershgorin()
    lo_o, hi_o = S.gershgorin(pr["A"])
    assert abs(lo - lo_o) <= 1e-14 * max(1, abs(lo_o)) and abs(hi - hi_o) <= 1e-14 * abs(hi_o)


# ------------------------------------------------------------------------- ortho
def _ortho_case(tsg, X, s, algo):
    n, k = X.shape
    Xt = _dev(X.T)  # (k, n) contiguous = column-major n x k
    _, R, oerr = tsg.orthogonalize(Xt, s=s, algo=algo, orth_err=True)
    Q = Xt.cpu().numpy().T
    Rg = R.cpu().numpy()
    Qo, Ro = BO.orthogonalize(X, s, algo)
    return Q, Rg, Qo, Ro, oerr


@pytest.mark.parametrize("algo", ["two_stage", "bcgs_pip2", "bcgs2_cholqr2"])
@pytest.mark.parametrize("n,k,s", [(100003, 61, 5), (20000, 61, 10), (7777, 14, 5), (4096, 1, 5),
                                   (129, 64, 16), (300, 9, 3)])
def test_orthogonalize_matches_oracle(tsg, algo, n, k, s):
    _say("case ortho", algo, n, k, s)
    X = W.gaussian_block(n, k, seed=n + k)
    Q, R, Qo, Ro, oerr = _ortho_case(tsg, X, s, algo)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 1e-12
    assert np.linalg.norm(Q - Qo) / np.sqrt(k) <= 1e-12
    assert D.orth_error(Q) <= 1e-13
    assert abs(oerr - D.orth_error(Q)) <= 1e-14
    assert D.repr_error(X, Q, R) <= 1e-14


@pytest.mark.parametrize("n,k,s,s_hat", [(100003, 61, 5, 5), (100003, 61, 5, 10), (100003, 61, 5, 20),
                                         (100003, 61, 5, 30), (20011, 47, 5, 10), (4096, 64, 3, 21),
                                         (300, 61, 10, 20)])
def test_orthogonalize_big_panels_match_oracle(tsg, n, k, s, s_hat):
    """Two-stage with several big panels (Sec. V, Fig. 5 with s_hat < k - 1): stage 1 per panel
    against every earlier column, stage 2 = BCGS-PIP of each big panel against the final
    columns before it, explicit Q per big panel -- against the oracle's same scheme."""
    _say("case ortho big panels", n, k, s, s_hat)
    X = W.gaussian_block(n, k, seed=n + k + s_hat)
    Xt = _dev(X.T)
    _, R, oerr = tsg.orthogonalize(Xt, s=s, algo="two_stage", orth_err=True, s_hat=s_hat)
    Q = Xt.cpu().numpy().T
    Rg = R.cpu().numpy()
    Qo, Ro = BO.two_stage(X, s, s_hat)
    eR = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
    eQ = np.linalg.norm(Q - Qo) / np.sqrt(k)
    _say(f"  |R - Ro| {eR:.2e} |Q - Qo| {eQ:.2e} orth {D.orth_error(Q):.2e}")
    assert np.allclose(np.tril(Rg, -1), 0)
    assert eR <= 1e-12 and eQ <= 1e-12
    assert D.orth_error(Q) <= 1e-13 and abs(oerr - D.orth_error(Q)) <= 1e-14
    assert D.repr_error(X, Q, Rg) <= 1e-14


def test_orthogonalize_big_panels_glued(tsg):
    """Fig. 8's glued matrix (panel condition 1e7, cumulative conditioning growing by 2 per
    panel) with s_hat = 20: O(eps) orthogonality, the unique QR to kappa eps."""
    _say("case ortho big panels glued")
    V = W.glued_block(20000, 12, 5, 1e7, seed=1)
    Xt = _dev(V.T)
    _, R = tsg.orthogonalize(Xt, s=5, algo="two_stage", s_hat=20)
    Q = Xt.cpu().numpy().T
    Qo, Ro = BO.two_stage(V, 5, 20)
    assert D.orth_error(Q) <= 1e-13
    assert D.repr_error(V, Q, R.cpu().numpy()) <= 1e-15
    assert np.linalg.norm(R.cpu().numpy() - Ro) / np.linalg.norm(Ro) <= 1e-8


def test_orthogonalize_glued_matrix(tsg):
    _say("case ortho glued")
    V = W.glued_block(20000, 12, 5, 1e7, seed=1)  # 61 columns, panel condition 1e7
    for algo in ("two_stage", "bcgs_pip2", "bcgs2_cholqr2"):
        Q, R, Qo, Ro, _ = _ortho_case(tsg, V, 5, algo)
        assert D.orth_error(Q) <= 1e-13, algo
        assert D.repr_error(V, Q, R) <= 1e-15, algo
        # both are the unique QR up to kappa * eps
        assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 1e-8, algo


def test_orthogonalize_breakdown_is_reported(tsg):
    _say("case ortho breakdown")
    # a zero column gives an exactly zero Cholesky pivot (an exactly duplicated column only
    # gives a rounding-noise pivot of either sign, so it is not a reliable breakdown)
    X = W.gaussian_block(5000, 11, seed=2)
    X[:, 7] = 0.0
    with pytest.raises(D.CholeskyBreakdown):
        BO.orthogonalize(X, 5, "two_stage")
    for algo in ("two_stage", "bcgs_pip2", "bcgs2_cholqr2"):
        with pytest.raises(tsg.TSGError) as ei:
            _ortho_case(tsg, X, 5, algo)
        assert ei.value.status == 2


# ------------------------------------------------------------------------- solves
VARIANTS = [("two_stage", "two_stage"), ("bcgs_pip2", "bcgs_pip2"),
            ("bcgs2_cholqr2", "bcgs2_cholqr2"), ("cgs2", "cgs2")]


def _oracle_run(pr, variant, **kw):
    if variant == "cgs2":
        return G.gmres(pr["A"], pr["b"], ortho="cgs2", m=kw["m"], tol=kw["tol"])
    return G.sstep_gmres(pr["A"], pr["b"], ortho=variant, m=kw["m"], s=kw["s"], tol=kw["tol"],
                         basis=kw.get("basis", "monomial"))


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("variant,_o", VARIANTS)
def test_solve_laplace64_matches_oracle(tsg, seed, variant, _o):
    """The 64 x 64 2D Laplace configuration: m = 60, s = 5, tol 1e-10, x0 = 0."""
    _say("case solve laplace64", variant, seed)
    pr = W.make_problem("laplace2d", 64, seed=seed)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=5, tol=1e-10, ortho=variant)
    xg = x.cpu().numpy()
    ref = _oracle_run(pr, variant, m=60, s=5, tol=1e-10)
    bn = np.linalg.norm(pr["b"])
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / bn
    assert info.converged and relres <= 1e-10, (info, relres)
    assert abs(info.relres - relres) <= 1e-3 * relres + 1e-16
    assert info.iters == ref["iters"] and info.cycles == ref["cycles"], (info.iters, ref["iters"])
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10
    lmin, lmax = W.laplace_extreme_eigs(64, 2)
    xt = pr["x_true"]
    assert np.linalg.norm(xg - xt) / np.linalg.norm(xt) <= 2 * 1e-10 * lmax / lmin


@pytest.mark.parametrize("variant,_o", VARIANTS)
def test_solve_laplace3d_matches_oracle(tsg, variant, _o):
    """3D Laplace 7-point, 24^3 (n = 13824; the generated stand-in for Table 4's Laplace3D at
    a size the oracle finishes in seconds): m = 60, s = 5, tol 1e-10, every variant."""
    _say("case solve laplace3d 24", variant)
    pr = W.make_problem("laplace3d", 24, seed=2)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=5, tol=1e-10, ortho=variant)
    xg = x.cpu().numpy()
    ref = _oracle_run(pr, variant, m=60, s=5, tol=1e-10)
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    _say(f"  iters {info.iters} oracle {ref['iters']}; relres {relres:.2e}")
    assert info.converged and relres <= 1e-10, (info, relres)
    assert info.iters == ref["iters"] and info.cycles == ref["cycles"], (info.iters, ref["iters"])
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10
    lmin, lmax = W.laplace_extreme_eigs(24, 3)
    xt = pr["x_true"]
    assert np.linalg.norm(xg - xt) / np.linalg.norm(xt) <= 2 * 1e-10 * lmax / lmin


@pytest.mark.parametrize("variant,_o", VARIANTS)
def test_solve_convdiff_ragged(tsg, variant, _o):
    """Nonsymmetric operator, n = 93^2 (not a multiple of any tile), s = 5 / m = 30."""
    _say("case solve convdiff93", variant)
    pr = W.make_problem("convdiff2d", 93, seed=4)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=30, s=5, tol=1e-10, ortho=variant)
    xg = x.cpu().numpy()
    ref = _oracle_run(pr, variant, m=30, s=5, tol=1e-10)
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert info.converged and relres <= 1e-10
    assert info.iters == ref["iters"], (info.iters, ref["iters"])
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


def test_solve_shifted_basis_s10(tsg):
    _say("case solve shifted s10")
    pr = W.make_problem("laplace2d", 48, seed=5)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=10, tol=1e-10, basis="shifted")
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=10, tol=1e-10, basis="shifted")
    xg = x.cpu().numpy()
    assert info.converged and info.iters == ref["iters"]
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


@pytest.mark.parametrize("s_hat", [5, 10, 20, 30])
def test_solve_big_panels_match_oracle(tsg, s_hat):
    """Two-stage with big panels s_hat < m: stage 2 of every completed big panel against the
    final columns, residual checked at each big-panel end (Table 2's check points)."""
    _say("case solve big panels", s_hat)
    pr = W.make_problem("laplace2d", 64, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=5, tol=1e-10, s_hat=s_hat)
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-10, s_hat=s_hat)
    xg = x.cpu().numpy()
    _say(f"  iters gpu {info.iters} oracle {ref['iters']}")
    assert info.converged and info.iters == ref["iters"] and info.cycles == ref["cycles"]
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert relres <= 1e-10


def test_solve_big_panels_convdiff_s10(tsg):
    _say("case solve big panels convdiff")
    pr = W.make_problem("convdiff2d", 93, seed=2)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=10, tol=1e-10, s_hat=20, basis="shifted")
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=10, tol=1e-10, s_hat=20, basis="shifted")
    assert info.converged and info.iters == ref["iters"]
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


@pytest.mark.parametrize("kind,N", [("laplace2d", 64), ("convdiff2d", 64)])
def test_solve_monomial_s10_explicit_second_pass(tsg, kind, N):
    """Monomial panels at s = 10 are beyond PIP's stability limit (Sec. IV-C): their relative
    pivots are 5e-12 .. 1.5e-9, below the stage-1 trigger of 1e-8, so every panel takes the
    explicit second pass on both sides, decided with a wide margin (the Pythagorean pivots'
    rounding is <= 2e-9), and the second pass's own pivots (>= 3.7e-12 against a threshold of
    1e-12, rounding <= 5e-13) are decided alike: equal pass counts, iteration and cycle counts,
    and iterates within 1e-10."""
    _say("case solve monomial s10 second pass", kind, N)
    pr = W.make_problem(kind, N, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=10, tol=1e-10, basis="monomial")
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=10, tol=1e-10, basis="monomial")
    xg = x.cpu().numpy()
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    _say(f"  fallbacks gpu {info.pip_fallbacks} oracle {ref['fallbacks']}; shifted {info.shifted_passes} "
         f"{ref['shifted']}; iters {info.iters} {ref['iters']}; |x - x_oracle| = {err:.2e}")
    assert ref["fallbacks"] >= 1 and info.pip_fallbacks == ref["fallbacks"]
    assert info.redone_cycles == 1  # the first cycle meets the fallback; the full cycle from then on
    assert info.shifted_passes == ref["shifted"]
    assert info.converged and info.iters == ref["iters"] and info.cycles == ref["cycles"]
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert relres <= 1e-10
    assert err <= 1e-10


def test_solve_tiny_system_with_breakdown(tsg):
    """n = 144 converges inside a cycle; the two-stage cycle truncates at the Cholesky
    breakdown (numerically invariant Krylov space) on both sides."""
    _say("case solve tiny breakdown")
    pr = W.make_problem("convdiff2d", 12, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=30, s=5, tol=1e-10)
    xg = x.cpu().numpy()
    x_lu, M = G.dense_solve(pr["A"], pr["b"])
    assert info.converged
    assert np.linalg.norm(xg - x_lu) / np.linalg.norm(x_lu) <= 2e-10 * np.linalg.cond(M)


def test_solve_max_iters_and_x0(tsg):
    _say("case solve max_iters")
    pr = W.make_problem("laplace2d", 64, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=5, tol=1e-10, max_iters=120)
    assert info.status == 1 and info.iters == 120 and info.cycles == 2
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-10, max_iters=120)
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10
    # restart from the returned x (resume): finishes like an uninterrupted solve
    x2, info2 = tsg.solve(A, _dev(pr["b"]), x=x.clone(), m=60, s=5, tol=1e-10)
    assert info2.converged and info2.iters == 360 - 120


def test_zero_rhs(tsg):
    pr = W.make_problem("laplace2d", 16, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x0 = torch.ones(A.n, dtype=torch.float64, device="cuda")
    x, info = tsg.solve(A, torch.zeros_like(x0), x=x0, m=60, s=5)
    assert info.converged and float(x.abs().max()) == 0.0


@pytest.mark.parametrize("kind,N,prec", [("laplace2d", 64, "fp64"), ("convdiff2d", 93, "fp64"),
                                         ("convdiff2d", 93, "fp32_ir"), ("laplace3d", 17, "fp64")])
def test_packed_operator_equals_csr(tsg, kind, N, prec):
    """The packed SELL-64 operator and the CSR kernels give the same solve bit for bit
    (same products, rounded the same way, summed in the same order)."""
    _say("case packed vs csr", kind, N, prec)
    pr = W.make_problem(kind, N, seed=4)
    b = _dev(pr["b"])
    kw = dict(m=60, s=5, tol=1e-10, precision=prec, basis="shifted")
    Ac = tsg.CSRMatrix.from_host(pr["A"], pack=False)
    Ap = tsg.CSRMatrix.from_host(pr["A"], pack=True)
    xc, ic = tsg.solve(Ac, b, **kw)
    xp, ip = tsg.solve(Ap, b, **kw)
    assert torch.equal(xc, xp)
    assert (ic.iters, ic.cycles) == (ip.iters, ip.cycles)
    Ap.unpack()
    xu, iu = tsg.solve(Ap, b, **kw)
    assert torch.equal(xc, xu)


def test_packed_operator_wide_columns(tsg):
    """A matrix whose column deltas exceed int16 uses the int32 packed columns."""
    _say("case packed int32 columns")
    import scipy.sparse as sp
    n = 70000
    rng = np.random.default_rng(5)
    rows = np.repeat(np.arange(n), 4)
    cols = rng.integers(0, n, size=4 * n)  # far columns: deltas beyond int16
    M = sp.csr_matrix((rng.uniform(0, 1, 4 * n), (rows, cols)), shape=(n, n)) + sp.eye(n, format="csr") * 8.0
    M = M.tocsr()
    M.sum_duplicates()
    M.sort_indices()
    A = W.CSR(n=n, row_ptr=M.indptr.astype(np.int32), col=M.indices.astype(np.int32), val=M.data.astype(np.float64))
    b = rng.uniform(-1, 1, n)
    Ac = tsg.CSRMatrix.from_host(A, pack=False)
    Ap = tsg.CSRMatrix.from_host(A, pack=True)
    x = _dev(rng.uniform(-1, 1, n))
    kw = dict(m=30, s=5, tol=1e-12, basis="shifted")
    xc, ic = tsg.solve(Ac, _dev(b), **kw)
    xp, ip = tsg.solve(Ap, _dev(b), **kw)
    assert torch.equal(xc, xp)
    ref = G.sstep_gmres(A, b, m=30, s=5, tol=1e-12, basis="shifted")
    assert ic.iters == ref["iters"]


@pytest.mark.parametrize("n,far,prec", [(2909, False, "fp64"), (2909, False, "fp32_ir"), (33309, True, "fp64")])
def test_packed_operator_variable_widths(tsg, n, far, prec):
    """Slices of every width 1 .. 20 (the packed SpMV's groups of 8 and every remainder,
    a ragged last slice): packed and CSR solves equal bit for bit; 16-bit deltas for the
    banded operator, 32-bit columns for the one with far columns."""
    _say("case packed variable widths", n, far, prec)
    A = W.variable_width(n, seed=7, far=far)
    b = W.uniform_vector(n, seed=8)
    kw = dict(m=30, s=5, tol=1e-12, precision=prec, basis="shifted")
    Ac = tsg.CSRMatrix.from_host(A, pack=False)
    Ap = tsg.CSRMatrix.from_host(A, pack=True)
    xc, ic = tsg.solve(Ac, _dev(b), **kw)
    xp, ip = tsg.solve(Ap, _dev(b), **kw)
    assert ic.converged and torch.equal(xc, xp)
    assert (ic.iters, ic.cycles) == (ip.iters, ip.cycles)
    if prec == "fp64" and n < 10000:
        ref = G.sstep_gmres(A, b, m=30, s=5, tol=1e-12, basis="shifted")
        assert ic.iters == ref["iters"]
        assert np.linalg.norm(xc.cpu().numpy() - ref["x"]) <= 1e-10 * np.linalg.norm(ref["x"])


def test_determinism(tsg):
    _say("case determinism")
    pr = W.make_problem("convdiff2d", 64, seed=1)
    A = tsg.CSRMatrix.from_host(pr["A"])
    b = _dev(pr["b"])
    x1, _ = tsg.solve(A, b, m=60, s=5, tol=1e-10)
    x2, _ = tsg.solve(A, b, m=60, s=5, tol=1e-10)
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("ortho,prec", [("two_stage", "fp64"), ("bcgs_pip2", "fp64"),
                                        ("bcgs2_cholqr2", "fp64"), ("cgs2", "fp64"),
                                        ("two_stage", "fp32_ir")])
def test_graph_replay_matches_eager(tsg, ortho, prec):
    """One captured restart cycle replayed once per cycle (many replays, with the host's
    read-back and synchronization between them, and directly launched timed cycles mixed
    in) gives the eager launches' iterate bit for bit."""
    _say("case graph vs eager", ortho, prec)
    pr = W.make_problem("convdiff2d", 64, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"])
    b = _dev(pr["b"])
    kw = dict(m=30, s=5, tol=1e-10, ortho=ortho, precision=prec, basis="shifted")
    xe, ie = tsg.solve(A, b, graph=False, **kw)
    assert ie.cycles >= 4
    for timing in (0, 3):
        _say("  graph, timing", timing)
        xg, ig = tsg.solve(A, b, graph=True, timing=timing, **kw)
        assert torch.equal(xe, xg)
        assert (ig.iters, ig.cycles, ig.status) == (ie.iters, ie.cycles, ie.status)
        assert ig.relres == ie.relres
    # sampled timing: passes 0, 3, 6, ... are timed, with the same launches per pass as
    # timing every pass of an eager solve.  A converged solve enqueues cycles + 1 passes:
    # the last one computes the final residual, which stops it (the rest is gated off).
    assert ig.timed_cycles == -(-(ie.cycles + 1) // 3)
    _, it = tsg.solve(A, b, graph=False, timing=1, **kw)
    assert it.timed_cycles == ie.cycles + 1
    assert it.redone_cycles == ig.redone_cycles == ie.redone_cycles
    if ie.redone_cycles:
        # a two-stage cycle that met a fallback ran twice (the first time cut short) and the
        # full sequence ran from then on: the cycles' launches differ, only the results agree
        return
    assert it.kernel_classes().keys() == ig.kernel_classes().keys()
    for name, (_, cnt, by) in it.kernel_classes().items():  # every cycle has the same launches
        _, cg, bg = ig.kernel_classes()[name]
        assert cnt * ig.timed_cycles == cg * it.timed_cycles, name
        assert by * ig.timed_cycles == bg * it.timed_cycles, name


# ------------------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("kind,N,basis", [("laplace2d", 128, "shifted"), ("convdiff2d", 160, "shifted"),
                                          ("convdiff2d", 48, "shifted")])
def test_mixed_precision_refinement(tsg, kind, N, basis):
    """FP32 basis / SpMV / tall-skinny products, FP64 Cholesky, least squares and outer residual:
    every restart cycle is one refinement step, so the FP64 gates still hold at tol 1e-10.
    The FP32 iterates have no oracle of their own (parity unpinned); the final x is compared
    with the FP64 oracle's x and with x_true within 2 tol kappa_2(A) (two solutions whose
    relative residuals are at most tol differ by at most that): kappa_2 in closed form for the
    Laplacian, from the SVD of the assembled operator for convection-diffusion on 48^2."""
    _say("case mixed", kind, N, basis)
    pr = W.make_problem(kind, N, seed=6)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=5, tol=1e-10, basis=basis, precision="fp32_ir")
    xg = x.cpu().numpy()
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert info.converged and relres <= 1e-10, (info, relres)
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-10, basis=basis)
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    if kind == "laplace2d":
        lmin, lmax = W.laplace_extreme_eigs(N, 2)
        kap = lmax / lmin
    elif N <= 64:
        kap = np.linalg.cond(G.dense_solve(pr["A"], pr["b"])[1])
    else:
        kap = None  # too large for the SVD here: the 48^2 case carries the kappa gate
    if kap is not None:
        assert err <= 2 * 1e-10 * kap
        xt = pr["x_true"]
        assert np.linalg.norm(xg - xt) / np.linalg.norm(xt) <= 2 * 1e-10 * kap
    _say(f"  mixed {kind}: iters {info.iters} (fp64 oracle {ref['iters']}), |x - x_fp64| = {err:.2e}")


@pytest.mark.parametrize("kind,N,s", [("laplace2d", 40, 12), ("laplace2d", 64, 15), ("convdiff2d", 40, 15)])
def test_solve_monomial_shifted_cholqr_pass(tsg, kind, N, s):
    """Monomial panels at s >= 12 are beyond the explicit second pass; both sides take the
    shifted Cholesky QR pass and converge.  Which panels take it is decided by pivots near
    the threshold (as for the explicit pass), so the gates are the explicit residual and
    ||x_gpu - x_oracle|| <= 2 tol kappa(A) ||x_oracle||."""
    _say("case solve monomial shifted pass", kind, N, s)
    pr = W.make_problem(kind, N, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=60, s=s, tol=1e-10)
    ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=s, tol=1e-10)
    xg = x.cpu().numpy()
    _say(f"  iters gpu {info.iters} oracle {ref['iters']}; shifted gpu {info.shifted_passes} oracle {ref['shifted']}")
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert info.converged and relres <= 1e-10
    assert info.shifted_passes > 0 and ref["shifted"] > 0
    if kind == "laplace2d":
        lmin, lmax = W.laplace_extreme_eigs(N, 2)
        kap = lmax / lmin
    else:
        kap = np.linalg.cond(G.dense_solve(pr["A"], pr["b"])[1])
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 2 * 1e-10 * kap


@pytest.mark.parametrize("m,s,basis,ortho,kind,N", [
    (63, 9, "shifted", "two_stage", "laplace2d", 40),   # m + 1 = 64 columns, s >= 8
    (63, 9, "shifted", "bcgs_pip2", "laplace2d", 40),
    (48, 16, "leja", "two_stage", "convdiff2d", 40),    # the largest step
    (63, 3, "shifted", "two_stage", "convdiff2d", 33),  # ragged n = 1089
])
def test_solve_largest_parameters_match_oracle(tsg, m, s, basis, ortho, kind, N):
    _say("case solve largest parameters", m, s, basis, ortho, kind, N)
    pr = W.make_problem(kind, N, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=m, s=s, tol=1e-10, basis=basis, ortho=ortho)
    ref = G.sstep_gmres(pr["A"], pr["b"], m=m, s=s, tol=1e-10, basis=basis, ortho=ortho)
    xg = x.cpu().numpy()
    _say(f"  iters gpu {info.iters} oracle {ref['iters']}")
    assert info.converged and info.iters == ref["iters"] and info.cycles == ref["cycles"]
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


@pytest.mark.parametrize("ortho", ["two_stage", "bcgs_pip2", "bcgs2_cholqr2", "cgs2"])
def test_solve_restart_length_one(tsg, ortho):
    """GMRES(1): one Krylov vector per cycle (the degenerate restart length), stopped by
    max_iters before convergence: 50 cycles equal the oracle's iterate."""
    _say("case solve m = 1", ortho)
    pr = W.make_problem("convdiff2d", 10, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"])
    x, info = tsg.solve(A, _dev(pr["b"]), m=1, s=1, tol=1e-10, max_iters=50, ortho=ortho)
    if ortho == "cgs2":
        ref = G.gmres(pr["A"], pr["b"], m=1, tol=1e-10, max_iters=50, ortho="cgs2")
    else:
        ref = G.sstep_gmres(pr["A"], pr["b"], m=1, s=1, tol=1e-10, max_iters=50, ortho=ortho)
    assert info.status == 1 and info.iters == ref["iters"] == 50 and info.cycles == 50
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10
