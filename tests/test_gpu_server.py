"""The solve server (continuous batching, tsg_server_* through the C ABI).

A request computes bit for bit what tsg_solve computes for it, whatever else shares the
batched launches: checked with requests of different sizes and operators submitted
together, arriving while others run, and admitted one by one through an arena too small
to hold them all; and served results against the oracle directly.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import gmres as G
from oracle import sparse as S

pytestmark = pytest.mark.gpu

KW = dict(m=60, s=5, tol=1e-8, basis="shifted", precision="fp32_ir")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def tsg():
    import paper_2402_15033_amd as m

    m.load_library()
    return m


def _requests(tsg, specs):
    out = []
    for i, (kind, N) in enumerate(specs):
        pr = W.make_problem(kind, N, seed=100 + i, rhs="uniform", pe_range=(1.0, 100.0))
        A = tsg.CSRMatrix.from_host(pr["A"])
        b = torch.as_tensor(pr["b"], device="cuda")
        out.append((pr, A, b))
    return out


SPECS = [("laplace2d", 32), ("convdiff2d", 40), ("laplace2d", 48), ("convdiff2d", 24), ("laplace2d", 20)]


def _alone(tsg, reqs, **kw):
    res = []
    for pr, A, b in reqs:
        x, info = tsg.solve(A, b, **dict(KW, **kw))
        res.append((x, info))
    return res


def _drain(srv, n):
    got = {}
    steps = 0
    while len(got) < n:
        srv.step()
        for tag, x, info in srv.poll():
            got[tag] = (x, info)
        steps += 1
        assert steps < 100000
    return got


def test_mix_equals_alone(tsg):
    _say("case server mix == alone")
    reqs = _requests(tsg, SPECS)
    alone = _alone(tsg, reqs)
    srv = tsg.Server(1 << 30, **KW)
    for i, (pr, A, b) in enumerate(reqs):
        srv.submit(i, A, b)
    got = _drain(srv, len(reqs))
    for i, (pr, A, b) in enumerate(reqs):
        xa, ia = alone[i]
        xm, im = got[i]
        assert torch.equal(xa, xm), i
        assert (ia.iters, ia.cycles, ia.status) == (im.iters, im.cycles, im.status)
        relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xm.cpu().numpy())) / np.linalg.norm(pr["b"])
        assert im.converged and relres <= 1e-8
    srv.close()


def test_continuous_admission_and_budget(tsg):
    """Requests arrive while others are active, and an arena that holds two requests at a
    time admits the rest as memory frees up; every result is still the solo result."""
    _say("case server admission")
    reqs = _requests(tsg, SPECS)
    alone = _alone(tsg, reqs)
    probe = tsg.Server(1 << 30, **KW)
    sizes = [probe.request_bytes(A) for _, A, _ in reqs]
    probe.close()
    top2 = sum(sorted(sizes)[-2:])
    # launch images (256 slots x 512 KiB) + heads + room for the two largest requests
    arena = 8 * 512 * 1024 + (1 << 20) + top2 + 4096
    srv = tsg.Server(arena, max_active=8, **KW)
    srv.submit(0, *reqs[0][1:])
    srv.submit(1, *reqs[1][1:])
    got = {}
    max_active = 0
    for step in range(3):
        na, nq = srv.step()
        max_active = max(max_active, na)
        for tag, x, info in srv.poll():
            got[tag] = (x, info)
    for i in range(2, len(reqs)):
        srv.submit(i, *reqs[i][1:])
    while len(got) < len(reqs):
        na, nq = srv.step()
        max_active = max(max_active, na)
        assert na <= 2
        for tag, x, info in srv.poll():
            got[tag] = (x, info)
    for i in range(len(reqs)):
        assert torch.equal(alone[i][0], got[i][0]), i
        assert alone[i][1].iters == got[i][1].iters
    assert max_active == 2
    srv.close()


def test_fp64_requests_and_zero_rhs(tsg):
    _say("case server fp64 + b=0")
    reqs = _requests(tsg, SPECS[:3])
    kw = dict(precision="fp64", basis="monomial", tol=1e-10)
    alone = _alone(tsg, reqs, **kw)
    srv = tsg.Server(1 << 30, **dict(KW, **kw))
    for i, (pr, A, b) in enumerate(reqs):
        srv.submit(i, A, b)
    zb = torch.zeros_like(reqs[0][2])
    x0 = torch.ones_like(zb)
    srv.submit(99, reqs[0][1], zb, x0)
    got = _drain(srv, len(reqs) + 1)
    for i in range(len(reqs)):
        assert torch.equal(alone[i][0], got[i][0])
    x, info = got[99]
    assert info.converged and info.iters == 0 and float(x.abs().max()) == 0.0
    srv.close()


@pytest.mark.parametrize("kw", [dict(precision="fp64", basis="leja", s=10, tol=1e-10),
                                dict(precision="fp32_ir", basis="leja", s=10, tol=1e-8)])
def test_leja_basis_requests_equal_alone(tsg, kw):
    """Every request finds its own Newton shifts (Ritz values of its first cycle) inside the
    batched launches, and takes the shifted Cholesky QR pass where its panels need it."""
    _say("case server leja", kw)
    reqs = _requests(tsg, SPECS)
    alone = _alone(tsg, reqs, **kw)
    srv = tsg.Server(1 << 30, **dict(KW, **kw))
    for i, (pr, A, b) in enumerate(reqs):
        srv.submit(i, A, b)
    got = _drain(srv, len(reqs))
    for i in range(len(reqs)):
        xa, ia = alone[i]
        xm, im = got[i]
        assert torch.equal(xa, xm), i
        assert (ia.iters, ia.newton_from_cycle, ia.shifted_passes) == (im.iters, im.newton_from_cycle,
                                                                       im.shifted_passes)
        assert im.converged
    srv.close()


def test_request_larger_than_arena_is_rejected(tsg):
    _say("case server reject")
    reqs = _requests(tsg, [("laplace2d", 128)])
    srv = tsg.Server(256 * 512 * 1024 + (1 << 20) + (1 << 16), **KW)
    with pytest.raises(tsg.TSGError):
        srv.submit(0, *reqs[0][1:])
    srv.close()


def test_served_results_match_oracle(tsg):
    """Served requests against the oracle, not against tsg_solve: a batch of operators and
    sizes submitted together plus one arriving while they run.  FP64 requests (monomial and
    shifted bases): the oracle's iteration count and x within 1e-10 wherever the oracle's
    cycles took no fallback pass and no truncation (else x within 2 tol kappa_2(A)).  Mixed-form requests
    (FP32 basis, FP64 refinement, tol 1e-8): the explicit residual at most tol, and x within
    2 tol kappa_2(A) of the oracle's FP64 x (kappa_2 in closed form for the Laplacian, from
    the SVD of the assembled operator for convection-diffusion)."""
    _say("case server vs oracle")
    specs = SPECS[:4]
    reqs = _requests(tsg, specs)
    for kw in (dict(precision="fp64", basis="monomial", tol=1e-10),
               dict(precision="fp64", basis="shifted", tol=1e-10),
               dict(precision="fp32_ir", basis="shifted", tol=1e-8)):
        srv = tsg.Server(1 << 30, **dict(KW, **kw))
        for i, (pr, A, b) in enumerate(reqs[:3]):
            srv.submit(i, A, b)
        got = {}
        for step in range(4):
            srv.step()
            for tag, x, info in srv.poll():
                got[tag] = (x, info)
        srv.submit(3, reqs[3][1], reqs[3][2])
        got.update(_drain(srv, len(reqs) - len(got)))
        srv.close()
        for i, (pr, A, b) in enumerate(reqs):
            x, info = got[i]
            xg = x.cpu().numpy()
            relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
            assert info.converged and relres <= kw["tol"], (i, kw, relres)
            kind, N = specs[i]
            if kw["precision"] == "fp64":
                ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-10, basis=kw["basis"], record=True)
                err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
                clean = ref["fallbacks"] == 0 and all(r["Qhat"].shape[1] == 61 for r in ref["records"])
                _say(f"  {kw['basis']} {specs[i]}: iters served {info.iters} oracle {ref['iters']}, "
                     f"|x - x_oracle| {err:.1e}{'' if clean else ' (oracle took fallback passes or truncated)'}")
                if clean:
                    assert info.iters == ref["iters"] and info.cycles == ref["cycles"]
                    assert err <= 1e-10
                else:
                    # the monomial basis of the strongly convective 24^2 operator: the oracle's
                    # pass and truncation decisions sit at rounding level (both sides converge);
                    # two solutions with relative residuals <= tol differ by <= 2 tol kappa
                    kap = np.linalg.cond(G.dense_solve(pr["A"], pr["b"])[1])
                    assert err <= 2 * 1e-10 * kap
            else:
                ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=5, tol=1e-12, basis="shifted")
                if kind == "laplace2d":
                    lmin, lmax = W.laplace_extreme_eigs(N, 2)
                    kap = lmax / lmin
                else:
                    kap = np.linalg.cond(G.dense_solve(pr["A"], pr["b"])[1])
                err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
                _say(f"  mixed {specs[i]}: iters {info.iters}, |x - x_fp64| {err:.1e}, bound {2 * 1e-8 * kap:.1e}")
                assert err <= 2 * 1e-8 * kap

