"""GPU parity of right preconditioning by multicolor Gauss-Seidel (precond = 'mcgs').

* Coloring (Jones-Plassmann rounds on the device) equal, row by row, to the oracle's
  greedy coloring in decreasing SplitMix64 priority (integer result: bit-exact).
* One sweep z = M^{-1} w against the oracle's sweep (1e-13 relative: the GPU sweeps the
  color-ordered system, whose rows hold their entries in renamed-column order).
* Preconditioned solves of every variant against the oracle: iteration and cycle
  counts equal, x within 1e-10; two-stage with s_hat < m and the Leja basis; graph
  replay against direct launches; the explicit FP64 residual gate.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gmres as G
from oracle import precond as PC
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


@pytest.mark.parametrize("kind,N", [("laplace2d", 37), ("laplace3d", 11), ("convdiff2d", 45), ("laplace2d", 300)])
def test_coloring_and_sweep_match_oracle(tsg, kind, N):
    _say("case precond coloring", kind, N)
    pr = W.make_problem(kind, N, seed=1)
    A = tsg.CSRMatrix.from_host(pr["A"]).precond_setup()
    ref = PC.coloring(pr["A"])
    got = A.colors().cpu().numpy()
    assert np.array_equal(got, ref)
    assert A.ncolors == int(ref.max()) + 1
    w = np.random.default_rng(N).uniform(-1, 1, pr["A"].n)
    z = tsg.precond_apply(A, torch.as_tensor(w, device="cuda")).cpu().numpy()
    zr = PC.mcgs_apply(pr["A"], ref, w)
    assert np.max(np.abs(z - zr)) <= 1e-13 * np.max(np.abs(zr))


def test_coloring_sweep_and_solve_variable_widths(tsg):
    """Rows of 1 .. 32 nonzeros (symmetrized random pattern): the sweep's groups of 4 and
    every remainder; coloring bit-exact, one sweep and a preconditioned solve against the
    oracle."""
    _say("case precond variable widths")
    A0 = W.variable_width(2909, seed=9, symmetric=True)
    A = tsg.CSRMatrix.from_host(A0).precond_setup()
    ref = PC.coloring(A0)
    assert np.array_equal(A.colors().cpu().numpy(), ref)
    w = np.random.default_rng(10).uniform(-1, 1, A0.n)
    z = tsg.precond_apply(A, torch.as_tensor(w, device="cuda")).cpu().numpy()
    zr = PC.mcgs_apply(A0, ref, w)
    assert np.max(np.abs(z - zr)) <= 1e-13 * np.max(np.abs(zr))
    # the preconditioned Krylov basis of this operator converges within ~20 vectors: with
    # s = 5 its panels' Pythagorean pivots sit at the rounding level (a pass decision either
    # way is correct, so counts are not unique); with s = 2 every relative pivot is >= 3e-4
    b = W.uniform_vector(A0.n, seed=11)
    x, info = tsg.solve(A, torch.as_tensor(b, device="cuda"), m=10, s=2, tol=1e-10, precond="mcgs")
    out = G.sstep_gmres(A0, b, m=10, s=2, tol=1e-10, precond=PC.MulticolorGS(A0))
    assert info.converged and info.iters == out["iters"]
    assert np.linalg.norm(x.cpu().numpy() - out["x"]) <= 1e-10 * np.linalg.norm(out["x"])


PRECOND_CASES = [("two_stage", "laplace2d", 64, 5, 0, "monomial"), ("bcgs_pip2", "laplace2d", 64, 5, 0, "monomial"),
                 ("bcgs2_cholqr2", "convdiff2d", 45, 5, 0, "monomial"), ("cgs2", "convdiff2d", 45, 5, 0, "monomial"),
                 ("two_stage", "convdiff2d", 93, 5, 20, "monomial"), ("two_stage", "laplace2d", 64, 10, 0, "leja")]


@pytest.mark.parametrize("ortho,kind,N,s,s_hat,basis", PRECOND_CASES)
def test_preconditioned_solve_matches_oracle(tsg, ortho, kind, N, s, s_hat, basis):
    _say("case precond solve", ortho, kind, N, s, s_hat, basis)
    pr = W.make_problem(kind, N, seed=2)
    A = tsg.CSRMatrix.from_host(pr["A"]).precond_setup()
    b = torch.as_tensor(pr["b"], device="cuda")
    x, info = tsg.solve(A, b, m=60, s=s, tol=1e-10, ortho=ortho, basis=basis, s_hat=s_hat, precond="mcgs")
    P = PC.MulticolorGS(pr["A"])
    if ortho == "cgs2":
        ref = G.gmres(pr["A"], pr["b"], m=60, tol=1e-10, ortho="cgs2", precond=P)
    else:
        ref = G.sstep_gmres(pr["A"], pr["b"], m=60, s=s, tol=1e-10, ortho=ortho, basis=basis,
                            s_hat=s_hat or None, precond=P)
    xg = x.cpu().numpy()
    _say(f"  iters gpu {info.iters} oracle {ref['iters']}")
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], xg)) / np.linalg.norm(pr["b"])
    assert info.converged and relres <= 1e-10
    assert info.iters == ref["iters"] and info.cycles == ref["cycles"]
    assert np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-10


def test_preconditioned_graph_replay_matches_eager(tsg):
    _say("case precond graph vs eager")
    pr = W.make_problem("convdiff2d", 64, seed=3)
    A = tsg.CSRMatrix.from_host(pr["A"]).precond_setup()
    b = torch.as_tensor(pr["b"], device="cuda")
    xs = [tsg.solve(A, b, m=60, s=5, tol=1e-10, precond="mcgs", graph=g)[0].cpu().numpy() for g in (True, False)]
    assert np.array_equal(xs[0], xs[1])


def test_precond_requires_setup(tsg):
    pr = W.make_problem("laplace2d", 16, seed=0)
    A = tsg.CSRMatrix.from_host(pr["A"])
    with pytest.raises(tsg.TSGError):
        tsg.solve(A, torch.as_tensor(pr["b"], device="cuda"), m=30, s=5, precond="mcgs")


def test_server_rejects_precond(tsg):
    with pytest.raises(tsg.TSGError):
        tsg.Server(64 << 20, m=30, s=5, precision="fp64", precond="mcgs")


def test_precond_and_solve_use_caller_memory_only(tsg):
    """tsg_csr_precond builds everything in the caller's buffer (coloring scratch, P A P^T,
    its handle block and packed copy, the sweep layout) and a preconditioned solve runs in the
    caller's workspace: after a warm-up on another operator (every kernel loaded), the set-up
    and an eager solve leave the device's free memory unchanged -- the library's only device
    allocation is the handle's 4 KiB block, made by tsg_csr_create before."""
    lib = tsg.load_library()
    _say("case precond caller memory")
    pr0 = W.make_problem("convdiff2d", 40, seed=1)
    A0 = tsg.CSRMatrix.from_host(pr0["A"]).precond_setup()
    tsg.solve(A0, torch.as_tensor(pr0["b"], device="cuda"), m=30, s=5, tol=1e-8, precond="mcgs", graph=False)
    pr = W.make_problem("convdiff2d", 96, seed=4)
    A = tsg.CSRMatrix.from_host(pr["A"])
    nbytes = int(lib.tsg_csr_precond_bytes(A.handle))
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ptr = (buf.data_ptr() + 255) // 256 * 256
    b = torch.as_tensor(pr["b"], device="cuda")
    x = torch.zeros_like(b)
    need = tsg.solve_workspace_bytes(A, m=60, s=5, precond="mcgs")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert ws.data_ptr() % 256 == 0
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    assert lib.tsg_csr_precond(A.handle, ptr, nbytes, torch.cuda.current_stream().cuda_stream) == 0
    A._precond = buf  # the buffer lives as long as the handle
    x, info = tsg.solve(A, b, x=x, m=60, s=5, tol=1e-10, precond="mcgs", graph=False, workspace=ws)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    _say(f"  buffer {nbytes} bytes ({nbytes / (8 * A.n):.1f} doubles per row); free memory change {free0 - free1}")
    assert info.converged
    assert free1 == free0, (free0, free1)
    relres = np.linalg.norm(pr["b"] - S.spmv(pr["A"], x.cpu().numpy())) / np.linalg.norm(pr["b"])
    assert relres <= 1e-10
