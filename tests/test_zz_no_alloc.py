"""The no-allocation entry point tsg_orthogonalize_noalloc (its workspace is the library's
file-scope device array) against tsg_orthogonalize with a caller workspace, through the
C ABI: two calls in a row, the second with a smaller block (the array keeps the first
call's contents), for the two-stage scheme and BCGS-PIP2; both against the FP64 oracle.
The same kernels run on the same block decomposition, so the results must be equal bit
for bit; against the oracle the ortho parity tolerances apply (R within 1e-12 relative,
Q within 1e-12 sqrt(k), orthogonality 1e-13)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from oracle import blockortho as BO
from oracle import dense as D

pytestmark = pytest.mark.gpu

# (n, k, s): the first call is the larger block, the second a smaller one with a ragged
# last panel
CALLS = [(100003, 61, 5), (7777, 14, 3)]


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def tsg():
    import paper_2402_15033_amd as m

    m.load_library()
    return m


def _run(tsg, X, s, algo, noalloc):
    n, k = X.shape
    Xt = torch.as_tensor(np.ascontiguousarray(X.T), device="cuda")
    _, R, oerr = tsg.orthogonalize(Xt, s=s, algo=algo, orth_err=True, noalloc=noalloc)
    torch.cuda.synchronize()
    return Xt.cpu().numpy().T, R.cpu().numpy(), oerr


@pytest.mark.parametrize("algo", ["two_stage", "bcgs_pip2"])
def test_noalloc_matches_workspace_entry(tsg, algo):
    blocks = [W.gaussian_block(n, k, seed=11 + n + k) for n, k, _ in CALLS]
    got = []
    for (n, k, s), X in zip(CALLS, blocks):  # two no-allocation calls in a row, larger first
        _say("case noalloc", algo, n, k, s)
        got.append(_run(tsg, X, s, algo, noalloc=True))
    for (n, k, s), X, (Qn, Rn, en) in zip(CALLS, blocks, got):
        _say("case workspace", algo, n, k, s)
        Qw, Rw, ew = _run(tsg, X, s, algo, noalloc=False)
        assert np.array_equal(Qn, Qw) and np.array_equal(Rn, Rw), (n, k, s)
        assert en == ew
        Qo, Ro = BO.orthogonalize(X, s, algo)
        assert np.linalg.norm(Rn - Ro) / np.linalg.norm(Ro) <= 1e-12
        assert np.linalg.norm(Qn - Qo) / np.sqrt(k) <= 1e-12
        assert D.orth_error(Qn) <= 1e-13
        assert abs(en - D.orth_error(Qn)) <= 1e-14


def test_noalloc_allocates_no_device_memory(tsg):
    """After both entry points have run once (kernels loaded), further no-allocation calls
    leave the device's free memory unchanged."""
    lib = tsg.load_library()
    n, k, s = CALLS[0]
    X = W.gaussian_block(n, k, seed=5)
    Xt = torch.as_tensor(np.ascontiguousarray(X.T), device="cuda")
    R = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    X0 = Xt.clone()
    _run(tsg, X, s, "two_stage", noalloc=False)
    assert lib.tsg_orthogonalize_noalloc(n, k, Xt.data_ptr(), n, R.data_ptr(), k, s, 0, 0, stream, None) == 0
    torch.cuda.synchronize()
    for _ in range(3):
        Xt.copy_(X0)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert lib.tsg_orthogonalize_noalloc(n, k, Xt.data_ptr(), n, R.data_ptr(), k, s, 0, 0, stream, None) == 0
        torch.cuda.synchronize()
        free2, _ = torch.cuda.mem_get_info()
        assert free2 == free1, (free1, free2)


def test_noalloc_rejects_blocks_beyond_its_scratch(tsg):
    lib = tsg.load_library()
    assert lib.tsg_orthogonalize_noalloc_max_bytes() >= lib.tsg_orthogonalize_workspace_bytes(1 << 28, 64, 16)
    fake = C.c_void_p(256)  # never dereferenced: the size check comes before any device work
    st = lib.tsg_orthogonalize_noalloc((1 << 28) + 1, 61, fake, (1 << 28) + 1, fake, 61, 5, 0, 0, None, None)
    assert st == -1
    assert b"no-allocation" in lib.tsg_last_error()
