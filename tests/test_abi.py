"""The C-ABI library loads and exports every symbol declared in include/tsgmres.h, and
host-side argument validation works without a GPU (no device work is issued)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsgmres.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2402_15033_amd import binding

    path = binding.library_path()
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    return binding.load_library()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("tsg_csr_create", "tsg_csr_destroy", "tsg_spmv", "tsg_solve", "tsg_solve_workspace_bytes",
              "tsg_orthogonalize", "tsg_orthogonalize_workspace_bytes", "tsg_status_string",
              "tsg_last_error", "tsg_csr_gershgorin", "tsg_server_create", "tsg_server_destroy",
              "tsg_server_submit", "tsg_server_step", "tsg_server_poll", "tsg_server_request_bytes",
              "tsg_csr_pack", "tsg_csr_pack_bytes", "tsg_ritz_newton", "tsg_csr_precond", "tsg_csr_precond_bytes",
              "tsg_csr_ncolors", "tsg_csr_colors", "tsg_precond_apply"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_status_strings(lib):
    assert lib.tsg_status_string(0) == b"ok"
    assert lib.tsg_status_string(-1) == b"invalid argument"
    assert lib.tsg_status_string(2) == b"breakdown"


def test_host_side_validation(lib):
    from paper_2402_15033_amd import binding

    p = binding._Params()
    p.m, p.s, p.s_hat, p.ortho, p.basis, p.precision = 60, 5, 0, 0, 0, 0
    p.tol, p.max_iters = 1e-10, 1000
    # workspace query is pure host arithmetic
    nb = lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p))
    assert nb > 61 * 4096 * 8
    p.s = 7  # does not divide m
    assert lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p)) == 0
    p.s = 5
    p.m = 64  # m + 1 > 64 columns
    assert lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p)) == 0
    p.m = 60
    # NULL handle / pointers are rejected before any device call
    assert lib.tsg_solve(None, None, None, C.byref(p), None, 0, None, None) == -1
    assert b"NULL" in lib.tsg_last_error()
    h = C.c_void_p()
    assert lib.tsg_csr_create(0, 0, None, None, None, None, C.byref(h)) == -1
    assert lib.tsg_orthogonalize(100, 65, None, 100, None, 65, 5, 0, 0, None, 0, None, None) == -1
    assert lib.tsg_orthogonalize_workspace_bytes(100, 65, 5) == 0
    assert lib.tsg_orthogonalize_workspace_bytes(100, 61, 5) > 0
    # preconditioner entries reject NULL handles before any device work
    assert lib.tsg_csr_precond(None, None, 0, None) == -1
    assert lib.tsg_csr_precond_bytes(None) == 0
    assert lib.tsg_precond_apply(None, None, None, None) == -1
    assert lib.tsg_csr_ncolors(None) == 0
    # precond = MCGS is FP64 only; an unknown precond value is rejected
    p.precond, p.precision = 1, 1
    assert lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p)) == 0
    p.precision = 0
    assert lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p)) > nb  # + two n-vectors
    p.precond = 2
    assert lib.tsg_solve_workspace_bytes(4096, 20224, C.byref(p)) == 0
    p.precond = 0
    # Ritz/Newton entry: argument checks happen before any device work
    assert lib.tsg_ritz_newton(None, 10, 10, 5, 0.0, 1.0, None, None) == -1
    assert lib.tsg_ritz_newton(C.c_void_p(256), 10, 64, 5, 0.0, 1.0, C.c_void_p(256), None) == -1  # k > 63
    assert lib.tsg_ritz_newton(C.c_void_p(256), 10, 10, 11, 0.0, 1.0, C.c_void_p(256), None) == -1  # s > k
    assert lib.tsg_ritz_newton(C.c_void_p(256), 9, 10, 5, 0.0, 1.0, C.c_void_p(256), None) == -1  # ldh < k


def test_no_cpu_fallback(monkeypatch, tmp_path):
    """Without the library, the package raises instead of computing anything."""
    from paper_2402_15033_amd import binding

    monkeypatch.setenv("TSGMRES_LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.load_library()


def test_noalloc_entry_rejects_oversized_blocks_on_the_host(lib):
    """tsg_orthogonalize_noalloc checks sizes against its fixed scratch before any device
    work (the pointers below are never dereferenced)."""
    assert lib.tsg_orthogonalize_noalloc_max_bytes() == 12 << 20
    assert lib.tsg_orthogonalize_workspace_bytes(1 << 28, 64, 16) <= lib.tsg_orthogonalize_noalloc_max_bytes()
    fake = C.c_void_p(256)
    n = (1 << 28) + 1
    assert lib.tsg_orthogonalize_noalloc(n, 61, fake, n, fake, 61, 5, 0, 0, None, None) == -1
    assert b"no-allocation" in lib.tsg_last_error()
    assert lib.tsg_orthogonalize_noalloc(100, 65, fake, 100, fake, 65, 5, 0, 0, None, None) == -1
    assert lib.tsg_orthogonalize_noalloc(100, 61, None, 100, fake, 61, 5, 0, 0, None, None) == -1


def test_block_pip_argument_checks_on_the_host(lib):
    fake = C.c_void_p(256)
    ws = lib.tsg_block_pip_workspace_bytes(1000, 9, 5)
    assert ws > 0 and lib.tsg_block_pip_workspace_bytes(1000, 60, 5) == 0  # k + s > 64
    assert lib.tsg_block_pip_workspace_bytes(1000, 9, 17) == 0
    args = dict(n=1000, k=9, s=5, V=fake, ldv=1000, pip=1e-8, piv=1e-12, chain=2, P=fake, ldp=9, R=fake, ldr=5)

    def call(**kw):
        a = dict(args, **kw)
        return lib.tsg_block_pip(a["n"], a["k"], a["s"], a["V"], a["ldv"], a["pip"], a["piv"], a["chain"], a["P"],
                                 a["ldp"], a["R"], a["ldr"], None, fake, ws, None)
    assert call(V=None) == -1
    assert call(s=0) == -1
    assert call(k=60) == -1           # k + s > 64
    assert call(n=10) == -1           # k + s > n
    assert call(ldv=999) == -1
    assert call(ldp=8) == -1
    assert call(chain=3) == -1
    assert call(piv=0.0) == -1        # the explicit pass needs a positive threshold
    assert call(pip=-1.0) == -1
    assert lib.tsg_block_pip(1000, 9, 5, fake, 1000, 1e-8, 1e-12, 2, fake, 9, fake, 5, None, C.c_void_p(257), ws,
                             None) == -3  # misaligned workspace
