"""ctypes binding of libtsgmres.so (the C ABI in include/tsgmres.h).

Argument marshalling only: tensors are checked (device, dtype, contiguity) and
passed as raw device pointers together with the current HIP stream.  Every step
of the computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libtsgmres.so"

ORTHO = {"two_stage": 0, "bcgs_pip2": 1, "bcgs2_cholqr2": 2, "cgs2": 3}
BASIS = {"monomial": 0, "shifted": 1, "newton": 2, "leja": 3}
PRECISION = {"fp64": 0, "fp32_ir": 1}
FLAG_EAGER = 1
STATUS = {0: "ok", 1: "not converged", 2: "breakdown", -1: "invalid argument",
          -2: "HIP runtime error", -3: "workspace", -4: "unsupported"}


class TSGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tsgmres status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class _Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("s", C.c_int32), ("s_hat", C.c_int32), ("ortho", C.c_int32),
                ("basis", C.c_int32), ("precision", C.c_int32), ("tol", C.c_double),
                ("max_iters", C.c_int64), ("newton_shifts", C.POINTER(C.c_double)),
                ("timing", C.c_int32), ("flags", C.c_int32), ("precond", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("cycles", C.c_int64), ("relres", C.c_double),
                ("relres_est", C.c_double), ("status", C.c_int32), ("truncated_cycles", C.c_int32),
                ("ms_total", C.c_double), ("ms_spmv", C.c_double), ("ms_ortho_reduce", C.c_double),
                ("ms_ortho_update", C.c_double), ("ms_small", C.c_double), ("ms_xupdate", C.c_double),
                ("ms_residual", C.c_double), ("n_ortho_reduce", C.c_int64),
                ("n_ortho_update", C.c_int64), ("n_spmv", C.c_int64),
                ("bytes_ortho_reduce", C.c_double), ("bytes_ortho_update", C.c_double),
                ("bytes_spmv", C.c_double), ("kc_ms", C.c_double * 16),
                ("kc_launches", C.c_int64 * 16), ("kc_bytes", C.c_double * 16),
                ("timed_cycles", C.c_int64), ("pip_fallbacks", C.c_int64),
                ("newton_from_cycle", C.c_int64), ("shifted_passes", C.c_int64),
                ("redone_cycles", C.c_int64)]


KERNEL_CLASSES = ["mpk", "gram", "gram_first", "update", "fused", "tail", "cycle_end", "xupdate",
                  "residual", "scale", "fallback", "stage2", "precond"]
PRECOND = {None: 0, "none": 0, "mcgs": 1}


@dataclass
class SolveInfo:
    status: int
    iters: int
    cycles: int
    relres: float
    relres_est: float
    truncated_cycles: int
    ms_total: float = 0.0
    ms_spmv: float = 0.0
    ms_ortho_reduce: float = 0.0
    ms_ortho_update: float = 0.0
    ms_small: float = 0.0
    ms_xupdate: float = 0.0
    ms_residual: float = 0.0
    n_ortho_reduce: int = 0
    n_ortho_update: int = 0
    n_spmv: int = 0
    bytes_ortho_reduce: float = 0.0
    bytes_ortho_update: float = 0.0
    bytes_spmv: float = 0.0
    kc_ms: tuple = ()
    kc_launches: tuple = ()
    kc_bytes: tuple = ()
    timed_cycles: int = 0
    pip_fallbacks: int = 0
    newton_from_cycle: int = 0
    shifted_passes: int = 0
    redone_cycles: int = 0

    def kernel_classes(self) -> dict:
        """{class: (ms, launches, algorithmic bytes)} for the classes that ran (timing mode)."""
        return {n: (self.kc_ms[i], self.kc_launches[i], self.kc_bytes[i])
                for i, n in enumerate(KERNEL_CLASSES) if i < len(self.kc_launches) and self.kc_launches[i]}

    @property
    def converged(self) -> bool:
        return self.status == 0


_lib = None


def library_path() -> str:
    return os.environ.get("TSGMRES_LIB", os.path.join(HERE, _LIB_NAME))


def load_library():
    """Load libtsgmres.so (raises if it has not been built; there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2402_15033_amd.build` "
                           "(or __graft_entry__.build()); no CPU fallback exists")
    lib = C.CDLL(path)
    vp, i32, i64, f64p = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.tsg_csr_create.argtypes = [i64, i64, vp, vp, vp, vp, C.POINTER(vp)]
    lib.tsg_csr_create.restype = C.c_int
    lib.tsg_csr_destroy.argtypes = [vp]
    lib.tsg_csr_destroy.restype = C.c_int
    lib.tsg_csr_gershgorin.argtypes = [vp, f64p, f64p]
    lib.tsg_csr_gershgorin.restype = C.c_int
    lib.tsg_csr_pack_bytes.argtypes = [vp]
    lib.tsg_csr_pack_bytes.restype = C.c_size_t
    lib.tsg_csr_pack.argtypes = [vp, vp, C.c_size_t, vp]
    lib.tsg_csr_pack.restype = C.c_int
    lib.tsg_spmv.argtypes = [vp, vp, vp, vp]
    lib.tsg_spmv.restype = C.c_int
    lib.tsg_solve_workspace_bytes.argtypes = [i64, i64, C.POINTER(_Params)]
    lib.tsg_solve_workspace_bytes.restype = C.c_size_t
    lib.tsg_solve.argtypes = [vp, vp, vp, C.POINTER(_Params), vp, C.c_size_t, vp, C.POINTER(_Info)]
    lib.tsg_solve.restype = C.c_int
    lib.tsg_orthogonalize_workspace_bytes.argtypes = [i64, i32, i32]
    lib.tsg_orthogonalize_workspace_bytes.restype = C.c_size_t
    lib.tsg_orthogonalize.argtypes = [i64, i32, vp, i64, vp, i32, i32, i32, i32, vp, C.c_size_t, vp, f64p]
    lib.tsg_orthogonalize.restype = C.c_int
    lib.tsg_block_pip_workspace_bytes.argtypes = [i64, i32, i32]
    lib.tsg_block_pip_workspace_bytes.restype = C.c_size_t
    lib.tsg_block_pip.argtypes = [i64, i32, i32, vp, i64, C.c_double, C.c_double, i32, vp, i32, vp, i32,
                                  C.POINTER(i32), vp, C.c_size_t, vp]
    lib.tsg_block_pip.restype = C.c_int
    lib.tsg_orthogonalize_noalloc.argtypes = [i64, i32, vp, i64, vp, i32, i32, i32, i32, vp, f64p]
    lib.tsg_orthogonalize_noalloc.restype = C.c_int
    lib.tsg_orthogonalize_noalloc_max_bytes.argtypes = []
    lib.tsg_orthogonalize_noalloc_max_bytes.restype = C.c_size_t
    lib.tsg_server_request_bytes.argtypes = [i64, i64, C.POINTER(_Params)]
    lib.tsg_server_request_bytes.restype = C.c_size_t
    lib.tsg_server_create.argtypes = [C.POINTER(_Params), vp, C.c_size_t, i32, vp, C.POINTER(vp)]
    lib.tsg_server_create.restype = C.c_int
    lib.tsg_server_destroy.argtypes = [vp]
    lib.tsg_server_destroy.restype = C.c_int
    lib.tsg_server_submit.argtypes = [vp, vp, vp, vp, i64]
    lib.tsg_server_submit.restype = C.c_int
    lib.tsg_server_step.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    lib.tsg_server_step.restype = C.c_int
    lib.tsg_server_poll.argtypes = [vp, C.POINTER(i64), C.POINTER(_Info), i32]
    lib.tsg_server_poll.restype = i32
    lib.tsg_csr_precond_bytes.argtypes = [vp]
    lib.tsg_csr_precond_bytes.restype = C.c_size_t
    lib.tsg_csr_precond.argtypes = [vp, vp, C.c_size_t, vp]
    lib.tsg_csr_precond.restype = C.c_int
    lib.tsg_csr_ncolors.argtypes = [vp]
    lib.tsg_csr_ncolors.restype = i32
    lib.tsg_csr_colors.argtypes = [vp, vp, vp]
    lib.tsg_csr_colors.restype = C.c_int
    lib.tsg_precond_apply.argtypes = [vp, vp, vp, vp]
    lib.tsg_precond_apply.restype = C.c_int
    lib.tsg_ritz_newton.argtypes = [vp, i64, i32, i32, C.c_double, C.c_double, vp, vp]
    lib.tsg_ritz_newton.restype = C.c_int
    lib.tsg_status_string.argtypes = [C.c_int]
    lib.tsg_status_string.restype = C.c_char_p
    lib.tsg_last_error.argtypes = []
    lib.tsg_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(status: int, allow_positive: bool = False) -> int:
    if status == 0 or (allow_positive and status > 0):
        return status
    msg = load_library().tsg_last_error().decode(errors="replace")
    raise TSGError(status, msg)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_tensor(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _workspace(nbytes: int, device, ws: torch.Tensor | None):
    """Device buffer of at least nbytes whose address is 256-byte aligned."""
    if ws is not None:
        p = ws.data_ptr()
        if p % 256 or ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small or not 256-byte aligned")
        return ws, p
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    p = buf.data_ptr()
    return buf, (p + 255) // 256 * 256


class CSRMatrix:
    """Handle on a device CSR matrix (borrows the three tensors; keeps references).

    pack=True (default) also builds the library's packed SELL-64 copy of the operator
    (tsg_csr_pack, device memory owned by this object), which every solve then uses; the
    results are identical to the CSR kernels'."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, pack: bool = True):
        lib = load_library()
        self.row_ptr = _dev_tensor(row_ptr, torch.int32, "row_ptr")
        self.col = _dev_tensor(col, torch.int32, "col")
        self.val = _dev_tensor(val, torch.float64, "val")
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        self.device = val.device
        h = C.c_void_p()
        _check(lib.tsg_csr_create(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                                  self.val.data_ptr(), _stream(self.device), C.byref(h)))
        self._h = h
        self._pack = None
        self._precond = None
        if pack:
            self.pack()

    def pack(self):
        """Build the packed copy (SELL-64) used by the solver's SpMVs."""
        lib = load_library()
        nbytes = int(lib.tsg_csr_pack_bytes(self._h))
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        p = (buf.data_ptr() + 255) // 256 * 256
        _check(lib.tsg_csr_pack(self._h, p, nbytes, _stream(self.device)))
        self._pack = buf
        return self

    def unpack(self):
        _check(load_library().tsg_csr_pack(self._h, None, 0, _stream(self.device)))
        self._pack = None
        return self

    def precond_setup(self):
        """Color the operator and build the sweep layout of the multicolor Gauss-Seidel
        preconditioner (precond='mcgs') in a device buffer this object owns (the size the
        library asks for); a second call does nothing."""
        if getattr(self, "_precond", None) is not None:
            return self
        lib = load_library()
        nbytes = int(lib.tsg_csr_precond_bytes(self._h))
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        p = (buf.data_ptr() + 255) // 256 * 256
        _check(lib.tsg_csr_precond(self._h, p, nbytes, _stream(self.device)))
        self._precond = buf
        return self

    @property
    def ncolors(self) -> int:
        return int(load_library().tsg_csr_ncolors(self._h))

    def colors(self) -> torch.Tensor:
        """The row colors of the preconditioner set-up (int32 device tensor)."""
        c = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(load_library().tsg_csr_colors(self._h, c.data_ptr(), _stream(self.device)))
        return c

    @classmethod
    def from_host(cls, A, device="cuda", pack: bool = True):
        """From any object with numpy row_ptr/col/val (e.g. workloads.CSR)."""
        return cls(torch.as_tensor(A.row_ptr, device=device), torch.as_tensor(A.col, device=device),
                   torch.as_tensor(A.val, device=device), pack=pack)

    @property
    def handle(self):
        return self._h

    def gershgorin(self):
        lo, hi = C.c_double(), C.c_double()
        _check(load_library().tsg_csr_gershgorin(self._h, C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tsg_csr_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmv(A: CSRMatrix, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
    _dev_tensor(x, torch.float64, "x")
    if y is None:
        y = torch.empty_like(x)
    _check(load_library().tsg_spmv(A.handle, x.data_ptr(), y.data_ptr(), _stream(x.device)))
    return y


def ritz_newton(H: torch.Tensor, s: int, lo: float, hi: float):
    """Newton-basis parameters of basis='leja' for the k x k upper Hessenberg H (float64
    device tensor, column-major: H.T contiguous, or any (k, k) tensor with stride (1, ld)).
    Returns dict(ritz=complex Leja-ordered Ritz values (host), theta, tau, sigma (device))."""
    lib = load_library()
    if H.dim() != 2 or H.shape[0] != H.shape[1] or H.dtype != torch.float64 or H.device.type != "cuda":
        raise ValueError("H must be a square float64 device tensor")
    if H.stride(0) != 1:
        raise ValueError("H must be column-major (stride (1, ld))")
    k = H.shape[0]
    ld = H.stride(1) if k > 1 else 1
    out = torch.empty(2 * k + 3 * int(s) + 1, dtype=torch.float64, device=H.device)
    _check(lib.tsg_ritz_newton(H.data_ptr(), ld, k, int(s), float(lo), float(hi), out.data_ptr(),
                               _stream(H.device)))
    o = out.cpu()
    ritz = torch.complex(o[:k], o[k:2 * k])
    s = int(s)
    return {"ritz": ritz, "theta": out[2 * k:2 * k + s], "tau": out[2 * k + s:2 * k + 2 * s],
            "sigma": out[2 * k + 2 * s:2 * k + 3 * s]}


def precond_apply(A: CSRMatrix, w: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
    """z = M^{-1} w for A's multicolor Gauss-Seidel preconditioner (A.precond_setup() first)."""
    _dev_tensor(w, torch.float64, "w")
    if z is None:
        z = torch.empty_like(w)
    _check(load_library().tsg_precond_apply(A.handle, w.data_ptr(), z.data_ptr(), _stream(w.device)))
    return z


def _params(m, s, ortho, basis, precision, tol, max_iters, shifts, timing, graph=True, s_hat=0, precond=None):
    p = _Params()
    p.m, p.s, p.s_hat = int(m), int(s), int(s_hat or 0)
    p.ortho = ORTHO[ortho] if isinstance(ortho, str) else int(ortho)
    p.basis = BASIS[basis] if isinstance(basis, str) else int(basis)
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.tol = float(tol)
    p.max_iters = int(max_iters)
    keep = None
    if shifts is not None:
        keep = (C.c_double * len(shifts))(*[float(v) for v in shifts])
        p.newton_shifts = C.cast(keep, C.POINTER(C.c_double))
    p.timing = int(timing)  # False/True -> 0/1; an int t > 1 times every t-th cycle
    p.flags = 0 if graph else FLAG_EAGER
    p.precond = PRECOND[precond] if (precond is None or isinstance(precond, str)) else int(precond)
    return p, keep


def solve_workspace_bytes(A: CSRMatrix, m=60, s=5, ortho="two_stage", basis="monomial",
                          precision="fp64", s_hat=0, precond=None) -> int:
    p, _ = _params(m, s, ortho, basis, precision, 1e-10, 1 << 40, None, False, s_hat=s_hat, precond=precond)
    return int(load_library().tsg_solve_workspace_bytes(A.n, A.nnz, C.byref(p)))


def solve(A: CSRMatrix, b: torch.Tensor, x: torch.Tensor | None = None, *, m: int = 60, s: int = 5,
          tol: float = 1e-10, max_iters: int = 1 << 40, ortho: str = "two_stage",
          basis: str = "monomial", precision: str = "fp64", shifts=None, timing: bool = False,
          graph: bool = True, s_hat: int = 0, workspace: torch.Tensor | None = None, precond=None):
    """Solve A x = b (x updated in place; zeros if None).  Returns (x, SolveInfo).

    graph=False launches every kernel directly instead of replaying one captured restart
    cycle per cycle (same results, bit for bit).  s_hat (two-stage): 0 or m for one big
    panel per cycle, else the big-panel size (s | s_hat | m).  precond='mcgs': right
    preconditioning by multicolor Gauss-Seidel (A.precond_setup() first; FP64)."""
    lib = load_library()
    _dev_tensor(b, torch.float64, "b")
    if x is None:
        x = torch.zeros_like(b)
    _dev_tensor(x, torch.float64, "x")
    p, keep = _params(m, s, ortho, basis, precision, tol, max_iters, shifts, timing, graph, s_hat, precond)
    need = int(lib.tsg_solve_workspace_bytes(A.n, A.nnz, C.byref(p)))
    if need == 0:
        _check(-1)
    ws, wp = _workspace(need, b.device, workspace)
    info = _Info()
    st = lib.tsg_solve(A.handle, b.data_ptr(), x.data_ptr(), C.byref(p), wp, need,
                       _stream(b.device), C.byref(info))
    _check(st, allow_positive=True)
    del keep, ws
    vals = {}
    for f, _ in _Info._fields_:
        v = getattr(info, f)
        vals[f] = tuple(v) if f.startswith("kc_") else v
    out = SolveInfo(**vals)
    return x, out


def _block_view(X: torch.Tensor, ldx):
    """(n, k, ld) of a float64 device tensor viewed as a column-major block."""
    if X.dim() != 2 or X.dtype != torch.float64 or X.device.type != "cuda":
        raise ValueError("X must be a 2-D float64 device tensor")
    if X.stride(0) == 1:  # (n, k) column-major view
        n, k = X.shape
        ld = X.stride(1) if k > 1 else n
    elif X.stride(1) == 1:  # (k, ld) rows are columns
        k = X.shape[0]
        n = X.shape[1] if ldx is None else int(ldx)
        ld = X.stride(0) if k > 1 else X.shape[1]
        n = min(n, X.shape[1])
    else:
        raise ValueError("X must be column-major")
    return n, k, ld


def orthogonalize(X: torch.Tensor, s: int = 5, algo: str = "two_stage", *, ldx: int | None = None,
                  orth_err: bool = False, workspace: torch.Tensor | None = None, noalloc: bool = False,
                  s_hat: int = 0):
    """Orthonormalize the n x k block in place.

    X is a float64 device tensor viewed as column-major: either a (k, ldx) contiguous tensor
    whose row c is column c of the block, or an (n, k) tensor with stride (1, ldx) (e.g. the
    transpose of a contiguous (k, n) tensor).  Returns (X, R[, ||I - Q^T Q||_F]).
    noalloc=True calls tsg_orthogonalize_noalloc (the library's own static scratch, no
    workspace).  s_hat (two-stage): 0 for one big panel, else the big-panel size (a multiple
    of s), each big panel's Q made final by its stage 2.
    """
    lib = load_library()
    n, k, ld = _block_view(X, ldx)
    R = torch.zeros((k, k), dtype=torch.float64, device=X.device)  # column-major: R_t[j, i] = R[i, j]
    a = ORTHO[algo] if isinstance(algo, str) else int(algo)
    err = C.c_double(0.0)
    if noalloc:
        st = lib.tsg_orthogonalize_noalloc(n, k, X.data_ptr(), ld, R.data_ptr(), k, int(s), int(s_hat), a,
                                           _stream(X.device), C.byref(err) if orth_err else None)
        _check(st)
    else:
        need = int(lib.tsg_orthogonalize_workspace_bytes(n, k, s))
        if need == 0:
            _check(-1)
        ws, wp = _workspace(need, X.device, workspace)
        st = lib.tsg_orthogonalize(n, k, X.data_ptr(), ld, R.data_ptr(), k, int(s), int(s_hat), a, wp, need,
                                   _stream(X.device), C.byref(err) if orth_err else None)
        _check(st)
        del ws
    Rt = R.t()  # R was written column-major
    if orth_err:
        return X, Rt, err.value
    return X, Rt


def block_pip(V: torch.Tensor, k: int, s: int, *, pip_tol: float = 1e-8, pivot_tol: float = 1e-12,
              chain: int = 2, ldv: int | None = None):
    """One stage-1 panel through the solver's fallback chain (tsg_block_pip): V is a float64
    device block viewed column-major as by orthogonalize(); its columns k .. k+s-1 are
    orthogonalized in place against columns 0 .. k-1.  Returns dict(status, passes,
    fail_col, P (k x s), R (s x s)); a breakdown is reported in status (2), not raised."""
    lib = load_library()
    n, ncol, ld = _block_view(V, ldv)
    if ncol < k + s:
        raise ValueError("V has fewer than k + s columns")
    P = torch.zeros((s, max(k, 1)), dtype=torch.float64, device=V.device)  # column-major k x s
    R = torch.zeros((s, s), dtype=torch.float64, device=V.device)
    need = int(lib.tsg_block_pip_workspace_bytes(n, int(k), int(s)))
    if need == 0:
        _check(-1)
    ws, wp = _workspace(need, V.device, None)
    out = (C.c_int32 * 2)(-1, -1)
    st = lib.tsg_block_pip(n, int(k), int(s), V.data_ptr(), ld, float(pip_tol), float(pivot_tol), int(chain),
                           P.data_ptr(), max(int(k), 1), R.data_ptr(), int(s), out, wp, need, _stream(V.device))
    _check(st, allow_positive=True)
    del ws
    return {"status": int(st), "passes": int(out[0]), "fail_col": int(out[1]),
            "P": P.t()[:k, :] if k > 0 else P.t()[:0, :], "R": R.t()}


def _info_to_py(info: _Info) -> SolveInfo:
    vals = {}
    for f, _ in _Info._fields_:
        v = getattr(info, f)
        vals[f] = tuple(v) if f.startswith("kc_") else v
    return SolveInfo(**vals)


class Server:
    """Continuous-batching solve server (tsg_server_* in the C ABI).

    Requests share the solver parameters; each brings its own CSR operator, right-hand side
    and solution vector (device tensors, kept referenced here until the request is polled).
    ``arena_bytes`` of device memory is allocated once (torch) and is the HBM budget that
    admission checks against; the library allocates nothing.
    """

    def __init__(self, arena_bytes: int, *, m: int = 60, s: int = 5, tol: float = 1e-8,
                 max_iters: int = 1 << 40, ortho: str = "two_stage", basis: str = "shifted",
                 precision: str = "fp32_ir", max_active: int = 256, s_hat: int = 0, device="cuda",
                 precond=None):
        lib = load_library()
        self._p, _ = _params(m, s, ortho, basis, precision, tol, max_iters, None, False, s_hat=s_hat,
                             precond=precond)
        self.device = torch.device(device)
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        base = (self._arena.data_ptr() + 255) // 256 * 256
        self.arena_bytes = int(arena_bytes)
        h = C.c_void_p()
        _check(lib.tsg_server_create(C.byref(self._p), base, self.arena_bytes, int(max_active),
                                     _stream(self.device), C.byref(h)))
        self._h = h
        self._live = {}  # tag -> (A, b, x) kept alive while the request is in the server

    def request_bytes(self, A: CSRMatrix) -> int:
        return int(load_library().tsg_server_request_bytes(A.n, A.nnz, C.byref(self._p)))

    def submit(self, tag: int, A: CSRMatrix, b: torch.Tensor, x: torch.Tensor | None = None) -> torch.Tensor:
        _dev_tensor(b, torch.float64, "b")
        if x is None:
            x = torch.zeros_like(b)
        _dev_tensor(x, torch.float64, "x")
        _check(load_library().tsg_server_submit(self._h, A.handle, b.data_ptr(), x.data_ptr(), int(tag)))
        self._live[int(tag)] = (A, b, x)
        return x

    def step(self):
        """One restart-cycle boundary.  Returns (active, queued)."""
        na, nq = C.c_int32(), C.c_int32()
        _check(load_library().tsg_server_step(self._h, C.byref(na), C.byref(nq)))
        return na.value, nq.value

    def poll(self, max_n: int = 1024):
        """Finished requests: list of (tag, x, SolveInfo)."""
        tags = (C.c_int64 * max_n)()
        infos = (_Info * max_n)()
        k = load_library().tsg_server_poll(self._h, tags, infos, max_n)
        out = []
        for i in range(k):
            A, b, x = self._live.pop(int(tags[i]))
            out.append((int(tags[i]), x, _info_to_py(infos[i])))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load_library().tsg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
