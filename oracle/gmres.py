"""Restarted GMRES(m) variants of the oracle, plain FP64 (test infrastructure only).

* ``gmres(..., ortho='mgs')``  -- standard GMRES(m), Arnoldi with modified
  Gram-Schmidt, one new vector per iteration (Sec. I); the backward-stable
  reference.
* ``gmres(..., ortho='cgs2')`` -- the same with classical Gram-Schmidt applied
  twice, the paper's "standard GMRES" baseline (Tables 2-4).
* ``sstep_gmres``              -- s-step GMRES(m) (Sec. III, Fig. 1): each panel is
  s SpMVs of the matrix-powers kernel followed by a block orthogonalization;
  ortho = 'two_stage' (Sec. V, Fig. 5 with s_hat = m), 'bcgs_pip2' (Fig. 4b) or
  'bcgs2_cholqr2' (Fig. 2b).  basis = 'monomial', 'shifted', 'newton' (given real
  shifts) or 'leja' (Newton basis from the Leja-ordered Ritz values of the first
  cycle, ``oracle.ritz``).

One restart cycle of every variant computes, in exact arithmetic, the same
iterate: x + argmin_{z in K_k(A, r)} ||b - A(x + z)||, with k the number of
basis vectors generated in that cycle.

Outer loop (all variants): r = b - A x, stop if ||r|| <= tol ||b|| (explicit
residual), else run one cycle.  Inside a cycle the implicit residual estimate
is checked after every new vector (standard), after every panel (one-stage
s-step) or once at the end of the cycle (two-stage with s_hat = m).  The
iteration count is the number of Krylov vectors generated.

s-step Hessenberg recovery (the small-matrix algebra implied by Fig. 1 and
Sec. VI; the paper's listing is not reproduced): with the basis
w_i = (A w_{i-1} - theta_i w_{i-1} + tau_i w_{i-2}) / sigma_i, w_0 = qhat_k
(tau_i != 0 only in the Newton basis, at the second step of a complex pair),
  A [w_0 .. w_{s-1}] = [w_0 .. w_s] B,   B(i,i) = theta_i, B(i+1,i) = sigma_i,
  B(i-1,i) = -tau_i,
and the panel factorization W = Qhat_{1:k} P + Qhat_{k+1:k+s} R gives
[w_0, W] = Qhat_{1:k+s} S with S(:,1) = e_k, S(:,2:s+1) = [P; R].  Splitting the
first k-1 rows off S(1:k+s-1,1:s) and using A Qhat_{1:k-1} = Qhat_{1:k} Hhat
yields, with T = S(k:k+s-1, 1:s) (upper triangular, T(1,1) = 1),
  Hhat(1:k+s, k:k+s-1) = (S B - [Hhat(1:k,1:k-1) S(1:k-1,1:s); 0]) T^{-1}.
Two-stage: Qhat = Q R2 with R2 = Chol(Qhat^T Qhat) (stage 2 = CholQR of the
m+1 columns), so A Q_{1:m} = Q_{1:m+1} H with H = R2 Hhat R2(1:m,1:m)^{-1}; the
projected problem is min || beta R2(1,1) e_1 - H y || and x += Qhat_{1:m} z with
z = R2(1:m,1:m)^{-1} y.

Breakdown (our reading; the paper does not treat it): if a panel's Cholesky
fails (a pivot at or below the relative threshold of ``dense.PIVOT_TOL``), the
panel lies numerically in the span of the basis -- the Krylov space is
(numerically) invariant.  The cycle then ends with the k columns built before
that panel; if the stage-2 Cholesky fails at pivot p, with the first p columns.
A cycle that can keep no column makes no progress and the solve stops.
"""
from __future__ import annotations

import numpy as np

from .dense import (PIP_TOL, PIVOT_TOL, CholeskyBreakdown, GivensState, chol_upper, givens_lsq,
                    right_solve_upper, solve_upper)
from .sparse import Operator, basis_params, gershgorin, spmv
from . import blockortho, ritz
from . import precond as precond_mod


# Two-stage stage 1 takes the shifted Cholesky QR pass (``blockortho.bcgs_pip_explicit``)
# where its explicit second pass fails, by default for s >= SHIFTED_MIN_S (smaller steps
# with a scaled basis stay far from that pass's limit, and a failure there means a
# numerically dependent panel).
SHIFTED_MIN_S = 8


def _outer(A, b, x0, tol, max_iters, cycle_fn, record):
    op = A if isinstance(A, Operator) else Operator(A)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(op.n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    iters = 0
    cycles = 0
    history = []
    estimates = []
    records = []
    converged = False
    while True:
        r = b - spmv(op, x)
        beta = float(np.linalg.norm(r))
        history.append(beta / bnorm)
        if beta <= tol * bnorm:
            converged = True
            break
        if iters >= max_iters:
            break
        dx, k_used, est, rec = cycle_fn(op, r, beta, tol * bnorm)
        x = x + dx
        iters += k_used
        cycles += 1
        estimates.append(est / bnorm)
        if record:
            records.append(rec)
        if k_used == 0:
            break
    return {
        "x": x, "iters": iters, "cycles": cycles, "converged": converged,
        "relres": history[-1], "history": history, "estimates": estimates,
        "records": records,
    }


def gmres(A, b, x0=None, m: int = 60, tol: float = 1e-10, max_iters: int = 10**9,
          ortho: str = "mgs", record: bool = False, precond=None):
    """Standard restarted GMRES(m) with MGS or CGS2 Arnoldi; precond: an object with
    apply(w) = M^{-1} w for right preconditioning (Arnoldi on A M^{-1}, x += M^{-1} Q y)."""
    prec = precond.apply if precond is not None else None

    def cycle(op, r, beta, tol_abs):
        n = op.n
        Q = np.zeros((n, m + 1), order="F")
        H = np.zeros((m + 1, m))
        Q[:, 0] = r / beta
        giv = GivensState(beta, m)
        k_used = m
        for j in range(m):
            w = spmv(op, Q[:, j] if prec is None else prec(Q[:, j]))
            h = np.zeros(j + 2)
            if ortho == "mgs":
                for i in range(j + 1):
                    h[i] = Q[:, i] @ w
                    w = w - h[i] * Q[:, i]
            elif ortho == "cgs2":
                Qj = Q[:, : j + 1]
                h1 = Qj.T @ w
                w = w - Qj @ h1
                h2 = Qj.T @ w
                w = w - Qj @ h2
                h[: j + 1] = h1 + h2
            else:
                raise ValueError(ortho)
            h[j + 1] = np.sqrt(w @ w)
            H[: j + 2, j] = h
            giv.add_column(h)
            if h[j + 1] == 0.0:  # happy breakdown: K_{j+1} is invariant
                k_used = j + 1
                break
            Q[:, j + 1] = w / h[j + 1]
            if giv.residual() <= tol_abs:
                k_used = j + 1
                break
        y = giv.solve(k_used)
        rec = {"Q": Q[:, : k_used + 1], "H": H[: k_used + 1, :k_used]} if record else None
        dx = Q[:, :k_used] @ y
        return (dx if prec is None else prec(dx)), k_used, giv.residual(), rec

    return _outer(A, b, x0, tol, max_iters, cycle, record)


def mpk(op, w0: np.ndarray, theta: np.ndarray, sigma: np.ndarray, tau=None, prec=None):
    """Matrix-powers kernel: s SpMVs in sequence (Sec. III).  Returns (W, B).

    Step i: w_{i+1} = (A w_i - theta_i w_i + tau_i w_{i-1}) / sigma_i (tau = 0 except at
    the second step of a complex pair of the Newton basis), so
    A w_i = sigma_i w_{i+1} + theta_i w_i - tau_i w_{i-1}: B(i+1,i) = sigma_i,
    B(i,i) = theta_i, B(i-1,i) = -tau_i.  With a right preconditioner (prec(w) = M^{-1} w)
    the product is A M^{-1} w_i.
    """
    s = len(theta)
    tau = np.zeros(s) if tau is None else np.asarray(tau, dtype=np.float64)
    W = np.zeros((op.n, s), order="F")
    B = np.zeros((s + 1, s))
    prev, w = None, w0
    for i in range(s):
        nxt = spmv(op, w if prec is None else prec(w)) - theta[i] * w
        if tau[i] != 0.0:
            nxt = nxt + tau[i] * prev
            B[i - 1, i] = -tau[i]
        prev, w = w, nxt / sigma[i]
        W[:, i] = w
        B[i, i] = theta[i]
        B[i + 1, i] = sigma[i]
    return W, B


class _Basis:
    """The s-step basis parameters of a solve.  basis = 'leja': the first cycle that keeps
    at least s columns runs with the shifted basis; its Ritz values then give the Newton
    basis of every later cycle (``ritz.leja_ritz_params``)."""

    def __init__(self, op, s, basis, shifts, prec=None):
        self.s = s
        self.lo, self.hi = gershgorin(op) if prec is None else precond_mod.PRECOND_INTERVAL
        self.theta, self.sigma = basis_params(op, s, "shifted" if basis == "leja" else basis, shifts,
                                              interval=(self.lo, self.hi))
        self.tau = np.zeros(s)
        self.pending = basis == "leja"
        self.switched_after = None

    def cycle_done(self, H_square: np.ndarray, cycle_index: int):
        if self.pending and H_square.shape[0] >= self.s:
            self.theta, self.tau, self.sigma = ritz.leja_ritz_params(H_square, self.s, self.lo, self.hi)
            self.pending = False
            self.switched_after = cycle_index

    def export(self, out):
        out["theta"], out["sigma"], out["tau"] = self.theta, self.sigma, self.tau
        out["basis_switched_after"] = self.switched_after


def hessenberg_block(Hh: np.ndarray, P: np.ndarray, R: np.ndarray, B: np.ndarray, k: int):
    """Columns k-1 .. k+s-2 (0-based) of the Hessenberg matrix of the basis, rows 0..k+s-1."""
    s = R.shape[0]
    S = np.zeros((k + s, s + 1))
    S[k - 1, 0] = 1.0
    S[:k, 1:] = P
    S[k:, 1:] = R
    T = S[k - 1: k - 1 + s, :s]
    M = S @ B
    if k > 1:
        M[:k, :] -= Hh[:k, : k - 1] @ S[: k - 1, :s]
    return right_solve_upper(M, T)


def sstep_gmres(A, b, x0=None, m: int = 60, s: int = 5, tol: float = 1e-10,
                max_iters: int = 10**9, ortho: str = "two_stage",
                basis: str = "monomial", shifts=None, record: bool = False, s_hat: int | None = None,
                shifted: bool | None = None, precond=None):
    """s-step GMRES(m) with one-stage or two-stage block orthogonalization.

    Two-stage with s_hat = m (default): stage 2 is one CholQR of the m+1 columns at the end
    of the cycle.  With s_hat < m (s | s_hat | m) the cycle's columns form big panels (the
    first holds column 1 plus s_hat columns, the others s_hat columns, as in the
    stand-alone scheme) and stage 2 runs when each big panel is complete (Sec. V, Fig. 5).
    """
    if m % s != 0:
        raise ValueError("s must divide m")
    if ortho == "two_stage" and s_hat is not None and s_hat < m:
        if s_hat % s != 0 or m % s_hat != 0:
            raise ValueError("need s | s_hat | m")
        return _sstep_gmres_shat(A, b, x0, m, s, s_hat, tol, max_iters, basis, shifts, record, shifted,
                                 precond)
    op = A if isinstance(A, Operator) else Operator(A)
    prec = precond.apply if precond is not None else None
    bp = _Basis(op, s, basis, shifts, prec)
    J = m // s
    one_stage = None if ortho == "two_stage" else blockortho.ONE_STAGE[ortho]
    stats = {"fallbacks": 0, "shifted": 0, "cycles": 0}  # panels that took the second / shifted pass
    use_shift = s >= SHIFTED_MIN_S if shifted is None else bool(shifted)

    def cycle(op, r, beta, tol_abs):
        n = op.n
        Qh = np.zeros((n, m + 1), order="F")
        Hh = np.zeros((m + 1, m))
        Qh[:, 0] = r / beta
        giv = GivensState(beta, m)
        panels = []
        k_used = m
        breakdown = None
        for j in range(J):
            k = j * s + 1
            W, B = mpk(op, Qh[:, k - 1], bp.theta, bp.sigma, bp.tau, prec)
            try:
                if one_stage is None:  # stage 1 (second pass only where PIP fails)
                    Qn, P, R, fb = blockortho.bcgs_pip_explicit(Qh[:, :k], W, PIVOT_TOL, use_shift,
                                                                pip_tol=PIP_TOL)
                    stats["fallbacks"] += int(fb >= 1)
                    stats["shifted"] += int(fb == 2)
                else:
                    Qn, P, R = one_stage(Qh[:, :k], W, PIVOT_TOL)
            except CholeskyBreakdown:
                # the panel is numerically in the span of the basis: keep the k columns
                # built so far (k-1 Hessenberg columns) and end the cycle there
                k_used = k - 1
                breakdown = ("panel", j)
                break
            Qh[:, k: k + s] = Qn
            Hh[: k + s, k - 1: k - 1 + s] = hessenberg_block(Hh, P, R, B, k)
            if record:
                panels.append({"k": k, "P": P, "R": R, "B": B})
            if one_stage is not None:
                for c in range(k - 1, k - 1 + s):
                    giv.add_column(Hh[: c + 2, c])
                if giv.residual() <= tol_abs:
                    k_used = k - 1 + s
                    break
        rec = None
        if k_used == 0:
            return np.zeros(n), 0, beta, {"breakdown": breakdown} if record else None
        if one_stage is None:
            kb = k_used + 1
            G2 = Qh[:, :kb].T @ Qh[:, :kb]
            try:
                R2 = chol_upper(G2, tol=PIVOT_TOL)  # stage 2: CholQR of the big panel
            except CholeskyBreakdown as e:
                kb = e.index  # leading kb columns factor cleanly
                k_used = kb - 1
                breakdown = ("stage2", kb)
                if k_used <= 0:
                    return np.zeros(n), 0, beta, {"breakdown": breakdown} if record else None
                R2 = chol_upper(G2[:kb, :kb], tol=PIVOT_TOL)
            H = right_solve_upper(R2 @ Hh[:kb, :k_used], R2[:k_used, :k_used])
            stats["cycles"] += 1
            bp.cycle_done(H[:k_used, :k_used], stats["cycles"])
            y, est = givens_lsq(H, beta * R2[0, 0])
            z = solve_upper(R2[:k_used, :k_used], y)
            dx = Qh[:, :k_used] @ z
            if prec is not None:
                dx = prec(dx)
            if record:
                rec = {"Qhat": Qh[:, :kb], "Hhat": Hh[:kb, :k_used], "R2": R2, "H": H, "y": y,
                       "z": z, "panels": panels, "beta": beta, "breakdown": breakdown}
            return dx, k_used, est, rec
        y = giv.solve(k_used)
        stats["cycles"] += 1
        bp.cycle_done(Hh[:k_used, :k_used], stats["cycles"])
        if record:
            rec = {"Q": Qh[:, : k_used + 1], "H": Hh[: k_used + 1, :k_used], "y": y,
                   "panels": panels, "beta": beta, "breakdown": breakdown}
        dx = Qh[:, :k_used] @ y
        return (dx if prec is None else prec(dx)), k_used, abs(giv.g[k_used]), rec

    out = _outer(op, b, x0, tol, max_iters, cycle, record)
    bp.export(out)
    out["fallbacks"] = stats["fallbacks"]
    out["shifted"] = stats["shifted"]
    return out


def _sstep_gmres_shat(A, b, x0, m, s, s_hat, tol, max_iters, basis, shifts, record, shifted=None,
                      precond=None):
    """Two-stage s-step GMRES(m) with big panels of s_hat < m columns.

    Within a cycle the basis Y holds final (orthonormal) columns for the completed big
    panels and pre-processed columns for the current one; the Hessenberg matrix H always
    describes A Y(:, :c-1) = Y(:, :c) H for the current Y.  Stage 1 of each panel and its
    Hessenberg block are as with s_hat = m.  When a big panel [b0, b1) is complete,
    stage 2 is one BCGS-PIP of it against the final columns (the explicit Q of Fig. 5):
      P2 = Y(:, :b0)^T Y(:, b0:b1),  R2 = Chol(Y_b^T Y_b - P2^T P2),
      Y(:, b0:b1) <- (Y(:, b0:b1) - Y(:, :b0) P2) R2^{-1},
    i.e. Y_old = Y_new M with M = I except M(:b0, b0:b1) = P2, M(b0:b1, b0:b1) = R2, so
    H <- M(:b1, :b1) H M(:b1-1, :b1-1)^{-1} (still upper Hessenberg) and the least-squares
    rhs beta e_1 becomes beta M(0, 0) e_1.  The next panel's matrix-powers kernel then starts
    from the final column (reading of the paper's silence on the start vector).  The
    residual is checked at the end of every big panel (least squares over the final
    columns); the cycle stops there when it is below tol.  A stage-1 breakdown ends the
    cycle with the columns of its completed big panels.
    """
    op = A if isinstance(A, Operator) else Operator(A)
    prec = precond.apply if precond is not None else None
    bp = _Basis(op, s, basis, shifts, prec)
    J = m // s
    bigs = blockortho.big_panel_bounds(m + 1, s, s_hat)
    stats = {"fallbacks": 0, "shifted": 0, "cycles": 0}
    use_shift = s >= SHIFTED_MIN_S if shifted is None else bool(shifted)

    def stage2(Y, H, done, b1, c_h):
        """Stage 2 on columns [done, b1); transforms H(:b1, :c_h).  Returns (kept, M00)."""
        Yb = Y[:, done:b1]
        P2 = Y[:, :done].T @ Yb
        Gb = Yb.T @ Yb
        G = Gb - P2.T @ P2
        kept = b1 - done
        try:
            R2 = chol_upper(G, ref_diag=np.diag(Gb), tol=PIVOT_TOL)
        except CholeskyBreakdown as e:
            kept = e.index
            if kept == 0:
                return 0, None
            R2 = chol_upper(G[:kept, :kept], ref_diag=np.diag(Gb)[:kept], tol=PIVOT_TOL)
            P2 = P2[:, :kept]
        e1 = done + kept
        Y[:, done:e1] = right_solve_upper(Y[:, done:e1] - Y[:, :done] @ P2, R2)
        M = np.eye(e1)
        M[:done, done:e1] = P2
        M[done:e1, done:e1] = R2
        c = min(c_h, e1 - 1)
        H[:e1, :c] = right_solve_upper(M @ H[:e1, :c], M[:c, :c])
        H[e1:, :c] = 0.0
        return kept, M[0, 0]

    def cycle(op, r, beta, tol_abs):
        n = op.n
        Y = np.zeros((n, m + 1), order="F")
        H = np.zeros((m + 1, m))
        Y[:, 0] = r / beta
        g0 = beta
        done = 0  # columns already final
        bi = 0
        k_used = m
        breakdown = None
        est = beta
        for j in range(J):
            k = j * s + 1
            W, B = mpk(op, Y[:, k - 1], bp.theta, bp.sigma, bp.tau, prec)
            try:
                Qn, P, R, fb = blockortho.bcgs_pip_explicit(Y[:, :k], W, PIVOT_TOL, use_shift, pip_tol=PIP_TOL)
                stats["fallbacks"] += int(fb >= 1)
                stats["shifted"] += int(fb == 2)
            except CholeskyBreakdown:
                # the cycle keeps the columns of its completed big panels (their stage 2
                # is done and their residual was checked); the unfinished big panel is
                # dropped
                k_used = done - 1
                breakdown = ("panel", j)
                break
            Y[:, k: k + s] = Qn
            H[: k + s, k - 1: k - 1 + s] = hessenberg_block(H, P, R, B, k)
            b0, b1 = bigs[bi]
            if k + s == b1:
                kept, m00 = stage2(Y, H, done, b1, b1 - 1)
                if done == 0 and kept > 0:
                    g0 = beta * m00
                if kept < b1 - done:  # stage-2 breakdown: keep the leading columns
                    k_used = done + kept - 1
                    breakdown = ("stage2", done + kept)
                    done = done + kept
                    break
                done = b1
                bi += 1
                _, est = givens_lsq(H[:b1, : b1 - 1], g0)
                if est <= tol_abs:
                    k_used = b1 - 1
                    break
        if k_used <= 0:
            return np.zeros(n), 0, beta, {"breakdown": breakdown} if record else None
        y, est = givens_lsq(H[: k_used + 1, :k_used], g0)
        stats["cycles"] += 1
        bp.cycle_done(H[:k_used, :k_used], stats["cycles"])
        dx = Y[:, :k_used] @ y
        if prec is not None:
            dx = prec(dx)
        rec = None
        if record:
            rec = {"Q": Y[:, : k_used + 1].copy(), "H": H[: k_used + 1, :k_used].copy(), "y": y,
                   "beta": beta, "g0": g0, "breakdown": breakdown}
        return dx, k_used, est, rec

    out = _outer(op, b, x0, tol, max_iters, cycle, record)
    bp.export(out)
    out["fallbacks"] = stats["fallbacks"]
    out["shifted"] = stats["shifted"]
    return out


def dense_solve(A, b):
    """Direct solve of a tiny system with LAPACK LU (numpy), for pins only."""
    M = np.zeros((A.n, A.n))
    for i in range(A.n):
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[p]] += A.val[p]
    return np.linalg.solve(M, b), M
