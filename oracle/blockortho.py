"""Block orthogonalization schemes of the paper, plain FP64 (test infrastructure only).

Each one-panel routine takes the already-orthonormal (or, in stage 1 of the
two-stage scheme, pre-processed) columns ``Q`` and a new panel ``V`` and
returns ``(Qnew, P, R)`` with  V = Q P + Qnew R,  R upper triangular with a
positive diagonal -- the BlkOrth contract of Fig. 1's caption.

* ``cholqr``        -- Sec. IV-B, Fig. 3a: G = V^T V, R = Chol(G), Q = V R^{-1}.
* ``cholqr2``       -- Fig. 3b: CholQR twice, R = R2 R1 (stable under Eq. (1), Thm. 1).
* ``bcgs``          -- Fig. 2a: P = Q^T V, Vhat = V - Q P.
* ``bcgs2_cholqr2`` -- Fig. 2b with CholQR2 as first and CholQR as second
                       intra-block step (the "original s-step" scheme, Sec. IV-B).
* ``bcgs_pip``      -- Sec. IV-C, Fig. 4a: one reduction [Q, V]^T V gives P and
                       V^T V; the Gram of V - QP follows from the block
                       Pythagorean identity  G = V^T V - P^T P.
* ``bcgs_pip2``     -- Fig. 4b: BCGS-PIP twice (Thm. 2).
* ``two_stage``     -- Sec. V, Fig. 5 and Thm. 3, on a whole n x k block:
                       stage 1 = one BCGS-PIP per s-column panel against every
                       previous column (pre-processing only); stage 2 = BCGS-PIP
                       of each big panel of s_hat columns against the final
                       columns of the earlier big panels.

Block layout used by ``orthogonalize``: column 1 is normalized on its own,
then panels of s columns follow (the last one may be short), mirroring an
s-step Krylov basis whose first vector is the normalized residual.
"""
from __future__ import annotations

import numpy as np

from .dense import PIVOT_TOL, chol_upper, right_solve_upper, CholeskyBreakdown  # noqa: F401


def cholqr(V: np.ndarray, tol: float = 0.0):
    """(Q, R) with Q = V R^{-1}, R = Chol(V^T V).  Fig. 3a."""
    G = V.T @ V
    R = chol_upper(G, tol=tol)
    return right_solve_upper(V, R), R


def cholqr2(V: np.ndarray, tol: float = 0.0):
    """(Q, R) from CholQR applied twice; R = R2 R1.  Fig. 3b."""
    Q1, R1 = cholqr(V, tol)
    Q, R2 = cholqr(Q1, tol)
    return Q, R2 @ R1


def bcgs(Q: np.ndarray, V: np.ndarray):
    """(P, Vhat) with P = Q^T V and Vhat = V - Q P.  Fig. 2a (one reduction)."""
    P = Q.T @ V
    return P, V - Q @ P


def bcgs2_cholqr2(Q: np.ndarray, V: np.ndarray, tol: float = 0.0):
    """BCGS2 with CholQR2 then CholQR (five reductions per panel).  Fig. 2b.

    V = Q P1 + Vhat;  Vhat = Qt Ra (CholQR2);  Qt = Q P2 + Y;  Y = Qnew Rc (CholQR)
    =>  V = Q (P1 + P2 Ra) + Qnew (Rc Ra).
    """
    P1, Vhat = bcgs(Q, V)
    Qt, Ra = cholqr2(Vhat, tol)
    P2, Y = bcgs(Q, Qt)
    Qnew, Rc = cholqr(Y, tol)
    return Qnew, P1 + P2 @ Ra, Rc @ Ra


def bcgs_pip(Q: np.ndarray, V: np.ndarray, tol: float = 0.0):
    """BCGS with Pythagorean inner product (one reduction).  Fig. 4a.

    [P; G_V] = [Q, V]^T V;  G = G_V - P^T P;  R = Chol(G);  Qnew = (V - Q P) R^{-1}.
    ``tol``: relative pivot threshold against diag(G_V) (0 = fail only if not SPD).
    """
    # the single fused reduction [Q, V]^T V, written as its two blocks
    P = Q.T @ V
    GV = V.T @ V
    G = GV - P.T @ P
    R = chol_upper(G, ref_diag=np.diag(GV), tol=tol)
    Qnew = right_solve_upper(V - Q @ P, R)
    return Qnew, P, R


def bcgs_pip_explicit(Q: np.ndarray, V: np.ndarray, tol: float = 0.0, shifted: bool = False,
                      pip_tol: float | None = None):
    """BCGS-PIP, with an explicit-Gram second pass where the Pythagorean Gram fails.

    The Pythagorean Gram G_V - P^T P loses all accuracy once [Q, V] is too ill-conditioned
    for the working precision (the stability condition of BCGS-PIP, Sec. IV-C).  When its
    Cholesky fails the pivot test (relative threshold pip_tol, default tol; the GMRES cycles
    pass dense.PIP_TOL), the projection is applied explicitly first,
    Y = V - Q P1, and Y is orthogonalized by a second BCGS-PIP pass whose Gram has no
    cancellation: P2 = Q^T Y, G = Y^T Y - P2^T P2, R = Chol(G), Qnew = (Y - Q P2) R^{-1},
    so V = Q (P1 + P2) + Qnew R.  A pivot of the second pass fails when it is at most
    tol * (Y^T Y)_jj (Y itself too ill-conditioned) or at most tol^2 * (V^T V)_jj (the
    column is numerically in span(Q): the pivot is at the rounding level of V).

    shifted = True: where the second pass fails, shifted Cholesky QR (Fukaya et al. 2020,
    the remedy the paper cites for CholQR's instability) takes over: with the second
    pass's Gram G, Rs = Chol(G + mu I), mu = 10 tol trace(G) (a shift well above the Gram's
    rounding level), Z = (Y - Q P2) Rs^{-1} is well conditioned, and one more BCGS-PIP pass
    orthogonalizes it: P3 = Q^T Z, R3 = Chol(Z^T Z - P3^T P3) (pivot test tol * (Z^T Z)_jj),
    Qnew = (Z - Q P3) R3^{-1}; V = Q (P1 + P2 + P3 Rs) + Qnew (R3 Rs).  A column whose final
    pivot (R3 Rs)_jj^2 is at most tol^2 * (V^T V)_jj is numerically in span(Q) and still
    breaks down.
    Returns (Qnew, P, R, passes): passes = 0 (PIP), 1 (second pass), 2 (shifted pass too).
    """
    try:
        Qn, P, R = bcgs_pip(Q, V, tol if pip_tol is None else pip_tol)
        return Qn, P, R, 0
    except CholeskyBreakdown:
        pass
    P1 = Q.T @ V
    Y = V - Q @ P1
    P2 = Q.T @ Y
    GY = Y.T @ Y
    G = GY - P2.T @ P2
    refV = np.diag(V.T @ V)
    thr = np.maximum(tol * np.diag(GY), tol * tol * refV)
    try:
        R = chol_upper(G, ref_diag=thr, tol=1.0 if tol > 0.0 else 0.0)
        Qnew = right_solve_upper(Y - Q @ P2, R)
        return Qnew, P1 + P2, R, 1
    except CholeskyBreakdown:
        if not shifted or tol <= 0.0:
            raise
    s = V.shape[1]
    mu = 10.0 * tol * float(np.trace(G))
    Rs = chol_upper(G + mu * np.eye(s))
    Z = right_solve_upper(Y - Q @ P2, Rs)
    P3 = Q.T @ Z
    GZ = Z.T @ Z
    R3 = chol_upper(GZ - P3.T @ P3, ref_diag=np.diag(GZ), tol=tol)
    R = R3 @ Rs
    bad = np.nonzero(np.diag(R) ** 2 <= tol * tol * refV)[0]
    if bad.size:
        err = CholeskyBreakdown("column numerically in span(Q)")
        err.index = int(bad[0])
        raise err
    Qnew = right_solve_upper(Z - Q @ P3, R3)
    return Qnew, P1 + P2 + P3 @ Rs, R, 2


def bcgs_pip2(Q: np.ndarray, V: np.ndarray, tol: float = 0.0):
    """BCGS-PIP twice (two reductions).  Fig. 4b.

    V = Q P1 + Qt R1;  Qt = Q P2 + Qnew R2  =>  V = Q (P1 + P2 R1) + Qnew (R2 R1).
    """
    Qt, P1, R1 = bcgs_pip(Q, V, tol)
    Qnew, P2, R2 = bcgs_pip(Q, Qt, tol)
    return Qnew, P1 + P2 @ R1, R2 @ R1


ONE_STAGE = {
    "bcgs2_cholqr2": bcgs2_cholqr2,
    "bcgs_pip2": bcgs_pip2,
    "bcgs_pip": bcgs_pip,
}


def panel_bounds(k: int, s: int):
    """Column ranges [c0, c1) of the panels after the first (normalized) column."""
    out = []
    c0 = 1
    while c0 < k:
        c1 = min(c0 + s, k)
        out.append((c0, c1))
        c0 = c1
    return out


def _normalize_first(X: np.ndarray):
    x = X[:, 0]
    nrm = np.sqrt(x @ x)
    if not nrm > 0.0:
        raise CholeskyBreakdown("zero first column")
    return x / nrm, nrm


def orthogonalize(X: np.ndarray, s: int, algo: str = "two_stage", s_hat: int | None = None):
    """Orthonormalize the n x k block X; returns (Q, R) with X = Q R.

    algo: 'two_stage' (Fig. 5), 'bcgs_pip2' (Fig. 4b), 'bcgs2_cholqr2' (Fig. 2b),
    'bcgs_pip' (Fig. 4a, one pass only: pre-processing, not orthonormal in general),
    'cholqr', 'cholqr2', 'householder'.
    """
    X = np.asarray(X, dtype=np.float64)
    n, k = X.shape
    if algo == "cholqr":
        return cholqr(X)
    if algo == "cholqr2":
        return cholqr2(X)
    if algo == "householder":
        from .dense import householder_qr
        return householder_qr(X)
    if algo == "two_stage":
        return two_stage(X, s, s_hat if s_hat is not None else k - 1)
    step = ONE_STAGE[algo]
    Q = np.zeros((n, k), order="F")
    R = np.zeros((k, k))
    Q[:, 0], R[0, 0] = _normalize_first(X)
    for c0, c1 in panel_bounds(k, s):
        Qn, P, Rp = step(Q[:, :c0], X[:, c0:c1])
        Q[:, c0:c1] = Qn
        R[:c0, c0:c1] = P
        R[c0:c1, c0:c1] = Rp
    return Q, R


def big_panel_bounds(k: int, s: int, s_hat: int):
    """Big panels of the two-stage scheme: the first holds column 1 plus s_hat columns,
    each later one s_hat columns (the last may be short).  s must divide s_hat unless one
    big panel covers the whole block."""
    if s_hat >= k - 1:
        return [(0, k)]
    if s_hat % s != 0:
        raise ValueError("s must divide s_hat")
    out = []
    c0 = 0
    c1 = min(1 + s_hat, k)
    while c0 < k:
        out.append((c0, c1))
        c0 = c1
        c1 = min(c0 + s_hat, k)
    return out


def two_stage(X: np.ndarray, s: int, s_hat: int, return_stage1: bool = False):
    """Two-stage block orthogonalization of X (n x k).  Sec. V, Fig. 5, Thm. 3.

    Stage 1 (every panel of s columns): one BCGS-PIP of the panel against all
    columns before it -- final columns Q_{1:l-1} of earlier big panels and the
    pre-processed columns Qhat_{l:j-1} of the current one.  The result only keeps
    the accumulated basis well conditioned.
    Stage 2 (when a big panel Qhat_{l:t} is complete): BCGS-PIP(Q_{1:l-1}, Qhat_{l:t}).
    With s_hat = k - 1 this is one CholQR of all k columns.

    Bookkeeping: X = Y Rh where Y holds the current (mixed final / pre-processed)
    columns; stage 2 writes Qhat_big = Q_{1:l-1} P2 + Q_big R2, i.e. Y = Y' M with
    M = [[I, P2], [0, R2]] on the rows of the big panel, so Rh <- M Rh.
    """
    X = np.asarray(X, dtype=np.float64)
    n, k = X.shape
    Y = np.zeros((n, k), order="F")
    Rh = np.zeros((k, k))
    Y[:, 0], Rh[0, 0] = _normalize_first(X)
    panels = panel_bounds(k, s)
    bigs = big_panel_bounds(k, s, s_hat)
    stage1 = None
    done = 0  # number of columns already final (orthonormal after stage 2)
    pi = 0
    for (b0, b1) in bigs:
        # stage 1 over the panels inside this big panel
        while pi < len(panels) and panels[pi][1] <= b1:
            c0, c1 = panels[pi]
            Qn, P, Rp = bcgs_pip(Y[:, :c0], X[:, c0:c1])
            Y[:, c0:c1] = Qn
            Rh[:c0, c0:c1] = P
            Rh[c0:c1, c0:c1] = Rp
            pi += 1
        if return_stage1 and stage1 is None:
            stage1 = (Y.copy(), Rh.copy())
        # stage 2 on the big panel [b0, b1)
        Qprev = Y[:, :done]
        Qb, P2, R2 = bcgs_pip(Qprev, Y[:, b0:b1])
        Y[:, b0:b1] = Qb
        rows_big = Rh[b0:b1, :].copy()
        Rh[:done, :] += P2 @ rows_big
        Rh[b0:b1, :] = R2 @ rows_big
        done = b1
    if return_stage1:
        return Y, Rh, stage1
    return Y, Rh
