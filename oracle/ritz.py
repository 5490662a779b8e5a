"""Newton basis from Leja-ordered Ritz values (test infrastructure only).

The paper runs its experiments with the monomial basis and names Newton and
Chebyshev bases (Bai, Hu and Reichel 1994) as the better-conditioned choice for
larger s (Sec. IV and Sec. VI).  This module states the Newton basis the way that
reference builds it, in plain FP64:

* ``ritz_values``    -- eigenvalues of the square k x k Hessenberg matrix of one
                        restart cycle (A Q_k = Q_{k+1} H): the Ritz values.  Library
                        primitive: numpy's LAPACK eigenvalue routine.
* ``leja_order``     -- the modified Leja ordering of a set closed under complex
                        conjugation: the point of largest modulus first, then each
                        next point maximizes the product of its distances to the
                        points already taken; the conjugate of a complex point is
                        taken right after it, so every pair is adjacent.
* ``capacity``       -- the scaling of every Newton step: the geometric mean of the
                        distances of the last Leja point to all earlier ones (the
                        Leja products tend to the logarithmic capacity of the set).
* ``newton_params``  -- theta, tau, sigma of the real form of the first s Leja
                        points: a complex pair a +- ib in positions i-1, i is applied
                        as two real steps
                            w_{i-1} = (A - aI) w_{i-2} / sigma,
                            w_i     = ((A - aI) w_{i-1} + (b^2 / sigma) w_{i-2}) / sigma,
                        which equals (A - zI)(A - conj(z) I) w_{i-2} / sigma^2.

Readings (the paper gives no Newton-basis details): the Ritz values come from the
first restart cycle that keeps at least s columns (that cycle runs with the shifted
basis); all k Ritz values are Leja-ordered and the first s used, in every panel of
every later cycle; when position s holds the first point of a complex pair, its real
part is used alone; ties of the Leja products go to the larger imaginary part, then
to the lower index; a capacity that is not a positive finite number falls back to
the Gershgorin half-width.
"""
from __future__ import annotations

import numpy as np


def ritz_values(H: np.ndarray) -> np.ndarray:
    """Eigenvalues of the square upper Hessenberg matrix H (k x k), complex array."""
    H = np.asarray(H, dtype=np.float64)
    if H.shape[0] != H.shape[1]:
        raise ValueError("square Hessenberg matrix expected")
    return np.linalg.eigvals(H).astype(np.complex128)


def _partner(z: np.ndarray, used: np.ndarray, i: int) -> int:
    """Index of the unused conjugate of z[i] (exact conjugates, as eigenvalue routines
    return them for real matrices; else the nearest unused point)."""
    want = np.conj(z[i])
    best, dist = -1, np.inf
    for j in range(len(z)):
        if used[j] or j == i:
            continue
        d = abs(z[j] - want)
        if d < dist:
            best, dist = j, d
    return best


def leja_order(z) -> tuple[np.ndarray, np.ndarray]:
    """Modified Leja ordering.  Returns (ordered points, second_of_pair flags)."""
    z = np.asarray(z, dtype=np.complex128)
    k = len(z)
    used = np.zeros(k, dtype=bool)
    logsum = np.zeros(k)  # sum of log|z_j - w| over the points w taken so far
    order, second = [], []

    def take(i, is_second):
        used[i] = True
        order.append(i)
        second.append(is_second)
        with np.errstate(divide="ignore"):
            for j in range(k):
                if not used[j]:
                    logsum[j] += np.log(abs(z[j] - z[i]))

    def pick(score):
        best = -1
        for j in range(k):
            if used[j]:
                continue
            if best < 0 or score[j] > score[best] or (score[j] == score[best] and z[j].imag > z[best].imag):
                best = j
        return best

    while len(order) < k:
        i = pick(np.abs(z) if not order else logsum)
        take(i, False)
        if z[i].imag != 0.0 and len(order) < k:
            p = _partner(z, used, i)
            if p >= 0:
                take(p, True)
    return z[order], np.array(second, dtype=bool)


def capacity(zl: np.ndarray) -> float:
    """Geometric mean of |z_k - z_j|, j < k, for the last Leja point z_k."""
    zl = np.asarray(zl, dtype=np.complex128)
    k = len(zl)
    if k < 2:
        return float("nan")
    with np.errstate(divide="ignore"):
        acc = 0.0
        for j in range(k - 1):
            acc += np.log(abs(zl[k - 1] - zl[j]))
    return float(np.exp(acc / (k - 1)))


def newton_params(zl: np.ndarray, second: np.ndarray, s: int, sigma: float):
    """(theta, tau, sigma) arrays of length s for the real form of the first s Leja points.

    Step i (0-based) computes w_{i+1} = ((A - theta_i I) w_i + tau_i w_{i-1}) / sigma_i;
    tau_i = Im(z_{i-1})^2 / sigma_{i-1} when z_i is the second point of a complex pair.
    """
    if len(zl) < s:
        raise ValueError("fewer Leja points than steps")
    theta = np.array([zl[i].real for i in range(s)])
    tau = np.zeros(s)
    sig = np.full(s, float(sigma))
    for i in range(1, s):
        if second[i]:
            tau[i] = zl[i - 1].imag ** 2 / sig[i - 1]
    return theta, tau, sig


def leja_ritz_params(H: np.ndarray, s: int, lo: float, hi: float):
    """theta, tau, sigma of the Newton basis from the k x k Hessenberg H of a cycle."""
    zl, second = leja_order(ritz_values(H))
    c = capacity(zl)
    if not (np.isfinite(c) and c > 0.0):
        c = 0.5 * (hi - lo)
    return newton_params(zl, second, s, c)
