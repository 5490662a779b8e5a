"""CSR operations of the oracle (test infrastructure only).

* ``spmv``        -- y = A x (the SpMV that the matrix-powers kernel applies s
                     times, Sec. III).  Library primitive: scipy's CSR product.
* ``spmv_plain``  -- the same product written as a plain row loop, for tiny
                     cross-checks.
* ``gershgorin``  -- real interval [lo, hi] containing the real parts of all
                     eigenvalues (Gershgorin discs); it fixes the scaling of the
                     monomial basis and the shift of the shifted basis.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def as_scipy(A) -> sp.csr_matrix:
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


class Operator:
    """Holds the scipy CSR matrix once so repeated products do not rebuild it."""

    def __init__(self, A):
        self.A = A
        self.n = A.n
        self.M = as_scipy(A)

    def __matmul__(self, x):
        return self.M @ x


def spmv(A, x: np.ndarray) -> np.ndarray:
    M = A.M if isinstance(A, Operator) else as_scipy(A)
    return M @ np.asarray(x, dtype=np.float64)


def spmv_plain(A, x: np.ndarray) -> np.ndarray:
    y = np.zeros(A.n)
    for i in range(A.n):
        acc = 0.0
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc += A.val[p] * x[A.col[p]]
        y[i] = acc
    return y


def gershgorin(A):
    """(lo, hi) = (min_i a_ii - r_i, max_i a_ii + r_i), r_i = sum_{j != i} |a_ij|."""
    A = A.A if isinstance(A, Operator) else A
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    is_diag = A.col == rows
    diag = np.zeros(A.n)
    np.add.at(diag, rows[is_diag], A.val[is_diag])
    rad = np.zeros(A.n)
    np.add.at(rad, rows[~is_diag], np.abs(A.val[~is_diag]))
    return float(np.min(diag - rad)), float(np.max(diag + rad))


def basis_params(A, s: int, basis: str = "monomial", shifts=None, interval=None):
    """Per-step shift theta_i and scale sigma_i of the s-step basis.

    The basis is built as w_i = (A w_{i-1} - theta_i w_{i-1}) / sigma_i.
    monomial: theta = 0, sigma = max(|lo|, |hi|);  shifted: theta = (lo+hi)/2,
    sigma = (hi-lo)/2;  newton: theta = given shifts, sigma = (hi-lo)/2.
    [lo, hi]: the Gershgorin interval of A, or the given interval (preconditioned operator).
    """
    lo, hi = gershgorin(A) if interval is None else interval
    if basis == "monomial":
        theta = np.zeros(s)
        sigma = np.full(s, max(abs(lo), abs(hi)))
    elif basis == "shifted":
        theta = np.full(s, 0.5 * (lo + hi))
        sigma = np.full(s, 0.5 * (hi - lo))
    elif basis == "newton":
        if shifts is None or len(shifts) != s:
            raise ValueError("newton basis needs s shifts")
        theta = np.asarray(shifts, dtype=np.float64)
        sigma = np.full(s, 0.5 * (hi - lo))
    else:
        raise ValueError(basis)
    return theta, sigma
