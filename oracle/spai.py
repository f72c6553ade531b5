"""SPAI construction and the column-wise reuse update.

* SPAI (Section III-A, eqs. gen-precond and gen-precond-par):
  ``min_P ||I - A_s P||_F^2`` splits into n independent problems
  ``min_p ||e_k - A_s p||_2``.  With the support of ``p`` fixed to ``J_k``
  only the rows ``I_k`` of ``A_s[:, J_k]`` are nonzero, so each problem is
  the small dense least-squares problem ``A_s[I_k, J_k] p = e_k[I_k]``.
* Reuse update (Section III-B, Table 2 second approach, and Section III-C for
  the horizontal and vertical directions): ``P_i = Q_i P_{i-1}`` with
  ``min_Q ||A_{i-1} - A_i Q||_F^2``, again n independent column problems
  ``min_q ||A_{i-1} e_k - A_i q||_2`` (the note under Algorithm 4 says these
  are solved like eq. gen-precond-par).  Here ``A_i = sigma_i E - A``.

Every column problem is solved with LAPACK least squares (``numpy.linalg.lstsq``)
on the dense local matrix; nothing is blocked or fused.

Pinned by: brute-force least squares over all n rows, the normal equations,
the full-pattern closed forms ``P = A_s^{-1}`` and
``Q_i = A_i^{-1} A_{i-1} = (I + (s_i - s_{i-1}) A_{i-1}^{-1} E)^{-1}``
(appendix B), and the static-pattern identity
``Q_i = I - (s_i - s_{i-1}) SPAI(A_i) E`` (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .pattern import column_support, shadow_rows, shifted_pattern_values


def _local_matrix(As: sp.csc_matrix, J: np.ndarray, I: np.ndarray) -> np.ndarray:
    """Dense ``As[I, J]`` (As is CSC with the pattern S)."""
    M = np.zeros((I.size, J.size))
    for a, j in enumerate(J):
        lo, hi = As.indptr[j], As.indptr[j + 1]
        M[np.searchsorted(I, As.indices[lo:hi]), a] = As.data[lo:hi]
    return M


def _column_rhs(As_prev: sp.csc_matrix, k: int, I: np.ndarray) -> np.ndarray:
    """Column k of ``As_prev`` restricted to the rows ``I``."""
    rhs = np.zeros(I.size)
    lo, hi = As_prev.indptr[k], As_prev.indptr[k + 1]
    rhs[np.searchsorted(I, As_prev.indices[lo:hi])] = As_prev.data[lo:hi]
    return rhs


def spai_column(A, e, sigma: float, k: int, As: sp.csc_matrix | None = None):
    """Column k of the SPAI of ``A_s = sigma E - A``: ``(J_k, p_k)``."""
    if As is None:
        As = shifted_pattern_values(A, e, sigma)
    J = column_support(As, k)
    I = shadow_rows(As, J)
    M = _local_matrix(As, J, I)
    rhs = (I == k).astype(np.float64)
    p, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    return J, p


def update_column(A, e, sigma_prev: float, sigma_new: float, k: int,
                  As_new: sp.csc_matrix | None = None, As_prev: sp.csc_matrix | None = None):
    """Column k of ``Q = argmin ||A_prev - A_new Q||_F`` on the pattern S: ``(J_k, q_k)``."""
    if As_new is None:
        As_new = shifted_pattern_values(A, e, sigma_new)
    if As_prev is None:
        As_prev = shifted_pattern_values(A, e, sigma_prev)
    J = column_support(As_new, k)
    I = shadow_rows(As_new, J)
    M = _local_matrix(As_new, J, I)
    rhs = _column_rhs(As_prev, k, I)
    q, *_ = np.linalg.lstsq(M, rhs, rcond=None)
    return J, q


def _assemble(n: int, cols) -> sp.csc_matrix:
    indptr = np.zeros(n + 1, dtype=np.int64)
    idx, val = [], []
    for k, (J, v) in enumerate(cols):
        indptr[k + 1] = indptr[k] + J.size
        idx.append(J)
        val.append(v)
    return sp.csc_matrix((np.concatenate(val), np.concatenate(idx), indptr), shape=(n, n))


def spai(A, e, sigma: float, columns=None) -> sp.csc_matrix:
    """SPAI factor ``P`` of ``sigma E - A`` (all columns, or ``columns`` only,
    the others left empty)."""
    n = A.shape[0]
    As = shifted_pattern_values(A, e, sigma)
    todo = range(n) if columns is None else set(int(c) for c in columns)
    cols = []
    for k in range(n):
        if k in todo:
            cols.append(spai_column(A, e, sigma, k, As=As))
        else:
            cols.append((np.zeros(0, dtype=np.int64), np.zeros(0)))
    return _assemble(n, cols)


def update(A, e, sigma_prev: float, sigma_new: float, columns=None) -> sp.csc_matrix:
    """Reuse factor ``Q`` with ``min ||(sigma_prev E - A) - (sigma_new E - A) Q||_F``."""
    n = A.shape[0]
    As_new = shifted_pattern_values(A, e, sigma_new)
    As_prev = shifted_pattern_values(A, e, sigma_prev)
    todo = range(n) if columns is None else set(int(c) for c in columns)
    cols = []
    for k in range(n):
        if k in todo:
            cols.append(update_column(A, e, sigma_prev, sigma_new, k, As_new=As_new, As_prev=As_prev))
        else:
            cols.append((np.zeros(0, dtype=np.int64), np.zeros(0)))
    return _assemble(n, cols)
