"""Static sparsity pattern of the preconditioner factors.

The SPAI column problem (Section III-A, eq. gen-precond-par) restricts column
k of the approximate inverse to a prescribed support.  Here that support is
the pattern of column k of ``A`` plus the diagonal entry (the paper's MSPAI
grows patterns adaptively; here they are fixed to A's pattern).  Because
``E`` is diagonal, ``sigma E - A`` has exactly this pattern ``S`` for every
shift, and the reuse factors ``Q_i`` are given the same support.

Pinned by: brute force against dense patterns on small matrices
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def shifted_pattern_values(A: sp.spmatrix, e: np.ndarray, sigma: float) -> sp.csc_matrix:
    """``sigma*diag(e) - A`` stored on the pattern ``S = pattern(A) + diag``.

    Explicit zeros are kept so that the structure never depends on values.
    Returns a CSC matrix with sorted row indices.
    """
    A = sp.coo_matrix(A)
    n = A.shape[0]
    rows = np.concatenate([A.row, np.arange(n)])
    cols = np.concatenate([A.col, np.arange(n)])
    vals = np.concatenate([-A.data.astype(np.float64), sigma * np.asarray(e, dtype=np.float64)])
    M = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))  # duplicates are summed
    M.sort_indices()
    return M


def pattern(A: sp.spmatrix) -> sp.csc_matrix:
    """Boolean-valued (1.0) CSC matrix of ``S = pattern(A) + diag``."""
    n = A.shape[0]
    S = shifted_pattern_values(A, np.zeros(n), 0.0)
    S.data[:] = 1.0
    return S


def column_support(S: sp.csc_matrix, k: int) -> np.ndarray:
    """``J_k``: rows of column k of S, i.e. the allowed nonzeros of column k of a factor."""
    return S.indices[S.indptr[k]:S.indptr[k + 1]].astype(np.int64)


def shadow_rows(S: sp.csc_matrix, J: np.ndarray) -> np.ndarray:
    """``I_k``: every row touched by the columns ``J`` of S (sorted, unique)."""
    parts = [S.indices[S.indptr[j]:S.indptr[j + 1]] for j in J]
    return np.unique(np.concatenate(parts)).astype(np.int64)
