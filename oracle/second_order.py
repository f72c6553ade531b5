"""Second-order systems with proportional damping, solved as AIRGA solves them.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section II's AIRGA model is ``M x'' + D x' + K x = F u``, ``y = C^T x`` with
``D = alpha M + beta K``; Algorithm 1 solves, at every expansion point s_i,

* line 4:  ``X_0(s_i) = A(s_i)^{-1} F``,
* line 10: ``X_j(s_i) = -A(s_i)^{-1} M V_j``, ``V_j`` the previous result,

with ``A(s) = s^2 M + s D + K``, and Section III-C reuses the preconditioner
of ``A(s_{i-1})`` for ``A(s_i)`` (horizontal) and of the first point of the
previous round for the first point of the next (vertical), in Algorithm 4's
order.  Here M is diagonal (a lumped mass, given as its diagonal ``m``).

Readings: line 10 normalises ``V_j`` to unit Frobenius norm; that scales
each moment and leaves its span unchanged, so the moments here are the
unnormalised recurrence ``X_j = -A(s)^{-1} M X_{j-1}``.  The transposed
systems (``A(s)^T Y_j = -M Y_{j-1}``, ``Y_0`` with C) are solved beside
them as in the first-order pair; the loop over points is read per point.

* :func:`matrix`  -- ``A(s)`` on the factor pattern S = pattern(K) + diag.
* :func:`direct`  -- lines 4 and 10 by sparse LU, the definition.
* :func:`factors` -- SPAI of ``A(s_1)`` and the updates
  ``min ||A(s_{i-1}) - A(s_i) Q||_F`` column by column, on these matrices.
* :func:`solve`   -- lines 4 and 10 by two-sided BiCG with those chains.
* :func:`reduce`, :func:`transfer` -- Section II's Ritz-Galerkin reduced
  model ``(V^T M V, V^T D V, V^T K V, V^T F, V^T C)`` and its transfer
  function ``C^T A(s)^{-1} F``.

Pinned by: the companion (first-order, 2n) linearisation of the model solved
densely, and the modal closed form ``X_j = (-1)^j Phi d(s)^{-(j+1)} Phi^T F``
for symmetric K (``K Phi = M Phi Lambda``, ``Phi^T M Phi = I``,
``d(s) = s^2 + s(alpha + beta lambda) + lambda``), and for the reduction:
interpolation of the full transfer function at the points whose solutions V
spans, and the exact model for a complete basis
(tests/test_oracle_second_order.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bicg, chain, spai
from .precision import round_storage


def matrix(m, K, alpha: float, beta: float, s: float) -> sp.csc_matrix:
    """``A(s) = s^2 M + s D + K`` with ``D = alpha M + beta K``, stored on the
    pattern ``pattern(K) + diag`` (explicit zeros kept), CSC, sorted rows."""
    K = sp.coo_matrix(K)
    n = K.shape[0]
    m = np.asarray(m, dtype=np.float64)
    s = float(s)
    rows = np.concatenate([K.row, np.arange(n)])
    cols = np.concatenate([K.col, np.arange(n)])
    # s^2 M + s (alpha M + beta K) + K: the K terms on K's entries, the M terms on the diagonal
    vals = np.concatenate([(s * beta + 1.0) * K.data.astype(np.float64),
                           (s * s + s * alpha) * m])
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))  # duplicates are summed
    A.sort_indices()
    return A


def direct(m, K, alpha, beta, F, C, points, nmom: int = 1):
    """Lines 4 and 10 by sparse LU: returns (X, Y) with moment j of column c of
    point i at column ``(j * npoint + i) * ncol + c``."""
    m = np.asarray(m, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64).reshape(m.size, -1)
    C = np.asarray(C, dtype=np.float64).reshape(m.size, -1)
    ncol, npt = F.shape[1], len(points)
    X = np.zeros((m.size, nmom * npt * ncol))
    Y = np.zeros((m.size, nmom * npt * ncol))
    for i, s in enumerate(points):
        lu = spla.splu(matrix(m, K, alpha, beta, s))
        x, y = F.copy(), C.copy()
        for j in range(nmom):
            x = lu.solve(x if j == 0 else -(m[:, None] * x))
            y = lu.solve(y if j == 0 else -(m[:, None] * y), trans="T")
            k = (j * npt + i) * ncol
            X[:, k:k + ncol], Y[:, k:k + ncol] = x, y
    return X, Y


def factors(m, K, alpha, beta, rounds, prec: str = "f64"):
    """Factors of Algorithm 4 for the second-order matrices: returns
    (factor list, chains) with ``chains[z][i]`` the factor indices of point i
    of round z in application order (as :func:`oracle.chain.schedule`)."""
    specs, chains = chain.schedule(rounds)
    n = np.asarray(m).size
    out = []
    for spec in specs:
        if spec[0] == "spai":
            As = matrix(m, K, alpha, beta, spec[1])
            cols = [spai.spai_column(None, None, None, k, As=As) for k in range(n)]
        else:
            Ap = matrix(m, K, alpha, beta, spec[1])
            An = matrix(m, K, alpha, beta, spec[2])
            cols = [spai.update_column(None, None, None, None, k, As_new=An, As_prev=Ap)
                    for k in range(n)]
        P = _assemble(n, cols)
        P.data = round_storage(P.data, prec)
        out.append(P.tocsr())
    return out, chains


def _assemble(n, cols):
    indptr = np.zeros(n + 1, dtype=np.int64)
    for k, (J, _) in enumerate(cols):
        indptr[k + 1] = indptr[k] + J.size
    idx = np.concatenate([J for J, _ in cols])
    val = np.concatenate([v for _, v in cols])
    return sp.csc_matrix((val, idx, indptr), shape=(n, n))


def solve(m, K, alpha, beta, F, C, rounds, nmom: int = 1, prec: str = "f64",
          tol: float = 1e-10, maxit=None, max_restarts: int = 3):
    """Every round's points, lines 4 and 10, by two-sided BiCG right-preconditioned
    with the chains of :func:`factors`.  Returns a list over rounds of
    (X, Y, stats) in :func:`direct`'s column order."""
    m = np.asarray(m, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64).reshape(m.size, -1)
    C = np.asarray(C, dtype=np.float64).reshape(m.size, -1)
    fs, chains = factors(m, K, alpha, beta, rounds, prec)
    ncol = F.shape[1]
    out = []
    for z, pts in enumerate(rounds):
        npt = len(pts)
        X = np.zeros((m.size, nmom * npt * ncol))
        Y = np.zeros((m.size, nmom * npt * ncol))
        stats = [None] * (nmom * npt * ncol)
        for i, s in enumerate(pts):
            As = matrix(m, K, alpha, beta, s).tocsr()
            AsT = As.T.tocsr()
            ch = chains[z][i]
            P = lambda v, ch=ch: chain.apply(fs, ch, v)
            PT = lambda v, ch=ch: chain.apply_transpose(fs, ch, v)
            for c in range(ncol):
                b, cc = F[:, c], C[:, c]
                for j in range(nmom):
                    res = bicg.solve(lambda v: As @ v, lambda v: AsT @ v, b, cc, P, PT, tol=tol,
                                     maxit=maxit, max_restarts=max_restarts)
                    k = (j * npt + i) * ncol + c
                    X[:, k], Y[:, k], stats[k] = res.x, res.y, res
                    b, cc = -(m * res.x), -(m * res.y)
        out.append((X, Y, stats))
    return out


def reduce(m, K, alpha, beta, F, C, V):
    """Ritz-Galerkin reduction on the orthonormalised columns of V (Householder
    QR): returns ``(Mh, Dh, Kh, Fh, Ch)`` with ``Dh = V^T D V``."""
    Q, _ = np.linalg.qr(np.asarray(V, dtype=np.float64), mode="reduced")
    m = np.asarray(m, dtype=np.float64)
    K = sp.csr_matrix(K)
    Mh = Q.T @ (m[:, None] * Q)
    Kh = Q.T @ (K @ Q)
    D = alpha * sp.diags(m) + beta * K
    Dh = Q.T @ (D @ Q)
    Fh = Q.T @ np.asarray(F, dtype=np.float64).reshape(m.size, -1)
    Ch = Q.T @ np.asarray(C, dtype=np.float64).reshape(m.size, -1)
    return Mh, Dh, Kh, Fh, Ch


def transfer(Mh, Dh, Kh, Fh, Ch, s: float) -> np.ndarray:
    """``Ch^T (s^2 Mh + s Dh + Kh)^{-1} Fh`` (dense)."""
    return Ch.T @ np.linalg.solve(s * s * Mh + s * Dh + Kh, Fh)


def full_transfer(m, K, alpha, beta, F, C, s: float) -> np.ndarray:
    """``C^T A(s)^{-1} F`` by sparse LU."""
    n = np.asarray(m).size
    X = spla.splu(matrix(m, K, alpha, beta, s)).solve(np.asarray(F, dtype=np.float64).reshape(n, -1))
    return np.asarray(C, dtype=np.float64).reshape(n, -1).T @ X
