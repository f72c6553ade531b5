"""Two-sided Petrov-Galerkin projection and transfer functions.

Section II (the text after the bilinear system and Algorithm 2, and the
QB-IHOMM description with Algorithm 3): with ``V`` and ``W`` spanning the
primal and transposed solutions at the interpolation points, ``x ~ V x^``
and ``W^T r = 0`` give the reduced model, whose transfer function and its
derivative match the full ones at those points.  For a descriptor system
``E x' = A x + B u``, ``y = C^T x`` the reduced matrices are
``Ar = W^T A V``, ``Er = W^T E V``, ``Br = W^T B``, ``Cr = V^T C``; when
``E = I`` and ``W^T V`` is invertible this is the same transfer function as
the paper's ``(W^T V)^{-1} W^T K V`` form.  ``orth`` is a thin Householder QR.

``H(s) = C^T (s E - A)^{-1} B``,
``H'(s) = -C^T (s E - A)^{-1} E (s E - A)^{-1} B``, and in general
``H^(k)(s) = (-1)^k k! C^T [(s E - A)^{-1} E]^k (s E - A)^{-1} B`` (each
derivative of ``(s E - A)^{-1}`` brings a factor ``-(s E - A)^{-1} E``).
Projecting on J moments per shift on both sides (the moments
``X_j = (s E - A)^{-1} E X_{j-1}``) matches derivatives up to order 2J - 1.

Pinned by: exact Hermite interpolation at every shift with solutions from a
sparse direct solver, a nonzero error away from the shifts, the two-way
identity ``c^T x = y^T b``, the k-th derivatives against central
differences of the (k-1)-th, and matching to order 2J - 1 with J moments
(tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def orth(X: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return Q


def reduce(A: sp.spmatrix, e: np.ndarray, B: np.ndarray, C: np.ndarray,
           X: np.ndarray, Y: np.ndarray, orthonormalize: bool = True):
    """Reduced descriptor model ``(Ar, Er, Br, Cr)`` from primal solutions X
    and transposed solutions Y (columns)."""
    V = orth(X) if orthonormalize else np.asarray(X, dtype=np.float64)
    W = orth(Y) if orthonormalize else np.asarray(Y, dtype=np.float64)
    Ar = W.T @ (A @ V)
    Er = W.T @ (np.asarray(e)[:, None] * V)
    Br = W.T @ np.asarray(B).reshape(A.shape[0], -1)
    Cr = V.T @ np.asarray(C).reshape(A.shape[0], -1)
    return Ar, Er, Br, Cr


def transfer(Ar, Er, Br, Cr, s: float) -> np.ndarray:
    return Cr.T @ np.linalg.solve(s * Er - Ar, Br)


def transfer_derivative(Ar, Er, Br, Cr, s: float) -> np.ndarray:
    M = s * Er - Ar
    return -Cr.T @ np.linalg.solve(M, Er @ np.linalg.solve(M, Br))


def transfer_derivative_k(Ar, Er, Br, Cr, s: float, k: int) -> np.ndarray:
    """``H_r^(k)(s)`` of the reduced model, written out from the closed form."""
    M = s * Er - Ar
    Z = np.linalg.solve(M, Br)
    for _ in range(k):
        Z = np.linalg.solve(M, Er @ Z)
    return (-1) ** k * float(np.prod(np.arange(1, k + 1))) * (Cr.T @ Z)


def full_transfer_derivative_k(A, e, B, C, s: float, k: int) -> np.ndarray:
    """``H^(k)(s)`` of the full model via a sparse LU factorisation."""
    n = A.shape[0]
    ev = np.asarray(e, dtype=np.float64)
    lu = spla.splu((s * sp.diags(ev) - A).tocsc())
    Z = lu.solve(np.asarray(B, dtype=np.float64).reshape(n, -1))
    for _ in range(k):
        Z = lu.solve(ev[:, None] * Z)
    C2 = np.asarray(C, dtype=np.float64).reshape(n, -1)
    return (-1) ** k * float(np.prod(np.arange(1, k + 1))) * (C2.T @ Z)


def full_transfer(A, e, B, C, s: float):
    """``H(s)`` and ``H'(s)`` of the full model via a sparse LU factorisation."""
    n = A.shape[0]
    M = (s * sp.diags(np.asarray(e, dtype=np.float64)) - A).tocsc()
    lu = spla.splu(M)
    B2 = np.asarray(B, dtype=np.float64).reshape(n, -1)
    C2 = np.asarray(C, dtype=np.float64).reshape(n, -1)
    X = lu.solve(B2)
    Yt = lu.solve(C2, trans="T")
    H = C2.T @ X
    dH = -Yt.T @ (np.asarray(e)[:, None] * X)
    return H, dH
