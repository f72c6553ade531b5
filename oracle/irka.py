"""IRKA-style outer loop with computed shifts (test infrastructure).

BIRKA (Algorithm 2) without its bilinear terms is the iterative rational
Krylov algorithm: each round diagonalises the reduced matrix (line 3) and
solves the full systems at the mirror images of the reduced poles (lines 4
and 5), then projects (lines 6 and 7).  For a descriptor SISO system
``E x' = A x + b u``, ``y = c^T x``, a round at shifts ``sigma_i`` solves
``(sigma_i E - A) v_i = b`` and ``(sigma_i E - A)^T w_i = c``, projects with
``V = orth([v_i])``, ``W = orth([w_i])`` to ``(Ar, Er)``, and the next shifts
are ``-lambda_i`` for the eigenvalues ``lambda_i`` of the pencil
``(Ar, Er)``.  Rounds stop when the largest relative change of the sorted
shifts is at most ``tol``.

Readings (the paper gives the algorithm, not these): the shifts are kept in
ascending order; a round whose reduced pencil has a complex eigenvalue pair
ends the loop with status "complex" (the solver path works with real shifts
only); the returned model is the last one projected, built at the returned
shifts.  The solves here are exact (sparse LU), so the iterates depend only
on the subspaces; the GPU path reaches the same subspaces to its solve
tolerance.

The MIMO form (:func:`run_tangential`) solves one tangential pair per shift,
``(sigma_i E - A) v_i = B b_i`` and ``(sigma_i E - A)^T w_i = C c_i``, and
takes from the reduced pencil's eigenvectors both the next shifts and the
next directions: ``b_i = Br^T y_i`` and ``c_i = Cr^T x_i`` for the left and
right eigenvectors ``y_i``, ``x_i`` of the pole ``lambda_i`` (Algorithm 2's
line 3 with ``R`` the right eigenvectors: ``R^{-1} Er^{-1} Br`` and
``Cr^T R``), each scaled to unit length with its largest entry positive.

Pinned by (tests/test_oracle_pins.py): a full-order model (r = n) whose
shifts become the mirror images of the full system's poles after one round
and then stay fixed; at a converged fixed point, the mirror images of the
reduced poles equal the shifts and the reduced transfer function and its
derivative interpolate the full ones there (the first-order conditions of
H2-optimality for SISO systems); real poles for a symmetric system with
c = b.  The MIMO form (tests/test_oracle_irka_tangential.py): equal to the
SISO loop for m = q = 1, the tangential interpolation conditions of every
model it returns, and the directions reproducing themselves at a converged
fixed point.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import projection


@dataclasses.dataclass
class IrkaResult:
    sigmas: np.ndarray   # shifts of the returned model (ascending)
    rounds: int          # solve + project rounds run
    change: float        # relative change of the mirror images against sigmas
    status: str          # "converged", "max_rounds" or "complex"
    Ar: np.ndarray
    Er: np.ndarray
    Br: np.ndarray
    Cr: np.ndarray
    poles: np.ndarray    # eigenvalues of (Ar, Er)


def mirror_shifts(Ar: np.ndarray, Er: np.ndarray):
    """Eigenvalues of the pencil and their mirror images, ascending."""
    lam = sla.eigvals(Ar, Er)
    return lam, np.sort(-lam.real), float(np.max(np.abs(lam.imag)) / np.max(np.abs(lam)))


def run(A, e, b, c, sigmas, max_rounds: int = 20, tol: float = 1e-6,
        complex_tol: float = 1e-10) -> IrkaResult:
    n = A.shape[0]
    ev = np.asarray(e, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(n)
    c = np.asarray(c, dtype=np.float64).reshape(n)
    sig = np.sort(np.asarray(sigmas, dtype=np.float64))
    for z in range(1, max_rounds + 1):
        X = np.zeros((n, sig.size))
        Y = np.zeros((n, sig.size))
        for i, s in enumerate(sig):
            lu = spla.splu((s * sp.diags(ev) - A).tocsc())
            X[:, i] = lu.solve(b)
            Y[:, i] = lu.solve(c, trans="T")
        Ar, Er, Br, Cr = projection.reduce(A, ev, b, c, X, Y)
        lam, new, imag = mirror_shifts(Ar, Er)
        if imag > complex_tol:
            return IrkaResult(sig, z, np.inf, "complex", Ar, Er, Br, Cr, lam)
        change = float(np.max(np.abs(new - sig) / np.abs(sig)))
        if change <= tol:
            return IrkaResult(sig, z, change, "converged", Ar, Er, Br, Cr, lam)
        if z == max_rounds:
            return IrkaResult(sig, z, change, "max_rounds", Ar, Er, Br, Cr, lam)
        sig = new
    raise AssertionError("unreachable")


@dataclasses.dataclass
class TangentialResult:
    sigmas: np.ndarray   # shifts of the returned model (ascending)
    bdir: np.ndarray     # m x r: column i the right direction of shift i
    cdir: np.ndarray     # q x r: column i the left direction of shift i
    rounds: int
    change: float
    status: str          # "converged", "max_rounds" or "complex"
    Ar: np.ndarray
    Er: np.ndarray
    Br: np.ndarray       # r x m
    Cr: np.ndarray       # r x q
    poles: np.ndarray


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    k = int(np.argmax(np.abs(v)))
    return v * (np.sign(v[k]) / np.linalg.norm(v))


def tangent_directions(Ar, Er, Br, Cr):
    """Poles of the pencil and, in ascending order of their mirror images,
    the next shifts and directions (``Br^T y_i``, ``Cr^T x_i``)."""
    lam, vl, vr = sla.eig(Ar, Er, left=True, right=True)
    order = np.argsort(-lam.real)
    sig = -lam.real[order]
    bd = np.stack([_unit((Br.T @ np.conj(vl[:, i])).real) for i in order], axis=1)
    cd = np.stack([_unit((Cr.T @ vr[:, i]).real) for i in order], axis=1)
    return lam, sig, bd, cd


def run_tangential(A, e, B, C, sigmas, bdir, cdir, max_rounds: int = 20, tol: float = 1e-6,
                   complex_tol: float = 1e-10) -> TangentialResult:
    n = A.shape[0]
    ev = np.asarray(e, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    C = np.asarray(C, dtype=np.float64).reshape(n, -1)
    order = np.argsort(np.asarray(sigmas, dtype=np.float64))
    sig = np.asarray(sigmas, dtype=np.float64)[order]
    bd = np.asarray(bdir, dtype=np.float64).reshape(B.shape[1], -1)[:, order]
    cd = np.asarray(cdir, dtype=np.float64).reshape(C.shape[1], -1)[:, order]
    for z in range(1, max_rounds + 1):
        X = np.zeros((n, sig.size))
        Y = np.zeros((n, sig.size))
        for i, s in enumerate(sig):
            lu = spla.splu((s * sp.diags(ev) - A).tocsc())
            X[:, i] = lu.solve(B @ bd[:, i])
            Y[:, i] = lu.solve(C @ cd[:, i], trans="T")
        Ar, Er, Br, Cr = projection.reduce(A, ev, B, C, X, Y)
        lam = sla.eigvals(Ar, Er)
        if float(np.max(np.abs(lam.imag)) / np.max(np.abs(lam))) > complex_tol:
            return TangentialResult(sig, bd, cd, z, np.inf, "complex", Ar, Er, Br, Cr, lam)
        _, new, nbd, ncd = tangent_directions(Ar, Er, Br, Cr)
        change = float(np.max(np.abs(new - sig) / np.abs(sig)))
        if change <= tol:
            return TangentialResult(sig, bd, cd, z, change, "converged", Ar, Er, Br, Cr, lam)
        if z == max_rounds:
            return TangentialResult(sig, bd, cd, z, change, "max_rounds", Ar, Er, Br, Cr, lam)
        sig, bd, cd = new, nbd, ncd
    raise AssertionError("unreachable")
