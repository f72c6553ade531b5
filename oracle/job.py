"""A whole multi-round shifted-solve job, in the order of Algorithm 4.

For every round z and shift i (chain order) the preconditioner factors are
built as :func:`oracle.chain.schedule` lists them (SPAI once, then reuse
updates), stored at the requested precision, and every column pair
``(b_j, c_j)`` is solved by two-sided BiCG with the chained preconditioner.
After each round the solutions are projected (Section II).

``columns_only`` restricts factor construction to a subset of columns (for
sampled comparisons on large systems); solves then cannot run.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bicg, chain, projection, spai
from .precision import round_storage


def build_factors(A, e, specs, prec: str = "f64", columns=None):
    """Build every factor of ``specs`` (FP64 least squares, values rounded to ``prec``)."""
    factors = []
    for spec in specs:
        if spec[0] == "spai":
            F = spai.spai(A, e, spec[1], columns=columns)
        else:
            F = spai.update(A, e, spec[1], spec[2], columns=columns)
        F = F.copy()
        F.data = round_storage(F.data, prec)
        factors.append(F.tocsr())
    return factors


SCHEDULES = {"reuse": chain.schedule, "direct": chain.schedule_direct,
             "first": chain.schedule_first}


def moments(A, e, B, C, sigmas, nmom: int, prec: str = "f64", tol: float = 1e-10,
            policy: str = "reuse", maxit=None, max_restarts: int = 3):
    """Moments ``X_j = (s E - A)^{-1} E X_{j-1}`` (``X_0`` solves with B) and the
    transposed ones with C, j < nmom, at every shift of one round, with the
    round's preconditioner chains (built once) and two-sided BiCG.  Returns
    (X, Y, stats) with moment j of column c of shift i at column
    ``(j * nshift + i) * m + c``."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    e = np.asarray(e, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    C = np.asarray(C, dtype=np.float64).reshape(n, -1)
    m, ns = B.shape[1], len(sigmas)
    specs, chains = SCHEDULES[policy]([list(sigmas)])
    factors = build_factors(A, e, specs, prec)
    E = sp.diags(e)
    X = np.zeros((n, nmom * ns * m))
    Y = np.zeros((n, nmom * ns * m))
    stats = [None] * (nmom * ns * m)
    for i, s in enumerate(sigmas):
        As = (float(s) * E - A).tocsr()
        AsT = As.T.tocsr()
        ch = chains[0][i]
        P = lambda v, ch=ch: chain.apply(factors, ch, v)
        PT = lambda v, ch=ch: chain.apply_transpose(factors, ch, v)
        for c in range(m):
            b, cc = B[:, c], C[:, c]
            for j in range(nmom):
                res = bicg.solve(lambda v: As @ v, lambda v: AsT @ v, b, cc, P, PT, tol=tol,
                                 maxit=maxit, max_restarts=max_restarts)
                k = (j * ns + i) * m + c
                X[:, k], Y[:, k], stats[k] = res.x, res.y, res
                b, cc = e * res.x, e * res.y
    return X, Y, stats


def run(A, e, B, C, rounds, prec: str = "f64", tol: float = 1e-10, want_dual: bool = True,
        maxit=None, max_restarts: int = 3, project: bool = True, factors=None,
        apply_prec: str = "f64", policy: str = "reuse"):
    """Return a dict with factor specs, factors, per-(round, shift, column)
    solutions and stats, and the reduced model of each round.

    ``prec`` is the storage precision of the factor values, ``apply_prec``
    the precision of the preconditioner apply (:func:`oracle.chain.apply`),
    ``policy`` the factor schedule: "reuse" (Algorithm 4), "direct" (a SPAI
    per shift) or "first" (Table 2's first approach)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    e = np.asarray(e, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    C = np.asarray(C, dtype=np.float64).reshape(n, -1)
    specs, chains = SCHEDULES[policy](rounds)
    if factors is None:
        factors = build_factors(A, e, specs, prec)
    E = sp.diags(e)
    out = {"specs": specs, "chains": chains, "factors": factors, "rounds": []}
    for z, sig in enumerate(rounds):
        X = np.zeros((n, len(sig) * B.shape[1]))
        Y = np.zeros((n, len(sig) * B.shape[1]))
        stats = []
        for i, s in enumerate(sig):
            As = (float(s) * E - A).tocsr()
            AsT = As.T.tocsr()
            ch = chains[z][i]
            P = lambda v, ch=ch: chain.apply(factors, ch, v, apply_prec)
            PT = lambda v, ch=ch: chain.apply_transpose(factors, ch, v, apply_prec)
            for j in range(B.shape[1]):
                res = bicg.solve(lambda v: As @ v, lambda v: AsT @ v, B[:, j],
                                 C[:, j] if want_dual else None, P, PT, tol=tol,
                                 maxit=maxit, max_restarts=max_restarts)
                col = i * B.shape[1] + j
                X[:, col] = res.x
                if want_dual:
                    Y[:, col] = res.y
                stats.append(res)
        rd = {"X": X, "Y": Y, "stats": stats}
        if project and want_dual:
            rd["reduced"] = projection.reduce(A, e, B, C, X, Y)
        out["rounds"].append(rd)
    return out
