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
