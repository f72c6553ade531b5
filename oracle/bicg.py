"""Right-preconditioned two-sided BiCG for ``A_s x = b`` and ``A_s^T y = c``.

Section III-A defines the Krylov setting and right preconditioning
(``A P x~ = b``, ``x = P x~``, ``P ~ A^{-1}``).  The shifted solves come in
pairs: the columns of V solve ``(s E - A) x = B`` and the columns of W solve
the transposed systems with ``C`` (the two solve lines of Algorithms 2 and 3).
One biconjugate-gradient recurrence produces both: the shadow recurrence of
BiCG is exactly the transposed system, preconditioned with ``P^T``.

Readings where the paper is silent (it uses GMRES with tolerance 1e-6):

* stopping test: true, unpreconditioned 2-norm residual relative to ``||b||``
  (``||c||`` for the transposed system), per column, starting from zero;
  both must pass in pair mode;
* near-breakdown when ``|rho| <= 1e-14 ||z~|| ||r||`` or
  ``|delta| <= 1e-14 ||p~|| ||q||``: restart from the current iterates with
  the true residuals;
* after the recursive residuals pass, the true residuals are recomputed; if
  one fails the cycle restarts from the current iterates (refinement);
* at most ``maxit`` iterations per cycle, at most ``max_restarts`` restarts;
* a zero right-hand side has the zero solution and drops out of the test;
  in primal-only mode the shadow right-hand side is ``b``.

Pinned by: dense LU solves, the textbook conjugate-gradient iterates in the
symmetric case with ``c = b`` and no preconditioner, one-step convergence for
diagonal systems (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

Op = Callable[[np.ndarray], np.ndarray]

BREAKDOWN_EPS = 1e-14


@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    y: Optional[np.ndarray]
    iters: int
    restarts: int
    relres_primal: float
    relres_dual: float
    status: str  # "ok", "not_converged", "breakdown"


def _norm(v):
    return float(np.linalg.norm(v))


def _core(A: Op, AT: Op, P: Op, PT: Op, b, c, tol, maxit, max_restarts, check_dual):
    n = b.size
    x = np.zeros(n)
    xt = np.zeros(n)
    r = b.copy()
    rt = c.copy()
    nb, nc = _norm(b), _norm(c)
    iters = 0
    restarts = 0
    status = "not_converged"

    def passed(rp, rd):
        return rp <= tol * nb and (not check_dual or rd <= tol * nc)

    while True:
        broke = False
        rho_prev = None
        p = pt = None
        for _ in range(maxit):
            if passed(_norm(r), _norm(rt)):
                break
            z = P(r)
            zt = PT(rt)
            rho = float(zt @ r)
            if abs(rho) <= BREAKDOWN_EPS * _norm(zt) * _norm(r):
                broke = True
                break
            if rho_prev is None:
                p, pt = z, zt
            else:
                beta = rho / rho_prev
                p = z + beta * p
                pt = zt + beta * pt
            q = A(p)
            qt = AT(pt)
            delta = float(pt @ q)
            if abs(delta) <= BREAKDOWN_EPS * _norm(pt) * _norm(q):
                broke = True
                break
            alpha = rho / delta
            x = x + alpha * p
            xt = xt + alpha * pt
            r = r - alpha * q
            rt = rt - alpha * qt
            rho_prev = rho
            iters += 1
        # true residuals (refinement check)
        r = b - A(x)
        rt = c - AT(xt)
        rp, rd = _norm(r), _norm(rt)
        if passed(rp, rd):
            status = "ok"
            break
        if restarts >= max_restarts:
            status = "breakdown" if broke else "not_converged"
            break
        restarts += 1
    relp = rp / nb if nb > 0 else 0.0
    reld = rd / nc if nc > 0 else 0.0
    return x, xt, iters, restarts, relp, reld, status


def solve(A: Op, AT: Op, b: np.ndarray, c: Optional[np.ndarray] = None,
          P: Optional[Op] = None, PT: Optional[Op] = None, tol: float = 1e-10,
          maxit: Optional[int] = None, max_restarts: int = 3) -> SolveResult:
    """Solve ``A x = b`` and (if ``c`` is given) ``A^T y = c`` together.

    ``A``/``AT`` apply the operator and its transpose, ``P``/``PT`` the
    preconditioner and its transpose (identity when omitted)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    if maxit is None:
        maxit = min(n, 20000)
    ident = lambda v: np.asarray(v, dtype=np.float64)
    P = P or ident
    PT = PT or ident
    want_dual = c is not None
    c = np.asarray(c, dtype=np.float64) if want_dual else None
    nb = _norm(b)
    nc = _norm(c) if want_dual else 0.0
    zero = np.zeros(n)
    if nb == 0.0 and (not want_dual or nc == 0.0):
        return SolveResult(zero, zero.copy() if want_dual else None, 0, 0, 0.0, 0.0, "ok")
    if nb == 0.0:
        # only the transposed system is nontrivial: run it as the primal one
        y, _, it, rs, rel, _, st = _core(AT, A, PT, P, c, c, tol, maxit, max_restarts, False)
        return SolveResult(zero, y, it, rs, 0.0, rel, st)
    if want_dual and nc > 0.0:
        x, y, it, rs, relp, reld, st = _core(A, AT, P, PT, b, c, tol, maxit, max_restarts, True)
        return SolveResult(x, y, it, rs, relp, reld, st)
    x, _, it, rs, relp, _, st = _core(A, AT, P, PT, b, b.copy(), tol, maxit, max_restarts, False)
    return SolveResult(x, zero.copy() if want_dual else None, it, rs, relp, 0.0, st)
