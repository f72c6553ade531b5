"""Right-preconditioned restarted GMRES(m) for ``A_s x = b`` (and, run
separately, ``A_s^T y = c`` with ``P^T``).

The paper's experiments solve the shifted systems with GMRES (Section IV,
tolerance 1e-6) under the reused preconditioner chain; this is that solver
written out as the textbook generalized minimal residual method with right
preconditioning: Arnoldi on ``A P`` started from ``r_0 / ||r_0||`` (modified
Gram-Schmidt), Givens rotations reducing the Hessenberg matrix so that the
least-squares residual ``|g_{k+1}|`` is known at every step, and
``x = x_0 + P V_k y_k`` with ``y_k`` minimising ``|| ||r_0|| e_1 - H_k y ||``.

Readings where the paper is silent (the same as for BiCG where they apply):

* a cycle stops when ``|g_{k+1}| <= tol ||b||`` or after m steps; the true
  residual ``b - A x`` is then recomputed and the next cycle restarts from the
  current iterate until the true relative residual passes, at most
  ``max_restarts`` restarts beyond those the cycle length forces (a cycle
  that ends after m steps without meeting the estimate does not count as a
  restart);
* ``x_0 = 0``; a zero right-hand side has the zero solution;
* iterations are Arnoldi steps summed over all cycles.

Pinned by: dense LU solves, the minimal-residual property (after k steps of
the first cycle the iterate's residual equals the least-squares minimum over
``P K_k(A P, b)``, computed by brute force from an explicit Krylov basis), and
convergence within n steps for an n x n system (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

Op = Callable[[np.ndarray], np.ndarray]


@dataclasses.dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    cycles: int
    relres: float
    status: str  # "ok", "not_converged"


def _givens(a: float, b: float):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def cycle(A: Op, P: Op, x0: np.ndarray, r0: np.ndarray, m: int, stop: float,
          steps: Optional[int] = None):
    """One GMRES cycle from ``x0`` with residual ``r0``.  Returns
    ``(x, steps_taken, estimate)``; ``steps`` forces exactly that many steps
    (for the minimal-residual pin)."""
    n = r0.size
    beta = float(np.linalg.norm(r0))
    if beta == 0.0:
        return x0.copy(), 0, 0.0
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[:, 0] = r0 / beta
    k = 0
    limit = m if steps is None else steps
    for j in range(limit):
        w = A(P(V[:, j]))
        for i in range(j + 1):  # modified Gram-Schmidt
            H[i, j] = float(V[:, i] @ w)
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] > 0.0:
            V[:, j + 1] = w / H[j + 1, j]
        for i in range(j):  # earlier rotations on the new column
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        if steps is None and abs(g[k]) <= stop:
            break
        if H[j, j] == 0.0:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):  # back substitution with the rotated H
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    x = x0 + P(V[:, :k] @ y)
    return x, k, abs(g[k])


def solve(A: Op, b: np.ndarray, P: Optional[Op] = None, tol: float = 1e-10, m: int = 30,
          maxit: Optional[int] = None, max_restarts: int = 3) -> GmresResult:
    """Solve ``A x = b`` with right preconditioner ``P`` (identity when omitted).
    ``maxit`` bounds the Arnoldi steps over all cycles (default min(n, 20000))."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    P = P or (lambda v: np.asarray(v, dtype=np.float64))
    if maxit is None:
        maxit = min(n, 20000)
    nb = float(np.linalg.norm(b))
    x = np.zeros(n)
    if nb == 0.0:
        return GmresResult(x, 0, 0, 0.0, "ok")
    r = b.copy()
    iters = cycles = restarts = 0
    while True:
        x, k, est = cycle(A, P, x, r, m, tol * nb)
        iters += k
        cycles += 1
        r = b - A(x)
        rel = float(np.linalg.norm(r)) / nb
        if rel <= tol:
            return GmresResult(x, iters, cycles, rel, "ok")
        if iters >= maxit:
            return GmresResult(x, iters, cycles, rel, "not_converged")
        if est <= tol * nb or k < m:
            # the estimate passed (or the cycle broke down) but the true
            # residual did not: a refinement restart
            if restarts >= max_restarts:
                return GmresResult(x, iters, cycles, rel, "not_converged")
            restarts += 1


def solve_pair(A: Op, AT: Op, b: np.ndarray, c: np.ndarray, P: Optional[Op] = None,
               PT: Optional[Op] = None, **kw):
    """The primal and the transposed system, each by its own GMRES run."""
    return solve(A, b, P, **kw), solve(AT, c, PT, **kw)
