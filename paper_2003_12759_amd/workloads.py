"""Seeded synthetic inputs for the shifted-solve workloads.

This module only *generates inputs*: the system matrix ``A`` (CSR), the
diagonal of ``E``, the input/output blocks ``B`` and ``C`` and the shift
sets.  It holds none of the method's arithmetic (no preconditioner, no
Krylov step, no projection), so both the CPU oracle and the HIP path can be
fed from it.

The paper's own matrices (the academic and industrial disk-brake models of
the numerical-experiments section) are not available; stencil operators of
the same kind (sparse, nonsymmetric or symmetric, first-order descriptor form
``E x' = A x + B u``, ``y = C^T x``; appendix B writes the same pencil as
``sigma D - K``) stand in for them.

Conventions
-----------
* Grid points are numbered lexicographically, x fastest:
  ``idx = i + N*j (+ N*N*k)``.
* ``A = -K`` where ``K`` is the discretised (positive definite / M-matrix)
  diffusion(-convection) operator with homogeneous Dirichlet boundaries and
  mesh width ``h = 1/(N+1)``; the ``1/h^2`` scaling is kept, so ``A`` is
  stable and ``sigma*E - A`` is nonsingular for every ``sigma > 0``.
* Variable coefficients are cell-centred; the coupling between points ``p``
  and ``q`` uses the harmonic mean ``2 k_p k_q / (k_p + k_q)``.  A neighbour
  outside the domain contributes ``w * k_p / h^2`` to the diagonal only.
* 27-point weights are 1, 1/2, 1/3 for face, edge and corner neighbours.
* Random draws use ``numpy.random.default_rng(seed)`` in this order:
  coefficient field, E diagonal, B, C, shift jitter, request stream.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Workload",
    "laplacian_5pt",
    "convdiff_7pt_upwind",
    "varcoef_stencil",
    "make_workload",
    "ServingPool",
    "make_serving_pool",
    "centered_convection",
    "SecondOrderWorkload",
    "make_second_order",
    "WORKLOAD_NAMES",
]


@dataclasses.dataclass
class Workload:
    """One synthetic shifted-solve job.

    ``A`` is a scipy CSR matrix (float64, int32 indices, sorted columns);
    ``e`` the diagonal of ``E``; ``B`` (n x m) and ``C`` (n x q) are
    Fortran-ordered float64 blocks; ``rounds[z]`` is the shift list of outer
    round ``z`` in chain order; ``prec`` is the preconditioner storage
    precision ("f64", "f32" or "bf16"); ``r`` the reduced order per round.
    """

    name: str
    A: sp.csr_matrix
    e: np.ndarray
    B: np.ndarray
    C: np.ndarray
    rounds: List[np.ndarray]
    prec: str
    tol: float
    r: int
    meta: dict

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def nnz(self) -> int:
        return self.A.nnz


# ---------------------------------------------------------------------------
# stencil assembly helpers


def _grid_coords(N: int, dim: int):
    idx = np.arange(N**dim, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for _ in range(dim):
        coords.append(rem % N)
        rem //= N
    return idx, coords


def _assemble(n: int, rows, cols, vals) -> sp.csr_matrix:
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return M


def laplacian_5pt(N: int) -> sp.csr_matrix:
    """``A = -(1/h^2) (I (x) T + T (x) I)``, ``T = tridiag(-1, 2, -1)``, h = 1/(N+1)."""
    h = 1.0 / (N + 1)
    T = sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1])
    I = sp.identity(N)
    K = (sp.kron(I, T) + sp.kron(T, I)) / (h * h)
    A = (-K).tocsr()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def convdiff_7pt_upwind(N: int, b=(10.0, 5.0, 2.0)) -> sp.csr_matrix:
    """``-A = -Delta_h + b . grad_h`` on an N^3 grid, first-order upwind.

    With all ``b_d > 0`` the convection term uses backward differences
    ``b_d (u_p - u_{p - e_d}) / h``.  Row p of ``-A``: diagonal
    ``6/h^2 + sum_d b_d/h``, every in-domain neighbour ``-1/h^2`` and the
    lower neighbour in direction d an extra ``-b_d/h``.
    """
    n = N**3
    h = 1.0 / (N + 1)
    idx, (cx, cy, cz) = _grid_coords(N, 3)
    coords = (cx, cy, cz)
    strides = (1, N, N * N)
    rows, cols, vals = [idx], [idx], [np.full(n, -(6.0 / h**2 + sum(b) / h))]
    for d in range(3):
        for sgn in (-1, 1):
            ok = (coords[d] + sgn >= 0) & (coords[d] + sgn < N)
            p = idx[ok]
            w = 1.0 / h**2 + (b[d] / h if sgn < 0 else 0.0)
            rows.append(p)
            cols.append(p + sgn * strides[d])
            vals.append(np.full(p.size, w))  # A = -(-w) on off-diagonals
    return _assemble(n, rows, cols, vals)


def varcoef_stencil(N: int, dim: int, points: int, kappa: np.ndarray) -> sp.csr_matrix:
    """Variable-coefficient diffusion operator ``A = -K`` on an N^dim grid.

    ``points`` is 5 (dim 2), 7 (dim 3) or 27 (dim 3).  ``kappa`` holds one
    positive coefficient per grid point (cell centred).  Coupling weight for
    a neighbour at offset ``o`` is ``w(o) * 2 k_p k_q / (k_p + k_q) / h^2``
    with ``w = 1, 1/2, 1/3`` by the number of nonzero offset components;
    out-of-domain neighbours add ``w * k_p / h^2`` to the diagonal.
    """
    n = N**dim
    h2 = (1.0 / (N + 1)) ** 2
    idx, coords = _grid_coords(N, dim)
    strides = [N**d for d in range(dim)]
    if points in (5, 7):
        offsets = []
        for d in range(dim):
            for s in (-1, 1):
                o = [0] * dim
                o[d] = s
                offsets.append(tuple(o))
    elif points == 27 and dim == 3:
        offsets = [
            (a, b_, c)
            for c in (-1, 0, 1)
            for b_ in (-1, 0, 1)
            for a in (-1, 0, 1)
            if (a, b_, c) != (0, 0, 0)
        ]
    else:
        raise ValueError("unsupported stencil")
    kappa = np.asarray(kappa, dtype=np.float64).reshape(n)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for o in offsets:
        w = 1.0 / sum(abs(c) for c in o)
        ok = np.ones(n, dtype=bool)
        shift = 0
        for d in range(dim):
            ok &= (coords[d] + o[d] >= 0) & (coords[d] + o[d] < N)
            shift += o[d] * strides[d]
        p = idx[ok]
        q = p + shift
        kp, kq = kappa[p], kappa[q]
        coup = w * (2.0 * (kp * kq) / (kp + kq)) / h2
        diag[p] += coup
        out = idx[~ok]
        diag[out] += w * kappa[out] / h2
        rows.append(p)
        cols.append(q)
        vals.append(coup)  # off-diagonal of K is -coup, so A = +coup
    rows.append(idx)
    cols.append(idx)
    vals.append(-diag)
    return _assemble(n, rows, cols, vals)


# ---------------------------------------------------------------------------
# workloads


WORKLOAD_NAMES = (
    "laplace2d_n2025",  # 45x45 5-point, 6 shifts, FP64 factors
    "convdiff3d_n262144",  # 64^3 7-point upwind, 10 shifts x 3 rounds, FP32 factors
    "varcoef3d_n1191016_mimo4",  # 106^3 7-point, MIMO 4, 8 shifts
    "serving_pool16",  # 16 resident systems, request stream
    "varcoef27_n2097152",  # 128^3 27-point, 12 shifts, precision ladder
)


def _blocks(rng, n, m):
    B = np.asfortranarray(rng.standard_normal((n, m)))
    C = np.asfortranarray(rng.standard_normal((n, m)))
    return B, C


def make_workload(index: int, seed: int = 0, N: Optional[int] = None,
                  nshift: Optional[int] = None, nrounds: Optional[int] = None,
                  prec: Optional[str] = None) -> Workload:
    """Build workload ``index`` (0..4; 3 is the serving pool, see
    :func:`make_serving_pool`).  ``N`` overrides the grid size (the recipe is
    otherwise unchanged), ``nshift``/``nrounds`` shorten the shift schedule,
    ``prec`` overrides the preconditioner storage precision.
    """
    rng = np.random.default_rng(seed)
    if index == 0:
        N = N or 45
        A = laplacian_5pt(N)
        n = A.shape[0]
        e = rng.uniform(1.0, 2.0, n)
        B, C = _blocks(rng, n, 1)
        k = nshift or 6
        sig = 10.0 ** (3.0 * np.arange(6) / 5.0)[:k]
        rounds = [sig]
        return Workload(f"laplace2d_n{n}", A, e, B, C, rounds, prec or "f64",
                        1e-10, len(sig), {"grid": N, "stencil": "5pt"})
    if index == 1:
        N = N or 64
        A = convdiff_7pt_upwind(N)
        n = A.shape[0]
        e = rng.uniform(1.0, 2.0, n)
        B, C = _blocks(rng, n, 1)
        k = nshift or 10
        z = nrounds or 3
        base = 10.0 ** (-1.0 + 4.0 * np.arange(10) / 9.0)[:k]
        rounds = [base]
        for _ in range(1, z):
            jit = np.exp(rng.uniform(-math.log(1.2), math.log(1.2), base.size))
            rounds.append(rounds[-1] * jit)
        return Workload(f"convdiff3d_n{n}", A, e, B, C, rounds, prec or "f32",
                        1e-10, len(base), {"grid": N, "stencil": "7pt-upwind",
                                           "b": (10.0, 5.0, 2.0)})
    if index == 2:
        N = N or 106
        n = N**3
        kappa = 10.0 ** rng.uniform(-1.0, 1.0, n)
        A = varcoef_stencil(N, 3, 7, kappa)
        e = rng.uniform(1.0, 2.0, n)
        B, C = _blocks(rng, n, 4)
        k = nshift or 8
        sig = 10.0 ** (4.0 * np.arange(8) / 7.0)[:k]
        return Workload(f"varcoef3d_n{n}_mimo4", A, e, B, C, [sig], prec or "f64",
                        1e-10, 4 * len(sig), {"grid": N, "stencil": "7pt-varcoef"})
    if index == 4:
        N = N or 128
        n = N**3
        kappa = 10.0 ** rng.uniform(-1.0, 1.0, n)
        A = varcoef_stencil(N, 3, 27, kappa)
        e = rng.uniform(1.0, 2.0, n)
        B, C = _blocks(rng, n, 1)
        k = nshift or 12
        sig = 10.0 ** (4.0 * np.arange(12) / 11.0)[:k]
        return Workload(f"varcoef27_n{n}", A, e, B, C, [sig], prec or "bf16",
                        1e-10, len(sig), {"grid": N, "stencil": "27pt-varcoef"})
    raise ValueError("workload index must be 0, 1, 2 or 4 (3 is the serving pool)")


def centered_convection(N: int, b=(20.0, 10.0, 5.0)) -> sp.csr_matrix:
    """Skew-symmetric ``b . grad_h`` on an N^3 grid (central differences,
    Dirichlet boundaries): row p holds ``+b_d / 2h`` at the upper and
    ``-b_d / 2h`` at the lower neighbour in direction d."""
    n = N**3
    h = 1.0 / (N + 1)
    idx, coords = _grid_coords(N, 3)
    strides = (1, N, N * N)
    rows, cols, vals = [], [], []
    for d in range(3):
        for sgn in (-1, 1):
            ok = (coords[d] + sgn >= 0) & (coords[d] + sgn < N)
            p = idx[ok]
            rows.append(p)
            cols.append(p + sgn * strides[d])
            vals.append(np.full(p.size, sgn * b[d] / (2.0 * h)))
    return _assemble(n, rows, cols, vals)


@dataclasses.dataclass
class SecondOrderWorkload:
    """A proportionally damped second-order system ``M x'' + D x' + K x = F u``,
    ``y = C^T x``, ``D = alpha M + beta K``, with a lumped (diagonal) mass
    ``m``; ``rounds[z]`` are the expansion points of outer round z.  The
    first-order system the solver is given is ``A = -K``, ``E = diag(m)``."""

    name: str
    K: sp.csr_matrix
    m: np.ndarray
    alpha: float
    beta: float
    F: np.ndarray
    C: np.ndarray
    rounds: List[np.ndarray]
    prec: str
    tol: float
    meta: dict

    @property
    def n(self) -> int:
        return self.K.shape[0]

    @property
    def A(self) -> sp.csr_matrix:
        A = (-self.K).tocsr()
        A.sort_indices()
        A.indices = A.indices.astype(np.int32)
        A.indptr = A.indptr.astype(np.int32)
        return A


def make_second_order(seed: int = 0, N: int = 106, nround: int = 2, npoint: int = 4,
                      unit_io: bool = True, prec: str = "f64") -> SecondOrderWorkload:
    """Stand-in for the disk-brake models of the AIRGA experiments: stiffness
    ``K = K_E + K_R`` with ``K_E`` the 27-point variable-coefficient diffusion
    operator (coefficients log-uniform in [0.1, 10]) and ``K_R`` a
    skew-symmetric centred convection (the nonsymmetric part), lumped mass
    uniform in [1, 2], the paper's damping ``alpha = 5e-2``, ``beta = 5e-6``,
    ``npoint`` expansion points linearly spaced in [1, 500] (later rounds
    jittered by up to 10 %), and ``F = C = e_1`` (``unit_io``) or standard
    normal columns.  N = 106 gives n = 1,191,016, the size class of the
    industrial model.  Draws: coefficient field, mass, F, C, point jitter."""
    rng = np.random.default_rng(seed)
    n = N**3
    kappa = 10.0 ** rng.uniform(-1.0, 1.0, n)
    KE = -varcoef_stencil(N, 3, 27, kappa)
    K = (KE + centered_convection(N)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    K.indices = K.indices.astype(np.int32)
    K.indptr = K.indptr.astype(np.int32)
    m = rng.uniform(1.0, 2.0, n)
    if unit_io:
        F = np.zeros((n, 1), order="F")
        C = np.zeros((n, 1), order="F")
        F[0, 0] = C[0, 0] = 1.0
    else:
        F, C = _blocks(rng, n, 1)
    base = np.linspace(1.0, 500.0, npoint)
    rounds = [base]
    for _ in range(1, nround):
        rounds.append(rounds[-1] * (1.0 + rng.uniform(-0.1, 0.1, npoint)))
    return SecondOrderWorkload(f"airga_varcoef27_n{n}", K, m, 5e-2, 5e-6, F, C, rounds, prec,
                               1e-10, {"grid": N, "stencil": "27pt-varcoef + skew 7pt"})


@dataclasses.dataclass
class ServingPool:
    """Resident systems plus a Poisson request stream.

    ``systems[s] = (A, e)``; request ``t`` asks for the primal solve of
    ``(sigma_t E_s - A_s) x = b_t`` and arrives at ``arrival[t]`` (seconds,
    scaled by the offered rate chosen by the caller).
    """

    systems: list
    req_system: np.ndarray
    req_sigma: np.ndarray
    req_seed: np.ndarray
    gaps: np.ndarray  # unit-rate exponential inter-arrival gaps

    def rhs(self, t: int) -> np.ndarray:
        n = self.systems[self.req_system[t]][0].shape[0]
        return np.random.default_rng(int(self.req_seed[t])).standard_normal(n)


def make_serving_pool(seed: int = 0, nsys: int = 16, nreq: int = 10000,
                      nmin: int = 4096, nmax: int = 262144) -> ServingPool:
    """16 systems with ``n`` log-uniform in [nmin, nmax]; kinds alternate
    2-D 5-point / 3-D 7-point with coefficients uniform in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    systems = []
    for s in range(nsys):
        ns = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        if s % 2 == 0:
            N = max(3, int(round(math.sqrt(ns))))
            kappa = rng.uniform(0.5, 2.0, N * N)
            A = varcoef_stencil(N, 2, 5, kappa)
        else:
            N = max(3, int(round(ns ** (1.0 / 3.0))))
            kappa = rng.uniform(0.5, 2.0, N**3)
            A = varcoef_stencil(N, 3, 7, kappa)
        systems.append((A, rng.uniform(1.0, 2.0, A.shape[0])))
    req_system = rng.integers(0, nsys, nreq)
    req_sigma = np.exp(rng.uniform(0.0, math.log(1e3), nreq))
    req_seed = rng.integers(0, 2**62, nreq)
    gaps = rng.exponential(1.0, nreq)
    return ServingPool(systems, req_system, req_sigma, req_seed, gaps)
