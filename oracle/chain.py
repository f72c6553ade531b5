"""Which factors make up each preconditioner, and how they are applied.

Algorithm 4 (AIRGA with reuse of the SPAI preconditioner) builds, for outer
round z and shift i:

* z = 1, i = 1: ``P_1^(1)`` by SPAI at ``s_1^(1)``;
* z = 1, i > 1: ``Q_i^(1)`` from ``min ||A_{i-1}^(1) - A_i^(1) Q||_F``
  (horizontal direction);
* z > 1, i = 1: ``Q_1^(z)`` from ``min ||A_1^(z-1) - A_1^(z) Q||_F``
  (vertical direction, only between the first shifts of consecutive rounds);
* z > 1, i > 1: ``Q_i^(z)`` from ``min ||A_{i-1}^(z) - A_i^(z) Q||_F``;

and solves with the preconditioner
``Q_i^(z) ... Q_2^(z) Q_1^(z) ... Q_1^(2) P_1^(1)``, i.e. ``i + z - 1``
factors.  The product is never formed (Section III-B): applying it to a
vector means applying ``P_1^(1)`` first and ``Q_i^(z)`` last; its transpose
applies the transposed factors in the reverse order.

Applying in FP32 (the mixed-precision form of the method's preconditioner,
whose storage may already be FP32 or BF16) is defined here as: the input
vector rounded to FP32, then every factor product formed in FP64 and its
result rounded to FP32 before the next factor; the output is the last rounded
vector.  The Krylov recurrences that consume it stay FP64.

Two comparators use other schedules: :func:`schedule_direct` (a fresh SPAI
per shift, no reuse) and :func:`schedule_first` (Table 2's first approach,
every update taken from the first shift).  Serving uses
:func:`schedule_anchored`: a resident anchor chain and one update per request.

Pinned by: hand-written expected schedules (all four), the chain
apply against the explicitly formed dense product on small matrices, and for
the FP32 apply: exact agreement with the FP64 apply when every intermediate
is an FP32 number, a rounding-error bound per pass, and FP32-representable
outputs (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

FactorSpec = Tuple  # ("spai", sigma) or ("update", sigma_prev, sigma_new)


def schedule(rounds: Sequence[Sequence[float]]):
    """Return ``(specs, chains)``.

    ``specs[f]`` describes factor f; ``chains[z][i]`` is the list of factor
    indices of the preconditioner for shift i of round z, in application
    order (first applied first)."""
    specs: List[FactorSpec] = []
    chains: List[List[List[int]]] = []
    vertical: List[int] = []  # P_1^(1), Q_1^(2), ..., Q_1^(z)
    for z, sig in enumerate(rounds):
        sig = [float(s) for s in sig]
        if z == 0:
            specs.append(("spai", sig[0]))
        else:
            specs.append(("update", float(rounds[z - 1][0]), sig[0]))
        vertical.append(len(specs) - 1)
        horizontal: List[int] = []
        round_chains = [list(vertical)]
        for i in range(1, len(sig)):
            specs.append(("update", sig[i - 1], sig[i]))
            horizontal.append(len(specs) - 1)
            round_chains.append(list(vertical) + list(horizontal))
        chains.append(round_chains)
    return specs, chains


def _to_apply(v: np.ndarray, apply_prec: str) -> np.ndarray:
    if apply_prec == "f64":
        return v
    if apply_prec != "f32":
        raise ValueError(apply_prec)
    return v.astype(np.float32).astype(np.float64)


def schedule_direct(rounds: Sequence[Sequence[float]]):
    """Comparator without reuse: a fresh SPAI at every shift of every round,
    each preconditioner a single factor (the paper's plain SPAI columns in its
    preconditioner-time tables).  Same ``(specs, chains)`` form as
    :func:`schedule`."""
    specs: List[FactorSpec] = []
    chains: List[List[List[int]]] = []
    for sig in rounds:
        round_chains = []
        for s in sig:
            specs.append(("spai", float(s)))
            round_chains.append([len(specs) - 1])
        chains.append(round_chains)
    return specs, chains


def schedule_first(rounds: Sequence[Sequence[float]]):
    """Table 2's first approach, round by round: ``P_1`` by SPAI at the round's
    first shift, then ``P_i = Q_i P_1`` with ``Q_i`` from
    ``min ||A_1 - A_i Q||_F`` (an update from the first shift to shift i), so
    every chain is ``[P_1]`` or ``[P_1, Q_i]``."""
    specs: List[FactorSpec] = []
    chains: List[List[List[int]]] = []
    for sig in rounds:
        sig = [float(s) for s in sig]
        specs.append(("spai", sig[0]))
        p1 = len(specs) - 1
        round_chains = [[p1]]
        for i in range(1, len(sig)):
            specs.append(("update", sig[0], sig[i]))
            round_chains.append([p1, len(specs) - 1])
        chains.append(round_chains)
    return specs, chains


def anchor_shifts(count: int, lo: float, hi: float) -> List[float]:
    """``count`` anchor shifts log-spaced over ``[lo, hi]``: ``lo (hi/lo)^(k/(count-1))``."""
    if count == 1:
        return [lo * (hi / lo) ** 0.0]
    return [lo * (hi / lo) ** (k / (count - 1)) for k in range(count)]


def schedule_anchored(anchors: Sequence[float], sigma: float) -> List[FactorSpec]:
    """The serving reading of Table 2's second approach along the horizontal
    direction of Section III-C: a resident chain of anchors (SPAI at the
    first, an update between each pair of consecutive anchors) and, for a
    request at ``sigma``, one more update from its nearest anchor (smallest
    ``|log sigma - log a_k|``, the first on ties).  Returns the request's
    chain as factor specs in application order."""
    dist = [abs(math.log(sigma) - math.log(a)) for a in anchors]
    k = min(range(len(anchors)), key=lambda j: (dist[j], j))
    out: List[FactorSpec] = [("spai", float(anchors[0]))]
    for j in range(1, k + 1):
        out.append(("update", float(anchors[j - 1]), float(anchors[j])))
    out.append(("update", float(anchors[k]), float(sigma)))
    return out


def apply(factors, chain: Sequence[int], v: np.ndarray, apply_prec: str = "f64") -> np.ndarray:
    """``F_chain[-1] ( ... F_chain[1] (F_chain[0] v))``, factors never multiplied together.

    ``apply_prec="f32"`` rounds the input and every pass result to FP32."""
    out = _to_apply(np.asarray(v, dtype=np.float64), apply_prec)
    for f in chain:
        out = _to_apply(factors[f] @ out, apply_prec)
    return out


def apply_rows(factors, chain: Sequence[int], v: np.ndarray, rows: Sequence[int],
               transpose: bool = False, factors_t=None) -> np.ndarray:
    """Selected entries of :func:`apply` (or :func:`apply_transpose` when
    ``transpose``), FP64, for systems too large to apply whole: row ``i`` of
    the chain's product is formed as the sparse row vector
    ``e_i^T F_chain[-1] ... F_chain[0]`` (``e_i^T F_chain[0]^T ... F_chain[-1]^T``)
    one factor at a time, then multiplied with ``v``.  The product is the
    same linear map; only the summation order differs.  ``factors_t`` may
    hold the transposes in CSR form (formed here otherwise)."""
    import scipy.sparse as sp

    n = factors[chain[0]].shape[0]
    if transpose:
        if factors_t is None:
            factors_t = {f: factors[f].T.tocsr() for f in set(chain)}
        mats = factors_t
        order = list(chain)
    else:
        mats = factors
        order = list(reversed(chain))
    out = np.empty(len(rows))
    for k, i in enumerate(rows):
        r = sp.csr_matrix(([1.0], ([0], [int(i)])), shape=(1, n))
        for f in order:
            r = r @ mats[f]
        out[k] = (r @ np.asarray(v, dtype=np.float64))[0]
    return out


def apply_transpose(factors, chain: Sequence[int], v: np.ndarray,
                    apply_prec: str = "f64") -> np.ndarray:
    """Transpose of :func:`apply`: ``F_chain[0]^T ( ... (F_chain[-1]^T v))``."""
    out = _to_apply(np.asarray(v, dtype=np.float64), apply_prec)
    for f in reversed(chain):
        out = _to_apply(factors[f].T @ out, apply_prec)
    return out
