"""Storage precision of preconditioner factor values.

The factor values are computed in FP64 and stored rounded: FP64 -> FP32 with
round-to-nearest-even, then (for BF16) FP32 -> BF16 with round-to-nearest-even
on the upper 16 bits of the FP32 pattern.  Applying a stored factor converts
the stored value back to FP64 exactly.

Pinned by: hand-checked bit patterns (ties to even, carries into the
exponent, overflow to infinity) and agreement with an independent library
conversion (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import numpy as np


def round_storage(values: np.ndarray, prec: str) -> np.ndarray:
    """Return ``values`` rounded to the storage precision ``prec`` and widened
    back to float64 (``prec`` is "f64", "f32" or "bf16")."""
    v = np.asarray(values, dtype=np.float64)
    if prec == "f64":
        return v.copy()
    f32 = v.astype(np.float32)  # IEEE round-to-nearest-even
    if prec == "f32":
        return f32.astype(np.float64)
    if prec != "bf16":
        raise ValueError(prec)
    bits = f32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    nan = np.isnan(f32)
    out = rounded.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out
