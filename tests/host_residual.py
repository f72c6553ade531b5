"""True residuals recomputed on the host, with the recomputation's own error.

A solver that stops at ||b - M x|| <= tol ||b|| (its own FP64 residual) can
show a residual slightly above tol when the host recomputes it with another
summation order.  Each entry of the FP64 product b - M x is within
(w + 2) u (|b| + |M| |x|) of the exact residual (w the most entries in a row of
M, u = 2^-53), so the check is ||b - M x|| <= tol ||b|| + that bound's norm.
"""
import numpy as np
import scipy.sparse as sp

U = 2.0**-53


def residual_bound(M, x, b, tol=1e-10):
    """(||b - M x||, tol ||b|| + rounding bound) for a sparse or dense M."""
    if sp.issparse(M):
        Mc = M.tocsr()
        w = int(np.diff(Mc.indptr).max()) if Mc.shape[0] else 0
        aMx = abs(Mc) @ np.abs(x)
        r = b - Mc @ x
    else:
        w = M.shape[1]
        aMx = np.abs(M) @ np.abs(x)
        r = b - M @ x
    slack = (w + 2) * U * np.linalg.norm(np.abs(b) + aMx)
    return np.linalg.norm(r), tol * np.linalg.norm(b) + slack


def residual_ok(M, x, b, tol=1e-10):
    res, bound = residual_bound(M, x, b, tol)
    return res <= bound
