"""Convenience wrappers over the libmorx binding (marshalling only).

``Context`` and ``System`` own the C handles; ``System.solve_shifts`` and
``System.project`` move host arrays to the device, call the C entry points
and return torch tensors.  No step of the method runs here.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import morx


class Context:
    def __init__(self, device: int = 0):
        self.device = device
        self.handle = morx.morx_create(device)

    def close(self):
        if self.handle:
            morx.morx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_dev(a, dtype=torch.float64, device="cuda"):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def block_to_dev(M: np.ndarray, device="cuda") -> torch.Tensor:
    """Column-major (n, m) device block from a host array (n,) or (n, m)."""
    M = np.asarray(M, dtype=np.float64)
    if M.ndim == 1:
        M = M[:, None]
    t = torch.as_tensor(np.ascontiguousarray(M.T), device=device)
    return t.t()


class System:
    """Resident ``A`` (scipy CSR) and ``E = diag(e)`` on the context's device."""

    def __init__(self, ctx: Context, A, e, stream=None):
        self.ctx = ctx
        A = A.tocsr()
        A.sort_indices()
        self.n = A.shape[0]
        dev = f"cuda:{ctx.device}"
        rowptr = to_dev(A.indptr, torch.int32, dev)
        colind = to_dev(A.indices, torch.int32, dev)
        val = to_dev(A.data, torch.float64, dev)
        ed = to_dev(e, torch.float64, dev)
        self.handle = morx.morx_system_create(ctx.handle, rowptr, colind, val, ed, stream)
        self.nnz_pattern, self.resident_bytes = morx.morx_system_info(self.handle)
        self.device = dev

    def close(self):
        if self.handle:
            morx.morx_system_destroy(self.handle)
            self.handle = None

    def pattern(self):
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(self.nnz_pattern, dtype=torch.int32, device=self.device)
        morx.morx_system_pattern(self.handle, rp, ci)
        return rp.cpu().numpy(), ci.cpu().numpy()

    def solve_shifts(self, sigmas: Sequence[float], B, C=None, prec: str = "f64", tol: float = 1e-10,
                     batched: bool = True, next_round: bool = False, use_graph: bool = True,
                     poll_iters: int = 8, maxit: int = 0, max_restarts: int = 3,
                     raise_on_error: bool = True, apply: str = "f64", policy: str = "reuse"):
        """Returns (X, Y, status, stats); X, Y are column-major (n, m*nshift) tensors.

        ``prec`` is the storage precision of the factor values, ``apply`` the
        precision of the preconditioner apply ("f64" or "f32"), ``policy`` the
        factor schedule: "reuse" (Algorithm 4; ``next_round`` selects the
        vertical update), "direct" (a SPAI per shift) or "first" (Table 2's
        first approach)."""
        Bd = B if isinstance(B, torch.Tensor) else block_to_dev(B, self.device)
        Cd = None
        if C is not None:
            Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        m = Bd.shape[1]
        ns = len(sigmas)
        X = morx.colmajor(m * ns, self.n, device=self.device)
        Y = morx.colmajor(m * ns, self.n, device=self.device) if Cd is not None else None
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        if policy == "reuse":
            o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        else:
            o.chain = {"direct": morx.MORX_CHAIN_DIRECT, "first": morx.MORX_CHAIN_FIRST}[policy]
        o.want_dual = 1 if Cd is not None else 0
        o.batched = 1 if batched else 0
        o.use_graph = 1 if use_graph else 0
        o.poll_iters = poll_iters
        o.maxit = maxit
        o.max_restarts = max_restarts
        o.apply_prec = morx.PREC[apply]
        st, stats = morx.morx_solve_shifts(self.handle, sigmas, Bd, Cd, X, Y, o,
                                           raise_on_error=raise_on_error)
        return X, Y, st, stats

    def solve_moments(self, sigmas: Sequence[float], B, C=None, nmom: int = 2, prec: str = "f64",
                      tol: float = 1e-10, batched: bool = True, policy: str = "reuse",
                      next_round: bool = False, raise_on_error: bool = True):
        """Moments 0..nmom-1 at every shift; returns (X, Y, status, stats) with
        moment j of column c of shift i at column (j * nshift + i) * m + c."""
        Bd = B if isinstance(B, torch.Tensor) else block_to_dev(B, self.device)
        Cd = None
        if C is not None:
            Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        m = Bd.shape[1]
        ns = len(sigmas)
        X = morx.colmajor(nmom * m * ns, self.n, device=self.device)
        Y = morx.colmajor(nmom * m * ns, self.n, device=self.device) if Cd is not None else None
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        o.want_dual = 1 if Cd is not None else 0
        o.batched = 1 if batched else 0
        if policy == "reuse":
            o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        else:
            o.chain = {"direct": morx.MORX_CHAIN_DIRECT, "first": morx.MORX_CHAIN_FIRST}[policy]
        st, stats = morx.morx_solve_moments(self.handle, sigmas, Bd, Cd, nmom, X, Y, o,
                                            raise_on_error=raise_on_error)
        return X, Y, st, stats

    def solve_second_order(self, alpha: float, beta: float, points: Sequence[float], F, C=None,
                           nmom: int = 1, prec: str = "f64", tol: float = 1e-10,
                           batched: bool = True, next_round: bool = False,
                           raise_on_error: bool = True):
        """AIRGA's solves on a system made from A = -K and E = M (diagonal):
        ``X_0 = A(s)^{-1} F``, ``X_j = -A(s)^{-1} M X_{j-1}`` with
        ``A(s) = s^2 M + s (alpha M + beta K) + K``, and the transposed ones
        with C; returns (X, Y, status, stats) in solve_moments' layout."""
        Fd = F if isinstance(F, torch.Tensor) else block_to_dev(F, self.device)
        Cd = None
        if C is not None:
            Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        m = Fd.shape[1]
        npt = len(points)
        X = morx.colmajor(nmom * m * npt, self.n, device=self.device)
        Y = morx.colmajor(nmom * m * npt, self.n, device=self.device) if Cd is not None else None
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        o.want_dual = 1 if Cd is not None else 0
        o.batched = 1 if batched else 0
        o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        st, stats = morx.morx_solve_second_order(self.handle, alpha, beta, points, Fd, Cd, nmom,
                                                 X, Y, o, raise_on_error=raise_on_error)
        return X, Y, st, stats

    def gmres_shifts(self, sigmas: Sequence[float], B, C=None, restart: int = 30,
                     prec: str = "f64", tol: float = 1e-10, policy: str = "reuse",
                     next_round: bool = False, max_restarts: int = 3, maxit: int = 0,
                     raise_on_error: bool = True):
        """GMRES(restart) on the same chains; returns (X, Y, status, stats)."""
        Bd = B if isinstance(B, torch.Tensor) else block_to_dev(B, self.device)
        Cd = None
        if C is not None:
            Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        m = Bd.shape[1]
        ns = len(sigmas)
        X = morx.colmajor(m * ns, self.n, device=self.device)
        Y = morx.colmajor(m * ns, self.n, device=self.device) if Cd is not None else None
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        o.want_dual = 1 if Cd is not None else 0
        o.max_restarts = max_restarts
        o.maxit = maxit
        if policy == "reuse":
            o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        else:
            o.chain = {"direct": morx.MORX_CHAIN_DIRECT, "first": morx.MORX_CHAIN_FIRST}[policy]
        st, stats = morx.morx_gmres_shifts(self.handle, sigmas, Bd, Cd, restart, X, Y, o,
                                           raise_on_error=raise_on_error)
        return X, Y, st, stats

    def irka(self, sigmas: Sequence[float], b, c, max_rounds: int = 20, shift_tol: float = 1e-6,
             prec: str = "f64", tol: float = 1e-10, next_round: bool = False,
             raise_on_error: bool = True):
        """IRKA-style loop from the initial shifts (SISO b, c); returns
        (status, result dict) as morx.morx_irka."""
        bd = b if isinstance(b, torch.Tensor) else torch.as_tensor(
            np.ascontiguousarray(b, dtype=np.float64), device=self.device)
        cd = c if isinstance(c, torch.Tensor) else torch.as_tensor(
            np.ascontiguousarray(c, dtype=np.float64), device=self.device)
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        return morx.morx_irka(self.handle, sigmas, bd.reshape(-1).contiguous(),
                              cd.reshape(-1).contiguous(), max_rounds, shift_tol, o,
                              raise_on_error=raise_on_error)

    def solve_pairs(self, sigmas: Sequence[float], B, C=None, prec: str = "f64",
                    tol: float = 1e-10, batched: bool = True, next_round: bool = False,
                    raise_on_error: bool = True):
        """Column i of B (and C) is the right-hand side of shift i only; returns
        (X, Y, status, stats) in shift order."""
        Bd = B if isinstance(B, torch.Tensor) else block_to_dev(B, self.device)
        Cd = None
        if C is not None:
            Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        ns = len(sigmas)
        X = morx.colmajor(ns, self.n, device=self.device)
        Y = morx.colmajor(ns, self.n, device=self.device) if Cd is not None else None
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        o.want_dual = 1 if Cd is not None else 0
        o.batched = 1 if batched else 0
        o.chain = morx.MORX_CHAIN_NEXT_ROUND if next_round else morx.MORX_CHAIN_RESET
        st, stats = morx.morx_solve_pairs(self.handle, sigmas, Bd, Cd, X, Y, o,
                                          raise_on_error=raise_on_error)
        return X, Y, st, stats

    def irka_tangential(self, sigmas: Sequence[float], B, C, bdir, cdir, max_rounds: int = 20,
                        shift_tol: float = 1e-6, prec: str = "f64", tol: float = 1e-10,
                        raise_on_error: bool = True):
        """The MIMO (tangential) IRKA-style loop; returns (status, result dict)
        as morx.morx_irka_tangential."""
        Bd = B if isinstance(B, torch.Tensor) else block_to_dev(B, self.device)
        Cd = C if isinstance(C, torch.Tensor) else block_to_dev(C, self.device)
        o = morx.morx_opts_default()
        o.tol = tol
        o.precond_prec = morx.PREC[prec]
        return morx.morx_irka_tangential(self.handle, sigmas, Bd, Cd, bdir, cdir, max_rounds,
                                         shift_tol, o, raise_on_error=raise_on_error)

    def autotune(self, sigma: float, ncols: int, chain_len: int = 1, prec: str = "f64") -> dict:
        """Time the launch-shape candidates on this system and keep the fastest."""
        return morx.morx_autotune(self.handle, sigma, ncols, chain_len, prec)

    def set_tune(self, factor_kernel: int = -1, cols_per_wave: int = -1,
                 slices_per_wave: int = -1, spmv_cols_per_wave: int = -1,
                 chain_kernel: int = -1) -> None:
        morx.morx_system_set_tune(self.handle, factor_kernel, cols_per_wave, slices_per_wave,
                                  spmv_cols_per_wave, chain_kernel)

    def get_tune(self) -> dict:
        return morx.morx_system_get_tune(self.handle)

    def project(self, V, W, B=None, C=None, orthonormalize=True):
        return morx.morx_project(self.handle, V, W, B, C, orthonormalize)
