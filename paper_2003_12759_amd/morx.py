"""Thin ctypes binding of libmorx (include/morx.h).

Argument marshalling only: every function forwards to the C entry point of
the same name; torch tensors supply device pointers and streams.  Dense
blocks are column-major ``(n, m)`` tensors (``stride(0) == 1``, e.g.
``torch.empty(m, n).t()``) or 1-D vectors.  A non-OK status raises
:class:`MorxError`.  Importing this module fails loudly when the library has
not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmorx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2003_12759_amd.build` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

MORX_OK = 0
STATUS = {
    0: "MORX_OK", -1: "MORX_E_INVALID", -2: "MORX_E_NOMEM", -3: "MORX_E_HIP",
    -4: "MORX_E_SINGULAR_LS", -5: "MORX_E_NOT_CONVERGED", -6: "MORX_E_BREAKDOWN",
    -7: "MORX_E_NONFINITE", -8: "MORX_E_ADMISSION", -9: "MORX_E_UNSUPPORTED",
    -10: "MORX_E_PENDING",
}
PREC = {"f64": 0, "f32": 1, "bf16": 2}
MORX_CHAIN_RESET = 0
MORX_CHAIN_NEXT_ROUND = 1
MORX_CHAIN_DIRECT = 2
MORX_CHAIN_FIRST = 3


class morx_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("precond_prec", ctypes.c_int32),
                ("chain", ctypes.c_int32), ("want_dual", ctypes.c_int32),
                ("batched", ctypes.c_int32), ("poll_iters", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("apply_prec", ctypes.c_int32)]


class morx_col_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("relres_primal", ctypes.c_double), ("relres_dual", ctypes.c_double)]


class morx_trace_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class morx_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("slots_per_system", ctypes.c_int32),
                ("anchors", ctypes.c_int32), ("anchor_min", ctypes.c_double),
                ("anchor_max", ctypes.c_double), ("segment_iters", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class morx_tune(ctypes.Structure):
    _fields_ = [("factor_kernel", ctypes.c_int32), ("cols_per_wave", ctypes.c_int32),
                ("slices_per_wave", ctypes.c_int32), ("spmv_cols_per_wave", ctypes.c_int32),
                ("chain_kernel", ctypes.c_int32), ("halo_stride", ctypes.c_int32),
                ("factor_ms", ctypes.c_double), ("iter_ms", ctypes.c_double)]


class morx_factor_spec(ctypes.Structure):
    _fields_ = [("is_spai", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sigma_prev", ctypes.c_double), ("sigma_new", ctypes.c_double)]


class morx_serve_counts(ctypes.Structure):
    _fields_ = [("admitted", ctypes.c_uint64), ("joined_running", ctypes.c_uint64),
                ("segments", ctypes.c_uint64), ("systems_made", ctypes.c_uint64),
                ("systems_evicted", ctypes.c_uint64), ("resident", ctypes.c_int32),
                ("max_running", ctypes.c_int32)]


class MorxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.morx_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)} ({msg})")


_p = ctypes.c_void_p
_i32, _i64, _d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIG = {
    "morx_opts_default": (None, [ctypes.POINTER(morx_opts)]),
    "morx_status_str": (ctypes.c_char_p, [_i32]),
    "morx_last_error": (ctypes.c_char_p, []),
    "morx_create": (_i32, [ctypes.POINTER(_p), ctypes.c_int]),
    "morx_destroy": (_i32, [_p]),
    "morx_system_create": (_i32, [_p, _i64, _i64, _p, _p, _p, _p, _p, ctypes.POINTER(_p)]),
    "morx_system_destroy": (_i32, [_p]),
    "morx_system_info": (_i32, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "morx_system_pattern": (_i32, [_p, _p, _p, _p]),
    "morx_shifted_apply": (_i32, [_p, _d, _i32, _i32, _p, _i64, _p, _i64, _p]),
    "morx_factor_spai": (_i32, [_p, _d, _i32, _p, ctypes.POINTER(_p)]),
    "morx_factor_update": (_i32, [_p, _d, _d, _i32, _p, ctypes.POINTER(_p)]),
    "morx_factor_values": (_i32, [_p, _p, _p]),
    "morx_factor_destroy": (_i32, [_p]),
    "morx_chain_apply": (_i32, [_p, _i32, ctypes.POINTER(_p), _i32, _i32, _p, _i64, _p, _i64, _p]),
    "morx_chain_apply_batch": (_i32, [_p, _i32, _i32, ctypes.POINTER(_p), ctypes.POINTER(_i32),
                                      _p, _i64, _p, _i64, _p, _i64, _p, _i64, _i32, _p]),
    "morx_shifted_apply_pair": (_i32, [_p, _i32, ctypes.POINTER(_d), _p, _i64, _p, _i64, _p, _i64,
                                       _p, _i64, _p]),
    "morx_factor_build": (_i32, [_p, _i32, ctypes.POINTER(morx_factor_spec), _i32, _p,
                                 ctypes.POINTER(_p)]),
    "morx_factor_import": (_i32, [_p, _p, _i32, _p, ctypes.POINTER(_p)]),
    "morx_last_chains": (_i32, [_p, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                ctypes.POINTER(morx_factor_spec)]),
    "morx_solve_shifts": (_i32, [_p, _i32, ctypes.POINTER(_d), _i32, _p, _i64, _p, _i64, _p, _i64,
                                 _p, _i64, ctypes.POINTER(morx_opts),
                                 ctypes.POINTER(morx_col_stats), _p]),
    "morx_solve_moments": (_i32, [_p, _i32, ctypes.POINTER(_d), _i32, _p, _i64, _p, _i64, _i32,
                                  _p, _i64, _p, _i64, ctypes.POINTER(morx_opts),
                                  ctypes.POINTER(morx_col_stats), _p]),
    "morx_solve_second_order": (_i32, [_p, _d, _d, _i32, ctypes.POINTER(_d), _i32, _p, _i64, _p,
                                       _i64, _i32, _p, _i64, _p, _i64, ctypes.POINTER(morx_opts),
                                       ctypes.POINTER(morx_col_stats), _p]),
    "morx_gmres_shifts": (_i32, [_p, _i32, ctypes.POINTER(_d), _i32, _p, _i64, _p, _i64, _i32,
                                 _p, _i64, _p, _i64, ctypes.POINTER(morx_opts),
                                 ctypes.POINTER(morx_col_stats), _p]),
    "morx_project": (_i32, [_p, _i32, _p, _i64, _p, _i64, _i32, _p, _i64, _i32, _p, _i64,
                            ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                            ctypes.POINTER(_d), _i32, _p]),
    "morx_project_noalloc": (_i32, [_p, _i32, _p, _i64, _p, _i64, _i32, _p, _i64, _i32, _p, _i64,
                                    ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                    ctypes.POINTER(_d), _p]),
    "morx_pencil_eigvals": (_i32, [_i32, ctypes.POINTER(_d), ctypes.POINTER(_d),
                                   ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "morx_irka": (_i32, [_p, _i32, ctypes.POINTER(_d), _p, _p, _i32, _d, ctypes.POINTER(morx_opts),
                         ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                         ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                         ctypes.POINTER(_i32), ctypes.POINTER(_d), ctypes.POINTER(morx_col_stats),
                         _p]),
    "morx_irka_tangential": (_i32, [_p, _i32, ctypes.POINTER(_d), _i32, _p, _i64, _i32, _p, _i64,
                                    ctypes.POINTER(_d), ctypes.POINTER(_d), _i32, _d,
                                    ctypes.POINTER(morx_opts), ctypes.POINTER(_d),
                                    ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                    ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_i32),
                                    ctypes.POINTER(_d), ctypes.POINTER(morx_col_stats), _p]),
    "morx_solve_pairs": (_i32, [_p, _i32, ctypes.POINTER(_d), _p, _i64, _p, _i64, _p, _i64, _p,
                                _i64, ctypes.POINTER(morx_opts), ctypes.POINTER(morx_col_stats),
                                _p]),
    "morx_system_get_tune": (_i32, [_p, ctypes.POINTER(morx_tune)]),
    "morx_chain_kernel_name": (_i32, [_p, _i32, _i32, _i32, ctypes.c_char_p, _i32]),
    "morx_system_set_tune": (_i32, [_p, ctypes.POINTER(morx_tune)]),
    "morx_autotune": (_i32, [_p, _d, _i32, _i32, _i32, ctypes.POINTER(morx_tune), _p]),
    "morx_serve_config_default": (None, [ctypes.POINTER(morx_serve_config)]),
    "morx_serve_start": (_i32, [_p, ctypes.POINTER(morx_serve_config), ctypes.POINTER(morx_opts),
                                ctypes.POINTER(_p)]),
    "morx_serve_submit": (_i32, [_p, _p, _d, _p, _p, ctypes.POINTER(ctypes.c_uint64)]),
    "morx_serve_poll": (_i32, [_p, ctypes.c_uint64, ctypes.POINTER(morx_col_stats),
                               ctypes.POINTER(_d)]),
    "morx_serve_wait": (_i32, [_p, ctypes.c_uint64, ctypes.POINTER(morx_col_stats),
                               ctypes.POINTER(_d)]),
    "morx_serve_info": (_i32, [_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                               ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64)]),
    "morx_serve_stop": (_i32, [_p]),
    "morx_serve_counts_get": (_i32, [_p, ctypes.POINTER(morx_serve_counts)]),
    "morx_serve_footprint": (_i32, [ctypes.POINTER(morx_serve_config), ctypes.POINTER(morx_opts),
                                    _p, ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "morx_serve_chain": (_i32, [_p, ctypes.c_uint64, _i32, ctypes.POINTER(_i32),
                                ctypes.POINTER(morx_factor_spec)]),
    "morx_trace_enable": (_i32, [_p, _i32]),
    "morx_trace_read": (_i32, [_p, ctypes.POINTER(morx_trace_entry), _i32, ctypes.POINTER(_i32)]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols() -> Sequence[str]:
    return tuple(_SIG)


def _check(status: int, where: str):
    if status != MORX_OK:
        raise MorxError(status, where)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous() and t.dim() == 1:
        raise TypeError(f"{name} must be contiguous")
    return t.data_ptr()


def _block(t: torch.Tensor, name: str):
    """(pointer, ld, ncols) of a column-major float64 block or a vector."""
    _dev(t, torch.float64, name)
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise TypeError(f"{name} must be contiguous")
        return t.data_ptr(), t.shape[0], 1
    if t.dim() == 2 and (t.stride(0) == 1 or t.shape[0] == 1):
        return t.data_ptr(), max(t.stride(1), t.shape[0]), t.shape[1]
    raise TypeError(f"{name} must be a column-major (n, m) block (stride(0) == 1)")


def colmajor(m: int, n: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    """An uninitialised column-major (n, m) block."""
    return torch.empty(m, n, device=device, dtype=dtype).t()


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)


def morx_opts_default() -> morx_opts:
    o = morx_opts()
    _lib.morx_opts_default(ctypes.byref(o))
    return o


def morx_status_str(status: int) -> str:
    return _lib.morx_status_str(status).decode()


def morx_last_error() -> str:
    return _lib.morx_last_error().decode(errors="replace")


def morx_create(device: int = 0) -> int:
    h = _p()
    _check(_lib.morx_create(ctypes.byref(h), device), "morx_create")
    return h.value


def morx_destroy(ctx: int) -> None:
    _check(_lib.morx_destroy(ctx), "morx_destroy")


def morx_system_create(ctx: int, rowptr: torch.Tensor, colind: torch.Tensor, val: torch.Tensor,
                       e_diag: torch.Tensor, stream=None) -> int:
    n = rowptr.numel() - 1
    nnz = colind.numel()
    h = _p()
    _check(_lib.morx_system_create(
        ctx, n, nnz, _dev(rowptr, torch.int32, "rowptr"), _dev(colind, torch.int32, "colind"),
        _dev(val, torch.float64, "val"), _dev(e_diag, torch.float64, "e_diag"), _stream(stream),
        ctypes.byref(h)), "morx_system_create")
    return h.value


def morx_system_destroy(sys: int) -> None:
    _check(_lib.morx_system_destroy(sys), "morx_system_destroy")


def morx_system_info(sys: int):
    a, b = _i64(), _i64()
    _check(_lib.morx_system_info(sys, ctypes.byref(a), ctypes.byref(b)), "morx_system_info")
    return a.value, b.value


def _tune_dict(t: morx_tune) -> dict:
    return {"factor_kernel": t.factor_kernel, "cols_per_wave": t.cols_per_wave,
            "slices_per_wave": t.slices_per_wave, "spmv_cols_per_wave": t.spmv_cols_per_wave,
            "chain_kernel": t.chain_kernel, "halo_stride": t.halo_stride,
            "factor_ms": t.factor_ms, "iter_ms": t.iter_ms}


def morx_system_get_tune(sys: int) -> dict:
    t = morx_tune()
    _check(_lib.morx_system_get_tune(sys, ctypes.byref(t)), "morx_system_get_tune")
    return _tune_dict(t)


def morx_chain_kernel_name(sys: int, ncol: int, prec: str = "f64", apply: str = "f64") -> str:
    buf = ctypes.create_string_buffer(128)
    _check(_lib.morx_chain_kernel_name(sys, int(ncol), PREC[prec], PREC[apply], buf, 128),
           "morx_chain_kernel_name")
    return buf.value.decode()


def morx_system_set_tune(sys: int, factor_kernel: int = -1, cols_per_wave: int = -1,
                         slices_per_wave: int = -1, spmv_cols_per_wave: int = -1,
                         chain_kernel: int = -1) -> None:
    t = morx_tune(factor_kernel, cols_per_wave, slices_per_wave, spmv_cols_per_wave,
                  chain_kernel, 0, 0.0, 0.0)
    _check(_lib.morx_system_set_tune(sys, ctypes.byref(t)), "morx_system_set_tune")


def morx_autotune(sys: int, sigma: float, ncols: int, chain_len: int = 1, prec: str = "f64",
                  stream=None) -> dict:
    t = morx_tune()
    _check(_lib.morx_autotune(sys, float(sigma), int(ncols), int(chain_len), PREC[prec],
                              ctypes.byref(t), _stream(stream)), "morx_autotune")
    return _tune_dict(t)


def morx_system_pattern(sys: int, rowptr: torch.Tensor, colind: torch.Tensor, stream=None) -> None:
    _check(_lib.morx_system_pattern(sys, _dev(rowptr, torch.int32, "rowptr"),
                                    _dev(colind, torch.int32, "colind"), _stream(stream)),
           "morx_system_pattern")


def morx_shifted_apply(sys: int, sigma: float, trans: bool, X: torch.Tensor, Y: torch.Tensor,
                       stream=None) -> None:
    px, ldx, nc = _block(X, "X")
    py, ldy, nc2 = _block(Y, "Y")
    if nc != nc2:
        raise ValueError("X and Y column counts differ")
    _check(_lib.morx_shifted_apply(sys, float(sigma), int(bool(trans)), nc, px, ldx, py, ldy,
                                   _stream(stream)), "morx_shifted_apply")


def morx_factor_spai(sys: int, sigma: float, prec: str = "f64", stream=None) -> int:
    h = _p()
    _check(_lib.morx_factor_spai(sys, float(sigma), PREC[prec], _stream(stream), ctypes.byref(h)),
           "morx_factor_spai")
    return h.value


def morx_factor_update(sys: int, sigma_prev: float, sigma_new: float, prec: str = "f64",
                       stream=None) -> int:
    h = _p()
    _check(_lib.morx_factor_update(sys, float(sigma_prev), float(sigma_new), PREC[prec],
                                   _stream(stream), ctypes.byref(h)), "morx_factor_update")
    return h.value


def morx_factor_values(f: int, val: torch.Tensor, stream=None) -> None:
    _check(_lib.morx_factor_values(f, _dev(val, torch.float64, "val"), _stream(stream)),
           "morx_factor_values")


def morx_factor_destroy(f: int) -> None:
    _check(_lib.morx_factor_destroy(f), "morx_factor_destroy")


def morx_chain_apply(sys: int, chain: Sequence[int], trans: bool, X: torch.Tensor, Y: torch.Tensor,
                     stream=None) -> None:
    arr = (_p * len(chain))(*chain)
    px, ldx, nc = _block(X, "X")
    py, ldy, nc2 = _block(Y, "Y")
    if nc != nc2:
        raise ValueError("X and Y column counts differ")
    _check(_lib.morx_chain_apply(sys, len(chain), arr, int(bool(trans)), nc, px, ldx, py, ldy,
                                 _stream(stream)), "morx_chain_apply")


def _spec_tuple(sp: morx_factor_spec):
    """("spai", sigma) or ("update", sigma_prev, sigma_new), the oracle's form."""
    if sp.is_spai:
        return ("spai", sp.sigma_new)
    return ("update", sp.sigma_prev, sp.sigma_new)


def _opt_block(t, name):
    if t is None:
        return None, 1, 0
    return _block(t, name)


def morx_chain_apply_batch(sys: int, chains: Sequence[Sequence[int]], X: Optional[torch.Tensor],
                           Y: Optional[torch.Tensor], Xt: Optional[torch.Tensor] = None,
                           Yt: Optional[torch.Tensor] = None, apply: str = "f64",
                           stream=None) -> None:
    """Column c of X times chain c (chains[c][0] applied first), column c of
    Xt times its transpose, with the solve's chain kernels."""
    ncol = len(chains)
    lcap = max(len(ch) for ch in chains)
    tab = (_p * (ncol * lcap))()
    lens = (_i32 * ncol)()
    for c, ch in enumerate(chains):
        lens[c] = len(ch)
        for k, f in enumerate(ch):
            tab[c * lcap + k] = f
    px, ldx, n1 = _opt_block(X, "X")
    py, ldy, n2 = _opt_block(Y, "Y")
    pxt, ldxt, n3 = _opt_block(Xt, "Xt")
    pyt, ldyt, n4 = _opt_block(Yt, "Yt")
    for nn in (n1, n2, n3, n4):
        if nn not in (0, ncol):
            raise ValueError("column counts differ from the number of chains")
    _check(_lib.morx_chain_apply_batch(sys, ncol, lcap, tab, lens, px, ldx, py, ldy, pxt, ldxt,
                                       pyt, ldyt, PREC[apply], _stream(stream)),
           "morx_chain_apply_batch")


def morx_shifted_apply_pair(sys: int, sigmas: Sequence[float], X: Optional[torch.Tensor],
                            Y: Optional[torch.Tensor], Xt: Optional[torch.Tensor] = None,
                            Yt: Optional[torch.Tensor] = None, stream=None) -> None:
    ncol = len(sigmas)
    sig = (_d * ncol)(*[float(x) for x in sigmas])
    px, ldx, n1 = _opt_block(X, "X")
    py, ldy, n2 = _opt_block(Y, "Y")
    pxt, ldxt, n3 = _opt_block(Xt, "Xt")
    pyt, ldyt, n4 = _opt_block(Yt, "Yt")
    for nn in (n1, n2, n3, n4):
        if nn not in (0, ncol):
            raise ValueError("column counts differ from the number of shifts")
    _check(_lib.morx_shifted_apply_pair(sys, ncol, sig, px, ldx, py, ldy, pxt, ldxt, pyt, ldyt,
                                        _stream(stream)), "morx_shifted_apply_pair")


def morx_factor_build(sys: int, specs, prec: str = "f64", stream=None):
    """Factors of the given specs (("spai", s) or ("update", s_prev, s_new))
    built in one launch; returns their handles."""
    nj = len(specs)
    arr = (morx_factor_spec * nj)()
    for j, sp in enumerate(specs):
        if sp[0] == "spai":
            arr[j] = morx_factor_spec(1, 0, 0.0, float(sp[1]))
        else:
            arr[j] = morx_factor_spec(0, 0, float(sp[1]), float(sp[2]))
    out = (_p * nj)()
    _check(_lib.morx_factor_build(sys, nj, arr, PREC[prec], _stream(stream), out),
           "morx_factor_build")
    return [out[j] for j in range(nj)]


def morx_factor_import(sys: int, val: torch.Tensor, prec: str = "f64", stream=None) -> int:
    h = _p()
    _check(_lib.morx_factor_import(sys, _dev(val, torch.float64, "val"), PREC[prec],
                                   _stream(stream), ctypes.byref(h)), "morx_factor_import")
    return h.value


def morx_last_chains(sys: int, cap_shifts: int = 1024, ldspec: int = 64):
    """Per shift of the last solve call, its chain as a list of spec tuples."""
    ns = _i32()
    lens = (_i32 * cap_shifts)()
    specs = (morx_factor_spec * (cap_shifts * ldspec))()
    _check(_lib.morx_last_chains(sys, cap_shifts, ldspec, ctypes.byref(ns), lens, specs),
           "morx_last_chains")
    return [[_spec_tuple(specs[i * ldspec + k]) for k in range(min(lens[i], ldspec))]
            for i in range(min(ns.value, cap_shifts))]


def morx_solve_shifts(sys: int, sigmas: Sequence[float], B: torch.Tensor, C: Optional[torch.Tensor],
                      X: torch.Tensor, Y: Optional[torch.Tensor], opts: Optional[morx_opts] = None,
                      stream=None, raise_on_error: bool = True):
    """Returns (status, list of morx_col_stats)."""
    if opts is None:
        opts = morx_opts_default()
    pb, ldb, m = _block(B, "B")
    px, ldx, mx = _block(X, "X")
    if C is not None:
        pc, ldc, mc = _block(C, "C")
        py, ldy, _ = _block(Y, "Y")
    else:
        pc, ldc, py, ldy = None, B.shape[0], None, B.shape[0]
    ns = len(sigmas)
    sig = (_d * ns)(*[float(s) for s in sigmas])
    stats = (morx_col_stats * (ns * m))()
    st = _lib.morx_solve_shifts(sys, ns, sig, m, pb, ldb, pc, ldc, px, ldx, py, ldy,
                                ctypes.byref(opts), stats, _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_solve_shifts")
    return st, list(stats)


def morx_solve_moments(sys: int, sigmas: Sequence[float], B: torch.Tensor,
                       C: Optional[torch.Tensor], nmom: int, X: torch.Tensor,
                       Y: Optional[torch.Tensor], opts: Optional[morx_opts] = None, stream=None,
                       raise_on_error: bool = True):
    """Returns (status, list of morx_col_stats); X, Y hold nmom * len(sigmas) * m columns."""
    if opts is None:
        opts = morx_opts_default()
    pb, ldb, m = _block(B, "B")
    px, ldx, _ = _block(X, "X")
    if C is not None:
        pc, ldc, _ = _block(C, "C")
        py, ldy, _ = _block(Y, "Y")
    else:
        pc, ldc, py, ldy = None, B.shape[0], None, B.shape[0]
    ns = len(sigmas)
    sig = (_d * ns)(*[float(s) for s in sigmas])
    stats = (morx_col_stats * (nmom * ns * m))()
    st = _lib.morx_solve_moments(sys, ns, sig, m, pb, ldb, pc, ldc, int(nmom), px, ldx, py, ldy,
                                 ctypes.byref(opts), stats, _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_solve_moments")
    return st, list(stats)


def morx_solve_second_order(sys: int, alpha: float, beta: float, points: Sequence[float],
                            F: torch.Tensor, C: Optional[torch.Tensor], nmom: int,
                            X: torch.Tensor, Y: Optional[torch.Tensor],
                            opts: Optional[morx_opts] = None, stream=None,
                            raise_on_error: bool = True):
    """Returns (status, list of morx_col_stats); X, Y hold nmom * len(points) * m columns."""
    if opts is None:
        opts = morx_opts_default()
    pf, ldf, m = _block(F, "F")
    px, ldx, _ = _block(X, "X")
    if C is not None:
        pc, ldc, _ = _block(C, "C")
        py, ldy, _ = _block(Y, "Y")
    else:
        pc, ldc, py, ldy = None, F.shape[0], None, F.shape[0]
    npt = len(points)
    pts = (_d * npt)(*[float(s) for s in points])
    stats = (morx_col_stats * (nmom * npt * m))()
    st = _lib.morx_solve_second_order(sys, float(alpha), float(beta), npt, pts, m, pf, ldf, pc,
                                      ldc, int(nmom), px, ldx, py, ldy, ctypes.byref(opts), stats,
                                      _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_solve_second_order")
    return st, list(stats)


def morx_gmres_shifts(sys: int, sigmas: Sequence[float], B: torch.Tensor,
                      C: Optional[torch.Tensor], restart: int, X: torch.Tensor,
                      Y: Optional[torch.Tensor], opts: Optional[morx_opts] = None, stream=None,
                      raise_on_error: bool = True):
    """Returns (status, list of morx_col_stats)."""
    if opts is None:
        opts = morx_opts_default()
    pb, ldb, m = _block(B, "B")
    px, ldx, _ = _block(X, "X")
    if C is not None:
        pc, ldc, _ = _block(C, "C")
        py, ldy, _ = _block(Y, "Y")
    else:
        pc, ldc, py, ldy = None, B.shape[0], None, B.shape[0]
    ns = len(sigmas)
    sig = (_d * ns)(*[float(s) for s in sigmas])
    stats = (morx_col_stats * (ns * m))()
    st = _lib.morx_gmres_shifts(sys, ns, sig, m, pb, ldb, pc, ldc, int(restart), px, ldx, py, ldy,
                                ctypes.byref(opts), stats, _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_gmres_shifts")
    return st, list(stats)


def morx_project(sys: int, V: torch.Tensor, W: torch.Tensor, B: Optional[torch.Tensor],
                 C: Optional[torch.Tensor], orthonormalize: bool = True, stream=None):
    """Returns numpy arrays (Ar, Er, Br, Cr) (column-major data, shapes r x r, r x m, r x q)."""
    import numpy as np

    pv, ldv, r = _block(V, "V")
    pw, ldw, r2 = _block(W, "W")
    if r != r2:
        raise ValueError("V and W column counts differ")
    pb, ldb, m = _block(B, "B") if B is not None else (None, V.shape[0], 0)
    pc, ldc, q = _block(C, "C") if C is not None else (None, V.shape[0], 0)
    Ar = (_d * (r * r))()
    Er = (_d * (r * r))()
    Br = (_d * max(r * m, 1))()
    Cr = (_d * max(r * q, 1))()
    _check(_lib.morx_project(sys, r, pv, ldv, pw, ldw, m, pb, ldb, q, pc, ldc, Ar, Er, Br, Cr,
                             int(bool(orthonormalize)), _stream(stream)), "morx_project")

    def mat(buf, rows, cols):
        return np.frombuffer(buf, dtype=np.float64, count=rows * cols).reshape(cols, rows).T.copy()

    return mat(Ar, r, r), mat(Er, r, r), mat(Br, r, m), mat(Cr, r, q)


def morx_project_noalloc(sys: int, V: torch.Tensor, W: torch.Tensor, B: Optional[torch.Tensor],
                         C: Optional[torch.Tensor], stream=None):
    """morx_project of V and W as given, through the allocation-free entry
    point; returns numpy (Ar, Er, Br, Cr)."""
    import numpy as np

    pv, ldv, r = _block(V, "V")
    pw, ldw, r2 = _block(W, "W")
    if r != r2:
        raise ValueError("V and W column counts differ")
    pb, ldb, m = _block(B, "B") if B is not None else (None, V.shape[0], 0)
    pc, ldc, q = _block(C, "C") if C is not None else (None, V.shape[0], 0)
    Ar = (_d * (r * r))()
    Er = (_d * (r * r))()
    Br = (_d * max(r * m, 1))()
    Cr = (_d * max(r * q, 1))()
    _check(_lib.morx_project_noalloc(sys, r, pv, ldv, pw, ldw, m, pb, ldb, q, pc, ldc, Ar, Er, Br,
                                     Cr, _stream(stream)), "morx_project_noalloc")

    def mat(buf, rows, cols):
        return np.frombuffer(buf, dtype=np.float64, count=rows * cols).reshape(cols, rows).T.copy()

    return mat(Ar, r, r), mat(Er, r, r), mat(Br, r, m), mat(Cr, r, q)


def morx_pencil_eigvals(Ar, Er):
    """Eigenvalues of the pencil (Ar, Er) (numpy r x r arrays): (wr, wi),
    ascending by real part."""
    import numpy as np

    Ar = np.asarray(Ar, dtype=np.float64)
    Er = np.asarray(Er, dtype=np.float64)
    r = Ar.shape[0]
    a = (_d * (r * r))(*Ar.T.ravel().tolist())
    e = (_d * (r * r))(*Er.T.ravel().tolist())
    wr = (_d * r)()
    wi = (_d * r)()
    _check(_lib.morx_pencil_eigvals(r, a, e, wr, wi), "morx_pencil_eigvals")
    return np.array(wr[:]), np.array(wi[:])


def morx_irka(sys: int, sigmas: Sequence[float], b: torch.Tensor, c: torch.Tensor,
              max_rounds: int = 20, tol: float = 1e-6, opts: Optional[morx_opts] = None,
              stream=None, raise_on_error: bool = True):
    """Returns (status, dict): sigmas, Ar, Er, Br, Cr, poles (complex), rounds,
    change, stats (the last round's)."""
    import numpy as np

    if opts is None:
        opts = morx_opts_default()
    r = len(sigmas)
    if b.dim() != 1 or c.dim() != 1 or not b.is_contiguous() or not c.is_contiguous():
        raise ValueError("b and c must be contiguous device vectors")
    sig = (_d * r)(*[float(x) for x in sigmas])
    Ar = (_d * (r * r))()
    Er = (_d * (r * r))()
    Br = (_d * r)()
    Cr = (_d * r)()
    pr = (_d * r)()
    pi = (_d * r)()
    rounds = _i32(0)
    change = _d(0.0)
    stats = (morx_col_stats * r)()
    st = _lib.morx_irka(sys, r, sig, b.data_ptr(), c.data_ptr(), int(max_rounds), float(tol),
                        ctypes.byref(opts), Ar, Er, Br, Cr, pr, pi, ctypes.byref(rounds),
                        ctypes.byref(change), stats, _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_irka")

    def mat(buf, rows, cols):
        return np.frombuffer(buf, dtype=np.float64, count=rows * cols).reshape(cols, rows).T.copy()

    return st, {"sigmas": np.array(sig[:]), "Ar": mat(Ar, r, r), "Er": mat(Er, r, r),
                "Br": np.array(Br[:]).reshape(r, 1), "Cr": np.array(Cr[:]).reshape(r, 1),
                "poles": np.array(pr[:]) + 1j * np.array(pi[:]), "rounds": rounds.value,
                "change": change.value, "stats": list(stats)}


def morx_solve_pairs(sys: int, sigmas: Sequence[float], B: torch.Tensor,
                     C: Optional[torch.Tensor], X: torch.Tensor, Y: Optional[torch.Tensor],
                     opts: Optional[morx_opts] = None, stream=None, raise_on_error: bool = True):
    """Column i of B and C belongs to shift i; returns (status, list of morx_col_stats)."""
    if opts is None:
        opts = morx_opts_default()
    pb, ldb, _ = _block(B, "B")
    px, ldx, _ = _block(X, "X")
    if C is not None:
        pc, ldc, _ = _block(C, "C")
        py, ldy, _ = _block(Y, "Y")
    else:
        pc, ldc, py, ldy = None, B.shape[0], None, B.shape[0]
    ns = len(sigmas)
    sig = (_d * ns)(*[float(s) for s in sigmas])
    stats = (morx_col_stats * ns)()
    st = _lib.morx_solve_pairs(sys, ns, sig, pb, ldb, pc, ldc, px, ldx, py, ldy,
                               ctypes.byref(opts), stats, _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_solve_pairs")
    return st, list(stats)


def morx_irka_tangential(sys: int, sigmas: Sequence[float], B: torch.Tensor, C: torch.Tensor,
                         bdir, cdir, max_rounds: int = 20, tol: float = 1e-6,
                         opts: Optional[morx_opts] = None, stream=None,
                         raise_on_error: bool = True):
    """bdir (m x r) and cdir (q x r): column i the directions of shift i.
    Returns (status, dict): sigmas, bdir, cdir, Ar, Er, Br (r x m), Cr (r x q),
    poles (complex), rounds, change, stats (the last round's)."""
    import numpy as np

    if opts is None:
        opts = morx_opts_default()
    r = len(sigmas)
    pb, ldb, m = _block(B, "B")
    pc, ldc, q = _block(C, "C")
    bd = np.asfortranarray(np.asarray(bdir, dtype=np.float64).reshape(m, r))
    cd = np.asfortranarray(np.asarray(cdir, dtype=np.float64).reshape(q, r))
    sig = (_d * r)(*[float(x) for x in sigmas])
    bb = (_d * (m * r))(*bd.ravel(order="F"))
    cb = (_d * (q * r))(*cd.ravel(order="F"))
    Ar = (_d * (r * r))()
    Er = (_d * (r * r))()
    Br = (_d * (r * m))()
    Cr = (_d * (r * q))()
    pr = (_d * r)()
    pi = (_d * r)()
    rounds = _i32(0)
    change = _d(0.0)
    stats = (morx_col_stats * r)()
    st = _lib.morx_irka_tangential(sys, r, sig, m, pb, ldb, q, pc, ldc, bb, cb, int(max_rounds),
                                   float(tol), ctypes.byref(opts), Ar, Er, Br, Cr, pr, pi,
                                   ctypes.byref(rounds), ctypes.byref(change), stats,
                                   _stream(stream))
    if raise_on_error and st != MORX_OK:
        raise MorxError(st, "morx_irka_tangential")

    def mat(buf, rows, cols):
        return np.frombuffer(buf, dtype=np.float64, count=rows * cols).reshape(cols, rows).T.copy()

    return st, {"sigmas": np.array(sig[:]), "bdir": mat(bb, m, r), "cdir": mat(cb, q, r),
                "Ar": mat(Ar, r, r), "Er": mat(Er, r, r), "Br": mat(Br, r, m),
                "Cr": mat(Cr, r, q), "poles": np.array(pr[:]) + 1j * np.array(pi[:]),
                "rounds": rounds.value, "change": change.value, "stats": list(stats)}


def morx_trace_enable(ctx: int, enable: bool) -> None:
    _check(_lib.morx_trace_enable(ctx, int(bool(enable))), "morx_trace_enable")


def morx_trace_read(ctx: int):
    """{class name: (launches, total_ms, alg_bytes)}."""
    buf = (morx_trace_entry * 16)()
    cnt = _i32()
    _check(_lib.morx_trace_read(ctx, buf, 16, ctypes.byref(cnt)), "morx_trace_read")
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].alg_bytes)
            for i in range(min(cnt.value, 16))}


# ---------------------------------------------------------------------------
# serving


def morx_serve_config_default() -> morx_serve_config:
    c = morx_serve_config()
    _lib.morx_serve_config_default(ctypes.byref(c))
    return c


def morx_serve_start(ctx: int, cfg: Optional[morx_serve_config] = None,
                     opts: Optional[morx_opts] = None) -> int:
    cfg = cfg or morx_serve_config_default()
    opts = opts or morx_opts_default()
    h = _p()
    _check(_lib.morx_serve_start(ctx, ctypes.byref(cfg), ctypes.byref(opts), ctypes.byref(h)),
           "morx_serve_start")
    return h.value


def morx_serve_submit(srv: int, sys: int, sigma: float, b: torch.Tensor, x: torch.Tensor) -> int:
    t = ctypes.c_uint64()
    _check(_lib.morx_serve_submit(srv, sys, float(sigma), _dev(b, torch.float64, "b"),
                                  _dev(x, torch.float64, "x"), ctypes.byref(t)),
           "morx_serve_submit")
    return t.value


def _serve_take(fn, srv, ticket):
    st = morx_col_stats()
    lat = _d()
    status = fn(srv, ticket, ctypes.byref(st), ctypes.byref(lat))
    return status, st, lat.value


def morx_serve_poll(srv: int, ticket: int):
    """(status, morx_col_stats, latency_s); status -10 (pending) while running."""
    return _serve_take(_lib.morx_serve_poll, srv, ticket)


def morx_serve_wait(srv: int, ticket: int):
    return _serve_take(_lib.morx_serve_wait, srv, ticket)


def morx_serve_info(srv: int):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    c, d = _i32(), _i32()
    e = _i64()
    _check(_lib.morx_serve_info(srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                ctypes.byref(d), ctypes.byref(e)), "morx_serve_info")
    return {"submitted": a.value, "completed": b.value, "running": c.value, "queued": d.value,
            "bytes_in_use": e.value}


def morx_serve_footprint(sys: int, cfg: Optional[morx_serve_config] = None,
                         opts: Optional[morx_opts] = None):
    """(system_bytes, request_bytes) a server counts for sys."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.morx_serve_footprint(ctypes.byref(cfg) if cfg is not None else None,
                                     ctypes.byref(opts) if opts is not None else None, sys,
                                     ctypes.byref(a), ctypes.byref(b)), "morx_serve_footprint")
    return a.value, b.value


def morx_serve_counts_get(srv: int) -> dict:
    c = morx_serve_counts()
    _check(_lib.morx_serve_counts_get(srv, ctypes.byref(c)), "morx_serve_counts_get")
    return {name: getattr(c, name) for name, _ in c._fields_}


def morx_serve_chain(srv: int, ticket: int, cap: int = 64):
    """The request's chain as spec tuples, or None while it waits for admission."""
    n = _i32()
    specs = (morx_factor_spec * cap)()
    st = _lib.morx_serve_chain(srv, ticket, cap, ctypes.byref(n), specs)
    if st == -10:
        return None
    _check(st, "morx_serve_chain")
    return [_spec_tuple(specs[k]) for k in range(min(n.value, cap))]


def morx_serve_stop(srv: int) -> None:
    _check(_lib.morx_serve_stop(srv), "morx_serve_stop")
