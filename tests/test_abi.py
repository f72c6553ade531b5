"""The C-ABI library loads and exports every entry point include/morx.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "morx.h")
LIB = os.path.join(ROOT, "paper_2003_12759_amd", "_lib", "libmorx.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(morx_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("morx_create", "morx_system_create", "morx_factor_spai", "morx_factor_update",
                 "morx_chain_apply", "morx_shifted_apply", "morx_solve_shifts", "morx_project"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run python -m paper_2003_12759_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_2003_12759_amd import morx

    assert set(declared_functions()) <= set(morx.exported_symbols())


def test_status_strings_and_defaults_without_gpu():
    from paper_2003_12759_amd import morx

    o = morx.morx_opts_default()
    assert o.tol == 1e-10 and o.max_restarts == 3 and o.want_dual == 1 and o.batched == 1
    assert morx.morx_status_str(0) == "ok"
    assert "converged" in morx.morx_status_str(-5)
