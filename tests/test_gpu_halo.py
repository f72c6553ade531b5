"""The chain step on the halo layout against the gather kernel and exact
solves, through the C ABI.

Patterns with rows of at most 32 entries get, per block of 256 rows, the list
of distinct columns the block touches (when it has at most 2048, 1024 for
rows of at most 8 entries); the halo kernel copies the input vectors at those
columns into LDS and sums each row from there.  Both kernels sum a row's
slots in the same order, so the chain outputs agree; the BiCG runs differ
only through the grouping of the rho partial sums.  Tolerances as in the other solve tests: true relative residual
<= 1e-10 (recomputed here in FP64), ||x - x_ref|| <= ||A_s^{-1}|| (||r|| +
||r_ref||) against a sparse direct solve with ||A_s^{-1}|| = 1 / sigma_min
from a dense SVD, and iteration counts of the two kernels within
max(3, 5 %) (FP64 apply) or 20 % (FP32 apply) of each other.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from paper_2003_12759_amd.workloads import make_workload

from host_residual import residual_ok  # noqa: E402

pytestmark = pytest.mark.gpu

MORX_E_INVALID = -1
MORX_E_UNSUPPORTED = -9


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _wide_random(n, per_row, seed):
    """Nonsymmetric, diagonally dominant, about per_row random entries a row."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=per_row / n, random_state=rng, format="csr")
    M.data = 0.3 * rng.standard_normal(M.nnz)
    M = (M + sp.diags(-6.0 - rng.uniform(0, 1, n))).tocsr()
    M.sort_indices()
    return M, np.random.default_rng(seed + 1).uniform(1, 2, n)


def _varcoef27(N):
    w = make_workload(4, N=N)
    return w.A, w.e


def _convdiff(N):
    w = make_workload(1, N=N)
    return w.A, w.e


def _dense(n, seed, per_row=None):
    """Diagonally dominant; every entry stored (per_row None) or about
    per_row random entries a row."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) * 0.2
    if per_row is not None:
        M *= rng.random((n, n)) < per_row / n
    M -= np.diag(1.0 + np.abs(M).sum(axis=1))
    return sp.csr_matrix(M), rng.uniform(1, 2, n)


# 27-point on 11^3 = 1331 rows: 21 slices, so the last block of four slices
# has one; the random pattern has no stencil structure and rows of ~11
# entries; the 7-point operator takes the halo kernel for rows of at most 8;
# the small dense systems have one slice (three waves of the block without
# rows), rows of 9 and of 31 entries, and a partial slice of 70 rows with
# ~20 entries a row
CASES = {
    "varcoef27_n1331": lambda: _varcoef27(11),
    "random_wide_n1300": lambda: _wide_random(1300, 10, 7),
    "convdiff_n1331": lambda: _convdiff(11),
    "dense_n9": lambda: _dense(9, 1),
    "dense_n31": lambda: _dense(31, 2),
    "random_n70": lambda: _dense(70, 3, per_row=20),
}


def _relres(M, x, b):
    return np.linalg.norm(b - M @ x) / np.linalg.norm(b)


@pytest.mark.parametrize("prec,apply,policy", [("bf16", "f64", "reuse"), ("f64", "f64", "first"),
                                               ("f32", "f32", "reuse")])
@pytest.mark.parametrize("name", list(CASES))
def test_halo_kernel_against_gather_kernel_and_direct_solves(ctx, name, prec, apply, policy):
    """policy "first" gives chunks whose pairs apply different factors."""
    from paper_2003_12759_amd import api

    A, e = CASES[name]()
    n = A.shape[0]
    rng = np.random.default_rng(11)
    B = rng.standard_normal((n, 1))
    C = rng.standard_normal((n, 1))
    sig = list(np.logspace(0, 3, 6))
    S = api.System(ctx, A, e)
    runs = {}
    for k in (1, 0):
        S.set_tune(chain_kernel=k)
        assert S.get_tune()["chain_kernel"] == k
        _say(f"{name} chain_kernel={k} prec={prec} apply={apply} policy={policy}")
        X, Y, st, stats = S.solve_shifts(sig, B, C, prec=prec, apply=apply, policy=policy)
        runs[k] = (X.cpu().numpy(), Y.cpu().numpy(), stats)
    S.close()
    allow = 0.2 if apply == "f32" else 0.05
    for i, s in enumerate(sig):
        M = (s * sp.diags(e) - A).tocsc()
        xr = spla.spsolve(M, B[:, 0])
        yr = spla.spsolve(M.T.tocsc(), C[:, 0])
        smin = np.linalg.svd(M.toarray(), compute_uv=False)[-1]
        for k in (1, 0):
            Xg, Yg, stats = runs[k]
            assert stats[i].status == 0
            rp = _relres(M, Xg[:, i], B[:, 0])
            rd = _relres(M.T, Yg[:, i], C[:, 0])
            assert residual_ok(M, Xg[:, i], B[:, 0]) and residual_ok(M.T, Yg[:, i], C[:, 0]), (k, i)
            rpr = _relres(M, xr, B[:, 0])
            rdr = _relres(M.T, yr, C[:, 0])
            assert np.linalg.norm(Xg[:, i] - xr) <= (rp + rpr) * np.linalg.norm(B) / smin * 1.01
            assert np.linalg.norm(Yg[:, i] - yr) <= (rd + rdr) * np.linalg.norm(C) / smin * 1.01
        ih, ig = runs[1][2][i].iters, runs[0][2][i].iters
        assert abs(ih - ig) <= max(3, allow * ig), (i, ih, ig)


def test_halo_layout_absent_on_scattered_pattern(ctx):
    """Random rows over 20,000 columns: a block of 256 rows touches about
    2,400 distinct columns, over the cap, so the system keeps no halo layout,
    rejects chain_kernel 1 and solves with the gather kernel."""
    from paper_2003_12759_amd import api, morx

    A, e = _wide_random(20000, 9, 3)
    S = api.System(ctx, A, e)
    assert S.get_tune()["chain_kernel"] == 0
    with pytest.raises(morx.MorxError) as ei:
        S.set_tune(chain_kernel=1)
    assert ei.value.status == MORX_E_UNSUPPORTED
    rng = np.random.default_rng(5)
    B = rng.standard_normal((A.shape[0], 1))
    _say("scattered n=20000, gather kernel")
    X, Y, st, stats = S.solve_shifts([1.0, 10.0], B, B, prec="f32")
    Xg = X.cpu().numpy()
    for i, s in enumerate([1.0, 10.0]):
        assert stats[i].status == 0
        assert residual_ok(s * sp.diags(e) - A, Xg[:, i], B[:, 0])
    S.close()


def test_chain_kernel_tune_values(ctx):
    from paper_2003_12759_amd import api, morx

    # a 7-point pattern has a halo layout, used on request only
    w = make_workload(1, N=8, nshift=2)
    S = api.System(ctx, w.A, w.e)
    assert S.get_tune()["chain_kernel"] == 0
    S.set_tune(chain_kernel=1)
    assert S.get_tune()["chain_kernel"] == 1
    S.close()
    # a 27-point pattern has one, used by default
    A, e = _varcoef27(6)
    S = api.System(ctx, A, e)
    assert S.get_tune()["chain_kernel"] == 1
    for bad in (2, -2):
        with pytest.raises(morx.MorxError) as ei:
            S.set_tune(chain_kernel=bad)
        assert ei.value.status == MORX_E_INVALID
    S.set_tune(chain_kernel=0)
    assert S.get_tune()["chain_kernel"] == 0
    S.set_tune(chain_kernel=-1)
    assert S.get_tune()["chain_kernel"] == 1
    S.close()


@pytest.mark.parametrize("name", ["varcoef7_n1000_mimo", "varcoef27_n729_mimo"])
def test_halo_kernels_widest_tiles(ctx, name):
    """32 columns (8 shifts x 4 inputs) with the chain tile pinned at 16 and the
    shifted pair's at 8: the widest instances of both halo kernels (8-slot
    forms for the 7-point operator, 32-slot forms for the 27-point one)
    against the gather kernels (both solutions within their residuals of the
    exact one), and every pair's true residuals."""
    from paper_2003_12759_amd import api

    if name.startswith("varcoef7"):
        w = make_workload(2, N=10, nshift=8)
        A, e, B, C, sig = w.A, w.e, w.B, w.C, w.rounds[0]
    else:
        A, e = _varcoef27(9)
        rng = np.random.default_rng(21)
        B = rng.standard_normal((A.shape[0], 4))
        C = rng.standard_normal((A.shape[0], 4))
        sig = list(np.logspace(0, 3, 8))
    m = B.shape[1]
    S = api.System(ctx, A, e)
    runs = {}
    for k in (1, 0):
        S.set_tune(cols_per_wave=16, spmv_cols_per_wave=8, chain_kernel=k)
        _say(f"{name} tile 16/8 chain_kernel={k}")
        X, Y, st, stats = S.solve_shifts(sig, B, C, prec="f64")
        runs[k] = (X.cpu().numpy(), Y.cpu().numpy(), stats)
    S.close()
    for i, s in enumerate(sig):
        M = (s * sp.diags(e) - A).tocsr()
        smin = np.abs(np.linalg.eigvalsh(M.toarray())).min()  # both operators are symmetric
        for j in range(m):
            c = i * m + j
            res = {}
            for k in (1, 0):
                Xg, Yg, stats = runs[k]
                assert stats[c].status == 0
                res[k] = _relres(M, Xg[:, c], B[:, j])
                assert residual_ok(M, Xg[:, c], B[:, j])
                assert residual_ok(M.T, Yg[:, c], C[:, j])
            # both within their residual of the exact solution
            xh, xg = runs[1][0][:, c], runs[0][0][:, c]
            bound = (res[1] + res[0]) * np.linalg.norm(B[:, j]) / smin * 1.01
            assert np.linalg.norm(xh - xg) <= bound, (i, j)
