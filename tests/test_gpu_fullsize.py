"""Full-size checks of the benchmark job (64^3 convection-diffusion, n = 262,144),
in the launch configurations bench.py times (batched, FP32 factors, 3 rounds,
preconditioner applied in FP64 and in FP32; launch shapes built in, and
autotuned on the system as bench.py does, which takes the halo chain kernel
where it is faster).

At this size the oracle cannot solve every system, so the checks are:
* sampled factor columns against the oracle's column least squares;
* properties that hold at any size: every true relative residual, recomputed
  here in FP64 on the CPU, is <= 1e-10 (primal and dual); the two-way transfer
  identity c^T x = y^T b; the reduced model interpolates the transfer function
  values c^T x at every shift.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import pattern as opattern
from oracle import projection as oproj
from oracle import spai as ospai
from oracle.precision import round_storage
from paper_2003_12759_amd.workloads import make_workload

from host_residual import residual_ok  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2003_12759_amd import api

    w = make_workload(1)
    ctx = api.Context(0)
    S = api.System(ctx, w.A, w.e)
    yield w, ctx, S
    S.close()
    ctx.close()


@pytest.mark.parametrize("launch", ["built-in", "autotuned"])
@pytest.mark.parametrize("apply", ["f64", "f32"])
def test_bench_job_fullsize_residuals_and_interpolation(setup, apply, launch):
    from paper_2003_12759_amd import api

    w, ctx, S = setup
    if launch == "autotuned":
        S.autotune(float(w.rounds[0][0]), ncols=len(w.rounds[0]) * w.B.shape[1],
                   chain_len=len(w.rounds[0]) + len(w.rounds) - 1, prec=w.prec)
    else:
        S.set_tune()
    Bd, Cd = api.block_to_dev(w.B), api.block_to_dev(w.C)
    E = sp.diags(w.e)
    for z, sig in enumerate(w.rounds):
        print(f"[case] full-size round {z} apply={apply} launch={launch} tune={S.get_tune()}",
              flush=True)
        X, Y, st, stats = S.solve_shifts(sig, Bd, Cd, prec="f32", next_round=z > 0, apply=apply)
        Ar, Er, Br, Cr = S.project(X, Y, Bd, Cd)
        Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
        for i, s in enumerate(sig):
            assert stats[i].status == 0
            M = (s * E - w.A).tocsr()
            assert residual_ok(M, Xg[:, i], w.B[:, 0]), (z, i)
            assert residual_ok(M.T, Yg[:, i], w.C[:, 0]), (z, i)
            h1 = w.C[:, 0] @ Xg[:, i]
            h2 = Yg[:, i] @ w.B[:, 0]
            assert abs(h1 - h2) <= 1e-7 * abs(h1)
            hr = oproj.transfer(Ar, Er, Br, Cr, s)[0, 0]
            assert abs(hr - h1) <= 1e-7 * abs(h1)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_factor_columns_sampled_fullsize(setup, prec):
    from paper_2003_12759_amd import morx

    w, ctx, S = setup
    rp, ci = S.pattern()
    cols = np.random.default_rng(7).choice(w.n, 300, replace=False)
    s0, s1 = float(w.rounds[0][0]), float(w.rounds[0][1])
    for kind in ("spai", "update"):
        print(f"[case] full-size {kind} {prec}", flush=True)
        if kind == "spai":
            f = morx.morx_factor_spai(S.handle, s0, prec)
        else:
            f = morx.morx_factor_update(S.handle, s0, s1, prec)
        vals = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
        morx.morx_factor_values(f, vals)
        F = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=(w.n, w.n)).tocsc()
        As0 = opattern.shifted_pattern_values(w.A, w.e, s0)
        As1 = opattern.shifted_pattern_values(w.A, w.e, s1)
        for k in cols:
            if kind == "spai":
                J, q = ospai.spai_column(w.A, w.e, s0, int(k), As=As0)
            else:
                J, q = ospai.update_column(w.A, w.e, s0, s1, int(k), As_new=As1, As_prev=As0)
            got = F[:, int(k)].toarray().ravel()[J]
            if prec == "f64":
                assert np.linalg.norm(got - q) <= 1e-11 * np.linalg.norm(q)
            else:
                want = round_storage(q, prec)
                assert np.all(np.abs(got - want) <= np.abs(want) * 2.0**-23)
        morx.morx_factor_destroy(f)
