"""Full-size checks of the two large workloads, in the launch configuration
bench.py times for them (shapes autotuned on the system, which takes the halo
chain kernel and shifted pair for these patterns):

* 128^3 27-point variable-coefficient operator (n = 2,097,152), 12 shifts,
  BF16 factor storage applied with FP64 vectors;
* 106^3 7-point variable-coefficient operator (n = 1,191,016), four inputs
  and outputs, 8 shifts, FP64 factors, batched.

The oracle cannot solve these systems, so the checks are properties that hold
at any size: every true relative residual, recomputed here in FP64 on the
CPU, is <= 1e-10 (primal and dual); the two-way transfer identity
c_j^T x_ij = y_ij^T b_j to 1e-7; and, for the 27-point operator, sampled
SPAI and update columns against the oracle's column least squares, to one
BF16 storage step.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import pattern as opattern
from oracle import spai as ospai
from oracle.precision import round_storage
from paper_2003_12759_amd.workloads import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _check_solves(w, sig, X, Y, stats):
    m = w.B.shape[1]
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    A = w.A.tocsr()
    AT = A.T  # a CSC view, no copy
    for i, s in enumerate(sig):
        for j in range(m):
            k = i * m + j
            assert stats[k].status == 0
            x, y = Xg[:, k], Yg[:, k]
            # (s E - A) x and (s E - A)^T y without forming the shifted matrix
            rp = np.linalg.norm(w.B[:, j] - (s * w.e * x - A @ x)) / np.linalg.norm(w.B[:, j])
            rd = np.linalg.norm(w.C[:, j] - (s * w.e * y - AT @ y)) / np.linalg.norm(w.C[:, j])
            assert rp <= 1.01e-10 and rd <= 1.01e-10, (i, j, rp, rd)
            h1 = w.C[:, j] @ x
            h2 = y @ w.B[:, j]
            assert abs(h1 - h2) <= 1e-7 * abs(h1)


def test_varcoef27_fullsize_autotuned_bf16(ctx):
    from paper_2003_12759_amd import api, morx

    w = make_workload(4)
    S = api.System(ctx, w.A, w.e)
    sig = w.rounds[0]
    _say(f"27-point n={w.n} autotune")
    t = S.autotune(float(sig[0]), ncols=len(sig) * w.B.shape[1], chain_len=len(sig), prec="bf16")
    _say(f"27-point solve, tune {t}")
    X, Y, st, stats = S.solve_shifts(sig, w.B, w.C, prec="bf16")
    _check_solves(w, sig, X, Y, stats)
    # sampled factor columns at the first two shifts
    rp, ci = S.pattern()
    cols = np.random.default_rng(7).choice(w.n, 200, replace=False)
    s0, s1 = float(sig[0]), float(sig[1])
    As0 = opattern.shifted_pattern_values(w.A, w.e, s0)
    As1 = opattern.shifted_pattern_values(w.A, w.e, s1)
    for kind in ("spai", "update"):
        _say(f"27-point sampled {kind} columns")
        f = (morx.morx_factor_spai(S.handle, s0, "bf16") if kind == "spai"
             else morx.morx_factor_update(S.handle, s0, s1, "bf16"))
        vals = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
        morx.morx_factor_values(f, vals)
        F = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=(w.n, w.n)).tocsc()
        for k in cols:
            if kind == "spai":
                J, q = ospai.spai_column(w.A, w.e, s0, int(k), As=As0)
            else:
                J, q = ospai.update_column(w.A, w.e, s0, s1, int(k), As_new=As1, As_prev=As0)
            got = F[:, int(k)].toarray().ravel()[J]
            want = round_storage(q, "bf16")
            assert np.all(np.abs(got - want) <= np.abs(want) * 2.0**-7), (kind, k)
        morx.morx_factor_destroy(f)
    S.close()


def test_mimo_fullsize_autotuned_batched(ctx):
    from paper_2003_12759_amd import api

    w = make_workload(2)
    S = api.System(ctx, w.A, w.e)
    sig = w.rounds[0]
    _say(f"MIMO n={w.n} autotune")
    t = S.autotune(float(sig[0]), ncols=len(sig) * w.B.shape[1], chain_len=len(sig), prec="f64")
    _say(f"MIMO solve, tune {t}")
    X, Y, st, stats = S.solve_shifts(sig, w.B, w.C, prec="f64")
    _check_solves(w, sig, X, Y, stats)
    S.close()
