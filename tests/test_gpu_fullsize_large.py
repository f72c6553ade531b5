"""Full-size checks of the two large workloads, in the launch configuration
bench.py times for them (shapes autotuned on the system, which takes the halo
chain kernel and shifted pair for these patterns):

* 128^3 27-point variable-coefficient operator (n = 2,097,152), 12 shifts,
  factors stored in FP64, FP32 and BF16 (the precision ladder) and applied
  with FP64 vectors;
* 106^3 7-point variable-coefficient operator (n = 1,191,016), four inputs
  and outputs, 8 shifts, FP64 factors, batched.

The oracle cannot solve these systems, so the checks are properties that hold
at any size: every true relative residual, recomputed here in FP64 on the
CPU, is <= 1e-10 (primal and dual) up to the recomputation's own rounding;
the two-way transfer identity c_j^T x_ij = y_ij^T b_j to 1e-7; sampled SPAI
and update columns against the oracle's column least squares (to 1e-11 in
FP64; in FP32/BF16 one storage step plus that FP64 difference, which can
move a small entry's rounding by more than a step); and sampled rows of the chain step's
output, at the solve's launch shape, against the oracle's row-by-row chain
product.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import chain as ochain
from oracle import pattern as opattern
from oracle import spai as ospai
from oracle.precision import round_storage
from paper_2003_12759_amd.workloads import make_workload

pytestmark = pytest.mark.gpu

U = 2.0**-53


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def w27(ctx):
    from paper_2003_12759_amd import api

    w = make_workload(4)
    S = api.System(ctx, w.A, w.e)
    yield w, S
    S.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _check_solves(w, sig, X, Y, stats):
    """Host true residuals (tolerance plus the FP64 recomputation's rounding
    bound (w + 2) u (|b| + |s E x| + |A||x|), w <= 27 entries per row) and the
    two-way transfer identity."""
    m = w.B.shape[1]
    Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
    A = w.A.tocsr()
    AT = A.T  # a CSC view, no copy
    aA, aAT = abs(A), abs(A).T
    g = 29 * U
    for i, s in enumerate(sig):
        for j in range(m):
            k = i * m + j
            assert stats[k].status == 0
            assert stats[k].relres_primal <= 1e-10 and stats[k].relres_dual <= 1e-10
            x, y = Xg[:, k], Yg[:, k]
            b, c = w.B[:, j], w.C[:, j]
            # (s E - A) x and (s E - A)^T y without forming the shifted matrix
            rp = np.linalg.norm(b - (s * w.e * x - A @ x))
            rd = np.linalg.norm(c - (s * w.e * y - AT @ y))
            sp_ = g * np.linalg.norm(np.abs(b) + np.abs(s * w.e * x) + aA @ np.abs(x))
            sd_ = g * np.linalg.norm(np.abs(c) + np.abs(s * w.e * y) + aAT @ np.abs(y))
            assert rp <= 1e-10 * np.linalg.norm(b) + sp_, (i, j, rp / np.linalg.norm(b))
            assert rd <= 1e-10 * np.linalg.norm(c) + sd_, (i, j, rd / np.linalg.norm(c))
            h1 = c @ x
            h2 = y @ b
            assert abs(h1 - h2) <= 1e-7 * abs(h1)


@pytest.mark.parametrize("prec", ["bf16", "f32", "f64"])
def test_varcoef27_fullsize_autotuned(w27, prec):
    from paper_2003_12759_amd import morx

    w, S = w27
    sig = w.rounds[0]
    _say(f"27-point n={w.n} autotune {prec}")
    t = S.autotune(float(sig[0]), ncols=len(sig) * w.B.shape[1], chain_len=len(sig), prec=prec)
    _say(f"27-point solve {prec}, tune {t}")
    X, Y, st, stats = S.solve_shifts(sig, w.B, w.C, prec=prec)
    _check_solves(w, sig, X, Y, stats)
    del X, Y
    # sampled factor columns at the first two shifts
    rp, ci = S.pattern()
    cols = np.random.default_rng(7).choice(w.n, 200, replace=False)
    s0, s1 = float(sig[0]), float(sig[1])
    As0 = opattern.shifted_pattern_values(w.A, w.e, s0)
    As1 = opattern.shifted_pattern_values(w.A, w.e, s1)
    for kind in ("spai", "update"):
        _say(f"27-point sampled {kind} columns {prec}")
        f = (morx.morx_factor_spai(S.handle, s0, prec) if kind == "spai"
             else morx.morx_factor_update(S.handle, s0, s1, prec))
        vals = torch.empty(S.nnz_pattern, dtype=torch.float64, device="cuda")
        morx.morx_factor_values(f, vals)
        F = sp.csr_matrix((vals.cpu().numpy(), ci, rp), shape=(w.n, w.n)).tocsc()
        for k in cols:
            if kind == "spai":
                J, q = ospai.spai_column(w.A, w.e, s0, int(k), As=As0)
            else:
                J, q = ospai.update_column(w.A, w.e, s0, s1, int(k), As_new=As1, As_prev=As0)
            got = F[:, int(k)].toarray().ravel()[J]
            if prec == "f64":
                assert np.linalg.norm(got - q) <= 1e-11 * np.linalg.norm(q), (kind, k)
            else:
                # the FP64 solutions before rounding agree to 1e-11 ||q||;
                # rounding to storage (monotonic) adds at most one step
                want = round_storage(q, prec)
                step = 2.0**-23 if prec == "f32" else 2.0**-7
                tol = np.abs(want) * step + 1e-11 * np.linalg.norm(q)
                assert np.all(np.abs(got - want) <= tol), (kind, k)
        morx.morx_factor_destroy(f)


@pytest.mark.parametrize("prec", ["bf16", "f64"])
def test_varcoef27_fullsize_chain_rows(w27, prec):
    """The chain step at full size and the bench's launch shape (autotuned for
    12 column pairs with chains of up to 12 factors): 12 columns, column c
    preconditioned by the first c + 1 factors of a list of 12 (three imported
    random factors, each used four times), forward and transposed at once;
    96 sampled rows per direction against the oracle's row-by-row product,
    within 4 L gamma (|F_L| ... |F_1| |x|)_i."""
    from paper_2003_12759_amd import morx

    w, S = w27
    sig = w.rounds[0]
    _say(f"27-point chain rows {prec}: autotune")
    S.autotune(float(sig[0]), ncols=12, chain_len=12, prec=prec)
    rp, ci = S.pattern()
    rng = np.random.default_rng(41)
    nnz = len(ci)
    rows_of = np.repeat(np.arange(w.n, dtype=np.int64), np.diff(rp))
    diag = ci == rows_of
    del rows_of
    mats, handles = [], []
    for k in range(3):
        v = rng.standard_normal(nnz)
        v[diag] += 3.0
        v /= 4.0
        handles.append(morx.morx_factor_import(S.handle, torch.as_tensor(v, device="cuda"), prec))
        mats.append(sp.csr_matrix((round_storage(v, prec), ci, rp), shape=(w.n, w.n)))
        del v
    amats = [abs(M) for M in mats]
    mats_t = [M.T.tocsr() for M in mats]
    amats_t = [abs(M) for M in mats_t]
    chain = [0, 1, 2] * 4
    ncol = 12
    X = rng.standard_normal((w.n, ncol))
    Xt = rng.standard_normal((w.n, ncol))
    Xd = torch.as_tensor(np.ascontiguousarray(X.T), device="cuda").t()
    Xtd = torch.as_tensor(np.ascontiguousarray(Xt.T), device="cuda").t()
    Y = morx.colmajor(ncol, w.n)
    Yt = morx.colmajor(ncol, w.n)
    _say(f"27-point chain rows {prec}: apply")
    morx.morx_chain_apply_batch(S.handle, [[handles[k] for k in chain[:c + 1]] for c in range(ncol)],
                                Xd, Y, Xtd, Yt)
    got, gott = Y.cpu().numpy(), Yt.cpu().numpy()
    g = 27 * U * 1.01
    for c in range(ncol):
        ch = chain[:c + 1]
        rows = rng.choice(w.n, 8, replace=False)
        rows[0] = w.n - 1  # the ragged end of the last row block
        for trans, V, G in ((False, X, got), (True, Xt, gott)):
            ref = ochain.apply_rows(mats, ch, V[:, c], rows, transpose=trans, factors_t=mats_t)
            absp = ochain.apply_rows(amats, ch, np.abs(V[:, c]), rows, transpose=trans,
                                     factors_t=amats_t)
            bound = 4.0 * len(ch) * g * absp
            err = np.abs(G[rows, c] - ref)
            assert np.all(err <= bound), (c, trans, np.max(err / bound))
    for h in handles:
        morx.morx_factor_destroy(h)


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
