"""Edge cases of the HIP path through the C ABI: systems smaller than one
64-row slice and on slice boundaries, more columns than one wave carries,
primal-only solves, reported non-convergence, and rejected inputs (malformed
CSR, non-finite values, bad arguments, a rank-deficient local least-squares
problem).  Solutions are checked against dense solves of sigma E - A.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from host_residual import residual_ok  # noqa: E402

pytestmark = pytest.mark.gpu

MORX_E_INVALID = -1
MORX_E_SINGULAR_LS = -4
MORX_E_NOT_CONVERGED = -5
MORX_E_NONFINITE = -7


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _rand_system(n, seed):
    rng = np.random.default_rng(seed)
    if n == 1:
        A = sp.csr_matrix(np.array([[-3.0]]))
    else:
        M = sp.random(n, n, density=min(1.0, 3.0 / n), random_state=rng, format="csr")
        M.data = rng.standard_normal(M.nnz)
        A = (M + sp.diags(-5.0 - rng.uniform(0, 1, n))).tocsr()
        A.sort_indices()
    e = rng.uniform(1, 2, n)
    return A, e


def _check_dense(A, e, sig, X, Y, B, C, m):
    Ad = A.toarray()
    for i, s in enumerate(sig):
        M = s * np.diag(e) - Ad
        for j in range(m):
            k = i * m + j
            x = np.linalg.solve(M, B[:, j])
            assert residual_ok(M, X[:, k], B[:, j])
            assert np.linalg.norm(X[:, k] - x) <= 1e-8 * np.linalg.norm(x)
            if Y is not None:
                y = np.linalg.solve(M.T, C[:, j])
                assert np.linalg.norm(Y[:, k] - y) <= 1e-8 * np.linalg.norm(y)


@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 127, 128])
@pytest.mark.parametrize("batched", [True, False])
def test_sizes_around_the_slice_height(ctx, n, batched):
    from paper_2003_12759_amd import api

    A, e = _rand_system(n, 100 + n)
    rng = np.random.default_rng(n)
    m = 2
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((n, m))
    sig = [0.5, 3.0, 20.0]
    S = api.System(ctx, A, e)
    _say(f"n={n} batched={batched}")
    X, Y, st, stats = S.solve_shifts(sig, B, C, prec="f64", batched=batched)
    assert all(c.status == 0 for c in stats)
    _check_dense(A, e, sig, X.cpu().numpy(), Y.cpu().numpy(), B, C, m)
    S.close()


def test_more_columns_than_one_wave_and_primal_only(ctx):
    """9 right-hand sides x 3 shifts = 27 columns (several column chunks),
    without C: the shadow recurrence uses b and Y is not produced."""
    from paper_2003_12759_amd import api

    n, m = 300, 9
    A, e = _rand_system(n, 7)
    B = np.random.default_rng(8).standard_normal((n, m))
    sig = [0.7, 4.0, 30.0]
    S = api.System(ctx, A, e)
    for batched in (True, False):
        _say(f"27 columns primal only batched={batched}")
        X, Y, st, stats = S.solve_shifts(sig, B, None, prec="f32", batched=batched)
        assert Y is None and all(c.status == 0 for c in stats) and len(stats) == 27
        _check_dense(A, e, sig, X.cpu().numpy(), None, B, None, m)
    S.close()


def test_not_converged_is_reported(ctx):
    from paper_2003_12759_amd import api
    from paper_2003_12759_amd.workloads import make_workload

    w = make_workload(0)
    S = api.System(ctx, w.A, w.e)
    _say("two iterations, no restart")
    X, Y, st, stats = S.solve_shifts(w.rounds[0][:2], w.B, w.C, maxit=2, max_restarts=0,
                                     raise_on_error=False)
    assert st == MORX_E_NOT_CONVERGED
    for c in stats:
        assert c.status == MORX_E_NOT_CONVERGED and c.iters == 2 and c.restarts == 0
        assert c.relres_primal > 1e-10
    # the system is still usable
    _, _, st, stats = S.solve_shifts(w.rounds[0][:2], w.B, w.C)
    assert st == 0
    S.close()


def test_rejected_arguments(ctx):
    from paper_2003_12759_amd import api, morx
    from paper_2003_12759_amd.workloads import make_workload

    w = make_workload(0, N=12, nshift=2)
    S = api.System(ctx, w.A, w.e)
    Bd, Cd = api.block_to_dev(w.B), api.block_to_dev(w.C)
    X = morx.colmajor(2, w.n)
    Y = morx.colmajor(2, w.n)
    _say("rejected arguments")
    with pytest.raises(morx.MorxError) as ei:
        morx.morx_solve_shifts(S.handle, [], Bd, Cd, X, Y)
    assert ei.value.status == MORX_E_INVALID
    with pytest.raises(morx.MorxError) as ei:
        morx.morx_solve_shifts(S.handle, [1.0, float("nan")], Bd, Cd, X, Y)
    assert ei.value.status == MORX_E_NONFINITE
    Bn = Bd.clone()
    Bn[3, 0] = float("inf")
    with pytest.raises(morx.MorxError) as ei:
        morx.morx_solve_shifts(S.handle, [1.0, 2.0], Bn, Cd, X, Y)
    assert ei.value.status == MORX_E_NONFINITE
    o = morx.morx_opts_default()
    o.chain = 7
    with pytest.raises(morx.MorxError) as ei:
        morx.morx_solve_shifts(S.handle, [1.0, 2.0], Bd, Cd, X, Y, o)
    assert ei.value.status == MORX_E_INVALID
    S.close()


def _create(ctx, rowptr, colind, val, e):
    from paper_2003_12759_amd import morx

    dev = torch.device("cuda")
    return morx.morx_system_create(
        ctx.handle, torch.tensor(rowptr, dtype=torch.int32, device=dev),
        torch.tensor(colind, dtype=torch.int32, device=dev),
        torch.tensor(val, dtype=torch.float64, device=dev),
        torch.tensor(e, dtype=torch.float64, device=dev))


@pytest.mark.parametrize("case,status", [
    ("unsorted", MORX_E_INVALID), ("duplicate", MORX_E_INVALID),
    ("out_of_range", MORX_E_INVALID), ("rowptr_end", MORX_E_INVALID),
    ("nan_value", MORX_E_NONFINITE), ("inf_e", MORX_E_NONFINITE)])
def test_malformed_systems_rejected(ctx, case, status):
    from paper_2003_12759_amd import morx

    rowptr, colind = [0, 2, 4, 6], [0, 1, 0, 1, 1, 2]
    val, e = [-4.0, 1.0, 1.0, -4.0, 1.0, -4.0], [1.0, 1.5, 2.0]
    if case == "unsorted":
        colind = [1, 0, 0, 1, 1, 2]
    elif case == "duplicate":
        colind = [0, 0, 0, 1, 1, 2]
    elif case == "out_of_range":
        colind = [0, 1, 0, 1, 1, 3]
    elif case == "rowptr_end":
        rowptr = [0, 2, 4, 5]
    elif case == "nan_value":
        val[3] = float("nan")
    else:
        e[1] = float("inf")
    _say(f"malformed system {case}")
    with pytest.raises(morx.MorxError) as ei:
        _create(ctx, rowptr, colind, val, e)
    assert ei.value.status == status


def test_rank_deficient_local_problem(ctx):
    """Column 1 of sigma E - A is zero (A has no entry in column 1 and e_1 =
    0): its SPAI least-squares problem has no unique solution."""
    from paper_2003_12759_amd import morx

    h = _create(ctx, [0, 1, 2, 3], [0, 1, 2], [-3.0, 0.0, -3.0], [1.0, 0.0, 1.0])
    _say("rank-deficient local problem")
    with pytest.raises(morx.MorxError) as ei:
        morx.morx_factor_spai(h, 2.0, "f64")
    assert ei.value.status == MORX_E_SINGULAR_LS
    morx.morx_system_destroy(h)
