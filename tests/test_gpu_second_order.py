"""Second-order solves (AIRGA, Algorithm 1 lines 4 and 10, proportional
damping) through the C ABI against the second-order oracle.

Bars: every moment's true residual on its own second-order system
(recomputed here in FP64) <= 1e-10 plus the recomputation's rounding bound;
solutions against the oracle's sparse LU within cond(A(s)) times that
residual; iteration counts within max(3, 5 %) of the oracle's BiCG run with
the paper's reuse on the second-order matrices themselves; with
alpha = beta = 0 the results equal morx_solve_moments at sigma = s^2 bit for
bit (up to the sign of odd moments).
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import second_order as oso
from paper_2003_12759_amd.workloads import make_second_order

from host_residual import residual_ok  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2003_12759_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _say(msg):
    print(f"[case] {msg}", flush=True)


@functools.lru_cache(maxsize=1)
def _oracle_case():
    w = make_second_order(N=10, nround=2, npoint=4, unit_io=False)
    return w, oso.solve(w.m, w.K, w.alpha, w.beta, w.F, w.C, w.rounds, nmom=2)


@pytest.mark.parametrize("batched", [True, False])
def test_second_order_matches_oracle(ctx, batched):
    from paper_2003_12759_amd import api

    w, ref = _oracle_case()
    nmom = 2
    S = api.System(ctx, w.A, w.m)
    for z, pts in enumerate(w.rounds):
        _say(f"second order n={w.n} round {z} nmom={nmom} batched={batched}")
        X, Y, st, stats = S.solve_second_order(w.alpha, w.beta, pts, w.F, w.C, nmom=nmom,
                                               batched=batched, next_round=z > 0)
        assert st == 0 and len(stats) == nmom * len(pts)
        Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
        Xd, Yd = oso.direct(w.m, w.K, w.alpha, w.beta, w.F, w.C, pts, nmom)
        _, _, ostats = ref[z]
        ns = len(pts)
        for i, s in enumerate(pts):
            A = oso.matrix(w.m, w.K, w.alpha, w.beta, s).tocsr()
            cond = np.linalg.cond(A.toarray())
            for j in range(nmom):
                k = j * ns + i
                assert stats[k].status == 0
                b = w.F[:, 0] if j == 0 else -(w.m * Xg[:, k - ns])
                c = w.C[:, 0] if j == 0 else -(w.m * Yg[:, k - ns])
                assert residual_ok(A, Xg[:, k], b) and residual_ok(A.T, Yg[:, k], c), (s, j)
                for got, want in ((Xg[:, k], Xd[:, k]), (Yg[:, k], Yd[:, k])):
                    assert np.linalg.norm(got - want) <= 4e-10 * cond * np.linalg.norm(want)
                oi = ostats[k].iters
                assert abs(stats[k].iters - oi) <= max(3, 0.05 * oi), (s, j, stats[k].iters, oi)
    S.close()


def test_undamped_second_order_equals_moments_at_s_squared(ctx):
    """alpha = beta = 0: A(s) = s^2 M + K = sigma E - A at sigma = s^2, and
    X_j = (-1)^j Z_j for the moments Z_j of morx_solve_moments."""
    from paper_2003_12759_amd import api

    w = make_second_order(N=9, nround=1, npoint=3, unit_io=False)
    S = api.System(ctx, w.A, w.m)
    pts = list(w.rounds[0])
    _say(f"undamped second order n={w.n}")
    X2, Y2, st2, s2 = S.solve_second_order(0.0, 0.0, pts, w.F, w.C, nmom=3)
    X1, Y1, st1, s1 = S.solve_moments([s * s for s in pts], w.F, w.C, nmom=3)
    assert st1 == st2 == 0
    ns = len(pts)
    for j in range(3):
        sl = slice(j * ns, (j + 1) * ns)
        sgn = -1.0 if j % 2 else 1.0
        assert torch.equal(X2[:, sl], sgn * X1[:, sl]) and torch.equal(Y2[:, sl], sgn * Y1[:, sl])
    assert [c.iters for c in s1] == [c.iters for c in s2]
    S.close()


def test_second_order_rejects_bad_arguments(ctx):
    from paper_2003_12759_amd import api, morx

    w = make_second_order(N=6, nround=1, npoint=2, unit_io=False)
    S = api.System(ctx, w.A, w.m)
    _say("second order argument checks")
    code = {name: v for v, name in morx.STATUS.items()}
    invalid, nonfinite = code["MORX_E_INVALID"], code["MORX_E_NONFINITE"]
    for alpha, beta, pts, want in ((0.05, -0.5, [2.0, 3.0], invalid),  # 1 + beta s = 0
                                   (float("nan"), 0.0, [2.0], nonfinite),
                                   (0.05, 5e-6, [1.0, float("inf")], nonfinite),
                                   (0.05, 5e-6, [1e300], invalid)):  # sigma overflows
        _, _, st, _ = S.solve_second_order(alpha, beta, pts, w.F, w.C, raise_on_error=False)
        assert st == want, (alpha, beta, pts, st)
    S.close()


def test_second_order_full_size_unit_io(ctx):
    """The 106^3 stand-in for the industrial model (n = 1,191,016, F = C = e_1,
    four points in [1, 500], the paper's alpha and beta), one round and its
    vertical successor: every point's true residual on A(s) <= 1e-10."""
    from paper_2003_12759_amd import api

    w = make_second_order()
    S = api.System(ctx, w.A, w.m)
    for z, pts in enumerate(w.rounds):
        _say(f"second order full size n={w.n} round {z}")
        X, Y, st, stats = S.solve_second_order(w.alpha, w.beta, pts, w.F, w.C, next_round=z > 0)
        assert st == 0
        Xg, Yg = X.cpu().numpy(), Y.cpu().numpy()
        for i, s in enumerate(pts):
            A = oso.matrix(w.m, w.K, w.alpha, w.beta, s).tocsr()
            assert residual_ok(A, Xg[:, i], w.F[:, 0]) and residual_ok(A.T, Yg[:, i], w.C[:, 0])
    S.close()


def test_galerkin_projection_interpolates_the_second_order_transfer_function(ctx):
    """Section II's reduction through morx_project with W = V: K^ = -Ar,
    M^ = Er, D^ = alpha Er - beta Ar, F^ = Br, C^ = Cr; the reduced
    H(s) = C^T (s^2 M^ + s D^ + K^)^{-1} F^ equals the full one at every point
    (the basis spans the GPU's solutions there)."""
    from paper_2003_12759_amd import api

    w = make_second_order(N=10, nround=1, npoint=4, unit_io=False)
    S = api.System(ctx, w.A, w.m)
    pts = list(w.rounds[0])
    _say(f"second order projection n={w.n}")
    X, _, st, _ = S.solve_second_order(w.alpha, w.beta, pts, w.F, None)
    assert st == 0
    Ar, Er, Br, Cr = S.project(X, X, api.block_to_dev(w.F), api.block_to_dev(w.C))
    Kh, Mh, Dh = -Ar, Er, w.alpha * Er - w.beta * Ar
    for s in pts:
        full = oso.full_transfer(w.m, w.K, w.alpha, w.beta, w.F, w.C, s)
        red = oso.transfer(Mh, Dh, Kh, Br, Cr, s)
        assert abs(red - full).max() <= 1e-8 * abs(full).max(), s
    S.close()
