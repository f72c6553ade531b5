"""The allocation-free projection (morx_project_noalloc, a fixed device
scratch instead of allocations) against morx_project with orthonormalize = 0
through the C ABI: two calls in a row, the second on a smaller system with
fewer columns, each equal to the allocating entry point bit for bit (they run
the same kernels over the same row slabs) and within the FP64 contraction
bound of the plain products W^T A V, W^T E V, W^T B, V^T C."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from paper_2003_12759_amd.workloads import make_workload

pytestmark = pytest.mark.gpu


def _dev(X):
    return torch.as_tensor(np.ascontiguousarray(X.T), device="cuda").t()


@pytest.mark.parametrize("first,second", [((4, 11, 12, 2, 3), (1, 8, 5, 1, 1))])
def test_project_noalloc_equals_project(first, second):
    from paper_2003_12759_amd import api, morx

    ctx = api.Context(0)
    for wl, N, r, m, q in (first, second):
        w = make_workload(wl, N=N)
        S = api.System(ctx, w.A, w.e)
        n = w.n
        rng = np.random.default_rng(N * 100 + r)
        V, W = rng.standard_normal((n, r)), rng.standard_normal((n, r))
        B, C = rng.standard_normal((n, m)), rng.standard_normal((n, q))
        print(f"[case] project_noalloc n={n} r={r} m={m} q={q}", flush=True)
        got = morx.morx_project_noalloc(S.handle, _dev(V), _dev(W), _dev(B), _dev(C))
        ref = morx.morx_project(S.handle, _dev(V), _dev(W), _dev(B), _dev(C), orthonormalize=False)
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b)
        A = w.A.tocsr()
        E = sp.diags(w.e)
        g = 64 * 2.0**-53  # rows of A of at most 27 terms, then n-long sums in slabs
        exact = (W.T @ (A @ V), W.T @ (E @ V), W.T @ B, V.T @ C)
        scale = (np.abs(W).T @ (abs(A) @ np.abs(V)), np.abs(W).T @ (E @ np.abs(V)),
                 np.abs(W).T @ np.abs(B), np.abs(V).T @ np.abs(C))
        for a, x, sc in zip(got, exact, scale):
            assert np.all(np.abs(a - x) <= (n * 2.0**-53 + g) * sc), np.max(np.abs(a - x) / sc)
        S.close()
    ctx.close()
