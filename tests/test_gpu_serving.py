"""Serving: continuous batching of shifted solves on resident systems.

Every request's result is checked against the plain definition (sparse LU of
sigma E - A) and its true residual; a request gives the same result alone and
in a mix of concurrent requests on several systems; admission by device
memory refuses what can never fit and queues what fits later.
"""
import threading
import time

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from paper_2003_12759_amd.workloads import make_serving_pool

pytestmark = pytest.mark.gpu

MORX_E_ADMISSION = -8


@pytest.fixture(scope="module")
def pool():
    from paper_2003_12759_amd import api

    p = make_serving_pool(seed=3, nsys=4, nreq=60, nmin=400, nmax=6000)
    ctx = api.Context(0)
    systems = [api.System(ctx, A, e) for (A, e) in p.systems]
    yield p, ctx, systems
    for S in systems:
        S.close()
    ctx.close()


def _serve(ctx, systems, p, reqs, cfg=None, threads=1, gap=0.0, opts=None):
    from paper_2003_12759_amd import morx

    srv = morx.morx_serve_start(ctx.handle, cfg, opts)
    bs, xs, tickets = {}, {}, {}
    for t in reqs:
        n = systems[p.req_system[t]].n
        bs[t] = torch.as_tensor(p.rhs(t), device="cuda")
        xs[t] = torch.zeros(n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lock = threading.Lock()

    def client(part):
        for t in part:
            tk = morx.morx_serve_submit(srv, systems[p.req_system[t]].handle, p.req_sigma[t],
                                        bs[t], xs[t])
            with lock:
                tickets[t] = tk
            if gap:
                time.sleep(gap)

    parts = [reqs[i::threads] for i in range(threads)]
    ths = [threading.Thread(target=client, args=(pp,)) for pp in parts]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    out = {}
    for t in reqs:
        out[t] = morx.morx_serve_wait(srv, tickets[t])
    info = morx.morx_serve_info(srv)
    morx.morx_serve_stop(srv)
    return {t: xs[t].cpu().numpy() for t in reqs}, out, info


def _check_exact(p, t, x, tol=1e-10):
    A, e = p.systems[p.req_system[t]]
    M = (p.req_sigma[t] * sp.diags(e) - A).tocsc()
    b = p.rhs(t)
    assert np.linalg.norm(b - M @ x) <= 1.01 * tol * np.linalg.norm(b)
    xe = spla.splu(M).solve(b)
    assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe)


def test_serving_results_match_direct_solves(pool):
    p, ctx, systems = pool
    reqs = list(range(40))
    print("[case] serving 40 requests, 4 systems, 3 client threads", flush=True)
    xs, out, info = _serve(ctx, systems, p, reqs, threads=3)
    assert info["completed"] == 40
    for t in reqs:
        status, st, lat = out[t]
        assert status == 0 and st.status == 0, (t, status)
        assert st.relres_primal <= 1e-10 and lat > 0
        _check_exact(p, t, xs[t])


def test_serving_fp32_storage_and_apply(pool):
    from paper_2003_12759_amd import morx

    p, ctx, systems = pool
    o = morx.morx_opts_default()
    o.precond_prec = morx.PREC["f32"]
    o.apply_prec = morx.PREC["f32"]
    reqs = list(range(20))
    print("[case] serving 20 requests, FP32 factors applied in FP32", flush=True)
    xs, out, info = _serve(ctx, systems, p, reqs, threads=2, opts=o)
    for t in reqs:
        status, st, lat = out[t]
        assert status == 0 and st.status == 0, (t, status)
        _check_exact(p, t, xs[t])


def test_serving_alone_equals_mix(pool):
    p, ctx, systems = pool
    picks = [1, 7, 22]
    mix = list(range(45))
    print("[case] serving alone vs mix", flush=True)
    xm, om, _ = _serve(ctx, systems, p, mix, threads=2)
    for t in picks:
        xa, oa, _ = _serve(ctx, systems, p, [t])
        assert oa[t][0] == 0 and om[t][0] == 0
        assert np.linalg.norm(xa[t] - xm[t]) <= 1e-8 * np.linalg.norm(xa[t])


def test_serving_admission(pool):
    from paper_2003_12759_amd import morx

    p, ctx, systems = pool
    cfg = morx.morx_serve_config_default()
    cfg.hbm_budget_bytes = 1 << 16  # far below one system's footprint
    print("[case] serving admission refusal", flush=True)
    _, out, _ = _serve(ctx, systems, p, [0, 1], cfg=cfg)
    assert all(out[t][0] == MORX_E_ADMISSION for t in (0, 1))
    # enough for one system plus a request at a time: everything still finishes
    # one system's slot batch and anchors (padding of the sliced layout
    # allowed for), plus room for two request factors
    npad = max(-(-S.n // 64) * 64 for S in systems)
    fbytes = max(2 * S.nnz_pattern for S in systems) * 8 * 1.5
    cfg.slots_per_system = 8
    cfg.hbm_budget_bytes = int(16 * 8 * npad * 8 + 8 * 8 * 1024 * 8 + (cfg.anchors + 2) * fbytes)
    reqs = list(range(16))
    print("[case] serving under a tight budget", flush=True)
    xs, out, info = _serve(ctx, systems, p, reqs, cfg=cfg)
    for t in reqs:
        if out[t][0] == 0:
            _check_exact(p, t, xs[t])
    assert sum(out[t][0] == 0 for t in reqs) >= 1


def test_serving_poisson_arrivals_latency(pool):
    p, ctx, systems = pool
    reqs = list(range(30))
    print("[case] serving with spaced arrivals", flush=True)
    xs, out, info = _serve(ctx, systems, p, reqs, gap=0.002)
    lats = sorted(out[t][2] for t in reqs)
    assert all(out[t][0] == 0 for t in reqs)
    assert lats[0] > 0 and lats[-1] < 60
    for t in reqs[:5]:
        _check_exact(p, t, xs[t])
