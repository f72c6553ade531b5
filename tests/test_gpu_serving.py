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


def _serve(ctx, systems, p, reqs, cfg=None, threads=1, gap=0.0, opts=None, chains=None):
    """Submit `reqs` from `threads` client threads (each waiting `gap` s
    between submissions), wait for all; returns (x per request, wait result
    per request, morx_serve_info, morx_serve_counts_get).  `chains` (a dict)
    receives each request's preconditioner chain, read once it is admitted."""
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
        if chains is not None:
            ch = None
            while ch is None:
                ch = morx.morx_serve_chain(srv, tickets[t])
                if ch is None:
                    time.sleep(0.0005)
            chains[t] = ch
        out[t] = morx.morx_serve_wait(srv, tickets[t])
    info = morx.morx_serve_info(srv)
    counts = morx.morx_serve_counts_get(srv)
    morx.morx_serve_stop(srv)
    return {t: xs[t].cpu().numpy() for t in reqs}, out, info, counts


def _check_exact(p, t, x, tol=1e-10, lu_max=None):
    """True residual of request t recomputed on the host against the
    request's tolerance (plus the host recomputation's own rounding bound),
    and the distance to a sparse direct solve (systems of at most lu_max
    rows)."""
    A, e = p.systems[p.req_system[t]]
    M = (p.req_sigma[t] * sp.diags(e) - A).tocsr()
    b = p.rhs(t)
    # |b - M x| recomputed in FP64: each entry within (w + 1) u (|b| + |M||x|)
    # of the exact residual, w <= 8 entries per row
    slack = 9 * 2.0**-53 * np.linalg.norm(np.abs(b) + abs(M) @ np.abs(x))
    assert np.linalg.norm(b - M @ x) <= tol * np.linalg.norm(b) + slack
    if lu_max is None or A.shape[0] <= lu_max:
        xe = spla.splu(M.tocsc()).solve(b)
        assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe)


def test_serving_results_match_direct_solves(pool):
    p, ctx, systems = pool
    reqs = list(range(40))
    print("[case] serving 40 requests, 4 systems, 3 client threads", flush=True)
    xs, out, info, counts = _serve(ctx, systems, p, reqs, threads=3)
    assert info["completed"] == 40 and counts["admitted"] == 40
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
    xs, out, info, _ = _serve(ctx, systems, p, reqs, threads=2, opts=o)
    for t in reqs:
        status, st, lat = out[t]
        assert status == 0 and st.status == 0, (t, status)
        _check_exact(p, t, xs[t])


def test_serving_alone_equals_mix(pool):
    """The same requests alone and in a mix of 45 concurrent ones (two client
    threads over four systems) agree to 1e-8; the mix did overlap: requests
    joined batches that were already iterating."""
    p, ctx, systems = pool
    picks = [1, 7, 22]
    mix = list(range(45))
    print("[case] serving alone vs mix", flush=True)
    xm, om, _, cm = _serve(ctx, systems, p, mix, threads=2)
    assert cm["max_running"] >= 2 and cm["joined_running"] >= 1, cm
    for t in picks:
        xa, oa, _, ca = _serve(ctx, systems, p, [t])
        assert ca["joined_running"] == 0 and ca["max_running"] == 1
        assert oa[t][0] == 0 and om[t][0] == 0
        assert np.linalg.norm(xa[t] - xm[t]) <= 1e-8 * np.linalg.norm(xa[t])


def test_serving_joins_a_running_batch(pool):
    """A request submitted while another request of its system iterates is
    admitted into that running batch (continuous batching, not a queue): the
    first request is hard (a small shift on the largest system), the second
    is submitted once the first has been admitted."""
    from paper_2003_12759_amd import morx

    p, ctx, systems = pool
    s = int(np.argmax([S.n for S in systems]))
    S = systems[s]
    srv = morx.morx_serve_start(ctx.handle, None, None)
    rng = np.random.default_rng(5)
    b1 = torch.as_tensor(rng.standard_normal(S.n), device="cuda")
    b2 = torch.as_tensor(rng.standard_normal(S.n), device="cuda")
    x1 = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    x2 = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    print("[case] serving: a request joins a running batch", flush=True)
    t1 = morx.morx_serve_submit(srv, S.handle, 1.0, b1, x1)
    while morx.morx_serve_chain(srv, t1) is None:
        time.sleep(0.0002)
    t2 = morx.morx_serve_submit(srv, S.handle, 3.0, b2, x2)
    r1 = morx.morx_serve_wait(srv, t1)
    r2 = morx.morx_serve_wait(srv, t2)
    counts = morx.morx_serve_counts_get(srv)
    morx.morx_serve_stop(srv)
    assert r1[0] == 0 and r2[0] == 0
    # the first needs more than one segment, so the second joined it
    assert r1[1].iters > 8
    assert counts["joined_running"] == 1 and counts["max_running"] == 2, counts
    A, e = p.systems[s]
    for sig, b, x in ((1.0, b1, x1), (3.0, b2, x2)):
        M = (sig * sp.diags(e) - A).tocsc()
        xe = spla.splu(M).solve(b.cpu().numpy())
        assert np.linalg.norm(x.cpu().numpy() - xe) <= 1e-8 * np.linalg.norm(xe)


def test_serving_chains_follow_the_anchored_schedule(pool):
    """Every request's chain, spec by spec and bit for bit: the system's
    anchor prefix up to the nearest anchor and one update to the request's
    shift (the oracle's anchored schedule)."""
    from oracle import chain as ochain
    from paper_2003_12759_amd import morx

    p, ctx, systems = pool
    cfg = morx.morx_serve_config_default()
    anchors = ochain.anchor_shifts(cfg.anchors, cfg.anchor_min, cfg.anchor_max)
    reqs = list(range(24))
    chains = {}
    print("[case] serving chains vs the anchored schedule", flush=True)
    xs, out, _, _ = _serve(ctx, systems, p, reqs, threads=2, chains=chains)
    for t in reqs:
        assert out[t][0] == 0
        assert chains[t] == ochain.schedule_anchored(anchors, float(p.req_sigma[t])), t


def _budget_one_system(systems, cfg, opts=None):
    """A budget that holds the largest system with every slot busy, and no
    two systems at once."""
    from paper_2003_12759_amd import morx

    fp = [morx.morx_serve_footprint(S.handle, cfg, opts) for S in systems]
    need = max(a + cfg.slots_per_system * b for a, b in fp)
    smallest_pair = min(fp[i][0] + fp[j][0] + fp[i][1]
                        for i in range(len(fp)) for j in range(len(fp)) if i != j)
    return need, smallest_pair


def test_serving_admission(pool):
    """A budget below any system's footprint refuses every request; a budget
    for one system at a time (but every slot) completes every request,
    releasing idle systems least recently used first."""
    from paper_2003_12759_amd import morx

    p, ctx, systems = pool
    cfg = morx.morx_serve_config_default()
    cfg.hbm_budget_bytes = 1 << 16  # far below one system's footprint
    print("[case] serving admission refusal", flush=True)
    _, out, _, counts = _serve(ctx, systems, p, [0, 1], cfg=cfg)
    assert all(out[t][0] == MORX_E_ADMISSION for t in (0, 1))
    assert counts["systems_made"] == 0
    cfg.slots_per_system = 8
    need, pair = _budget_one_system(systems, cfg)
    cfg.hbm_budget_bytes = need
    reqs = list(range(16))
    print("[case] serving under a one-system budget", flush=True)
    xs, out, info, counts = _serve(ctx, systems, p, reqs, cfg=cfg)
    for t in reqs:
        assert out[t][0] == 0, (t, out[t][0])
        _check_exact(p, t, xs[t])
    assert info["completed"] == 16
    if need < pair:  # the pool's systems cannot be resident two at a time
        nsys = len(set(int(p.req_system[t]) for t in reqs))
        assert counts["systems_made"] >= nsys and counts["systems_evicted"] >= nsys - 1, counts
    assert counts["resident"] >= 1


def test_serving_cycles_through_more_systems_than_fit():
    """Four systems of about the same size, a budget for one at a time, and
    requests that cycle over all four: each system is made resident again
    after being released, and every request completes with the direct
    solve's answer."""
    from paper_2003_12759_amd import api, morx

    p = make_serving_pool(seed=7, nsys=4, nreq=24, nmin=2500, nmax=2600)
    ctx = api.Context(0)
    systems = [api.System(ctx, A, e) for (A, e) in p.systems]
    cfg = morx.morx_serve_config_default()
    cfg.slots_per_system = 4
    need, pair = _budget_one_system(systems, cfg)
    assert need < pair
    cfg.hbm_budget_bytes = need
    p.req_system[:] = np.arange(24) % 4
    reqs = list(range(24))
    print("[case] serving: requests cycling over 4 systems, room for 1", flush=True)
    xs, out, info, counts = _serve(ctx, systems, p, reqs, cfg=cfg, gap=0.001)
    for t in reqs:
        assert out[t][0] == 0, (t, out[t][0])
        _check_exact(p, t, xs[t])
    assert counts["systems_evicted"] >= 3 and counts["systems_made"] >= 4, counts
    for S in systems:
        S.close()
    ctx.close()


def test_serving_poisson_arrivals_latency(pool):
    p, ctx, systems = pool
    reqs = list(range(30))
    print("[case] serving with spaced arrivals", flush=True)
    xs, out, info, counts = _serve(ctx, systems, p, reqs, gap=0.002)
    lats = sorted(out[t][2] for t in reqs)
    assert all(out[t][0] == 0 for t in reqs)
    assert lats[0] > 0 and lats[-1] < 60
    for t in reqs[:5]:
        _check_exact(p, t, xs[t])
