"""Serving at the configured pool sizes: 16 resident systems with n
log-uniform in [4096, 262144] (2-D 5-point and 3-D 7-point stencils,
coefficients uniform in [0.5, 2]), shapes autotuned per system as bench.py
does, and a few hundred requests (shifts log-uniform in [1, 1e3]) arriving
with Poisson gaps from two client threads.

Every request's true relative residual is recomputed on the host (tolerance
1e-10 plus the FP64 recomputation's rounding bound), requests on systems of
at most 10,000 rows are compared with a sparse direct solve, and the run
must show continuous batching: requests admitted into batches that were
already iterating, several requests on the device at once.
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

NREQ = 300


def test_serving_pool16_at_configured_sizes():
    from paper_2003_12759_amd import api, morx

    p = make_serving_pool(seed=0, nreq=NREQ)
    ctx = api.Context(0)
    systems = [api.System(ctx, A, e) for (A, e) in p.systems]
    assert min(S.n for S in systems) >= 3000 and max(S.n for S in systems) <= 270000
    cfg = morx.morx_serve_config_default()
    cfg.slots_per_system = 16
    o = morx.morx_opts_default()
    o.precond_prec = morx.PREC["f32"]
    print(f"[case] serving pool: 16 systems, n {min(S.n for S in systems)}.."
          f"{max(S.n for S in systems)}, autotune", flush=True)
    for S in systems:
        S.autotune(float(np.sqrt(cfg.anchor_min * cfg.anchor_max)), ncols=cfg.slots_per_system,
                   chain_len=cfg.anchors + 1, prec="f32")
    bs, xs = [], []
    for t in range(NREQ):
        bs.append(torch.as_tensor(p.rhs(t), device="cuda"))
        xs.append(torch.zeros(systems[p.req_system[t]].n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    srv = morx.morx_serve_start(ctx.handle, cfg, o)
    tickets = [None] * NREQ
    # mean gap 1 ms: faster than requests finish, so batches are busy when
    # later requests arrive
    gaps = p.gaps * 1e-3

    def client(part):
        for t in part:
            time.sleep(gaps[t])
            tickets[t] = morx.morx_serve_submit(srv, systems[p.req_system[t]].handle,
                                                float(p.req_sigma[t]), bs[t], xs[t])

    print(f"[case] serving pool: {NREQ} Poisson requests", flush=True)
    ths = [threading.Thread(target=client, args=(list(range(k, NREQ, 2)),)) for k in range(2)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    res = [morx.morx_serve_wait(srv, tk) for tk in tickets]
    counts = morx.morx_serve_counts_get(srv)
    morx.morx_serve_stop(srv)
    print(f"[case] serving pool: counts {counts}", flush=True)
    assert counts["admitted"] == NREQ
    assert counts["joined_running"] >= NREQ // 10 and counts["max_running"] >= 4, counts
    lu_done = 0
    for t in range(NREQ):
        status, st, lat = res[t]
        assert status == 0 and st.status == 0 and st.relres_primal <= 1e-10, (t, status)
        assert lat > 0
        A, e = p.systems[p.req_system[t]]
        M = (float(p.req_sigma[t]) * sp.diags(e) - A).tocsr()
        b = p.rhs(t)
        x = xs[t].cpu().numpy()
        slack = 9 * 2.0**-53 * np.linalg.norm(np.abs(b) + abs(M) @ np.abs(x))
        assert np.linalg.norm(b - M @ x) <= 1e-10 * np.linalg.norm(b) + slack, t
        if A.shape[0] <= 10000 and lu_done < 20:
            xe = spla.splu(M.tocsc()).solve(b)
            assert np.linalg.norm(x - xe) <= 1e-8 * np.linalg.norm(xe), t
            lu_done += 1
    assert lu_done >= 5
    for S in systems:
        S.close()
    ctx.close()
