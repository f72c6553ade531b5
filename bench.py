"""Throughput of the shifted-solve hot path on one MI355X.

One step = the whole job of the 64^3 convection-diffusion workload
(n = 262,144, 7-point upwind stencil, E = diag U[1,2], SISO): three rounds of
ten shifts (rounds 2 and 3 jittered, vertical reuse between rounds), SPAI at
the first shift and the column-wise reuse update for every other one (FP32
factor storage), two-sided BiCG to a true relative residual of 1e-10 for all
30 primal + dual pairs, and the Petrov-Galerkin projection after each round.
Inputs are resident on the device before the clock starts.

Printed JSON (one line): value = shifted solves per second (a solve is one
primal + dual pair meeting 1e-10 on both), batched multi-shift path;
``plain`` is the one-shift-one-column path on the same job; ``roofline`` is
measured on the dominant kernel (the chain step) with HIP events around its
launches in one extra traced step; ``cpu_baseline`` times the CPU oracle on a
bounded sample (one factor build + one pair solve, the per-shift unit).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shifted solves/sec to rel-res 1e-10 (batched vs plain); HBM GB/s; p99 lat"
HBM_PEAK_GBPS = 8000.0
DOMINANT = "chain_step"


def traffic_file(workload: str) -> str:
    """Measured HBM traffic of the chain step on a workload (rocprofv3 counters)."""
    return os.path.join(ROOT, "profiles", f"traffic_chain_step_{workload}.json")


def kernel_source_hash() -> str:
    """sha256 of the chain step's sources (the kernels, their launches and the
    shared helpers)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("chain_kernels.h", "chain_f64.hip", "chain_f32.hip", "chain_bf16.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2003_12759_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def chain_kernel_name(A, vt: str, at: str, ncol: int, ncmax: int, halo: bool) -> str:
    """Instance of the chain step the library launches for this batch: the
    halo variant when the system uses it (`halo`, from the tune the library
    reports), else the narrow variant when every row of S = pattern(A) +
    diagonal and of S^T has at most 8 entries, else the general one, at the
    tile width of the library's column split (equal chunks of at most ncmax
    columns, rounded up to an instantiated width)."""
    import numpy as np
    import scipy.sparse as sp

    P = sp.csr_matrix(A, copy=True)
    P.data[:] = 1.0
    P = (P + sp.identity(P.shape[0], format="csr")).tocsr()
    width = max(int(np.diff(P.indptr).max()), int(np.diff(P.tocsc().indptr).max()))
    ncmax = ncmax if ncmax > 0 else 8
    chunks = -(-ncol // ncmax)
    nc = -(-ncol // chunks)
    nc = nc if nc <= 8 else (10 if nc <= 10 else (12 if nc <= 12 else 16))
    kind = "k_chain_halo" if halo else ("k_chain_narrow" if width <= 8 else "k_chain_step")
    return f"{kind}<{vt}, {at}, {nc}>"


def default_apply(prec: str) -> str:
    """Apply precision used unless --apply says otherwise: FP64 vectors for
    every storage precision (FP32 and BF16 factor values are widened as they
    are loaded).  Rounding the chain's vectors to FP32 costs far more BiCG
    iterations at 64^3 than it saves in bytes."""
    return "f64"


def run_job(S, w, Bd, Cd, batched: bool, apply: str, use_graph: bool = True, prec=None,
            keep=None, policy: str = "reuse"):
    """One step: every round's shifted solves and projection.  ``keep`` (a
    list) receives the last round's (X, Y)."""
    stats_all = []
    for z, sig in enumerate(w.rounds):
        X, Y, st, stats = S.solve_shifts(sig, Bd, Cd, prec=prec or w.prec, tol=w.tol,
                                         batched=batched, next_round=z > 0, use_graph=use_graph,
                                         apply=apply, policy=policy)
        S.project(X, Y, Bd, Cd)
        stats_all.extend(stats)
    if keep is not None:
        keep[:] = [X, Y]
    return stats_all


def ladder(S, w, Bd, Cd, nsolves):
    """Precision ladder: the same job with FP64, FP32 and BF16 factor storage
    (chain applied with FP64 vectors, FP64 Krylov and refinement).  Per
    precision: one timed step after one untimed one, iterations per shift,
    the largest true relative residual recomputed on the host in FP64, and
    the largest relative distance of x and y from the FP64-storage solution."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    E = sp.diags(w.e)
    out, ref = {}, None
    for prec in ("f64", "f32", "bf16"):
        keep = []
        run_job(S, w, Bd, Cd, batched=True, apply="f64", prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = run_job(S, w, Bd, Cd, batched=True, apply="f64", prec=prec, keep=keep)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        check(st, w.tol)
        X, Y = keep[0].cpu().numpy(), keep[1].cpu().numpy()
        m = w.B.shape[1]
        res = 0.0
        for i, sig in enumerate(w.rounds[-1]):
            M = (sig * E - w.A).tocsr()
            for j in range(m):
                k = i * m + j
                res = max(res, np.linalg.norm(w.B[:, j] - M @ X[:, k]) / np.linalg.norm(w.B[:, j]),
                          np.linalg.norm(w.C[:, j] - M.T @ Y[:, k]) / np.linalg.norm(w.C[:, j]))
        if ref is None:
            ref = (X, Y)
        err = max(float(np.max(np.linalg.norm(X - ref[0], axis=0) / np.linalg.norm(ref[0], axis=0))),
                  float(np.max(np.linalg.norm(Y - ref[1], axis=0) / np.linalg.norm(ref[1], axis=0))))
        its = [x.iters for x in st[-len(w.rounds[-1]) * m:]]
        out[prec] = {"value": round(nsolves / dt, 3), "unit": "solves/s",
                     "iters_per_shift": its, "iters_total": sum(its),
                     "max_true_relres": float(f"{res:.3e}"),
                     "max_rel_diff_vs_f64_storage": float(f"{err:.3e}")}
    return out


def check(stats, tol):
    bad = [(k, s.status, s.relres_primal, s.relres_dual) for k, s in enumerate(stats)
           if s.status != 0 or s.relres_primal > tol or s.relres_dual > tol]
    if bad:
        raise SystemExit(f"accuracy check failed: {bad[:5]}")


def cpu_baseline(w, apply):
    """Oracle on one factor build + one pair solve (round 1, shift 1)."""
    import numpy as np
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits

    from oracle import bicg as obicg
    from oracle import chain as ochain
    from oracle import job as ojob

    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        specs, chains = ochain.schedule([w.rounds[0][:1]])
        factors = ojob.build_factors(w.A, w.e, specs, w.prec)
        s = float(w.rounds[0][0])
        As = (s * sp.diags(w.e) - w.A).tocsr()
        AsT = As.T.tocsr()
        res = obicg.solve(lambda v: As @ v, lambda v: AsT @ v, w.B[:, 0], w.C[:, 0],
                          lambda v: ochain.apply(factors, [0], v, apply),
                          lambda v: ochain.apply_transpose(factors, [0], v, apply), tol=w.tol)
        dt = time.perf_counter() - t0
    assert res.status == "ok"
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one SPAI factor build (n={w.n}, {w.prec.upper()} storage, "
                      f"{apply.upper()} apply) + one primal+dual "
                      f"BiCG pair solve to 1e-10 ({res.iters} iterations), {dt:.1f} s, "
                      "single-threaded NumPy/SciPy"}


def serving_bench(args):
    """Serving workload: 16 resident systems, Poisson request stream.

    First a closed-loop run (every request submitted at once) gives the
    maximum throughput; then the stream is replayed with Poisson arrivals at
    0.5, 0.8 and 1.0 of that rate and p50 / p99 latency (submit to result)
    is reported.  A sample of results is checked against the true residual
    on the host."""
    import numpy as np
    import scipy.sparse as sp
    import threading
    import torch

    from paper_2003_12759_amd import api, morx
    from paper_2003_12759_amd.workloads import make_serving_pool

    pool = make_serving_pool(seed=0, nreq=args.requests)
    ctx = api.Context(0)
    systems = [api.System(ctx, A, e) for (A, e) in pool.systems]
    nreq = args.requests
    bs, xs = [], []
    for t in range(nreq):
        n = systems[pool.req_system[t]].n
        g = torch.Generator(device="cuda")
        g.manual_seed(int(pool.req_seed[t]) % (2**63))
        bs.append(torch.randn(n, dtype=torch.float64, device="cuda", generator=g))
        xs.append(torch.zeros(n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    cfg = morx.morx_serve_config_default()
    cfg.slots_per_system = args.slots
    prec = args.prec or "f32"
    apply = args.apply or default_apply(prec)
    opts = morx.morx_opts_default()
    opts.precond_prec = morx.PREC[prec]
    opts.apply_prec = morx.PREC[apply]
    if not args.no_autotune:
        # per system: slots columns, chains up to anchors + 1 factors
        for S in systems:
            S.autotune(float(cfg.anchor_min * (cfg.anchor_max / cfg.anchor_min) ** 0.5),
                       ncols=cfg.slots_per_system, chain_len=cfg.anchors + 1, prec=prec)
    srv = morx.morx_serve_start(ctx.handle, cfg, opts)
    # anchors of every system are built on its first request (not timed)
    # b and x must stay alive until the request is finished
    warm_b = [torch.ones(S.n, dtype=torch.float64, device="cuda") for S in systems]
    warm_x = [torch.zeros(S.n, dtype=torch.float64, device="cuda") for S in systems]
    warm = [morx.morx_serve_submit(srv, S.handle, 10.0, b, x)
            for S, b, x in zip(systems, warm_b, warm_x)]
    for k in warm:
        morx.morx_serve_wait(srv, k)

    def run(times):
        tickets = [None] * nreq
        t0 = time.perf_counter()

        def client():
            for t in range(nreq):
                if times is not None:
                    delay = t0 + times[t] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                tickets[t] = morx.morx_serve_submit(srv, systems[pool.req_system[t]].handle,
                                                    pool.req_sigma[t], bs[t], xs[t])

        th = threading.Thread(target=client)
        th.start()
        th.join()
        res = [morx.morx_serve_wait(srv, k) for k in tickets]
        wall = time.perf_counter() - t0
        bad = [t for t, r in enumerate(res) if r[0] != 0 or r[1].relres_primal > 1e-10]
        if bad:
            raise SystemExit(f"serving: {len(bad)} requests failed, e.g. {bad[:5]}")
        lat = np.array([r[2] for r in res])
        its = np.array([r[1].iters for r in res])
        return wall, lat, its

    wall, lat, its = run(None)
    lam_max = nreq / wall
    out = {"closed_loop": {"requests_per_s": round(lam_max, 2), "wall_s": round(wall, 3),
                           "p50_s": round(float(np.percentile(lat, 50)), 4),
                           "p99_s": round(float(np.percentile(lat, 99)), 4),
                           "mean_iters": round(float(its.mean()), 1)}}
    # host check of a sample of results against their true residuals
    rng = np.random.default_rng(1)
    for t in rng.choice(nreq, 16, replace=False):
        A, e = pool.systems[pool.req_system[t]]
        M = (pool.req_sigma[t] * sp.diags(e) - A).tocsr()
        b, x = bs[t].cpu().numpy(), xs[t].cpu().numpy()
        rr = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
        if rr > 1.01e-10:
            raise SystemExit(f"serving: request {t} true residual {rr}")
    loads = {}
    for rho in args.loads:
        times = np.cumsum(pool.gaps) / (rho * lam_max)
        wall, lat, its = run(times)
        loads[str(rho)] = {"offered_per_s": round(rho * lam_max, 2),
                           "achieved_per_s": round(nreq / wall, 2),
                           "p50_s": round(float(np.percentile(lat, 50)), 4),
                           "p99_s": round(float(np.percentile(lat, 99)), 4)}
    info = morx.morx_serve_info(srv)
    morx.morx_serve_stop(srv)
    hi = loads.get("0.8") or next(iter(loads.values()), out["closed_loop"])
    line = {"metric": METRIC, "value": round(lam_max, 3), "unit": "solves/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * out["closed_loop"]["wall_s"], 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "serving_pool16", "systems": len(systems),
                       "n_range": [min(S.n for S in systems), max(S.n for S in systems)],
                       "requests": nreq, "slots_per_system": args.slots, "anchors": cfg.anchors,
                       "precond_storage": prec, "precond_apply": apply, "krylov": "f64",
                       "tol": 1e-10, "mode": "continuous batching",
                       "launch_shapes": "built-in" if args.no_autotune else "autotuned per system"},
            "p50_s": hi["p50_s"], "p99_s": hi["p99_s"], "serving": out, "loads": loads,
            "server_bytes": info["bytes_in_use"], "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)
    for S in systems:
        S.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="convdiff3d_n262144",
                    choices=["convdiff3d_n262144", "laplace2d_n2025", "varcoef3d_n1191016_mimo4",
                             "varcoef27_n2097152", "serving_pool16"])
    ap.add_argument("--prec", default=None, choices=[None, "f64", "f32", "bf16"],
                    help="factor storage precision (default: the workload's)")
    ap.add_argument("--apply", default=None, choices=[None, "f64", "f32"],
                    help="preconditioner apply precision (default: FP64)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of timing candidates first")
    ap.add_argument("--shapes", default=None,
                    help="pin the launch shapes instead of autotuning: "
                         "factor_kernel,cols_per_wave,slices_per_wave"
                         "[,spmv_cols_per_wave[,chain_kernel]]")
    ap.add_argument("--compare-policies", action="store_true",
                    help="also time the comparator schedules: a SPAI per shift, and "
                         "Table 2's first approach")
    ap.add_argument("--moments", type=int, default=0,
                    help="also time morx_solve_moments with this many moments per shift "
                         "(every round of the job; each moment pair counts as a solve)")
    ap.add_argument("--gmres", type=int, default=0,
                    help="also time the job with GMRES(this restart length) instead of BiCG "
                         "(one system at a time, the paper's solver)")
    ap.add_argument("--irka", type=int, default=0,
                    help="also run the IRKA-style shift loop for at most this many rounds")
    ap.add_argument("--irka-tol", type=float, default=1e-4,
                    help="relative change of the shifts that ends the IRKA loop")
    ap.add_argument("--requests", type=int, default=10000, help="serving: number of requests")
    ap.add_argument("--slots", type=int, default=16, help="serving: slots per system")
    ap.add_argument("--loads", type=float, nargs="*", default=[0.5, 0.8, 1.0],
                    help="serving: offered loads as fractions of the closed-loop rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path is one system per GPU); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2003_12759_amd import api, morx
    from paper_2003_12759_amd.workloads import make_workload

    if args.workload == "serving_pool16":
        serving_bench(args)
        return
    index = {"laplace2d_n2025": 0, "convdiff3d_n262144": 1, "varcoef3d_n1191016_mimo4": 2,
             "varcoef27_n2097152": 4}[args.workload]
    w = make_workload(index, prec=args.prec)
    apply = args.apply or default_apply(w.prec)
    nsolves = sum(len(r) for r in w.rounds) * w.B.shape[1]
    ctx = api.Context(0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    S = api.System(ctx, w.A, w.e)  # host CSR -> device, then morx_system_create
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    Bd = api.block_to_dev(w.B)
    Cd = api.block_to_dev(w.C)
    torch.cuda.synchronize()

    # launch shapes: timed on this system before the clock starts (a
    # one-time cost per system, like building it)
    tuned = None
    if args.shapes:
        sh = [int(x) for x in args.shapes.split(",")] + [-1, -1]
        S.set_tune(factor_kernel=sh[0], cols_per_wave=sh[1], slices_per_wave=sh[2],
                   spmv_cols_per_wave=sh[3], chain_kernel=sh[4])
        tuned = dict(S.get_tune(), pinned=True)
    elif not args.no_autotune:
        t_tune = time.perf_counter()
        tuned = S.autotune(float(w.rounds[0][0]), ncols=len(w.rounds[0]) * w.B.shape[1],
                           chain_len=len(w.rounds[0]) + len(w.rounds) - 1, prec=w.prec)
        tuned["seconds"] = round(time.perf_counter() - t_tune, 3)
        setup_s += tuned["seconds"]

    for _ in range(args.warmup):
        check(run_job(S, w, Bd, Cd, batched=True, apply=apply), w.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = run_job(S, w, Bd, Cd, batched=True, apply=apply)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    check(last, w.tol)
    value = nsolves * args.steps / dt
    iters = sum(st.iters for st in last)

    def timed(batched, ap_, steps):
        run_job(S, w, Bd, Cd, batched=batched, apply=ap_)  # first call sizes the slot batch
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            st_ = run_job(S, w, Bd, Cd, batched=batched, apply=ap_)
        torch.cuda.synchronize()
        check(st_, w.tol)
        return nsolves * steps / (time.perf_counter() - t1), sum(x.iters for x in st_)

    # the same batched job with the preconditioner applied in FP64
    f64_apply = None
    if apply != "f64" and args.plain_steps > 0:
        v64, it64 = timed(True, "f64", 1)
        f64_apply = {"value": round(v64, 3), "unit": "solves/s", "iters_per_step": it64,
                     "mode": "batched multi-shift, preconditioner applied in FP64"}

    plain_value = None
    if args.plain_steps > 0:
        plain_value, plain_iters = timed(False, "f64", args.plain_steps)

    roofline, kernels = None, None
    if not args.no_trace:
        morx.morx_trace_enable(ctx.handle, True)
        check(run_job(S, w, Bd, Cd, batched=True, apply=apply), w.tol)
        tr = morx.morx_trace_read(ctx.handle)
        morx.morx_trace_enable(ctx.handle, False)
        kernels = {}
        for name, (launches, ms, byts) in tr.items():
            if launches == 0:
                continue
            kernels[name] = {"launches": launches, "avg_us": 1e3 * ms / launches,
                             "total_ms": ms,
                             "GBps": (byts / (ms * 1e-3) / 1e9) if byts > 0 else None}
        launches, ms, byts = tr[DOMINANT]
        achieved = byts / (ms * 1e-3) / 1e9
        ncol = len(w.rounds[0]) * w.B.shape[1]
        ctype = {"f64": "double", "f32": "float", "bf16": "unsigned short"}
        tune_now = S.get_tune()
        roof_kernel = chain_kernel_name(w.A, ctype[w.prec], ctype[apply], ncol,
                                        tune_now["cols_per_wave"], tune_now["chain_kernel"] == 1)
        traffic = None
        if os.path.exists(traffic_file(w.name)):
            with open(traffic_file(w.name)) as f:
                tf = json.load(f)
            # counters describe the kernel source and instance they were taken on
            entry = tf.get("kernels", {}).get(roof_kernel)
            if (tf.get("source_sha256") == kernel_source_hash() and entry
                    and w.name in tf.get("workload", "")):
                traffic = entry.get("bytes_per_launch")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic,
                    "kernel": roof_kernel,
                    "avg_launch_us": round(1e3 * ms / launches, 2),
                    "alg_bytes_per_launch": byts / launches}

    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    lad = ladder(S, w, Bd, Cd, nsolves) if index == 4 and args.prec is None else None

    comparators = None
    if args.compare_policies:
        # the same batched job under the comparator factor schedules
        comparators = {}
        for pol in ("direct", "first"):
            run_job(S, w, Bd, Cd, batched=True, apply=apply, policy=pol)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st_ = run_job(S, w, Bd, Cd, batched=True, apply=apply, policy=pol)
            torch.cuda.synchronize()
            dt_ = time.perf_counter() - t1
            check(st_, w.tol)
            comparators[pol] = {"value": round(nsolves / dt_, 3), "unit": "solves/s",
                                "iters_per_step": sum(x.iters for x in st_)}

    moments = None
    if args.moments > 0:
        def moment_job():
            sts = []
            for z, sig in enumerate(w.rounds):
                _, _, _, st_ = S.solve_moments(list(sig), Bd, Cd, nmom=args.moments,
                                               prec=w.prec, tol=w.tol, next_round=z > 0)
                sts.extend(st_)
            return sts
        moment_job()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_ = moment_job()
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t1
        check(st_, w.tol)
        moments = {"moments_per_shift": args.moments, "solves_per_step": len(st_),
                   "value": round(len(st_) / dt_, 3), "unit": "solves/s",
                   "ms_per_step": round(1e3 * dt_, 3),
                   "iters_per_step": sum(x.iters for x in st_)}

    gm = None
    if args.gmres > 0:
        def gmres_job():
            sts = []
            for z, sig in enumerate(w.rounds):
                _, _, _, st_ = S.gmres_shifts(list(sig), Bd, Cd, restart=args.gmres, prec=w.prec,
                                              tol=w.tol, next_round=z > 0)
                sts.extend(st_)
            return sts
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_ = gmres_job()
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t1
        check(st_, w.tol)
        gm = {"restart": args.gmres, "value": round(nsolves / dt_, 3), "unit": "solves/s",
              "ms_per_step": round(1e3 * dt_, 3),
              "iters_per_step": sum(x.iters for x in st_),
              "mode": "GMRES, one system at a time, same chains"}

    ik = None
    if args.irka > 0:
        # IRKA-style loop from the workload's first-round shifts, SISO on B's
        # first column with c = b (a symmetric operator then has real reduced
        # poles; a complex pair ends the loop with MORX_E_UNSUPPORTED)
        b0 = Bd[:, 0].contiguous()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_, res = S.irka(list(w.rounds[0]), b0, b0, max_rounds=args.irka,
                          shift_tol=args.irka_tol, prec=w.prec, tol=w.tol, raise_on_error=False)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t1
        rounds = res["rounds"]
        r = len(w.rounds[0])
        ik = {"status": morx.morx_status_str(st_), "rounds": rounds, "shift_tol": args.irka_tol,
              "final_change": res["change"], "seconds": round(dt_, 3),
              "pairs_per_s": round(rounds * r / dt_, 3) if rounds else None,
              "shifts": [round(x, 6) for x in res["sigmas"]],
              "iters_last_round": sum(x.iters for x in res["stats"]),
              "mode": "IRKA (Algorithm 2 shift update), c = b, r = shifts per round"}
        print(f"[irka] {ik['status']} rounds={rounds} {dt_:.2f} s", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(w, apply)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "shifts_per_round": len(w.rounds[0]),
                   "rounds": len(w.rounds), "solves_per_step": nsolves, "precond_storage": w.prec,
                   "precond_apply": apply, "krylov": "f64", "tol": w.tol,
                   "mode": "batched multi-shift", "parallelism": "single GPU",
                   "launch_shapes": tuned or "built-in"},
        "iters_per_step": iters,
        # one step with the system's one-time set-up (host-to-device copy of A
        # and E, morx_system_create, autotune) added to the clock
        "with_setup": {"value": round(nsolves / (dt / args.steps + setup_s), 3),
                       "unit": "solves/s", "setup_s": round(setup_s, 3)},
        "batched_f64_apply": f64_apply,
        "plain": None if plain_value is None else {"value": round(plain_value, 3),
                                                    "unit": "solves/s",
                                                    "iters_per_step": plain_iters,
                                                    "mode": "one shift, one column at a time, "
                                                            "preconditioner applied in FP64"},
        "batched_over_plain": None if plain_value is None else round(value / plain_value, 3),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    if lad is not None:
        out["ladder"] = lad
    if comparators is not None:
        out["comparators"] = comparators
    if moments is not None:
        out["moments"] = moments
    if gm is not None:
        out["gmres"] = gm
    if ik is not None:
        out["irka"] = ik
    print(json.dumps(out), flush=True)
    S.close()
    ctx.close()


if __name__ == "__main__":
    main()
