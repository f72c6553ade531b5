"""Throughput of the shifted-solve hot path on one MI355X.

One step = the whole job of a workload, with inputs resident on the device
before the clock starts.  The default workload is the largest single-GPU
one, the 128^3 27-point variable-coefficient operator (n = 2,097,152, nnz =
55,742,968, E = diag U[1,2], SISO): 12 shifts log-spaced in [1, 1e4], SPAI at
the first and the column-wise reuse update for every other one (one factor
build of 12 jobs), factors stored in FP64 (the ladder adds FP32 and BF16),
two-sided BiCG to a true relative residual of 1e-10 for all 12 primal + dual
pairs, and the Petrov-Galerkin projection.

Printed JSON (one line): value = shifted solves per second (a solve is one
primal + dual pair meeting 1e-10 on both), batched multi-shift path;
``plain`` is the one-shift-one-column path on the same job; ``roofline`` is
measured on the dominant kernel (the chain step) with HIP events around its
launches in one extra traced step, and carries the HBM traffic measured by
rocprofv3 counters on the same kernel source; ``ladder`` is the same job at
each factor storage precision; ``cpu_baseline`` times the CPU oracle on a
bounded sample on a process pool of the host's cores (the sample is stated).
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
LLC_BYTES = 256e6  # MI355X last-level (Infinity) cache
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
    emin = float(np.min(w.e))
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
        res, ebound = 0.0, 0.0
        for i, sig in enumerate(w.rounds[-1]):
            M = (sig * E - w.A).tocsr()
            for j in range(m):
                k = i * m + j
                rp = np.linalg.norm(w.B[:, j] - M @ X[:, k])
                rd = np.linalg.norm(w.C[:, j] - M.T @ Y[:, k])
                res = max(res, rp / np.linalg.norm(w.B[:, j]), rd / np.linalg.norm(w.C[:, j]))
                # -A has a positive semidefinite symmetric part, so the
                # smallest singular value of s E - A is at least s min(e):
                # ||x - x_exact|| <= ||r|| / (s min(e))
                ebound = max(ebound, rp / (sig * emin * np.linalg.norm(X[:, k])),
                             rd / (sig * emin * np.linalg.norm(Y[:, k])))
        if ref is None:
            ref = (X, Y)
        err = max(float(np.max(np.linalg.norm(X - ref[0], axis=0) / np.linalg.norm(ref[0], axis=0))),
                  float(np.max(np.linalg.norm(Y - ref[1], axis=0) / np.linalg.norm(ref[1], axis=0))))
        its = [x.iters for x in st[-len(w.rounds[-1]) * m:]]
        out[prec] = {"value": round(nsolves / dt, 3), "unit": "solves/s",
                     "iters_per_shift": its, "iters_total": sum(its),
                     "max_true_relres": float(f"{res:.3e}"),
                     "max_rel_error_bound_vs_exact": float(f"{ebound:.3e}"),
                     "max_rel_diff_vs_f64_storage": float(f"{err:.3e}")}
    return out


def check(stats, tol):
    bad = [(k, s.status, s.relres_primal, s.relres_dual) for k, s in enumerate(stats)
           if s.status != 0 or s.relres_primal > tol or s.relres_dual > tol]
    if bad:
        raise SystemExit(f"accuracy check failed: {bad[:5]}")


def _host_cpu():
    """(model name, usable cores) of the host, from /proc/cpuinfo and the
    process's affinity."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


# state the pool's workers inherit (fork), so the large matrices are not copied
_POOL = {}


def _pool_columns(cols):
    """Oracle SPAI columns (single-threaded) for a list of column indices."""
    from threadpoolctl import threadpool_limits

    from oracle import spai as ospai

    g = _POOL
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for k in cols:
            ospai.spai_column(g["A"], g["e"], g["sigma"], int(k), As=g["As"])
        return time.perf_counter() - t0


def _pool_iterations(L):
    """Seconds per oracle BiCG iteration (single-threaded) with a chain of L
    factor passes per direction: the difference of runs with 3 and 1
    iterations, halved."""
    from threadpoolctl import threadpool_limits

    from oracle import bicg as obicg
    from oracle import chain as ochain

    g = _POOL
    F = [g["F"]]
    chain = [0] * L
    As, AsT = g["As_csr"], g["AsT"]
    b, c = g["b"], g["c"]
    with threadpool_limits(limits=1):
        out = []
        for it in (1, 3):
            t0 = time.perf_counter()
            obicg.solve(lambda v: As @ v, lambda v: AsT @ v, b, c,
                        lambda v: ochain.apply(F, chain, v, "f64"),
                        lambda v: ochain.apply_transpose(F, chain, v, "f64"), tol=0.0,
                        maxit=it, max_restarts=0)
            out.append(time.perf_counter() - t0)
    return (out[1] - out[0]) / 2.0


def cpu_sample(w):
    """Time the CPU oracle on a bounded sample of the workload, on a process
    pool of the host's cores (at most 16), each worker single-threaded:
    (a) SPAI columns of the first shift, 1500 per worker, from the oracle's
    column least squares; (b) oracle BiCG iterations on the full system with
    chains of 1 and 3 factor passes (factor values random on the pattern S:
    the cost does not depend on them), every worker at once.  Runs before
    the GPU is touched (the pool forks)."""
    import multiprocessing as mp

    import numpy as np
    import scipy.sparse as sp

    from oracle import pattern as opattern

    model, ncpu = _host_cpu()
    P = max(1, min(16, ncpu))
    sigma = float(w.rounds[0][0])
    As = opattern.shifted_pattern_values(w.A, w.e, sigma)
    rng = np.random.default_rng(5)
    Scsr = As.tocsr()
    fv = rng.standard_normal(Scsr.nnz)
    fv[Scsr.indices == np.repeat(np.arange(w.n), np.diff(Scsr.indptr))] += 3.0
    F = sp.csr_matrix((fv, Scsr.indices, Scsr.indptr), shape=Scsr.shape)
    _POOL.update(A=w.A, e=w.e, sigma=sigma, As=As, As_csr=Scsr, AsT=Scsr.T.tocsr(), F=F,
                 b=np.ascontiguousarray(w.B[:, 0]), c=np.ascontiguousarray(w.C[:, 0]))
    per = 1500
    cols = rng.choice(w.n, P * per, replace=False)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        pool.map(_pool_columns, [cols[k::P] for k in range(P)])
        t_cols = time.perf_counter() - t0
        it1 = pool.map(_pool_iterations, [1] * P)
        it3 = pool.map(_pool_iterations, [3] * P)
    wall = time.perf_counter() - t0
    _POOL.clear()
    t1, t3 = float(np.mean(it1)), float(np.mean(it3))
    tf = max((t3 - t1) / 2.0, 0.0)  # one factor pass per direction
    return {"model": model, "cores": P, "cols_per_s": P * per / t_cols,
            "iter_s_base": max(t1 - tf, 0.0), "iter_s_per_factor": tf, "wall_s": wall}


def cpu_baseline(w, sample, chain_lens, iters, nfactors):
    """The oracle's job time on the pool, from the sample: every factor's n
    column problems at the pool's column rate, then the shifts' BiCG solves
    spread over the workers (longest first), shift i taking iters[i]
    iterations at (base + L_i per-factor) seconds each; value = solves / time."""
    P = sample["cores"]
    t_factor = nfactors * w.n / sample["cols_per_s"]
    load = [0.0] * P
    for t in sorted((it * (sample["iter_s_base"] + L * sample["iter_s_per_factor"])
                     for it, L in zip(iters, chain_lens)), reverse=True):
        load[load.index(min(load))] += t
    t_solve = max(load)
    total = t_factor + t_solve
    return {"value": round(len(iters) / total, 6), "unit": "solves/s", "cores": P,
            "kind": "oracle", "cpu_model": sample["model"],
            "sample": (f"oracle on a pool of {P} single-threaded processes "
                       f"({sample['wall_s']:.1f} s): SPAI column least squares of the first "
                       f"shift ({sample['cols_per_s']:.0f} columns/s over the pool) and BiCG "
                       f"iterations on the full n={w.n} system with chains of 1 and 3 factors "
                       f"({sample['iter_s_base']:.3f} s + {sample['iter_s_per_factor']:.3f} s per "
                       f"factor per iteration, all workers at once); job time = {nfactors} factor "
                       f"builds at that rate ({t_factor:.0f} s) + the {len(iters)} shifts' solves "
                       f"at the GPU run's iteration counts spread over the workers "
                       f"({t_solve:.0f} s)"),
            "projected_job_s": round(total, 1)}


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
        # the host recomputation's own rounding, (w + 2) u (|b| + |M||x|), w <= 8
        rr = np.linalg.norm(b - M @ x)
        slack = 10 * 2.0**-53 * np.linalg.norm(np.abs(b) + abs(M) @ np.abs(x))
        if rr > 1e-10 * np.linalg.norm(b) + slack:
            raise SystemExit(f"serving: request {t} true residual {rr / np.linalg.norm(b)}")
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


def projection_bench(args, w):
    """The Petrov-Galerkin projection alone at the workload's n: r seeded
    random basis columns for V and W, the workload's B and C.  Times
    morx_project with and without orthonormalisation (HIP events around the
    calls, on the library's stream) and prints one JSON line."""
    import torch

    from paper_2003_12759_amd import api, morx

    r = args.projection
    ctx = api.Context(0)
    S = api.System(ctx, w.A, w.e)
    g = torch.Generator(device="cuda").manual_seed(1)
    V = torch.randn(r, w.A.shape[0], generator=g, device="cuda", dtype=torch.float64).t()
    W = torch.randn(r, w.A.shape[0], generator=g, device="cuda", dtype=torch.float64).t()
    Bd, Cd = api.block_to_dev(w.B), api.block_to_dev(w.C)
    out = {}
    for orth in (True, False):
        for _ in range(2):
            S.project(V, W, Bd, Cd, orthonormalize=orth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            S.project(V, W, Bd, Cd, orthonormalize=orth)
        torch.cuda.synchronize()
        out["orth" if orth else "plain"] = 1e3 * (time.perf_counter() - t0) / args.steps
    n, nnz = w.A.shape[0], w.A.nnz
    # W^T A V (A V formed on the fly), W^T E V, W^T B, C^T V: every operand read once
    byts = 8.0 * n * (2 * r + w.B.shape[1] + w.C.shape[1] + 1) + 12.0 * nnz + 4.0 * (n + 1)
    flops = 2.0 * n * r * r * 2 + 2.0 * nnz * r
    line = {"metric": "projection ms per call", "value": round(out["plain"], 3), "unit": "ms",
            "n_gpus": 1, "steps": args.steps, "warmup": 2, "higher_is_better": False,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": w.name, "n": n, "r": r, "m": int(w.B.shape[1]),
                       "q": int(w.C.shape[1])},
            "orthonormalize_ms": round(out["orth"], 3),
            "alg_bytes": byts, "GBps": round(byts / (out["plain"] * 1e-3) / 1e9, 1),
            "TFLOPs": round(flops / (out["plain"] * 1e-3) / 1e12, 3)}
    print(json.dumps(line), flush=True)
    S.close()
    ctx.close()


def second_order_bench(args):
    """AIRGA's solves on the proportionally damped second-order stand-in
    (106^3, 27-point stiffness with a skew part, lumped mass, the paper's
    alpha and beta, four points in [1, 500] and a jittered second round,
    F = C = e_1): every round through morx_solve_second_order with
    ``args.second_order`` moments per point, FP64 factors.  Prints one JSON
    line with second-order solve pairs per second."""
    import torch

    from paper_2003_12759_amd import api
    from paper_2003_12759_amd.workloads import make_second_order

    w = make_second_order()
    nmom = args.second_order
    ctx = api.Context(0)
    S = api.System(ctx, w.A, w.m)
    Fd, Cd = api.block_to_dev(w.F), api.block_to_dev(w.C)
    s0 = float(w.rounds[0][0])
    sig0 = (s0 * s0 + w.alpha * s0) / (1.0 + w.beta * s0)
    t0 = time.perf_counter()
    tuned = S.autotune(sig0, ncols=len(w.rounds[0]))
    tune_s = time.perf_counter() - t0

    def job():
        iters = []
        for z, pts in enumerate(w.rounds):
            _, _, st, stats = S.solve_second_order(w.alpha, w.beta, pts, Fd, Cd, nmom=nmom,
                                                   next_round=z > 0)
            if st != 0:
                raise RuntimeError(f"second-order solve failed in round {z}: status {st}")
            iters += [c.iters for c in stats]
        return iters

    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        iters = job()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    nsolves = sum(len(r) for r in w.rounds) * nmom
    line = {"metric": "second-order solve pairs per second", "value": round(nsolves / ms * 1e3, 3),
            "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 2), "higher_is_better": True, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": w.name, "n": w.n, "points": [list(map(float, r)) for r in w.rounds],
                       "alpha": w.alpha, "beta": w.beta, "moments": nmom, "prec": w.prec,
                       "tol": w.tol},
            "iters": iters, "autotune_s": round(tune_s, 3), "launch_shapes": tuned}
    print(json.dumps(line), flush=True)
    S.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ladder", action="store_true",
                    help="skip the precision ladder of the 27-point workload")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="varcoef27_n2097152",
                    choices=["convdiff3d_n262144", "laplace2d_n2025", "varcoef3d_n1191016_mimo4",
                             "varcoef27_n2097152", "serving_pool16"])
    ap.add_argument("--prec", default=None, choices=[None, "f64", "f32", "bf16"],
                    help="factor storage precision (default: FP64 for the 27-point "
                         "workload, whose ladder adds FP32 and BF16; the workload's otherwise)")
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
    ap.add_argument("--irka-tangential", type=int, default=0,
                    help="also run the MIMO (tangential) IRKA-style loop on all of B's columns "
                         "(C = B) for at most this many rounds")
    ap.add_argument("--irka-tol", type=float, default=1e-4,
                    help="relative change of the shifts that ends the IRKA loop")
    ap.add_argument("--projection", type=int, default=0,
                    help="time only the projection, with this many basis columns")
    ap.add_argument("--second-order", type=int, default=0,
                    help="time only AIRGA's second-order solves (proportional damping) on the "
                         "106^3 stand-in, with this many moments per point")
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

    if args.second_order:
        second_order_bench(args)
        return
    if args.workload == "serving_pool16":
        serving_bench(args)
        return
    index = {"laplace2d_n2025": 0, "convdiff3d_n262144": 1, "varcoef3d_n1191016_mimo4": 2,
             "varcoef27_n2097152": 4}[args.workload]
    w = make_workload(index, prec=args.prec or ("f64" if index == 4 else None))
    if args.projection:
        projection_bench(args, w)
        return
    apply = args.apply or default_apply(w.prec)
    nsolves = sum(len(r) for r in w.rounds) * w.B.shape[1]
    # the CPU oracle's sample runs first: its process pool forks, which is
    # done before anything touches the GPU
    sample = None if args.no_cpu_baseline else cpu_sample(w)
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
        # the instance the library launches, as rocprofv3 names it
        roof_kernel = morx.morx_chain_kernel_name(S.handle, ncol, w.prec, apply)
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
        if byts / launches < LLC_BYTES:
            # one launch's bytes fit the 256 MB last-level cache: the rate is
            # not an HBM rate
            roofline["cache_resident"] = True

    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    lad = (ladder(S, w, Bd, Cd, nsolves)
           if index == 4 and args.prec is None and not args.no_ladder else None)

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

    ikt = None
    if args.irka_tangential > 0:
        # the MIMO (tangential) loop from the workload's first-round shifts on
        # all of B's columns with C = B and equal seeded initial directions (a
        # symmetric operator then has real reduced poles)
        import numpy as np

        m = w.B.shape[1]
        d0 = np.random.default_rng(5).standard_normal((m, len(w.rounds[0])))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st_, res = S.irka_tangential(list(w.rounds[0]), Bd, Bd, d0, d0,
                                     max_rounds=args.irka_tangential, shift_tol=args.irka_tol,
                                     prec=w.prec, tol=w.tol, raise_on_error=False)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t1
        rounds = res["rounds"]
        r = len(w.rounds[0])
        ikt = {"status": morx.morx_status_str(st_), "rounds": rounds,
               "shift_tol": args.irka_tol, "final_change": res["change"],
               "seconds": round(dt_, 3),
               "pairs_per_s": round(rounds * r / dt_, 3) if rounds else None,
               "shifts": [round(x, 6) for x in res["sigmas"]],
               "iters_last_round": sum(x.iters for x in res["stats"]),
               "mode": f"tangential IRKA, m = q = {m}, C = B, r = shifts per round"}
        print(f"[irka-tangential] {ikt['status']} rounds={rounds} {dt_:.2f} s", file=sys.stderr,
              flush=True)

    cpu = None
    if sample is not None:
        from oracle import chain as ochain

        specs, chains = ochain.schedule(w.rounds)
        m = w.B.shape[1]
        lens = [len(chains[z][i]) for z in range(len(w.rounds))
                for i in range(len(w.rounds[z])) for _ in range(m)]
        cpu = cpu_baseline(w, sample, lens, [st.iters for st in last], len(specs))

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
    if ikt is not None:
        out["irka_tangential"] = ikt
    print(json.dumps(out), flush=True)
    S.close()
    ctx.close()


if __name__ == "__main__":
    main()
