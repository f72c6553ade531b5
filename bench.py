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
WORKLOAD_INDEX = 1
DOMINANT = "chain_step"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_chain_step_convdiff3d_n262144.json")


def kernel_source_hash() -> str:
    """sha256 of the sources of the iteration kernels (bicg.hip, common.h)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("bicg.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2003_12759_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def run_job(S, w, Bd, Cd, batched: bool, use_graph: bool = True):
    stats_all = []
    for z, sig in enumerate(w.rounds):
        X, Y, st, stats = S.solve_shifts(sig, Bd, Cd, prec=w.prec, tol=w.tol, batched=batched,
                                         next_round=z > 0, use_graph=use_graph)
        S.project(X, Y, Bd, Cd)
        stats_all.extend(stats)
    return stats_all


def check(stats, tol):
    bad = [(k, s.status, s.relres_primal, s.relres_dual) for k, s in enumerate(stats)
           if s.status != 0 or s.relres_primal > tol or s.relres_dual > tol]
    if bad:
        raise SystemExit(f"accuracy check failed: {bad[:5]}")


def cpu_baseline(w):
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
                          lambda v: ochain.apply(factors, [0], v),
                          lambda v: ochain.apply_transpose(factors, [0], v), tol=w.tol)
        dt = time.perf_counter() - t0
    assert res.status == "ok"
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one SPAI factor build (n={w.n}, FP32 storage) + one primal+dual "
                      f"BiCG pair solve to 1e-10 ({res.iters} iterations), {dt:.1f} s, "
                      "single-threaded NumPy/SciPy"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the path is one system per GPU); --gpus {args.gpus} "
              "is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2003_12759_amd import api, morx
    from paper_2003_12759_amd.workloads import make_workload

    w = make_workload(WORKLOAD_INDEX)
    nsolves = sum(len(r) for r in w.rounds) * w.B.shape[1]
    ctx = api.Context(0)
    S = api.System(ctx, w.A, w.e)
    Bd = api.block_to_dev(w.B)
    Cd = api.block_to_dev(w.C)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        check(run_job(S, w, Bd, Cd, batched=True), w.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = run_job(S, w, Bd, Cd, batched=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    check(last, w.tol)
    value = nsolves * args.steps / dt

    plain_value = None
    if args.plain_steps > 0:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.plain_steps):
            pst = run_job(S, w, Bd, Cd, batched=False)
        torch.cuda.synchronize()
        check(pst, w.tol)
        plain_value = nsolves * args.plain_steps / (time.perf_counter() - t1)

    roofline, kernels = None, None
    if not args.no_trace:
        morx.morx_trace_enable(ctx.handle, True)
        check(run_job(S, w, Bd, Cd, batched=True), w.tol)
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
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as f:
                tf = json.load(f)
            # counters describe the kernel source they were taken on
            if tf.get("source_sha256") == kernel_source_hash():
                traffic = tf.get("bytes_per_launch")
        ncol = len(w.rounds[0]) * w.B.shape[1]
        chunks = -(-ncol // 8)
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": traffic,
                    "kernel": f"k_chain_step<{ {'f64': 'double', 'f32': 'float', 'bf16': 'unsigned short'}[w.prec]}, {-(-ncol // chunks)}>",
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

    cpu = None if args.no_cpu_baseline else cpu_baseline(w)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "nnz": w.nnz, "shifts_per_round": len(w.rounds[0]),
                   "rounds": len(w.rounds), "solves_per_step": nsolves, "precond_storage": w.prec,
                   "tol": w.tol, "mode": "batched multi-shift", "parallelism": "single GPU"},
        "plain": None if plain_value is None else {"value": round(plain_value, 3),
                                                    "unit": "solves/s",
                                                    "mode": "one shift, one column at a time"},
        "batched_over_plain": None if plain_value is None else round(value / plain_value, 3),
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    S.close()
    ctx.close()


if __name__ == "__main__":
    main()
