#!/usr/bin/env python
"""Throughput of the inflation hot path on one MI355X.

Workload: N = 1e6 relative diameters from the truncated lognormal with
sigma_lnD = 1.0 and S = 1e3 (equal-probability quantiles), i.i.d. uniform
positions at phi = 0.6 in a periodic cube, FP64 throughout.  One step is one
inflation iteration of the default schedule's densification rung: energy
gradient over the neighbour list, Adam on positions and kappa, the tail
(schedule, stop and validity tests), and a list rebuild whenever the
validity test asks for one.  value = N x iterations / wall time.

The roofline entry is for the fused gradient + Adam kernel (k_iterate):
algorithmic bytes per launch = 180 N + 4 nnz (read x, D0, m, v, x_ref and
one row pointer, write x, m, v; 4 bytes per listed partner), divided by the
launch's average duration from HIP events recorded by the library on its
stream over the timed region.  The CPU baseline is the FP64 oracle
(OpenMP over rows) on the same state, gradient + Adam only.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (Adam iters/s × N) and % HBM peak; batched vs plain loop"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, skin_s, skin_g, target_s=12.0):
    """Oracle gradient + Adam iterations on the host cores (bounded sample)."""
    import oracle
    oracle.lib()
    threads = oracle.num_threads()
    t, npairs = oracle.time_iterations(w.x, w.d0, w.L, 1.0, 1e-2, 2, s=skin_s, g=skin_g)
    per = max(t / 2, 1e-6)
    iters = int(max(3, min(500, target_s / per)))
    t, npairs = oracle.time_iterations(w.x, w.d0, w.L, 1.0, 1e-2, iters, s=skin_s, g=skin_g)
    return {"value": w.n * iters / t, "unit": "particle-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d gradient+Adam iterations of the FP64 oracle on the same N=%d state "
                      "(list build excluded), %.1f s" % (iters, w.n, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--skin", type=float, default=2.0)
    ap.add_argument("--skin-g", type=float, default=0.02)
    ap.add_argument("--graph-iters", type=int, default=None)
    ap.add_argument("--fused-tail", type=int, default=None)
    ap.add_argument("--heavy-first", type=int, default=None)
    ap.add_argument("--xcd-remap", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(packings shard across GPUs without communication; see the design "
              "notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp

    w = ri.c3_lognormal_dense(seed=0, n=args.n)
    tun = rcp.make_tuning()
    if args.graph_iters is not None:
        tun.graph_iters = args.graph_iters
    if args.fused_tail is not None:
        tun.fused_tail = args.fused_tail
    if args.heavy_first is not None:
        tun.heavy_first = args.heavy_first
    if args.xcd_remap is not None:
        tun.xcd_remap = args.xcd_remap
    params = rcp.make_params(skin_s=args.skin, skin_g=args.skin_g)
    p = rcp.Packing(w.d0, w.L, 1.0, 0, init="none", params=params, tuning=tun)
    p.set_state(w.x, 1.0)
    p.run_start(rcp.default_schedule(w.n))
    log("warmup %d iterations" % args.warmup)
    p.run_continue(args.warmup)
    torch.cuda.synchronize()
    p.reset_stats()
    log("timed %d iterations" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.run_continue(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = p.stats()
    iters = st["iterations"]
    wall = t1 - t0
    value = w.n * iters / wall
    kern_s = st["iterate_ms"] * 1e-3 / max(iters, 1)
    nnz = st["nnz"]
    alg_bytes = 180.0 * w.n + 4.0 * nnz
    achieved = alg_bytes / kern_s / 1e9
    res = p.run_result()
    log("stats", st)
    log("state after timed region: kappa %.6f max_overlap %.3e rung %d" %
        (res["kappa_before_shrink"], res["max_overlap"], res["rung"]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / max(iters, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "lognormal sigma_lnD=1.0 S=1e3 N=%d i.i.d. uniform at phi=0.6, "
                        "3-D periodic, densification rung of the default schedule" % w.n,
            "n": w.n,
            "skin_s": args.skin,
            "skin_g": args.skin_g,
            "graph_iters": tun.graph_iters,
            "fused_tail": tun.fused_tail,
            "heavy_first": tun.heavy_first,
            "xcd_remap": tun.xcd_remap,
            "rebuilds_in_timed_region": st["rebuilds"],
            "rebuild_ms": st["rebuild_ms"],
            "iterate_ms": st["iterate_ms"],
            "nnz": nnz,
            "max_degree": st["max_degree"],
            "kernel_rate": w.n / kern_s,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_iterate",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": alg_bytes,
            "avg_launch_us": kern_s * 1e6,
        },
    }
    p.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, args.skin, args.skin_g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
