#!/usr/bin/env python
"""Throughput of the inflation hot path on one MI355X.

Workload: N = 1e6 relative diameters from the truncated lognormal with
sigma_lnD = 1.0 and S = 1e3 (equal-probability quantiles), placed by random
sequential addition at phi0 = 0.05 in a periodic cube (the paper's dilute,
non-overlapping start), FP64 throughout, the default schedule for that size
ratio.  One step is one inflation iteration: energy gradient over the
neighbour list, Adam on positions and kappa, the tail (schedule, stop and
validity tests), and a list rebuild whenever the validity test asks for
one.  After W untimed iterations, K iterations are timed;
value = N x K / wall time.

The roofline entry is for the fused gradient + Adam kernel (k_iterate):
algorithmic bytes per launch = 188 N + 4 nnz (read x, y, z, D0 as one
32-byte record, m, v, x_ref and a row pointer; write the position record,
m and v; 4 bytes per listed partner; partner gathers are assumed
cache-served), with nnz averaged over the timed launches, divided by the
kernel's mean duration from HIP events the library records on its stream
around the middle launch of every graph of the timed region (one launch in
graph_iters, a uniform sample: event nodes cost a few microseconds each;
--kernel-timing 2 brackets every launch, 0 none and omits the roofline
entry).
traffic is the HBM bytes per launch from the hardware counters committed
under profiles/ (FETCH_SIZE x 2 + WRITE_SIZE x 1, the scales measured with
a plain copy); it is null when the kernel sources differ from the ones the
counters were taken on.  The CPU baseline is the FP64 oracle (OpenMP over
rows) on the same diameters in the same box, gradient + Adam only.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (Adam iters/s × N) and % HBM peak; batched vs plain loop"
HBM_PEAK_GBS = 8000.0
C5_SKIN = 2048.0   # listing skin of the extreme size-ratio workload, in D0_min
KERNEL_SOURCES = ["paper_2608_12235_amd/csrc/k_iterate.hip", "paper_2608_12235_amd/csrc/rcp_dev.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iterate_traffic.json")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per k_iterate launch from the committed counter summary,
    or None when the kernel has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("source_sha256") != kernel_source_hash():
        return None, t
    b = 1024.0 * (t["fetch_kib_per_launch"] * t["fetch_scale"] +
                  t["write_kib_per_launch"] * t["write_scale"])
    return b, t


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(d0, L, phi, skin_s, skin_g, target_s=12.0):
    """Oracle gradient + Adam iterations on the host cores (bounded sample).

    State: the same diameters in the same box, i.i.d. uniform positions
    (seeded generator) at the scale kappa that gives the volume fraction the
    GPU run had reached, so the list density is comparable.
    """
    import oracle
    import rcp_inputs as ri
    oracle.lib()
    threads = oracle.num_threads()
    n = d0.shape[0]
    kappa = float((phi * L ** 3 / (np.pi / 6.0 * np.sum(d0 ** 3))) ** (1.0 / 3.0))
    x = ri.uniform_positions(n, L, 7)
    t, npairs = oracle.time_iterations(x, d0, L, kappa, 1e-2, 2, s=skin_s, g=skin_g)
    per = max(t / 2, 1e-6)
    iters = int(max(3, min(500, target_s / per)))
    t, npairs = oracle.time_iterations(x, d0, L, kappa, 1e-2, iters, s=skin_s, g=skin_g)
    return {"value": n * iters / t, "unit": "particle-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d gradient+Adam iterations of the FP64 oracle, N=%d, same diameters and "
                      "box, uniform positions at phi=%.3f (%d listed pairs; list build "
                      "excluded), %.1f s" % (iters, n, phi, npairs, t)}


def copy_reference(torch, mib):
    """Plain copy of a known size: each launch reads and writes mib MiB."""
    a = torch.empty(mib * 131072, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_mib": mib, "launches": 3}), flush=True)


def run_builds(torch, args):
    """List builds alone: the workload's state after --warmup iterations,
    then --builds rebuilds of its neighbour list timed one by one (the
    profiling target for the build kernels; no iteration in between)."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    if args.workload == "c5":
        w = ri.c5_extreme(n=3_000_000 if args.n == 1_000_000 else args.n)
        d0, L, seed = w.d0, w.L, w.seed
        skin = C5_SKIN if args.skin == 16.0 else args.skin
        tun = rcp.make_tuning(row_cost=16, item_work=4096)
        name = "lognormal sigma_lnD=2.5 S=5e5 N=%d" % len(d0)
    else:
        d0 = ri.lognormal_quantiles(args.n, 1.0, 1e3)
        L, seed, skin = ri.box_for_phi(d0, args.phi0), 0, args.skin
        tun = rcp.make_tuning()
        name = "lognormal sigma_lnD=1.0 S=1e3 N=%d" % len(d0)
    if args.variant is not None:
        tun.variant = args.variant
    S = float(d0.max() / d0.min())
    p = rcp.Packing(d0, L, 1.0, seed, init="rsa", params=rcp.make_params(skin_s=skin),
                    tuning=tun)
    p.run_start(rcp.default_schedule(len(d0), S=S))
    p.run_continue(args.warmup)
    torch.cuda.synchronize()
    it = p.run_result()["iterations"]
    ms = []
    npairs = 0
    for _ in range(args.builds):
        t0 = time.perf_counter()
        npairs = p.neighbor_build()
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
    p.close()
    out = {"metric": "list build time", "value": float(np.mean(ms)), "unit": "ms",
           "higher_is_better": False, "builds": args.builds, "median_ms": float(np.median(ms)),
           "config": {"workload": "%s, RSA start at phi0=0.05, state after %d iterations, "
                                  "skin %g D0_min" % (name, it, skin),
                      "listed_pairs": int(npairs), "variant": int(tun.variant)}}
    print(json.dumps(out), flush=True)


def _kernel_roofline(st, n):
    nl = max(st["kernel_launches"], 1)
    it_us = 1e3 * st["kernel_ms"] / nl
    nnz = st["kernel_nnz"] / nl
    b = 188.0 * n + 4.0 * nnz
    a = b / (it_us * 1e-6) / 1e9 if it_us > 0 else 0.0
    return {"bound": "hbm", "kernel": "k_iterate", "achieved": a, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": a / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": b,
            "avg_launch_us": it_us, "launches_timed": st["kernel_launches"]}


def run_c5(torch, args):
    """Extreme size ratio: one whole run to the stop criterion."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    n = 3_000_000 if args.n == 1_000_000 else args.n
    w = ri.c5_extreme(n=n)
    S = float(w.d0.max() / w.d0.min())
    # listing skin 2048 D0_min: on this workload the gradient kernel hardly
    # slows as the skin grows while rebuilds get rarer (whole runs: 1.18e10
    # updates/s at 256, 1.44e10 at 768, 1.52e10 at 1536, 1.53e10 at 3072,
    # where the kernel starts to slow)
    skin = C5_SKIN if args.skin == 16.0 else args.skin
    log("placement (random sequential addition, N=%d, S=%.3g)" % (n, S))
    # work cut 16 / 4096 measured faster than the library default on this
    # workload (176 against 196 us per iteration launch at skin 2048)
    tun = rcp.make_tuning(time_kernels=1, row_cost=16, item_work=4096)
    if args.row_cost is not None:
        tun.row_cost = args.row_cost
    if args.item_work is not None:
        tun.item_work = args.item_work
    if args.variant is not None:
        tun.variant = args.variant
    p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="rsa", params=rcp.make_params(skin_s=skin),
                    tuning=tun)
    p.run_start(rcp.default_schedule(n, S=S))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        act = p.run_continue(25000)
        torch.cuda.synchronize()
        log("  %d iterations, %.1f s" % (p.run_result()["iterations"], time.perf_counter() - t0))
        if act == 0:
            break
    wall = time.perf_counter() - t0
    st = p.stats()
    res = p.run_result()
    p.close()
    out = {"metric": METRIC, "value": n * res["iterations"] / wall, "unit": "particle-updates/s",
           "n_gpus": 1, "steps": res["iterations"], "warmup": 0,
           "ms_per_step": wall * 1e3 / max(res["iterations"], 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "lognormal sigma_lnD=2.5 S=5e5 N=%d, RSA start at phi0=0.05, "
                                  "3-D periodic, default schedule, whole run" % n,
                      "phi_final": res["phi"], "status": res["status"],
                      "max_overlap_before_shrink": res["max_overlap"], "skin_s": skin,
                      "row_cost": tun.row_cost, "item_work": tun.item_work,
                      "variant": tun.variant,
                      "rebuilds": st["rebuilds"], "rebuild_ms": st["rebuild_ms"],
                      "iterate_ms": st["iterate_ms"]},
           "roofline": _kernel_roofline(st, n)}
    print(json.dumps(out), flush=True)


def run_census(torch, args):
    """C4: 64 packings in one context against a loop of plain solves."""
    import rcp_inputs as ri
    from paper_2608_12235_amd import census
    wl = ri.census_draw(64)
    ntot = sum(w.n for w in wl)
    log("census: 64 packings, sum N = %d; batched" % ntot)
    res_b, tb, st = census.run_batched(wl)
    log("batched %.1f s; loop of plain solves" % tb)
    res_l, tl = census.run_loop(wl)
    log("loop %.1f s; autotuned" % tl)
    res_a, ta, info = census.run_autotuned(wl)
    ub = census.particle_updates(res_b, wl)
    phib = np.array([r["phi"] for r in res_b])
    phil = np.array([r["phi"] for r in res_l])
    phia = np.array([r["phi"] for r in res_a])
    out = {"metric": METRIC, "value": ub / tb, "unit": "particle-updates/s", "n_gpus": 1,
           "steps": int(max(r["iterations"] for r in res_b)), "warmup": 0,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "census of 64 packings (lognormal / power law / Weibull, "
                                  "S 2..100, N 1e3..2e5, sum N %d), whole runs" % ntot,
                      "batched_s": tb, "loop_s": tl, "autotuned_s": ta,
                      "speedup_batched": tl / tb, "speedup_autotuned": tl / ta,
                      "loop_value": census.particle_updates(res_l, wl) / tl,
                      "bit_identical_batched_vs_loop": bool(np.array_equal(phib, phil)),
                      "mean_phi_batched": float(phib.mean()),
                      "mean_phi_autotuned": float(phia.mean()),
                      "autotune_choice": info["best"],
                      "statuses": sorted(set(int(r["status"]) for r in res_b)),
                      "rebuilds_batched": st["rebuilds"], "rebuild_ms_batched": st["rebuild_ms"]}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--phi0", type=float, default=0.05)
    ap.add_argument("--skin", type=float, default=16.0)
    ap.add_argument("--skin-g", type=float, default=0.02)
    ap.add_argument("--graph-iters", type=int, default=None)
    ap.add_argument("--fused-tail", type=int, default=None)
    ap.add_argument("--row-cost", type=int, default=None)
    ap.add_argument("--item-work", type=int, default=None)
    ap.add_argument("--xcd-remap", type=int, default=None)
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-timing", type=int, default=1, choices=(0, 1, 2),
                    help="HIP events around 0: no launch (no roofline entry), 1: the middle "
                         "launch of every graph, 2: every launch")
    ap.add_argument("--workload", default="lognormal", choices=("lognormal", "c5", "census"),
                    help="lognormal: the default line; c5: lognormal sigma_lnD=2.5, S=5e5, "
                         "N=3e6 run to the stop criterion; census: 64 packings batched vs a loop "
                         "of plain solves")
    ap.add_argument("--builds", type=int, default=0, metavar="K",
                    help="only time K neighbour-list builds of the lognormal or c5 workload "
                         "after --warmup iterations and exit")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(the known-size reference for hardware byte counters) and exit")
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
    if args.copy_reference > 0:
        copy_reference(torch, args.copy_reference)
        return
    if args.builds > 0:
        run_builds(torch, args)
        return
    if args.workload == "c5":
        run_c5(torch, args)
        return
    if args.workload == "census":
        run_census(torch, args)
        return
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp

    d0 = ri.lognormal_quantiles(args.n, 1.0, 1e3)
    L = ri.box_for_phi(d0, args.phi0)
    S = float(d0.max() / d0.min())
    tun = rcp.make_tuning()
    tun.time_kernels = args.kernel_timing
    if args.graph_iters is not None:
        tun.graph_iters = args.graph_iters
    if args.fused_tail is not None:
        tun.fused_tail = args.fused_tail
    if args.row_cost is not None:
        tun.row_cost = args.row_cost
    if args.item_work is not None:
        tun.item_work = args.item_work
    if args.xcd_remap is not None:
        tun.xcd_remap = args.xcd_remap
    if args.variant is not None:
        tun.variant = args.variant
    params = rcp.make_params(skin_s=args.skin, skin_g=args.skin_g)
    log("placement (random sequential addition, N=%d)" % args.n)
    p = rcp.Packing(d0, L, 1.0, 0, init="rsa", params=params, tuning=tun)
    p.run_start(rcp.default_schedule(args.n, S=S))
    log("warmup %d iterations" % args.warmup)
    if args.warmup:
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
    value = args.n * iters / wall
    res = p.run_result()
    log("stats", st)
    nl = max(st["kernel_launches"], 1)
    it_us = 1e3 * st["kernel_ms"] / nl
    tail_us = 1e3 * st["tail_kernel_ms"] / nl
    nnz_mean = st["kernel_nnz"] / nl
    alg_bytes = 188.0 * args.n + 4.0 * nnz_mean
    achieved = alg_bytes / (it_us * 1e-6) / 1e9 if it_us > 0 else 0.0
    traffic, tinfo = counter_traffic()
    phi_now = float(np.pi / 6.0 * res["kappa_before_shrink"] ** 3 * np.sum(d0 ** 3) / L ** 3)
    log("state after the timed region: kappa %.6f phi %.4f max_overlap %.3e rung %d; "
        "k_iterate %.1f us, tail %.1f us (mean over %d timed launches)" %
        (res["kappa_before_shrink"], phi_now, res["max_overlap"], res["rung"], it_us, tail_us,
         st["kernel_launches"]))
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
            "workload": "lognormal sigma_lnD=1.0 S=1e3 N=%d, RSA start at phi0=%g, 3-D "
                        "periodic, default schedule, iterations %d..%d" %
                        (args.n, args.phi0, args.warmup, args.warmup + iters),
            "n": args.n,
            "phi_after_timed_region": phi_now,
            "skin_s": args.skin,
            "skin_g": args.skin_g,
            "graph_iters": tun.graph_iters,
            "fused_tail": tun.fused_tail,
            "row_cost": tun.row_cost,
            "item_work": tun.item_work,
            "xcd_remap": tun.xcd_remap,
            "variant": tun.variant,
            "rebuilds_in_timed_region": st["rebuilds"],
            "rebuild_ms": st["rebuild_ms"],
            "iterate_ms": st["iterate_ms"],
            "nnz_mean_per_launch": nnz_mean,
            "max_degree": st["max_degree"],
            "tail_us": tail_us,
            "kernel_rate": args.n / (it_us * 1e-6) if it_us > 0 else None,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_iterate",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": alg_bytes,
            "avg_launch_us": it_us,
            "launches_timed": st["kernel_launches"],
            "traffic_source": (tinfo or {}).get("summary") if traffic is not None else None,
        },
    }
    if args.kernel_timing == 0:
        del out["roofline"]
    p.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(d0, L, phi_now, args.skin, args.skin_g)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
