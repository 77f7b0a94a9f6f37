#!/usr/bin/env python
"""Throughput of the inflation hot path on one MI355X.

Primary workload (the one the line's value and roofline are for): the
dense random state of N = 1e6 spheres, relative diameters from the truncated
lognormal with sigma_lnD = 1.0 and S = 1e3 (equal-probability quantiles),
i.i.d. uniform positions at phi = 0.6 in a periodic cube (overlaps
allowed), FP64 throughout.  One step is one inflation iteration from that
state: energy gradient over the neighbour list, Adam on positions and kappa,
the tail (schedule, stop and validity tests), and a list rebuild whenever
the validity test asks for one.  mu and the step sizes are held at the
values the default schedule's final relaxation rung takes at this state,
the listing skin is 4 D0_min.  The list is built during the W untimed
warm-up iterations; K iterations are then timed with inputs resident in
device memory; value = N x K / wall time (rebuilds in the window included,
and reported separately).

The roofline entry is for the fused gradient + Adam kernel (k_iterate):
algorithmic bytes per launch = (176 + 4) N + 4 nnz (read x, D0, m, v, x_ref
and a row pointer; write x', m, v; 4 bytes per listed partner; partner
gathers assumed cache-served), nnz the listed partners (both directions)
averaged over the timed launches, divided by the kernel's mean duration from
HIP events the library records on its own stream around every launch of
the timed region.  traffic is the HBM bytes per launch from the hardware
counters committed under profiles/ (FETCH_SIZE x 2 + WRITE_SIZE x 1, the
scales measured with a plain copy), null when the kernel sources differ
from the ones the counters were taken on.

Secondary legs run first, each in a child process of its own (before this
process touches the GPU), and are reported as sub-objects: the C2 whole run
(power law p = -3, S = 20, N = 1e5, RSA start at phi0 = 0.05, to the stop
criterion), the RSA-start window of the lognormal S = 1e3 workload, and the
census of 64 packings batched against a loop of plain solves.  The CPU
baseline is the FP64 oracle (OpenMP over rows) on the primary state itself,
gradient + Adam only, timed on every host thread and on one.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-updates/s (Adam iters/s × N) and % HBM peak; batched vs plain loop"
HBM_PEAK_GBS = 8000.0
C5_SKIN = 2048.0   # listing skin of the extreme size-ratio workload, in D0_min
C3_SKIN = 4.0      # listing skin of the primary workload, in D0_min
KERNEL_SOURCES = ["paper_2608_12235_amd/csrc/k_iterate.hip", "paper_2608_12235_amd/csrc/rcp_dev.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iterate_traffic.json")
# algorithmic bytes per sphere update of the gradient + Adam kernel: read x
# (24), D0 (8), m (24), v (24), x_ref (24); write x' (24), m (24), v (24); one
# row pointer (4); plus 4 per listed partner
BYTES_PER_SPHERE = 176.0 + 4.0
BYTES_PER_PARTNER = 4.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(workload):
    """HBM bytes per k_iterate launch from the committed counter summary of
    this workload, or None when the kernel has changed since the counters
    were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("source_sha256") != kernel_source_hash() or t.get("workload") != workload:
        return None, t
    b = 1024.0 * (t["fetch_kib_per_launch"] * t["fetch_scale"] +
                  t["write_kib_per_launch"] * t["write_scale"])
    return b, t


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, d0, L, kappa, eta_x, skin_s, skin_g, target_s=10.0):
    """Oracle gradient + Adam iterations on the host cores (bounded samples)
    on the given state: every host thread, then one thread."""
    import oracle
    oracle.lib()
    threads = oracle.num_threads()
    n = d0.shape[0]
    out = {}
    for label, th in (("all", 0), ("one", 1)):
        t, npairs = oracle.time_iterations(x, d0, L, kappa, eta_x, 1, s=skin_s, g=skin_g,
                                           threads=th)
        per = max(t, 1e-6)
        iters = int(max(2, min(500, target_s / per)))
        t, npairs = oracle.time_iterations(x, d0, L, kappa, eta_x, iters, s=skin_s, g=skin_g,
                                           threads=th)
        out[label] = (n * iters / t, iters, t, npairs)
    v, iters, t, npairs = out["all"]
    v1, iters1, t1, _ = out["one"]
    return {"value": v, "unit": "particle-updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "value_1_thread": v1,
            "sample": "%d gradient+Adam iterations of the FP64 oracle on %d threads (%.1f s) "
                      "and %d on 1 thread (%.1f s), N=%d, the primary state itself (same "
                      "diameters, box, positions and kappa; %d listed pairs; list build "
                      "excluded)" % (iters, threads, t, iters1, t1, n, npairs)}


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
        skin = C5_SKIN if args.skin is None else args.skin
        tun = rcp.make_tuning(row_cost=16, item_work=4096)
        name = "lognormal sigma_lnD=2.5 S=5e5 N=%d" % len(d0)
    else:
        d0 = ri.lognormal_quantiles(args.n, 1.0, 1e3)
        L, seed = ri.box_for_phi(d0, 0.05), 0
        skin = 16.0 if args.skin is None else args.skin
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
    b = BYTES_PER_SPHERE * n + BYTES_PER_PARTNER * nnz
    a = b / (it_us * 1e-6) / 1e9 if it_us > 0 else 0.0
    return {"bound": "hbm", "kernel": "k_iterate", "achieved": a, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": a / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": b,
            "avg_launch_us": it_us, "launches_timed": st["kernel_launches"],
            "nnz_per_sphere": nnz / n}


def _apply_tuning_args(tun, args):
    for k in ("graph_iters", "fused_tail", "row_cost", "item_work", "xcd_remap", "variant"):
        v = getattr(args, k)
        if v is not None:
            setattr(tun, k, v)
    return tun


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
    skin = C5_SKIN if args.skin is None else args.skin
    log("placement (random sequential addition, N=%d, S=%.3g)" % (n, S))
    # the library's work cut (6 / 1536) is the fastest of those measured on
    # this workload: 135 us per iteration launch against 136, 137, 141, 144,
    # 149 and 153 us at 8 / 2048, 10 / 2560, 12 / 3072, 16 / 4096, 24 / 6144
    # and 32 / 8192 (skin 2048, whole runs)
    tun = rcp.make_tuning(time_kernels=1)
    _apply_tuning_args(tun, args)
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


# Table (tab:cap): lognormal width alpha, size ratio S = e^(2 a alpha)
# (the truncation, Eq. (S)), N, the paper's phi and compute minutes on 14
# CPU cores
TABCAP_ROWS = [(0.10, 3.0, 2000, 0.641, 0.0), (0.50, 116.0, 2000, 0.698, 0.1),
               (0.70, 773.0, 8784, 0.735, 0.2), (0.90, 5167.0, 75966, 0.772, 2.9),
               (1.00, 13360.0, 195929, 0.788, 12.8), (1.10, 34544.0, 413799, 0.799, 35.9),
               (1.25, 143631.0, 883556, 0.809, 98.3), (1.30, 230960.0, 1049699, 0.813, 124.2)]


def run_tabcap(torch, args):
    """Every row of Table (tab:cap), one seed: device RSA at phi0 = 0.05,
    the default schedule made `--tabcap-length` times longer, whole runs to
    the stop criterion and the shrink; phi and wall time beside the
    paper's.  Listing skin S / 250 D0_min above S = 1e3 (the largest cutoff
    stays below L / 2 on these rows, whose largest sphere spans about 0.4 L),
    the library default below, and the C5 work cut above S = 1e4."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    rows = [r for k, r in enumerate(TABCAP_ROWS)
            if args.tabcap_rows is None or str(k) in args.tabcap_rows.split(",")]
    out_rows = []
    t_all = time.perf_counter()
    upd = 0
    for alpha, S, n, phi_paper, minutes in rows:
        d0 = ri.lognormal_quantiles(n, alpha, S)
        L = ri.box_for_phi(d0, 0.05)
        Sr = float(d0.max() / d0.min())
        params = rcp.make_params(skin_s=S / 250.0) if S > 1e3 else rcp.make_params()
        tun = rcp.make_tuning(row_cost=16, item_work=4096) if S > 1e4 else rcp.make_tuning()
        sched = rcp.longer_schedule(rcp.default_schedule(n, S=Sr), args.tabcap_length)
        log("tab:cap alpha %.2f S %.6g N %d: placement" % (alpha, S, n))
        t0 = time.perf_counter()
        p = rcp.Packing(d0, L, 1.0, 0, init="rsa_device", params=params, tuning=tun)
        p.run_start(sched)
        while True:
            act = p.run_continue(100000)
            torch.cuda.synchronize()
            log("  %d iterations, %.1f s" % (p.run_result()["iterations"],
                                              time.perf_counter() - t0))
            if act == 0:
                break
        res = p.run_result()
        st = p.stats()
        p.close()
        wall = time.perf_counter() - t0
        upd += n * res["iterations"]
        row = {"alpha": alpha, "S": S, "N": n, "phi": res["phi"], "phi_paper": phi_paper,
               "status": res["status"], "iterations": res["iterations"], "seconds": wall,
               "paper_minutes_14_cores": minutes, "rebuilds": st["rebuilds"]}
        log("  phi %.4f (paper %.3f), %.1f s (paper %.1f min on 14 cores)" %
            (res["phi"], phi_paper, wall, minutes))
        out_rows.append(row)
    wall = time.perf_counter() - t_all
    out = {"metric": METRIC, "value": upd / wall, "unit": "particle-updates/s", "n_gpus": 1,
           "steps": sum(r["iterations"] for r in out_rows), "warmup": 0,
           "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "Table (tab:cap) lognormal rows, seed 0, RSA at phi0=0.05, "
                                  "default schedule x %d" % args.tabcap_length,
                      "rows": out_rows, "seconds": wall}}
    print(json.dumps(out), flush=True)


def run_placement(torch, args):
    """Initial placement of the extreme size-ratio packing (lognormal
    sigma_lnD = 2.5, S = 5e5, N = 3e6, phi0 = 0.05): random sequential
    addition on the host (RCP_INIT_RSA) against the rounds on the GPU
    (rcp_place_device, window RCP_PLACE_WINDOW).  Each time is the context
    creation with that placement minus the creation without placement."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    n = 3_000_000 if args.n == 1_000_000 else args.n
    w = ri.c5_extreme(n=n)
    out = {}
    for label in ("none", "rsa", "device"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if label == "device":
            p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="none")
            rounds = p.place_device(w.seed, rcp._lib.RCP_PLACE_WINDOW)
        else:
            p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init=label)
        torch.cuda.synchronize()
        out[label] = time.perf_counter() - t0
        log("%s: %.3f s" % (label, out[label]))
        p.close()
    res = {"metric": "initial placement time", "value": out["device"] - out["none"], "unit": "s",
           "higher_is_better": False,
           "config": {"workload": "lognormal sigma_lnD=2.5 S=5e5 N=%d at phi0=0.05" % n,
                      "host_rsa_s": out["rsa"] - out["none"],
                      "device_rounds_s": out["device"] - out["none"],
                      "device_rounds": rounds, "window": rcp._lib.RCP_PLACE_WINDOW,
                      "context_without_placement_s": out["none"]}}
    print(json.dumps(res), flush=True)


# ------------------------------------------------------------ secondary legs
def leg_c2(torch, args):
    """Power law p = -3 on [1, 20], N = 1e5, RSA at phi0 = 0.05, seed 0, the
    default schedule run to the stop criterion (whole run, rebuilds and
    shrink included)."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    w = ri.c2_powerlaw(seed=0)
    p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="rsa")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = p.inflate_run()[0]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = p.stats()
    p.close()
    return {"workload": "powerlaw p=-3 S=20 N=%d, RSA start at phi0=0.05, seed 0, default "
                        "schedule, whole run to the stop criterion" % w.n,
            "value": w.n * r["iterations"] / wall, "unit": "particle-updates/s",
            "seconds": wall, "iterations": r["iterations"], "phi_final": r["phi"],
            "status": r["status"], "max_overlap_before_shrink": r["max_overlap"],
            "rebuilds": st["rebuilds"], "rebuild_ms": st["rebuild_ms"]}


def leg_rsa(torch, args):
    """Lognormal S = 1e3, N = 1e6, RSA start at phi0 = 0.05, default
    schedule, listing skin 16 D0_min: iterations 200..2200 of the run."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    n = 1_000_000
    d0 = ri.lognormal_quantiles(n, 1.0, 1e3)
    L = ri.box_for_phi(d0, 0.05)
    tun = rcp.make_tuning(time_kernels=1)
    p = rcp.Packing(d0, L, 1.0, 0, init="rsa", params=rcp.make_params(skin_s=16.0), tuning=tun)
    p.run_start(rcp.default_schedule(n, S=float(d0.max() / d0.min())))
    p.run_continue(200)
    torch.cuda.synchronize()
    p.reset_stats()
    t0 = time.perf_counter()
    p.run_continue(2000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = p.stats()
    p.close()
    rf = _kernel_roofline(st, n)
    return {"workload": "lognormal sigma_lnD=1.0 S=1e3 N=1e6, RSA start at phi0=0.05, default "
                        "schedule, skin 16 D0_min, iterations 200..2200",
            "value": n * st["iterations"] / wall, "unit": "particle-updates/s",
            "k_iterate_us": rf["avg_launch_us"], "k_iterate_frac": rf["frac"],
            "nnz_per_sphere": rf["nnz_per_sphere"], "launches_timed": rf["launches_timed"],
            "rebuilds": st["rebuilds"], "rebuild_ms": st["rebuild_ms"]}


def leg_census(torch, args):
    """C4: 64 packings in one context against a loop of plain solves."""
    import rcp_inputs as ri
    from paper_2608_12235_amd import census
    wl = ri.census_draw(64)
    ntot = sum(w.n for w in wl)
    res_b, tb, st = census.run_batched(wl)
    res_l, tl = census.run_loop(wl)
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        res_a, ta, info = census.run_autotuned(wl, cache=os.path.join(td, "cache.json"))
    phib = np.array([r["phi"] for r in res_b])
    phil = np.array([r["phi"] for r in res_l])
    phia = np.array([r["phi"] for r in res_a])
    ub = census.particle_updates(res_b, wl)
    return {"workload": "census of 64 packings (lognormal / power law / Weibull, S 2..100, "
                        "N 1e3..2e5, sum N %d), whole runs" % ntot,
            "value": ub / tb, "unit": "particle-updates/s",
            "batched_s": tb, "loop_s": tl, "speedup_batched": tl / tb,
            "loop_value": census.particle_updates(res_l, wl) / tl,
            "autotuned_s": ta, "speedup_autotuned": tl / ta,
            "autotune_proxy_tuning_s": info["tuning_s"], "autotune_choice": info["best"],
            "bit_identical_batched_vs_loop": bool(np.array_equal(phib, phil)),
            "mean_phi": float(phib.mean()), "mean_phi_autotuned": float(phia.mean()),
            "statuses": sorted(set(int(r["status"]) for r in res_b)),
            "rebuilds": st["rebuilds"], "rebuild_ms": st["rebuild_ms"]}


def leg_cascade(torch, args):
    """Sequential multimodal cascade (Sec. 4, Table (tab:cascade)): 60
    coarse spheres, diameter ratio 7, three classes (N = 904534), seed 0,
    every stage and release to its stop criterion; phi after each class
    against the paper's 0.624 / 0.800 / 0.879."""
    from paper_2608_12235_amd import cascade
    torch.cuda.synchronize()
    out = cascade.run_cascade(60, 7.0, 3, 0)
    torch.cuda.synchronize()
    # sphere updates: every sphere of a stage's context, per iteration
    upd = 0
    for s in out["stages"]:
        nst = sum(out["counts"][:s["class"]])
        upd += nst * (s["iterations"] + s.get("iterations_frozen_stage", 0))
    return {"workload": "ternary cascade, 60 coarse spheres, diameter ratio 7, counts %s "
                        "(ideal void-filling cascade), seed 0, stages and releases to the stop "
                        "criterion" % out["counts"],
            "value": upd / out["seconds"], "unit": "particle-updates/s",
            "seconds": out["seconds"], "phi": out["phi"], "phi_paper": [0.624, 0.800, 0.879],
            "phi_ideal": [cascade.ideal_phi(c + 1) for c in range(3)],
            "statuses": [s["status"] for s in out["stages"]],
            "iterations": [s["iterations"] for s in out["stages"]],
            "iterations_frozen_stages": [s.get("iterations_frozen_stage") for s in out["stages"]]}


# algorithmic bytes per disk update of the two-coordinate kernel, by the
# same count as BYTES_PER_SPHERE: read x, y (16), D0 (8), m, v (32), x_ref
# (16); write x', y' (16), m, v (32); one row pointer (4); 4 per partner
BYTES_PER_DISK = 124.0


def leg_disks(torch, args):
    """Two dimensions: lognormal sigma_lnD = 1.0, S = 1e3, N = 1e6 disks,
    i.i.d. uniform at area fraction 0.6 (the C3 state in the plane), kappa
    1, mu and the step sizes of the final rung held fixed; 64 + 200
    iterations of the two-coordinate kernel, every launch timed."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    n = 1_000_000
    d0 = ri.lognormal_quantiles(n, 1.0, 1e3)
    L = float(np.sqrt(np.sum(d0 ** 2) / 0.6))   # (pi/4) sum D^2 / L^2 = 0.6
    x = ri.uniform_positions(n, L, 0)[:, :2]
    S = float(d0.max() / d0.min())
    ds = rcp.default_schedule(n, S=S, dim=2)
    r = ds.n_rungs - 1
    sched = rcp.schedule_from_rungs([(ds.mu[r], ds.eta_x[r], ds.eta_k[r], 1.0, 10 ** 6)],
                                    tol=-1.0)
    tun = rcp.make_tuning(graph_iters=64)
    p = rcp.Packing(d0, L, 1.0, 0, init="none", dim=2, tuning=tun,
                    params=rcp.make_params(skin_s=C3_SKIN, skin_g=0.02))
    p.set_state(x, 1.0)
    p.run_start(sched)
    p.run_continue(64)
    torch.cuda.synchronize()
    p.reset_stats()
    t0 = time.perf_counter()
    p.run_continue(200)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tun.time_kernels = 2
    p.set_tuning(tun)
    p.run_continue(64)
    torch.cuda.synchronize()
    p.reset_stats()
    p.run_continue(200)
    torch.cuda.synchronize()
    st = p.stats()
    p.close()
    nl = max(st["kernel_launches"], 1)
    it_us = 1e3 * st["kernel_ms"] / nl
    nnz = st["kernel_nnz"] / nl
    b = BYTES_PER_DISK * n + BYTES_PER_PARTNER * nnz
    return {"workload": "disks: lognormal sigma_lnD=1.0 S=1e3 N=1e6, uniform at area fraction "
                        "0.6, final-rung mu and steps, skin %g D0_min" % C3_SKIN,
            "value": n * 200 / wall, "unit": "particle-updates/s",
            "k_iterate_us": it_us, "bytes_per_launch": b,
            "k_iterate_frac": b / (it_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "tail_us": 1e3 * st["tail_kernel_ms"] / nl, "nnz_per_disk": nnz / n}


def leg_extreme2d(torch, args):
    """The two-dimensional packing of Fig. (extreme): truncated lognormal
    sigma_lnD = 1.3, N = 1e5, S = 8.4e3 realised, device RSA at area fraction
    0.05, seed 0, the default schedule for d = 2 made 8 times longer
    (longer_schedule; the default budgets end at the iteration cap on this
    set), listing skin 256 D0_min; phi after the shrink against the paper's
    0.91."""
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp
    d0 = ri.lognormal_quantiles(100_000, 1.3, 8.55e3)
    S = float(d0.max() / d0.min())
    L = float(np.sqrt(np.pi / 4.0 * np.sum(d0 ** 2) / 0.05))
    s = rcp.longer_schedule(rcp.default_schedule(d0.shape[0], dim=2, S=S), 8)
    t0 = time.perf_counter()
    p = rcp.Packing(d0, L, 1.0, 0, init="rsa_device", dim=2,
                    params=rcp.make_params(skin_s=256.0))
    res = p.inflate_run(s)[0]
    st = p.stats()
    p.close()
    wall = time.perf_counter() - t0
    return {"workload": "2-D truncated lognormal sigma_lnD=1.3 N=1e5 S=%.4g, RSA at area "
                        "fraction 0.05, default d=2 schedule 8 times longer" % S,
            "value": 1e5 * res["iterations"] / wall, "unit": "particle-updates/s",
            "seconds": wall, "iterations": res["iterations"], "phi": res["phi"],
            "phi_paper": 0.91, "status": res["status"], "rebuilds": st["rebuilds"]}


LEGS = {"c2": leg_c2, "rsa": leg_rsa, "census": leg_census, "cascade": leg_cascade,
        "disks": leg_disks, "extreme2d": leg_extreme2d}
LEG_KEYS = {"c2": "c2_whole_run", "rsa": "rsa_start_window", "census": "census",
            "cascade": "cascade", "disks": "disks_2d", "extreme2d": "extreme_2d"}
LEG_TIMEOUT = {"c2": 300, "rsa": 300, "census": 900, "cascade": 600, "disks": 300,
               "extreme2d": 300}


def run_legs(names):
    """Each leg in a child process of its own (started before this process
    initialises the GPU); returns {key: result or error}."""
    out = {}
    for name in names:
        log("leg %s (child process)" % name)
        t0 = time.perf_counter()
        try:
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--leg", name],
                               capture_output=True, text=True, timeout=LEG_TIMEOUT[name])
        except subprocess.TimeoutExpired:
            out[LEG_KEYS[name]] = {"error": "timed out after %d s" % LEG_TIMEOUT[name]}
            continue
        sys.stderr.write(r.stderr)
        res = None
        for line in r.stdout.splitlines():
            if line.startswith("{"):
                res = json.loads(line)
        if r.returncode != 0 or res is None:
            out[LEG_KEYS[name]] = {"error": "exit code %d" % r.returncode}
        else:
            out[LEG_KEYS[name]] = res
        log("leg %s done in %.1f s" % (name, time.perf_counter() - t0))
    return out


# ------------------------------------------------------------ primary
def run_primary(torch, args):
    import rcp_inputs as ri
    import paper_2608_12235_amd as rcp

    w = ri.c3_lognormal_dense(seed=0, n=args.n)
    n, d0, L = w.n, w.d0, w.L
    S = float(d0.max() / d0.min())
    skin = C3_SKIN if args.skin is None else args.skin
    tun = rcp.make_tuning()
    # no timing events in the warmup or the timed region: in a HIP graph each
    # event node adds a dispatch gap of several microseconds
    tun.time_kernels = 0
    _apply_tuning_args(tun, args)
    params = rcp.make_params(skin_s=skin, skin_g=args.skin_g)
    # mu and the step sizes of the default schedule's final rung, held fixed
    # (the budget covers the warmup, the timed region and the kernel-timing
    # pass after it)
    ds = rcp.default_schedule(n, S=S)
    r = ds.n_rungs - 1
    sched = rcp.schedule_from_rungs(
        [(ds.mu[r], ds.eta_x[r], ds.eta_k[r], 1.0, args.warmup + 3 * args.steps + 1)], tol=-1.0)
    log("primary: %s, kappa 1, skin %g D0_min" % (w.name, skin))
    # unless a graph length is asked for, the warmup runs as one graph of
    # `warmup` iterations and the timed region as one graph of `steps`
    # iterations, captured before the clock starts: every launch does work
    graph_fixed = args.graph_iters is not None
    if not graph_fixed and 1 <= args.warmup <= 4096:
        tun.graph_iters = args.warmup
    p = rcp.Packing(d0, L, 1.0, 0, init="none", params=params, tuning=tun)
    torch.cuda.synchronize()
    tu = time.perf_counter()
    p.set_state(w.x, 1.0)       # positions host -> device (N x 3 FP64)
    torch.cuda.synchronize()
    t_up = time.perf_counter() - tu
    p.run_start(sched)
    log("warmup %d iterations" % args.warmup)
    if args.warmup:
        p.run_continue(args.warmup)
    if not graph_fixed:
        tun.graph_iters = min(args.steps, 4096) if args.steps <= 4096 else 32
        p.set_tuning(tun)
        p.run_prepare()
    torch.cuda.synchronize()
    p.reset_stats()
    log("timed %d iterations" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p.run_continue(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st_timed = p.stats()
    st = st_timed
    if args.kernel_timing:
        # kernel-timing pass: `steps` iterations of the same state with HIP
        # events around every launch (kernel_timing 2) or around one launch
        # per graph (1), on the library's stream; the graph with the event
        # nodes runs once untimed first (its first launch is slower)
        log("kernel-timing pass: %d + %d iterations" % (args.steps, args.steps))
        tun.time_kernels = args.kernel_timing
        p.set_tuning(tun)
        p.run_prepare()
        p.run_continue(args.steps)
        torch.cuda.synchronize()
        p.reset_stats()
        p.run_continue(args.steps)
        torch.cuda.synchronize()
        st = p.stats()
    _, _, opt = p.get_optimizer(moments=False)
    res = p.run_result()
    torch.cuda.synchronize()
    td = time.perf_counter()
    xs, kap = p.get_state()     # positions device -> host
    t_down = time.perf_counter() - td
    p.close()
    iters = st_timed["iterations"]
    wall = t1 - t0
    value = n * iters / wall
    log("stats (timed region)", st_timed)
    log("stats (kernel-timing pass)", st)
    rf = _kernel_roofline(st, n)
    nl = max(st["kernel_launches"], 1)
    tail_us = 1e3 * st["tail_kernel_ms"] / nl
    wl_name = "c3_lognormal_S1e3_N%d_phi0.6_uniform" % n
    traffic, tinfo = counter_traffic(wl_name)
    rf["traffic"] = traffic
    rf["traffic_source"] = (tinfo or {}).get("summary") if traffic is not None else None
    phi_now = float(np.pi / 6.0 * kap ** 3 * np.sum(d0 ** 3) / L ** 3)
    log("after the timed region: kappa %.6f phi %.4f max_overlap %.3e; k_iterate %.2f us, tail "
        "%.2f us (mean over %d launches), nnz/N %.3f" %
        (kap, phi_now, res["max_overlap"], rf["avg_launch_us"], tail_us, st["kernel_launches"],
         rf["nnz_per_sphere"]))
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
            "workload": "lognormal sigma_lnD=1.0 S=1e3 N=%d, i.i.d. uniform positions at "
                        "phi=0.6 (kappa 1), 3-D periodic; Adam iterations %d..%d with mu, "
                        "eta_x, eta_k of the default schedule's final rung held fixed; "
                        "listing skin %g D0_min" % (n, args.warmup, args.warmup + iters, skin),
            "n": n,
            "nnz_per_sphere": rf["nnz_per_sphere"],
            "mu": opt["mu"], "eta_x": opt["eta_x"], "eta_k": opt["eta_k"],
            "phi_after_timed_region": phi_now,
            "skin_s": skin,
            "skin_g": args.skin_g,
            "graph_iters": tun.graph_iters,
            "fused_tail": tun.fused_tail,
            "row_cost": tun.row_cost,
            "item_work": tun.item_work,
            "xcd_remap": tun.xcd_remap,
            "variant": tun.variant,
            "rebuilds_in_timed_region": st_timed["rebuilds"],
            "rebuild_ms": st_timed["rebuild_ms"],
            "iterate_ms": st_timed["iterate_ms"],
            "max_degree": st_timed["max_degree"],
            "kernel_timing_pass": "roofline and tail_us: HIP events around every k_iterate and "
                                  "k_tail launch of iterations %d..%d, run right after the timed "
                                  "region and %d untimed iterations with the same graph (the "
                                  "timed region has no event nodes)"
                                  % (args.warmup + 2 * iters, args.warmup + 3 * iters, iters),
            "tail_us": tail_us,
            "kernel_rate": n / (rf["avg_launch_us"] * 1e-6) if rf["avg_launch_us"] > 0 else None,
            # a job that hands over host positions once and reads them back
            # once: the timed region plus those two copies (not `value`)
            "host_transfer_ms": {"positions_in": 1e3 * t_up, "positions_out": 1e3 * t_down},
            "value_with_host_transfers": n * iters / (wall + t_up + t_down),
        },
        "roofline": rf,
    }
    if args.kernel_timing == 0:
        del out["roofline"]
    return out, (w.x, d0, L, 1.0, opt["eta_x"], skin, args.skin_g)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--skin", type=float, default=None,
                    help="listing skin in D0_min (default 4; c5: 2048; --builds: 16)")
    ap.add_argument("--skin-g", type=float, default=0.02)
    ap.add_argument("--graph-iters", dest="graph_iters", type=int, default=None)
    ap.add_argument("--fused-tail", dest="fused_tail", type=int, default=None)
    ap.add_argument("--row-cost", dest="row_cost", type=int, default=None)
    ap.add_argument("--item-work", dest="item_work", type=int, default=None)
    ap.add_argument("--xcd-remap", dest="xcd_remap", type=int, default=None)
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", default="c2,rsa,census,cascade,disks,extreme2d",
                    help="secondary legs run first in child processes (comma list of c2, rsa, "
                         "census, cascade; empty for none)")
    ap.add_argument("--leg", default=None, choices=sorted(LEGS), help=argparse.SUPPRESS)
    ap.add_argument("--kernel-timing", type=int, default=2, choices=(0, 1, 2),
                    help="kernel-timing pass after the timed region (c3 workload), HIP "
                         "events around 0: no launch (no pass, no roofline entry), 1: the "
                         "middle launch of every graph, 2: every launch")
    ap.add_argument("--tabcap-length", dest="tabcap_length", type=int, default=8,
                    help="schedule length factor of --workload tabcap")
    ap.add_argument("--tabcap-rows", dest="tabcap_rows", default=None,
                    help="comma-separated row indices of --workload tabcap (default all)")
    ap.add_argument("--workload", default="c3", choices=("c3", "c5", "placement", "tabcap"),
                    help="c3: the default line; c5: lognormal sigma_lnD=2.5, S=5e5, N=3e6 run "
                         "to the stop criterion; placement: that packing's initial placement "
                         "on the host against the GPU")
    ap.add_argument("--builds", type=int, default=0, metavar="K",
                    help="only time K neighbour-list builds of the RSA-start lognormal (or c5) "
                         "workload after --warmup iterations and exit")
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(the known-size reference for hardware byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(packings shard across GPUs without communication; see the design "
              "notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    legs = {}
    if args.leg is None and args.copy_reference == 0 and args.builds == 0 and \
            args.workload == "c3" and args.legs:
        # before this process initialises the GPU
        legs = run_legs([s for s in args.legs.split(",") if s])

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.leg is not None:
        print(json.dumps(LEGS[args.leg](torch, args)), flush=True)
        return
    if args.copy_reference > 0:
        copy_reference(torch, args.copy_reference)
        return
    if args.builds > 0:
        run_builds(torch, args)
        return
    if args.workload == "c5":
        run_c5(torch, args)
        return
    if args.workload == "placement":
        run_placement(torch, args)
        return
    if args.workload == "tabcap":
        run_tabcap(torch, args)
        return
    out, cpu_state = run_primary(torch, args)
    out.update(legs)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(*cpu_state)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
