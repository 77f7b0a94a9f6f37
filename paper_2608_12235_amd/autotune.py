"""Autotuner for the listing skin and the launch tuning (performance only).

Two ways to use it:

* tune(packing): trials continue a running schedule, so no iteration is
  wasted: for each candidate the skin (rcp_set_skin) and the tuning
  (rcp_set_tuning) are applied and `trial_iters` iterations of every active
  packing are timed, list rebuilds included.

* tune_proxy(workloads) / cached(...): the trials run on a proxy, a context
  of a few of the workloads (the largest ones: they set the iteration time
  of a batch) started from their own placement, so the real run is not held
  up by trials; the winner is stored in a JSON cache keyed by the workload
  signature (sum of N, largest size ratio, number of packings, in
  logarithmic buckets) and the device architecture, and later runs of the
  same kind take it from there without trials.

The current settings are timed first; a candidate replaces the best only if
its particle-update rate is higher by the factor MARGIN (trial rates are
noisy and the run drifts from trial to trial).  The search is
coordinate-wise: the skin first (it trades list length against rebuild
frequency), then the iteration kernel variant, the work-item cut, and the
graph length.  Results do not depend on any of these beyond summation
order.
"""
import json
import math
import os
import time

from .api import Packing, make_params, make_tuning

# Candidates around the defaults; every trial runs part of the real
# schedule, so a poor candidate costs its trial's time.
SKINS = (0.5, 1.0, 2.0)
VARIANTS = (192, 208, 64)
WORK_CUTS = ((8, 2048), (6, 1536), (10, 2560), (16, 4096))
GRAPH_ITERS = (8, 16, 32)
MARGIN = 1.05
CACHE_ENV = "RCP_AUTOTUNE_CACHE"


def _sync():
    import torch
    torch.cuda.synchronize()


def _copy_tuning(t):
    c = make_tuning()
    for f, _ in t._fields_:
        setattr(c, f, getattr(t, f))
    return c


def _trial(packing, trial_iters):
    packing.reset_stats()
    _sync()
    t0 = time.perf_counter()
    active = packing.run_continue(trial_iters)
    _sync()
    dt = time.perf_counter() - t0
    st = packing.stats()
    return st["particle_updates"] / dt if dt > 0 else 0.0, active


def apply(packing, settings):
    """Apply a settings dict (skin_s, variant, row_cost, item_work,
    graph_iters) to a Packing."""
    t = _copy_tuning(packing.tuning)
    t.variant = settings["variant"]
    t.row_cost, t.item_work = settings["row_cost"], settings["item_work"]
    t.graph_iters = settings["graph_iters"]
    packing.set_skin(settings["skin_s"], packing.params.skin_g)
    packing.set_tuning(t)


def tune(packing, trial_iters=200, skins=SKINS, variants=VARIANTS, work_cuts=WORK_CUTS,
         graph_iters=GRAPH_ITERS, log=None):
    """Tune a Packing whose schedule is running (rcp_run_start done).
    Returns (best settings dict, list of (settings, rate)) and leaves the
    best settings applied."""
    trials = []
    best_t = _copy_tuning(packing.tuning)
    best = {"skin_s": packing.params.skin_s, "variant": best_t.variant,
            "row_cost": best_t.row_cost, "item_work": best_t.item_work,
            "graph_iters": best_t.graph_iters}
    best_rate = -1.0

    def run(settings):
        nonlocal best, best_rate
        try:
            apply(packing, settings)
        except Exception as e:   # a skin too large for some box
            if log:
                log("autotune: skip %s (%s)" % (settings, e))
            return True
        rate, active = _trial(packing, trial_iters)
        trials.append((dict(settings), rate))
        if log:
            log("autotune: %s -> %.4g updates/s" % (settings, rate))
        # a candidate must beat the best so far by a margin: trial rates
        # are noisy and the run's conditions drift from trial to trial
        if best_rate < 0 or rate > MARGIN * best_rate:
            best_rate, best = rate, dict(settings)
        return active > 0

    # the current settings first: the baseline every candidate must beat
    if not run(dict(best)):
        return best, trials

    axes = [("skin_s", [(s,) for s in skins]), ("variant", [(v,) for v in variants]),
            ("work", list(work_cuts)), ("graph_iters", [(k,) for k in graph_iters])]
    for name, values in axes:
        for v in values:
            s = dict(best)
            if name == "work":
                s["row_cost"], s["item_work"] = v
            else:
                s[name] = v[0]
            if any(s == t for t, _ in trials):
                continue
            if not run(s):
                break
    apply(packing, best)
    return best, trials


def signature(workloads, arch):
    """Cache key: sum of N (powers of 2), largest size ratio (half decades),
    number of packings (powers of 2) and the device architecture."""
    ntot = sum(w.n for w in workloads)
    smax = max(float(w.d0.max() / w.d0.min()) for w in workloads)
    return "%s|n2^%d|S10^%.1f|p2^%d" % (arch, int(round(math.log2(max(ntot, 1)))),
                                       round(2 * math.log10(max(smax, 1.0))) / 2,
                                       int(round(math.log2(max(len(workloads), 1)))))


def device_arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def tune_proxy(workloads, params=None, tuning=None, n_proxy=4, warmup=500, trial_iters=150,
               log=None):
    """Trials on a proxy context of the n_proxy largest workloads, started
    from their own placement and run `warmup` iterations of the default
    schedule first.  Returns the best settings dict."""
    params = params if params is not None else make_params()
    ws = sorted(workloads, key=lambda w: -w.n)[:n_proxy]
    p = Packing([w.d0 for w in ws], [w.L for w in ws], 1.0, [w.seed for w in ws],
                init="rsa_device", params=params, tuning=tuning)
    try:
        p.run_start(None)
        if warmup:
            p.run_continue(warmup)
        best, _ = tune(p, trial_iters=trial_iters, log=log)
        return best
    finally:
        p.close()


def _cache_path(path):
    if path:
        return path
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache",
                                                      "rcp_autotune.json")


def cached(workloads, path=None, params=None, tuning=None, log=None):
    """Settings for this kind of workload: from the cache when present,
    else from tune_proxy (and stored).  Returns (settings, hit, seconds spent
    tuning)."""
    path = _cache_path(path)
    key = signature(workloads, device_arch())
    try:
        with open(path) as fh:
            cache = json.load(fh)
    except (OSError, ValueError):
        cache = {}
    if key in cache:
        return cache[key], True, 0.0
    t0 = time.perf_counter()
    best = tune_proxy(workloads, params=params, tuning=tuning, log=log)
    dt = time.perf_counter() - t0
    cache[key] = best
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)
    return best, False, dt
