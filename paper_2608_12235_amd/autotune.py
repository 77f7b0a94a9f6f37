"""Autotuner for the listing skin and the launch tuning (performance only).

Trials continue a running schedule, so no iteration is wasted: for each
candidate the skin (rcp_set_skin) and the tuning (rcp_set_tuning) are
applied and `trial_iters` iterations of every active packing are timed,
list rebuilds included.  The current settings are timed first; a candidate
replaces the best only if its particle-update rate is higher by the factor
MARGIN (trial rates are noisy and the run drifts from trial to trial).  The
search is coordinate-wise: the skin first (it trades list length against
rebuild frequency), then the iteration kernel variant, the work-item cut,
and the graph length.  Results do not depend on any of these beyond
summation order.
"""
import time

from .api import make_tuning

# Candidates around the defaults; every trial runs part of the real
# schedule, so a poor candidate costs its trial's time.
SKINS = (1.0, 2.0, 4.0)
VARIANTS = (64, 65)
WORK_CUTS = ((10, 2560), (16, 4096))
GRAPH_ITERS = (8, 16, 32)
MARGIN = 1.05


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


def tune(packing, trial_iters=200, skins=SKINS, variants=VARIANTS, work_cuts=WORK_CUTS,
         graph_iters=GRAPH_ITERS, log=None):
    """Tune a Packing whose schedule is running (rcp_run_start done).
    Returns (best settings dict, list of (settings, rate)) and leaves the
    best settings applied."""
    trials = []
    g = packing.params.skin_g
    best_t = _copy_tuning(packing.tuning)
    best = {"skin_s": packing.params.skin_s, "variant": best_t.variant,
            "row_cost": best_t.row_cost, "item_work": best_t.item_work,
            "graph_iters": best_t.graph_iters}
    best_rate = -1.0

    def run(settings):
        nonlocal best, best_rate
        t = _copy_tuning(best_t)
        t.variant = settings["variant"]
        t.row_cost, t.item_work = settings["row_cost"], settings["item_work"]
        t.graph_iters = settings["graph_iters"]
        try:
            packing.set_skin(settings["skin_s"], g)
        except Exception as e:   # a skin too large for some box
            if log:
                log("autotune: skip %s (%s)" % (settings, e))
            return True
        packing.set_tuning(t)
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
    # leave the winner applied
    t = _copy_tuning(best_t)
    t.variant, t.row_cost, t.item_work = best["variant"], best["row_cost"], best["item_work"]
    t.graph_iters = best["graph_iters"]
    packing.set_skin(best["skin_s"], g)
    packing.set_tuning(t)
    return best, trials
