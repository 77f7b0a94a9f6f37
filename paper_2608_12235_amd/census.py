"""Batched census: many independent packings in one context.

Every iteration of a census is one launch of the gradient + Adam kernel over
the work items of all packings that are still running, and one tail launch
with a block per packing (each packing keeps its own kappa, Adam state,
schedule and flags), captured in HIP graphs; lists are rebuilt per packing
when its validity test asks for it.  A packing's trajectory depends only on
its own data, so the results equal those of plain solves bit for bit.
"""
import time

import numpy as np

from .api import Packing, make_params, make_tuning


def _sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except ImportError:
        pass


def census_tuning():
    """Library defaults with 8-iteration graphs: small packings ask for a
    list build every few tens of iterations and sit idle for the rest of the
    graph once they have asked (8 and 12 measured best on a 16-packing
    census, against 16 and 32)."""
    return make_tuning(graph_iters=8)


def run_batched(workloads, params=None, tuning=None, schedules=None, max_iters=0):
    """One context for all workloads (objects with d0, L, seed); returns
    (results, seconds of the inflation run, stats)."""
    params = params if params is not None else make_params()
    tuning = tuning if tuning is not None else census_tuning()
    p = Packing([w.d0 for w in workloads], [w.L for w in workloads], 1.0,
                [w.seed for w in workloads], init="rsa", params=params, tuning=tuning)
    try:
        _sync()
        t0 = time.perf_counter()
        res = p.inflate_run(schedules, max_iters=max_iters, allow_fail=True)
        _sync()
        dt = time.perf_counter() - t0
        return res, dt, p.stats()
    finally:
        p.close()


def run_loop(workloads, params=None, tuning=None, schedules=None, max_iters=0, log=None):
    """The same workloads as one plain solve each (library default tuning
    unless given); returns (results, summed seconds of the inflation
    runs)."""
    params = params if params is not None else make_params()
    out, total = [], 0.0
    for k, w in enumerate(workloads):
        p = Packing(w.d0, w.L, 1.0, w.seed, init="rsa", params=params, tuning=tuning)
        try:
            _sync()
            t0 = time.perf_counter()
            r = p.inflate_run(None if schedules is None else schedules[k], max_iters=max_iters,
                              allow_fail=True)[0]
            _sync()
            total += time.perf_counter() - t0
        finally:
            p.close()
        out.append(r)
        if log:
            log("plain solve %d/%d: N=%d phi=%.4f its=%d" % (k + 1, len(workloads), w.n,
                                                              r["phi"], r["iterations"]))
    return out, total


def particle_updates(results, workloads):
    return float(sum(r["iterations"] * w.n for r, w in zip(results, workloads)))


def run_autotuned(workloads, params=None, cache=None, log=None):
    """The batched census with the launch settings the autotuner chose for
    this kind of workload (taken from its cache, or found on a proxy of the
    largest workloads and stored there, see autotune.cached).  Returns
    (results, seconds of the census run, info: settings, cache hit, seconds
    spent tuning)."""
    from . import autotune
    params = params if params is not None else make_params()
    best, hit, t_tune = autotune.cached(workloads, path=cache, params=params,
                                        tuning=census_tuning(), log=log)
    p2 = make_params()
    for f, _ in params._fields_:
        setattr(p2, f, getattr(params, f))
    p2.skin_s = best["skin_s"]
    tun = census_tuning()
    tun.variant = best["variant"]
    tun.row_cost, tun.item_work = best["row_cost"], best["item_work"]
    tun.graph_iters = best["graph_iters"]
    res, dt, st = run_batched(workloads, params=p2, tuning=tun)
    return res, dt, {"best": best, "cache_hit": hit, "tuning_s": t_tune, "stats": st}
