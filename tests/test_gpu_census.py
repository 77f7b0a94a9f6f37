"""Batched census (many packings in one context) against plain solves and
against the FP64 oracle.

A packing's trajectory in a census depends only on its own data, so the
batched results must equal the plain solves bit for bit.  phi accuracy:
the 8 smallest packings of the census draw, 8 placement seeds each, batched
on the GPU against the oracle's stored whole runs; mean phi within 0.002 (the
whole-run bar), every GPU run stopped by the criterion."""
import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rcp():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2608_12235_amd as m
    m.lib()
    return m


def _say(*a):
    print(*a, flush=True)


def _smallest(k):
    wl = ri.census_draw(64)
    return sorted(wl, key=lambda w: w.n)[:k]


def test_census_equals_plain_solves(rcp):
    from paper_2608_12235_amd import census
    wl = _smallest(6)
    _say("census of", [w.n for w in wl])
    rb, _, _ = census.run_batched(wl)
    rl, _ = census.run_loop(wl)
    for a, b in zip(rb, rl):
        assert a == b


def test_census_phi_matches_oracle(rcp):
    # the 8 smallest packings of the census draw x 8 placement seeds, batched
    # in one context, against the oracle's whole runs of the same 64 cases
    # (stored by tests/golden/make_oracle_phi.py, which calls only oracle/)
    import json
    import os
    from paper_2608_12235_amd import census
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "census8_phi_oracle.json")) as fh:
        gold = json.load(fh)["runs"]
    base = _smallest(8)
    wl = []
    for w in base:
        for seed in range(8):
            wl.append(type(w)(w.name, w.d0, w.L, w.phi0, 1000 + seed, w.family, w.params))
    assert [(g["n"], g["seed"]) for g in gold] == [(w.n, w.seed) for w in wl]
    _say("census phi check:", len(wl), "packings, N", [w.n for w in base])
    res, _, _ = census.run_batched(wl)
    pg = np.array([r["phi"] for r in res])
    po = np.array([g["phi"] for g in gold])
    for w, r in zip(wl, res):
        assert r["status"] == 0 and r["max_overlap"] < 5e-4, r
    for k, w in enumerate(base):
        a, b = pg[8 * k:8 * k + 8], po[8 * k:8 * k + 8]
        _say("  %s: gpu %.5f +- %.5f oracle %.5f +- %.5f" % (w.name, a.mean(), a.std(),
                                                           b.mean(), b.std()))
    _say("phi gpu %.5f +- %.5f oracle %.5f +- %.5f" % (pg.mean(), pg.std(), po.mean(), po.std()))
    assert abs(pg.mean() - po.mean()) <= 0.002


def test_autotuned_census_phi_matches_oracle(rcp, tmp_path):
    # the same 64 cases with the settings the autotuner finds on a proxy of
    # the largest ones; a second call takes them from the cache
    import json
    import os
    from paper_2608_12235_amd import census
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "census8_phi_oracle.json")) as fh:
        po = np.array([g["phi"] for g in json.load(fh)["runs"]])
    wl = []
    for w in _smallest(8):
        for seed in range(8):
            wl.append(type(w)(w.name, w.d0, w.L, w.phi0, 1000 + seed, w.family, w.params))
    cache = str(tmp_path / "autotune.json")
    res, _, info = census.run_autotuned(wl, cache=cache)
    assert not info["cache_hit"]
    _say("autotuned settings", info["best"], "tuning %.2f s" % info["tuning_s"])
    pg = np.array([r["phi"] for r in res])
    assert all(r["status"] == 0 for r in res)
    _say("phi autotuned %.5f oracle %.5f" % (pg.mean(), po.mean()))
    assert abs(pg.mean() - po.mean()) <= 0.002
    res2, _, info2 = census.run_autotuned(wl, cache=cache)
    assert info2["cache_hit"] and info2["tuning_s"] == 0.0 and info2["best"] == info["best"]
    assert [r["phi"] for r in res2] == [r["phi"] for r in res]


def test_finished_packings_leave_the_work_table(rcp):
    # packings of very different length: the short ones finish first and
    # give up their work items (the iteration grid shrinks); the results are
    # those of plain solves all the same
    from paper_2608_12235_amd import census
    wl = _smallest(6)
    scheds = [rcp.default_schedule(w.n, S=float(w.d0.max() / w.d0.min()), Y=1 + k % 3)
              for k, w in enumerate(wl)]
    rb, _, _ = census.run_batched(wl, schedules=scheds)
    for k, w in enumerate(wl):
        p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="rsa")
        r = p.inflate_run(scheds[k])[0]
        p.close()
        assert r == rb[k], k


def test_census_box_failure_isolated(rcp):
    # a packing whose largest sphere cannot fit its box at the reached scale
    # is stopped with RCP_EBOX while the others finish
    from paper_2608_12235_amd import census
    ok = _smallest(2)
    d0 = np.array([10.0] + [1.0] * 29)
    L = ri.box_for_phi(d0, 0.03)   # fits at kappa = 1, not once phi nears jamming
    bad = type(ok[0])("tight", d0, L, 0.03, 7, "lognormal", {})
    res, _, _ = census.run_batched(ok + [bad])
    assert res[0]["status"] == 0 and res[1]["status"] == 0
    assert res[2]["status"] == -2
