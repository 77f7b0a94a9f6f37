"""Whole runs on the GPU against the oracle's stored whole runs (the oracle
takes minutes per run at these sizes; tests/golden/make_oracle_phi.py writes
its results and calls only oracle/).

Trajectories diverge chaotically, so the bar is statistical (the whole-run
bar): over seeds 0-7 the mean final phi is within 0.002 of the oracle's, and
every GPU run stops by the criterion (max overlap below 5e-4 before the
shrink)."""
import json
import os

import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def rcp():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2608_12235_amd as m
    m.lib()
    return m


def test_c2_whole_runs_match_oracle(rcp):
    # power law p = -3 on [1, 20], N = 1e5, RSA at phi0 = 0.05, default schedule
    with open(os.path.join(GOLD, "c2_phi_oracle.json")) as fh:
        gold = json.load(fh)["runs"]
    pg = []
    for g in gold:
        w = ri.c2_powerlaw(seed=g["seed"])
        assert w.n == g["n"]
        p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="rsa")
        r = p.inflate_run()[0]
        p.close()
        print("C2 seed %d: gpu phi %.5f (%d its), oracle %.5f (%d its)" %
              (g["seed"], r["phi"], r["iterations"], g["phi"], g["iterations"]), flush=True)
        assert r["status"] == 0 and r["max_overlap"] < 5e-4, r
        pg.append(r["phi"])
    pg = np.array(pg)
    po = np.array([g["phi"] for g in gold])
    print("phi gpu %.5f +- %.5f oracle %.5f +- %.5f" % (pg.mean(), pg.std(), po.mean(), po.std()))
    assert len(pg) == 8
    assert abs(pg.mean() - po.mean()) <= 0.002
