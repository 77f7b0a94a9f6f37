"""Frozen spheres and the sequential multimodal cascade (Sec. 4) on the GPU,
through the C ABI, against the FP64 CPU oracle.

Bars as for the plain protocol: seating bit for bit; energy terms and
gradients within 1e-10 per component relative to the sum of absolute pair
contributions; Adam steps within 1e-9 of the step size per step, frozen
spheres exactly still; whole cascades statistically against the oracle's
stored runs (tests/golden/make_oracle_phi.py).
"""
import json
import os

import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


def _mixed_case(n=4096, S=30.0, phi=0.5, seed=23, frac=0.3):
    w = ri.small_polydisperse(n, S, phi, seed=seed)
    mask = (np.random.default_rng(seed).random(n) < frac).astype(np.uint8)
    return w, mask


def _oracle_mixed_energy(orc, x, d0, mask, L, kappa, mu):
    sig = np.where(mask == 1, d0, kappa * d0)
    pi, pj = (orc.pairs_brute if len(d0) <= 4096 else orc.pairs_cells)(x, sig, L, 1.0, 0.0, 0.0)
    orc.set_frozen(mask)
    try:
        return orc.energy_grad(x, d0, L, kappa, mu, pi, pj)
    finally:
        orc.set_frozen(None)


@pytest.mark.parametrize("kappa", [0.8, 1.3])
def test_frozen_energy_grad_matches_oracle(rcp, orc, kappa):
    w, mask = _mixed_case()
    p = rcp.Packing(w.d0, w.L, 1.0, 0, init="none", params=rcp.make_params(skin_s=0.2))
    p.set_state(w.x, kappa)
    p.set_frozen(mask)
    e = p.energy_grad(mu=1e-3)
    r = _oracle_mixed_energy(orc, w.x, w.d0, mask, w.L, kappa, 1e-3)
    assert r["n_overlap"] > 1000
    err = np.abs(e["g"] - r["g"])
    assert np.all(err <= TOL * r["gscale"]), float(np.max(err / (r["gscale"] + 1e-300)))
    assert e["E_overlap"] == pytest.approx(r["E_ov"], rel=TOL)
    assert e["E_growth"] == pytest.approx(r["E_growth"], rel=TOL)
    assert e["dE_dkappa_overlap"] == pytest.approx(r["gk_ov"], rel=TOL)
    assert e["dE_dkappa_growth"] == pytest.approx(r["gk_growth"], rel=TOL)
    assert e["max_overlap"] == pytest.approx(r["max_delta"], rel=1e-13)
    assert e["n_overlap"] == r["n_overlap"]
    # freeing every sphere gives the plain protocol back
    p.set_frozen(None)
    e0 = p.energy_grad(mu=1e-3)
    pi, pj = orc.pairs_brute(w.x, w.d0, w.L, kappa, 0.0, 0.0)
    r0 = orc.energy_grad(w.x, w.d0, w.L, kappa, 1e-3, pi, pj)
    assert e0["E_overlap"] == pytest.approx(r0["E_ov"], rel=TOL)
    p.close()


@pytest.mark.parametrize("steps,graph", [(1, 1), (10, 16), (25, 4)])
def test_frozen_adam_steps_match_oracle(rcp, orc, steps, graph):
    w, mask = _mixed_case(n=2000, phi=0.55, seed=7)
    kappa, mu, ex, ek = 0.95, 2e-3, 2e-3, 2e-4
    P = orc.default_params(w.d0, s=0.3, g=0.02)
    p = rcp.Packing(w.d0, w.L, 1.0, 0, init="none",
                    params=rcp.make_params(skin_s=0.3, skin_g=0.02, eps_x=P.eps_x),
                    tuning=rcp.make_tuning(graph_iters=graph))
    p.set_state(w.x, kappa)
    p.set_frozen(mask)
    p.adam_step(mu, ex, ek, steps)
    xg, kg = p.get_state()
    p.close()
    orc.set_frozen(mask)
    try:
        st = orc.RunState(w.x, w.d0, w.L, kappa)
        orc.run(st, P, orc.oracle.absolute_schedule(mu, ex, ek, steps))
    finally:
        orc.set_frozen(None)
    fz = mask == 1
    assert np.array_equal(xg[fz], w.x[fz])          # held fixed, bit for bit
    assert np.array_equal(st.x[fz], w.x[fz])
    d = np.abs(xg - st.x)
    d = np.minimum(d, w.L - d)
    assert d.max() <= 1e-9 * ex * steps + 4e-16 * w.L, d.max()
    assert not np.array_equal(xg[~fz], w.x[~fz])    # the others moved
    assert kg == pytest.approx(st.kappa[0], rel=1e-12)


@pytest.mark.parametrize("k0", [0.3, 0.6])
def test_seating_bit_exact(rcp, orc, k0):
    d = np.concatenate([np.ones(40), np.full(20, 0.4)])
    L = float((np.pi / 6.0 * np.sum(d ** 3) / 0.3) ** (1.0 / 3.0))
    xb = orc.rsa(d, L, 1.0, 11)
    nf = 3000
    d0 = np.concatenate([d, np.full(nf, 0.1)])
    mask = np.concatenate([np.ones(d.shape[0], np.uint8), np.zeros(nf, np.uint8)])
    p = rcp.Packing(d0, L, 1.0, 0, init="none")
    p.set_state(np.concatenate([xb, np.zeros((nf, 3))]), 1.0)
    p.set_frozen(mask)
    p.seat(k0, 11)
    xg, kg = p.get_state()
    p.close()
    assert kg == k0
    orc.set_frozen(mask)
    try:
        xo = orc.seat(np.concatenate([xb, np.zeros((nf, 3))]), d0, L, k0, 11)
    finally:
        orc.set_frozen(None)
    assert np.array_equal(xg, xo)


def test_cascade_stage_holds_the_coarse_class(rcp, orc):
    # a frozen stage in full: the coarse spheres do not move, the new class
    # inflates until the stop criterion, the result reports phi unshrunk
    from paper_2608_12235_amd import cascade
    d = np.ones(20)
    L = float((np.pi / 6.0 * 20 / 0.05) ** (1.0 / 3.0))
    par = rcp.make_params(skin_s=0.05)
    p = rcp.Packing(d, L, 1.0, 3, init="rsa", params=par)
    r = p.inflate_run()[0]
    xb, _ = p.get_state()
    p.close()
    sig = d * r["kappa"]
    nf = 800
    dn = 2.0 * sig[0] / 7.0   # twice the nominal size, seated at half the scale
    d0 = np.concatenate([sig, np.full(nf, dn)])
    mask = np.concatenate([np.ones(20, np.uint8), np.zeros(nf, np.uint8)])
    p = rcp.Packing(d0, L, 1.0, 3, init="none", params=par)
    p.set_state(np.concatenate([xb, np.zeros((nf, 3))]), 1.0)
    p.set_frozen(mask)
    p.seat(0.5 * (0.05 / cascade.PHI1) ** (1.0 / 3.0), 3)
    rf = p.inflate_run(rcp.default_schedule(nf, S=1.0))[0]
    x, kf = p.get_state()
    p.close()
    assert rf["status"] == 0 and rf["max_overlap"] < 5e-4
    assert np.array_equal(x[:20], xb)
    assert 0.25 < kf < 1.0
    phi = np.pi / 6.0 * (np.sum(sig ** 3) + nf * (kf * dn) ** 3) / L ** 3
    assert rf["phi"] == pytest.approx(phi, rel=1e-12)
    assert rf["kappa"] == kf


def test_binary_cascade_matches_oracle(rcp):
    # 20 coarse spheres, ratio 7, two classes, seeds 0-7, against the
    # oracle's stored cascades: mean phi of each class within the bar
    from paper_2608_12235_amd import cascade
    with open(os.path.join(GOLD, "cascade_phi_oracle.json")) as fh:
        gold = json.load(fh)
    runs = gold["runs"]
    pg = []
    for g in runs:
        out = cascade.run_cascade(gold["n1"], gold["rho"], gold["classes"], g["seed"])
        assert out["counts"] == g["counts"]
        assert all(s["status"] == 0 for s in out["stages"]), out["stages"]
        _say("cascade seed %d: gpu %s oracle %s" % (g["seed"], np.round(out["phi"], 4),
                                                    np.round(g["phi"], 4)))
        pg.append(out["phi"])
    pg = np.array(pg)
    po = np.array([g["phi"] for g in runs])
    _say("mean phi gpu %s oracle %s; std gpu %s oracle %s" %
         (pg.mean(0), po.mean(0), pg.std(0), po.std(0)))
    # first class: the same placement and schedule; later classes: chaotic
    # divergence, so the bar is the statistical one of the whole runs
    bar = np.maximum(0.004, 3.0 * np.sqrt((pg.var(0) + po.var(0)) / len(runs)))
    assert np.all(np.abs(pg.mean(0) - po.mean(0)) <= bar), (pg.mean(0), po.mean(0), bar)
