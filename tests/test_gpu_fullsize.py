"""The fused gradient + Adam kernel at full size, and the optimiser state
across calls, against the FP64 oracle (through the C ABI).

Bars (per component; Adam as App. A applies it, Kingma and Ba with bias
correction):
  positions  |dx| <= 1e-10 * eta_x * steps + steps * ulp(x)  (eta_x is the
             largest step a coordinate can take per iteration, and the
             gradient bar of 1e-10 on the sum of |pair contributions| carries
             over to the step; a stored coordinate is known to its own ulp
             only, so each update may round to a neighbouring double);
  moments    |dm| <= 1e-10 * gs,  |dv| <= 2e-10 * gs^2, gs the component's
             largest sum of |pair contributions| over the gradients the run
             evaluated (m and v are averages of g and g^2 over the steps);
  kappa      relative 1e-12.
"""
import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def _true_pairs(orc, x, d0, L, kappa):
    f = orc.pairs_brute if len(d0) <= 4096 else orc.pairs_cells
    return f(x, d0, L, kappa, 0.0, 0.0)


def _gscale(orc, x, d0, L, kappa):
    pi, pj = _true_pairs(orc, x, d0, L, kappa)
    return orc.energy_grad(x, d0, L, kappa, 0.0, pi, pj)["gscale"]


def _check_state(orc, p, st, L, d0, eta_x, steps, gs, label):
    xg, kg = p.get_state()
    mg, vg, opt = p.get_optimizer()
    d = np.abs(xg - st.x)
    d = np.minimum(d, L - d)
    dm = np.abs(mg - st.m)
    dv = np.abs(vg - st.v)
    bx = TOL * eta_x * steps + steps * np.spacing(np.maximum(np.abs(xg), np.abs(st.x)))
    _say("%s: max |dx| %.3g (max |dx|/bar %.3g, %d over 1e-12 eta steps), max |dm|/gs %.3g, "
         "max |dv|/gs^2 %.3g, kappa rel %.3g" %
         (label, d.max(), float(np.max(d / bx)), int((d > 1e-12 * eta_x * steps).sum()),
          float(np.max(dm / (gs + 1e-300))), float(np.max(dv / (gs * gs + 1e-300))),
          abs(kg - st.kappa[0]) / st.kappa[0]))
    assert np.all(d <= bx), label
    assert np.all(dm <= TOL * gs), label
    assert np.all(dv <= 2 * TOL * gs * gs), label
    assert kg == pytest.approx(st.kappa[0], rel=1e-12), label
    assert opt["t"] == st.ctl[0], label
    assert opt["m_kappa"] == pytest.approx(st.mkvk[0], rel=1e-9, abs=1e-300), label
    assert opt["v_kappa"] == pytest.approx(st.mkvk[1], rel=1e-9, abs=1e-300), label


def _steps_vs_oracle(rcp, orc, d0, L, x, kappa, skin, mu, ex, ek, label, tuning=None,
                     boundary=None):
    """One Adam step, then nine more in a second call, from (x, kappa) with
    fresh moments: GPU against the oracle after 1 and after 10 steps (with
    the hard walls `boundary` = (walls, round) on both sides, if given)."""
    P = orc.default_params(d0, s=0.1, g=0.02)
    p = rcp.Packing(d0, L, kappa, 0, init="none",
                    params=rcp.make_params(skin_s=skin, skin_g=0.02, eps_x=P.eps_x),
                    tuning=tuning, boundary=boundary)
    p.set_state(x, kappa)
    st = orc.RunState(x, d0, L, kappa)
    gs = np.zeros((len(d0), 3))
    done = 0
    if boundary is not None:
        orc.set_boundary(*boundary)
    try:
        for k in (1, 9):
            p.adam_step(mu, ex, ek, k)
            st.new_schedule()
            orc.run(st, P, orc.oracle.absolute_schedule(mu, ex, ek, k), gsmax=gs)
            done += k
            _check_state(orc, p, st, L, d0, ex, done, gs, "%s after %d" % (label, done))
    finally:
        orc.set_boundary(0, 0)
    stats = p.stats()
    p.close()
    return stats


def test_c3_state_adam_steps_full_size(rcp, orc):
    # the primary bench state and launch configuration: N = 1e6 lognormal
    # S = 1e3 at phi = 0.6, skin 4 D0_min, default tuning
    w = ri.c3_lognormal_dense(seed=0)
    _say("C3 full-size Adam steps")
    st = _steps_vs_oracle(rcp, orc, w.d0, w.L, w.x, 1.0, 4.0, 1e-6, 0.0125, 1e-4, "C3")
    assert st["rebuilds"] == 1 and st["nnz"] > 2_000_000


def test_c3_state_in_a_walled_box_adam_steps_full_size(rcp, orc):
    # the same state and launch shape with flat walls across every axis
    # (the walls instantiation of the kernel: wall terms in the Adam phase,
    # no images), and in a cylinder along z (round over x and y)
    w = ri.c3_lognormal_dense(seed=0)
    for bnd, label in (((7, 0), "C3 walled box"), ((4, 3), "C3 cylinder")):
        _say("%s full-size Adam steps" % label)
        st = _steps_vs_oracle(rcp, orc, w.d0, w.L, w.x, 1.0, 4.0, 1e-6, 0.0125, 1e-4, label,
                              boundary=bnd)
        assert st["rebuilds"] == 1 and st["nnz"] > 2_000_000


@pytest.fixture(scope="module")
def c5dense():
    # C5's size distribution (lognormal sigma_lnD = 2.5, S = 5e5) at N = 5e5,
    # i.i.d. uniform at phi = 0.6: rows of hundreds of partners, ten grid
    # levels at the library's default skin
    n = 500_000
    d0 = ri.lognormal_quantiles(n, 2.5, 5e5)
    L = ri.box_for_phi(d0, 0.6)
    x = ri.uniform_positions(n, L, 13)
    return d0, L, x


def test_c5_distribution_dense_pairs_energy(rcp, orc, c5dense):
    d0, L, x = c5dense
    _say("C5 distribution dense: pairs and energy")
    p = rcp.Packing(d0, L, 1.0, 0, init="none", params=rcp.make_params(skin_s=0.5))
    p.set_state(x, 1.0)
    npairs = p.neighbor_build()
    assert p.stats()["levels"] >= 8
    gi, gj = p.pairs()
    oi, oj = orc.pairs_cells(x, d0, L, 1.0, 0.5, 0.02)
    assert npairs == len(oi) and np.array_equal(gi, oi) and np.array_equal(gj, oj)
    e = p.energy_grad(mu=1e-3)
    pi, pj = _true_pairs(orc, x, d0, L, 1.0)
    r = orc.energy_grad(x, d0, L, 1.0, 1e-3, pi, pj)
    err = np.abs(e["g"] - r["g"])
    assert np.all(err <= TOL * r["gscale"]), float(np.max(err / (r["gscale"] + 1e-300)))
    assert e["E_overlap"] == pytest.approx(r["E_ov"], rel=TOL)
    assert e["dE_dkappa_overlap"] == pytest.approx(r["gk_ov"], rel=TOL)
    assert e["n_overlap"] == r["n_overlap"]
    p.close()


def test_c5_distribution_dense_adam_steps(rcp, orc, c5dense):
    d0, L, x = c5dense
    _say("C5 distribution dense: Adam steps")
    st = _steps_vs_oracle(rcp, orc, d0, L, x, 1.0, 0.5, 1e-6, 0.005, 1e-4, "C5 dense")
    assert st["levels"] >= 8


def _dense_c1(orc, iters=1500):
    w = ri.c1_lognormal(0)
    x0 = orc.rsa(w.d0, w.L, 1.0, w.seed)
    st = orc.RunState(x0, w.d0, w.L, 1.0)
    orc.run(st, orc.default_params(w.d0, s=0.3, g=0.02), orc.default_schedule(w.n),
            max_iters=iters)
    return w, st.x.copy(), float(st.kappa[0])


def test_adam_step_calls_carry_the_moments(rcp, orc):
    # adam_step(a) then adam_step(b) continues the moments and the step
    # counter: the oracle runs the same two calls on one resumed state
    w, x, k = _dense_c1(orc)
    mu, ex, ek = 2e-3, 2e-3, 2e-4
    P = orc.default_params(w.d0, s=0.3, g=0.02)
    p = rcp.Packing(w.d0, w.L, k, 0, init="none",
                    params=rcp.make_params(skin_s=0.3, skin_g=0.02, eps_x=P.eps_x))
    p.set_state(x, k)
    m0, v0, o0 = p.get_optimizer()
    assert o0["t"] == 0 and not m0.any() and not v0.any()
    st = orc.RunState(x, w.d0, w.L, k)
    gs = np.zeros((w.n, 3))
    done = 0
    for n in (4, 6, 1):
        p.adam_step(mu, ex, ek, n)
        st.new_schedule()
        orc.run(st, P, orc.oracle.absolute_schedule(mu, ex, ek, n), gsmax=gs)
        done += n
        _check_state(orc, p, st, w.L, w.d0, ex, done, gs, "C1 calls %d" % done)
    p.close()


def test_optimizer_checkpoint_resumes_adam_steps(rcp, orc):
    w, x, k = _dense_c1(orc)
    mu, ex, ek = 2e-3, 2e-3, 2e-4
    mk = lambda: rcp.Packing(w.d0, w.L, k, 0, init="none",
                             params=rcp.make_params(skin_s=0.3, skin_g=0.02))
    a = mk()
    a.set_state(x, k)
    a.adam_step(mu, ex, ek, 12)
    xa, ka = a.get_state()
    b = mk()
    b.set_state(x, k)
    b.adam_step(mu, ex, ek, 5)
    xb, kb = b.get_state()
    mb, vb, ob = b.get_optimizer()
    b.close()
    c = mk()
    c.set_state(xb, kb)
    c.set_optimizer(ob, mb, vb)
    m2, v2, o2 = c.get_optimizer()
    assert np.array_equal(m2, mb) and np.array_equal(v2, vb) and o2 == ob
    c.adam_step(mu, ex, ek, 7)
    xc, kc = c.get_state()
    d = np.abs(xc - xa)
    d = np.minimum(d, w.L - d)
    assert np.all(d <= TOL * ex * 7 + 7 * np.spacing(np.abs(xa))), d.max()
    assert kc == pytest.approx(ka, rel=1e-12)
    a.close()
    c.close()


def test_optimizer_checkpoint_resumes_a_run(rcp, orc):
    # a run checkpointed mid-schedule (positions, kappa, moments, rung
    # position) and resumed in a new context follows the uninterrupted run
    w, x, k = _dense_c1(orc, iters=600)
    rungs = [(1e-2, 1e-2, 1e-3, 1.0, 40), (1e-3, 5e-3, 5e-4, 0.98, 40),
             (1e-5, 2e-3, 1e-4, 0.99, 40)]
    sched = rcp.schedule_from_rungs(rungs, tol=-1.0)
    mk = lambda: rcp.Packing(w.d0, w.L, k, 0, init="none",
                             params=rcp.make_params(skin_s=0.3, skin_g=0.02))
    a = mk()
    a.set_state(x, k)
    a.run_start(sched)
    a.run_continue(70)
    xa, ka = a.get_state()
    ma, va, oa = a.get_optimizer()
    assert oa["rung"] == 1 and oa["it_rung"] == 30 and oa["iterations"] == 70 and oa["t"] == 70
    a.run_continue(30)
    xa2, ka2 = a.get_state()
    b = mk()
    b.set_state(xa, ka)
    b.run_start(sched)
    b.set_optimizer(oa, ma, va)
    b.run_continue(30)
    xb, kb = b.get_state()
    _, _, ob = b.get_optimizer(moments=False)
    assert ob["iterations"] == 100 and ob["rung"] == 2 and ob["it_rung"] == 20
    d = np.abs(xb - xa2)
    d = np.minimum(d, w.L - d)
    assert np.all(d <= TOL * 1e-2 * k * 30 + 30 * np.spacing(np.abs(xa2))), d.max()
    assert kb == pytest.approx(ka2, rel=1e-12)
    a.close()
    b.close()


def test_optimizer_set_rejects_bad_values(rcp):
    w = ri.c1_lognormal(0)
    p = rcp.Packing(w.d0, w.L, 1.0, w.seed, init="rsa")
    _, _, o = p.get_optimizer(moments=False)
    for f, bad in (("t", -1), ("rung", 1), ("v_kappa", -1.0), ("mu", float("nan"))):
        oo = dict(o)
        oo[f] = bad
        with pytest.raises(rcp.RcpError):
            p.set_optimizer(oo)
    v = np.zeros((w.n, 3))
    v[3, 1] = -1.0
    with pytest.raises(rcp.RcpError):
        p.set_optimizer(o, None, v)
    p.close()


def test_every_overlapping_pair_is_listed_or_a_rebuild_follows(rcp, orc):
    # list validity (App. A rebuilds on accumulated displacement): after each
    # step either every overlapping pair of the new state is in the current
    # list, or the next call rebuilds before its gradient
    w, x, k = _dense_c1(orc)
    p = rcp.Packing(w.d0, w.L, k, 0, init="none",
                    params=rcp.make_params(skin_s=0.02, skin_g=0.002))
    p.set_state(x, k)
    p.adam_step(2e-3, 5e-3, 5e-4, 1)
    missed = 0
    for it in range(60):
        xs, ks = p.get_state()
        oi, oj = orc.pairs_brute(xs, w.d0, w.L, ks, 0.0, 0.0)
        gi, gj = p.pairs()
        listed = set(zip(gi.tolist(), gj.tolist()))
        ok = all(pr in listed for pr in zip(oi.tolist(), oj.tolist()))
        before = p.stats()["rebuilds"]
        p.adam_step(2e-3, 5e-3, 5e-4, 1)
        if not ok:
            missed += 1
            assert p.stats()["rebuilds"] > before, it
    _say("steps whose list had to be rebuilt before the next gradient:", missed)
    assert p.stats()["rebuilds"] > 3
    p.close()


def test_disks_state_adam_steps_full_size(rcp, orc):
    # the C3 state in the plane (N = 1e6 disks, area fraction 0.6) through the
    # kernel instantiated for two coordinates, against the oracle in 2-D
    n = 1_000_000
    d0 = ri.lognormal_quantiles(n, 1.0, 1e3)
    L = float(np.sqrt(np.sum(d0 ** 2) / 0.6))
    x = np.column_stack([ri.uniform_positions(n, L, 0)[:, :2], np.zeros(n)])
    mu, ex, ek = 1e-6, 0.0125, 1e-4
    P = orc.default_params(d0, s=0.1, g=0.02)
    p = rcp.Packing(d0, L, 1.0, 0, init="none", dim=2,
                    params=rcp.make_params(skin_s=4.0, skin_g=0.02, eps_x=P.eps_x))
    p.set_state(x[:, :2], 1.0)
    orc.set_dim(2)
    try:
        st = orc.RunState(x, d0, L, 1.0)
        gs = np.zeros((n, 3))
        done = 0
        for k in (1, 9):
            p.adam_step(mu, ex, ek, k)
            st.new_schedule()
            orc.run(st, P, orc.oracle.absolute_schedule(mu, ex, ek, k), gsmax=gs)
            done += k
            xg, kg = p.get_state()
            mg, vg, _ = p.get_optimizer()
            d = np.abs(xg - st.x[:, :2])
            d = np.minimum(d, L - d)
            bx = TOL * ex * done + done * np.spacing(np.maximum(np.abs(xg), np.abs(st.x[:, :2])))
            _say("disks after %d: max |dx|/bar %.3g, max |dm|/gs %.3g" %
                 (done, float(np.max(d / bx)),
                  float(np.max(np.abs(mg - st.m[:, :2]) / (gs[:, :2] + 1e-300)))))
            assert np.all(d <= bx)
            assert np.all(np.abs(mg - st.m[:, :2]) <= TOL * gs[:, :2])
            assert np.all(np.abs(vg - st.v[:, :2]) <= 2 * TOL * gs[:, :2] ** 2)
            assert np.all(st.x[:, 2] == 0.0)
            assert kg == pytest.approx(st.kappa[0], rel=1e-12)
    finally:
        orc.set_dim(3)
    assert p.stats()["nnz"] > 1_000_000
    p.close()
