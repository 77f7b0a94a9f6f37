"""Hard walls (Sec. 2: flat or curved hard walls per axis) on the GPU,
through the C ABI, against the FP64 CPU oracle with the same boundary.

Bars as for the periodic box: placements, pair sets and shrink scales bit
for bit; energy terms and gradients within 1e-10 per component relative to
the sum of absolute contributions; Adam steps within 1e-9 of the step size
per step; whole runs statistically (mean phi over 8 seeds); a census that
mixes a walled and a periodic packing bit-identical to separate runs.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-10
X, Y, Z = 1, 2, 4
BOUNDS = [(X | Y | Z, 0), (X, 0), (0, X | Y | Z), (Z, X | Y)]


@pytest.fixture(scope="module")
def rcp():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2608_12235_amd as m
    m.lib()
    return m


@pytest.fixture
def orw(orc):
    yield orc
    orc.set_boundary(0, 0)
    orc.set_dim(3)


def _say(*a):
    print(*a, flush=True)


def _poly(n, L, seed, lo=0.5, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, n), L


@pytest.mark.parametrize("walls,round_axes", BOUNDS)
def test_walled_placement_bit_exact(rcp, orw, walls, round_axes):
    d0, L = _poly(3000, 40.0, seed=walls * 8 + round_axes)
    _say("walled placement walls=%d round=%d" % (walls, round_axes))
    p = rcp.Packing(d0, L, 1.0, 21, init="rsa_device", boundary=(walls, round_axes))
    xg, _ = p.get_state()
    p.close()
    orw.set_boundary(walls, round_axes)
    xo, _ = orw.rsa_rounds(d0, L, 1.0, 21, rcp._lib.RCP_PLACE_WINDOW)
    assert np.array_equal(xg, xo)


def test_walled_placement_2d_circle(rcp, orw):
    # 2000 disks at area fraction 0.1 in the circle (pi/4) L^2
    d0, _ = _poly(2000, 0.0, seed=3)
    L = float(math.sqrt(np.sum(d0 ** 2) / 0.1))
    p = rcp.Packing(d0, L, 1.0, 5, init="rsa_device", dim=2, boundary=(0, X | Y))
    xg, _ = p.get_state()
    p.close()
    orw.set_dim(2)
    orw.set_boundary(0, X | Y)
    xo, _ = orw.rsa_rounds(d0, L, 1.0, 5, rcp._lib.RCP_PLACE_WINDOW)
    assert np.array_equal(xg, xo[:, :2])
    r = np.sqrt(np.sum((xg - 0.5 * L) ** 2, 1))
    assert np.all(r <= 0.5 * (L - d0))


def _overlapping_state(n, L, seed, bounded, spill=0.3):
    # positions spill past the walls by up to `spill` (the list build must
    # clamp them into the end cells), diameters 0.8-1.6, many overlaps;
    # periodic axes wrapped into [0, L) as the library stores them
    rng = np.random.default_rng(seed)
    x = rng.uniform(-spill, L + spill, (n, 3))
    for a in range(3):
        if not (bounded >> a) & 1:
            x[:, a] = np.where(x[:, a] < 0.0, x[:, a] + L, x[:, a])
            x[:, a] = np.where(x[:, a] >= L, x[:, a] - L, x[:, a])
    d0 = rng.uniform(0.8, 1.6, n)
    return x, d0


@pytest.mark.parametrize("walls,round_axes", BOUNDS)
def test_walled_pairs_energy_gradient(rcp, orw, walls, round_axes):
    L, kappa, mu = 14.0, 1.05, 2e-3
    x, d0 = _overlapping_state(3000, L, walls + 8 * round_axes, walls | round_axes)
    _say("walled energy walls=%d round=%d" % (walls, round_axes))
    p = rcp.Packing(d0, L, 1.0, 0, init="none", boundary=(walls, round_axes),
                    params=rcp.make_params(skin_s=0.2, skin_g=0.02))
    p.set_state(x, kappa)
    p.neighbor_build()
    gi, gj = p.pairs()
    orw.set_boundary(walls, round_axes)
    oi, oj = orw.pairs_brute(x, d0, L, kappa, 0.2, 0.02)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    e = p.energy_grad(mu=mu)
    ai, aj = orw.pairs_brute(x, d0, L, kappa, 0.0, 0.0)
    r = orw.energy_grad(x, d0, L, kappa, mu, ai, aj)
    p.close()
    assert r["n_overlap"] > 1000
    err = np.abs(e["g"] - r["g"])
    assert np.all(err <= TOL * r["gscale"]), float(np.max(err / (r["gscale"] + 1e-300)))
    assert e["E_overlap"] == pytest.approx(r["E_ov"], rel=TOL)
    assert e["dE_dkappa_overlap"] == pytest.approx(r["gk_ov"], rel=TOL)
    assert e["max_overlap"] == pytest.approx(r["max_delta"], rel=1e-13)
    assert e["n_overlap"] == r["n_overlap"]


@pytest.mark.parametrize("walls,round_axes,steps,graph",
                         [(X | Y | Z, 0, 1, 1), (X | Y | Z, 0, 10, 16), (0, X | Y | Z, 10, 4),
                          (Z, X | Y, 25, 16)])
def test_walled_adam_steps_match_oracle(rcp, orw, walls, round_axes, steps, graph):
    L = 12.0
    x, d0 = _overlapping_state(1500, L, 9, walls | round_axes, spill=0.2)
    mu, ex, ek = 2e-3, 2e-3, 2e-4
    P = orw.default_params(d0, s=0.3, g=0.02)
    p = rcp.Packing(d0, L, 1.0, 0, init="none", boundary=(walls, round_axes),
                    params=rcp.make_params(skin_s=0.3, skin_g=0.02, eps_x=P.eps_x),
                    tuning=rcp.make_tuning(graph_iters=graph))
    p.set_state(x, 0.95)
    p.adam_step(mu, ex, ek, steps)
    xg, kg = p.get_state()
    p.close()
    orw.set_boundary(walls, round_axes)
    st = orw.RunState(x, d0, L, 0.95)
    orw.run(st, P, orw.oracle.absolute_schedule(mu, ex, ek, steps))
    d = np.abs(xg - st.x)
    per = [not ((walls | round_axes) >> a & 1) for a in range(3)]
    for a in range(3):
        if per[a]:
            d[:, a] = np.minimum(d[:, a], L - d[:, a])
    assert d.max() <= 1e-9 * ex * steps + 4e-16 * L, d.max()
    assert kg == pytest.approx(st.kappa[0], rel=1e-12)
    # positions past a wall stay there (no wrap)
    b = [a for a in range(3) if not per[a]]
    assert np.any(xg[:, b] < 0.0)


def test_walled_shrink_lattices(rcp, orw):
    # cubic lattice touching the walls of a box: kappa' = 1, phi = pi / 6
    n = 5
    g = np.arange(n) + 0.5
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = rcp.Packing(np.ones(n ** 3), float(n), 1.0, 0, init="none", boundary=(X | Y | Z, 0),
                    params=rcp.make_params(skin_s=0.05, skin_g=0.02))
    p.set_state(x, 1.3)
    kp, phi = p.shrink()
    p.close()
    assert kp == 1.0 and phi == pytest.approx(math.pi / 6.0, rel=1e-15)
    # one sphere at the centre of a ball fills it
    p = rcp.Packing(np.ones(1), 10.0, 1.0, 0, init="none", boundary=(0, X | Y | Z),
                    params=rcp.make_params(skin_s=0.05, skin_g=0.02))
    p.set_state(np.array([[5.0, 5.0, 5.0]]), 4.0)
    kp, phi = p.shrink()
    p.close()
    assert kp == 4.0     # capped by the current kappa
    # seven disks in a circle of diameter 3: the oracle's scale, bit for bit
    t = np.arange(6) * math.pi / 3.0
    xd = np.full((7, 2), 1.5)
    xd[1:, 0] += np.cos(t)
    xd[1:, 1] += np.sin(t)
    p = rcp.Packing(np.ones(7), 3.0, 1.0, 0, init="none", dim=2, boundary=(0, X | Y),
                    params=rcp.make_params(skin_s=0.05, skin_g=0.02))
    p.set_state(xd, 1.2)
    kp, phi = p.shrink()
    p.close()
    orw.set_dim(2)
    orw.set_boundary(0, X | Y)
    x3 = np.column_stack([xd, np.zeros(7)])
    pi, pj = orw.pairs_brute(x3, np.ones(7), 3.0, 1.2, 0.0, 0.0)
    ko = orw.shrink(x3, np.ones(7), 3.0, 1.2, pi, pj)
    assert kp == ko and abs(kp - 1.0) < 4e-16
    assert phi == orw.phi(np.ones(7), 3.0, ko)


@pytest.mark.parametrize("walls,round_axes", [(X | Y | Z, 0), (0, X | Y | Z)])
def test_walled_whole_runs_match_oracle(rcp, orw, walls, round_axes):
    # 50:50 spheres of diameter ratio 1.4, N = 256, device RSA at phi0 = 0.1
    # in a walled cube and in a ball, default schedule, seeds 0-7: mean phi
    # within the statistical bar; every final state clear of the walls and
    # of every other sphere at kappa'
    n = 256
    d0 = np.where(np.arange(n) % 2 == 0, 1.0, 1.4)
    vol = math.pi / 6.0 * np.sum(d0 ** 3) / 0.1
    L = float((vol / (1.0 if round_axes == 0 else math.pi / 6.0)) ** (1.0 / 3.0))
    orw.set_boundary(walls, round_axes)
    pg, po = [], []
    for seed in range(8):
        p = rcp.Packing(d0, L, 1.0, seed, init="rsa_device", boundary=(walls, round_axes))
        r = p.inflate_run()[0]
        x, _ = p.get_state()
        kp = r["kappa"]
        p.close()
        assert r["status"] == 0 and r["max_overlap"] < 5e-4, r
        pi, pj = orw.pairs_brute(x, d0, L, kp, 0.0, 0.0)
        q = orw.energy_grad(x, d0, L, kp, 0.0, pi, pj, want_grad=False)
        # touching at most, walls included: the shrink's tests are exact in
        # squares, the energy's round-wall gap L - 2 sqrt(rho^2) rounds the
        # root, so a touching sphere may read an overlap of a few ulp
        assert q["max_delta"] <= 1e-12, q["max_delta"]
        pg.append(r["phi"])
        xo, _ = orw.rsa_rounds(d0, L, 1.0, seed, rcp._lib.RCP_PLACE_WINDOW)
        st = orw.RunState(xo, d0, L, 1.0)
        status, res, _ = orw.run(st, orw.default_params(d0), orw.default_schedule(n, S=1.4))
        assert status == 0
        po.append(res.phi)
    pg, po = np.array(pg), np.array(po)
    _say("walls=%d round=%d phi gpu %.5f +- %.5f oracle %.5f +- %.5f" %
         (walls, round_axes, pg.mean(), pg.std(), po.mean(), po.std()))
    bar = max(0.004, 3.0 * math.sqrt((pg.var() + po.var()) / 8))
    assert abs(pg.mean() - po.mean()) <= bar


def test_census_mixing_walled_and_periodic(rcp):
    # one context, a walled packing and a periodic one: each result is the
    # one its own context gives (the walled kernel leaves the periodic
    # packing's arithmetic as it is)
    n = 400
    d0 = np.where(np.arange(n) % 2 == 0, 1.0, 1.4)
    L = float((math.pi / 6.0 * np.sum(d0 ** 3) / 0.1) ** (1.0 / 3.0))
    both = rcp.Packing([d0, d0], [L, L], 1.0, [4, 5], init="rsa_device",
                       boundary=[(X | Y | Z, 0), (0, 0)])
    rb = both.inflate_run()
    xb = [both.get_state(k)[0] for k in range(2)]
    both.close()
    for k, bnd in enumerate([(X | Y | Z, 0), (0, 0)]):
        one = rcp.Packing(d0, L, 1.0, 4 + k, init="rsa_device", boundary=bnd)
        r1 = one.inflate_run()[0]
        x1, _ = one.get_state()
        one.close()
        assert r1["phi"] == rb[k]["phi"] and r1["iterations"] == rb[k]["iterations"]
        assert np.array_equal(x1, xb[k])
    assert rb[0]["phi"] < rb[1]["phi"]


def test_boundary_arguments_checked(rcp):
    d0 = np.ones(8)
    p = rcp.Packing(d0, 10.0, 1.0, 0, init="none")
    for w, r in ((8, 0), (0, 1), (X, X | Y), (0, 8)):
        with pytest.raises(rcp.RcpError):
            p.set_boundary(w, r)
    p.set_boundary(X, 0)
    with pytest.raises(rcp.RcpError):
        p.set_frozen(np.r_[np.ones(4), np.zeros(4)].astype(np.uint8))
    p.set_boundary(0, 0)
    p.set_frozen(np.r_[np.ones(4), np.zeros(4)].astype(np.uint8))
    with pytest.raises(rcp.RcpError):
        p.set_boundary(0, X | Y | Z)
    p.close()
    q = rcp.Packing(d0, 10.0, 1.0, 0, init="none", dim=2)
    with pytest.raises(rcp.RcpError):
        q.set_boundary(Z, 0)        # no z axis in two dimensions
    q.set_boundary(0, X | Y)
    q.close()


@pytest.mark.parametrize("n", [1, 2, 3, 40])
@pytest.mark.parametrize("walls,round_axes", [(X | Y | Z, 0), (0, X | Y | Z)])
def test_walled_pairs_tiny_grids(rcp, orw, n, walls, round_axes):
    # few spheres in a small walled box (class grids of fewer than 3 cells
    # per axis, positions up to 1 past the walls): no image pairs
    d0 = np.linspace(1.0, 2.0, n)
    L = 9.0
    x = np.random.default_rng(n).uniform(-1.0, L + 1.0, (n, 3))
    p = rcp.Packing(d0, L, 1.5, 0, init="none", boundary=(walls, round_axes),
                    params=rcp.make_params(skin_s=0.2, skin_g=0.02))
    p.set_state(x, 1.5)
    p.neighbor_build()
    gi, gj = p.pairs()
    e = p.energy_grad()
    p.close()
    orw.set_boundary(walls, round_axes)
    oi, oj = orw.pairs_brute(x, d0, L, 1.5, 0.2, 0.02)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    ai, aj = orw.pairs_brute(x, d0, L, 1.5, 0.0, 0.0)
    r = orw.energy_grad(x, d0, L, 1.5, 0.0, ai, aj)
    assert e["n_overlap"] == r["n_overlap"]
    assert e["E_overlap"] == pytest.approx(r["E_ov"], rel=TOL, abs=1e-300)
