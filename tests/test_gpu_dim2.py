"""Two dimensions (Sec. 2: the dimension is an input; Fig. 1 is a 2-D
packing) on the GPU, through the C ABI, against the FP64 CPU oracle in
two dimensions.

Bars as in three dimensions: placements and pair sets bit for bit; energy
terms and gradients within 1e-10 per component relative to the sum of
absolute pair contributions; Adam steps within 1e-9 of the step size per
step; whole runs statistically (mean phi over 8 seeds).
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


@pytest.fixture
def orc2(orc):
    orc.set_dim(2)
    yield orc
    orc.set_dim(3)


def _say(*a):
    print(*a, flush=True)


def _disks(n, S, phi, seed):
    w = ri.small_polydisperse(n, S, phi, seed=seed)
    L = float(np.sqrt(np.pi / 4.0 * np.sum(w.d0 ** 2) / phi))
    return w.d0, L


def _xy(x3):
    return np.ascontiguousarray(x3[:, :2])


@pytest.mark.parametrize("init", ["rsa", "rsa_device"])
def test_2d_placement_bit_exact(rcp, orc2, init):
    d0, L = _disks(3000, 20.0, 0.3, seed=4)
    p = rcp.Packing(d0, L, 1.0, 9, init=init, dim=2)
    x, k = p.get_state()
    p.close()
    assert x.shape == (3000, 2) and k == 1.0
    if init == "rsa":
        xo = orc2.rsa(d0, L, 1.0, 9)
    else:
        xo, _ = orc2.rsa_rounds(d0, L, 1.0, 9, 65536)
    assert np.all(xo[:, 2] == 0.0)
    assert np.array_equal(x, _xy(xo))


def test_2d_pairs_energy_gradient(rcp, orc2):
    d0, L = _disks(4000, 30.0, 0.75, seed=6)
    x = np.column_stack([ri.rng.uniform_positions(4000, L, 3)[:, :2], np.zeros(4000)])
    p = rcp.Packing(d0, L, 1.0, 0, init="none", dim=2,
                    params=rcp.make_params(skin_s=0.2, skin_g=0.02))
    p.set_state(_xy(x), 1.0)
    p.neighbor_build()
    gi, gj = p.pairs()
    oi, oj = orc2.pairs_brute(x, d0, L, 1.0, 0.2, 0.02)
    assert np.array_equal(gi, oi) and np.array_equal(gj, oj)
    e = p.energy_grad(mu=1e-3)
    ai, aj = orc2.pairs_brute(x, d0, L, 1.0, 0.0, 0.0)
    r = orc2.energy_grad(x, d0, L, 1.0, 1e-3, ai, aj)
    assert r["n_overlap"] > 1000
    assert e["g"].shape == (4000, 2)
    assert np.all(r["g"][:, 2] == 0.0)
    err = np.abs(e["g"] - r["g"][:, :2])
    assert np.all(err <= TOL * r["gscale"][:, :2]), float(np.max(err / (r["gscale"][:, :2] + 1e-300)))
    assert e["E_overlap"] == pytest.approx(r["E_ov"], rel=TOL)
    assert e["dE_dkappa_overlap"] == pytest.approx(r["gk_ov"], rel=TOL)
    assert e["n_overlap"] == r["n_overlap"]
    p.close()


@pytest.mark.parametrize("steps,graph", [(1, 1), (10, 16)])
def test_2d_adam_steps_match_oracle(rcp, orc2, steps, graph):
    d0, L = _disks(2000, 10.0, 0.8, seed=8)
    x = np.column_stack([ri.rng.uniform_positions(2000, L, 5)[:, :2], np.zeros(2000)])
    mu, ex, ek = 2e-3, 2e-3, 2e-4
    P = orc2.default_params(d0, s=0.3, g=0.02)
    p = rcp.Packing(d0, L, 1.0, 0, init="none", dim=2,
                    params=rcp.make_params(skin_s=0.3, skin_g=0.02, eps_x=P.eps_x),
                    tuning=rcp.make_tuning(graph_iters=graph))
    p.set_state(_xy(x), 1.0)
    p.adam_step(mu, ex, ek, steps)
    xg, kg = p.get_state()
    m, v, _ = p.get_optimizer()
    p.close()
    st = orc2.RunState(x, d0, L, 1.0)
    orc2.run(st, P, orc2.oracle.absolute_schedule(mu, ex, ek, steps))
    assert np.all(st.x[:, 2] == 0.0) and np.all(st.m[:, 2] == 0.0)
    d = np.abs(xg - st.x[:, :2])
    d = np.minimum(d, L - d)
    assert d.max() <= 1e-9 * ex * steps + 4e-16 * L, d.max()
    assert m.shape == (2000, 2) and v.shape == (2000, 2)
    assert kg == pytest.approx(st.kappa[0], rel=1e-12)


def test_2d_square_lattice_shrinks_to_touching(rcp):
    # n x n equal disks on a square lattice of spacing 1 at kappa 1.3: the
    # shrink lands on touching, kappa' = 1, area fraction pi / 4
    n = 8
    g = np.arange(n) + 0.5
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.column_stack([X.ravel(), Y.ravel()])
    p = rcp.Packing(np.ones(n * n), float(n), 1.0, 0, init="none", dim=2,
                    params=rcp.make_params(skin_s=0.05, skin_g=0.02))
    p.set_state(x, 1.3)
    kp, phi = p.shrink()
    p.close()
    assert kp == 1.0
    assert phi == pytest.approx(np.pi / 4.0, rel=1e-15)


def test_2d_whole_runs_match_oracle(rcp, orc2):
    # 50:50 disks of diameter ratio 1.4, N = 512, RSA at phi0 = 0.1, the
    # default schedule for d = 2, seeds 0-7: mean phi within 0.002
    n = 512
    d0 = np.where(np.arange(n) % 2 == 0, 1.0, 1.4)
    L = float(np.sqrt(np.pi / 4.0 * np.sum(d0 ** 2) / 0.1))
    pg, po = [], []
    for seed in range(8):
        p = rcp.Packing(d0, L, 1.0, seed, init="rsa", dim=2)
        r = p.inflate_run()[0]
        x, _ = p.get_state()
        p.close()
        assert r["status"] == 0 and r["max_overlap"] < 5e-4, r
        pg.append(r["phi"])
        st = orc2.RunState(orc2.rsa(d0, L, 1.0, seed), d0, L, 1.0)
        status, res, _ = orc2.run(st, orc2.default_params(d0),
                                  orc2.default_schedule(n, d=2, S=1.4))
        assert status == 0
        po.append(res.phi)
    pg, po = np.array(pg), np.array(po)
    _say("2-D phi gpu %.5f +- %.5f oracle %.5f +- %.5f" % (pg.mean(), pg.std(), po.mean(), po.std()))
    assert abs(pg.mean() - po.mean()) <= 0.002


def test_2d_kernel_equals_3d_kernel_on_the_plane(rcp):
    # the kernel instantiated for two coordinates leaves out terms that are
    # exactly zero on the plane: a 3-D context holding the same disks at
    # z = 0 must give the same positions and kappa, bit for bit
    d0, L = _disks(6000, 40.0, 0.8, seed=12)
    xy = ri.rng.uniform_positions(6000, L, 7)[:, :2]
    out = []
    for dim in (2, 3):
        p = rcp.Packing(d0, L, 1.0, 0, init="none", dim=dim,
                        params=rcp.make_params(skin_s=0.3, skin_g=0.02),
                        tuning=rcp.make_tuning(graph_iters=8))
        p.set_state(xy if dim == 2 else np.column_stack([xy, np.zeros(6000)]), 1.0)
        p.adam_step(2e-3, 2e-3, 2e-4, 24)
        x, k = p.get_state()
        p.close()
        out.append((x[:, :2], k, x))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert np.all(out[1][2][:, 2] == 0.0)


def test_2d_extreme_packing_reaches_the_papers_phi(rcp):
    # Fig. (extreme): truncated lognormal sigma_lnD = 1.3, N = 1e5,
    # S = 8.4e3, phi ~ 0.91 (2-D, periodic).  Device RSA at area fraction
    # 0.05, the default d = 2 schedule 8 times longer (the default lengths
    # end at the cap on this set)
    d0 = ri.lognormal_quantiles(100_000, 1.3, 8.55e3)
    S = float(d0.max() / d0.min())
    assert abs(S - 8.4e3) < 0.01 * 8.4e3
    L = float(np.sqrt(np.pi / 4.0 * np.sum(d0 ** 2) / 0.05))
    s = rcp.longer_schedule(rcp.default_schedule(d0.shape[0], dim=2, S=S), 8)
    p = rcp.Packing(d0, L, 1.0, 0, init="rsa_device", dim=2,
                    params=rcp.make_params(skin_s=256.0))
    r = p.inflate_run(s)[0]
    p.close()
    _say("2-D extreme packing: phi %.4f after %d iterations" % (r["phi"], r["iterations"]))
    assert r["status"] == 0 and r["max_overlap"] < 5e-4
    assert abs(r["phi"] - 0.91) <= 0.015
