"""Pins of the oracle's hard walls (Sec. 2: every axis periodic or bounded by
a flat or curved hard wall) against facts that do not come from the oracle:
hand-worked single-sphere cases (tests/golden/one_sphere_walls.txt), central
finite differences, the symmetries of the container (reflection across a
flat-walled axis, rotation of a round container), lattices whose contact
scale is known exactly, the closed-form volume of the container, brute-force
checks of the placement, and whole runs that must end clear of every wall.
"""
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")

X, Y, Z = 1, 2, 4   # axis bits


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()
        out[k] = float(v)
    return out


@pytest.fixture
def orw(orc):
    yield orc
    orc.set_boundary(0, 0)
    orc.set_dim(3)


def _eval(orc, x, d0, L, kappa, mu=0.0):
    pi, pj = orc.pairs_brute(x, d0, L, kappa, 0.0, 0.0)
    return orc.energy_grad(x, d0, L, kappa, mu, pi, pj)


# ------------------------------------------------------------ hand values
def test_one_sphere_flat_wall_hand_values(orw):
    gd = _golden("one_sphere_walls.txt")
    orw.set_boundary(walls=X)
    L, d0, kappa = 10.0, np.ones(1), 2.0
    for xpos, sgn in ((gd["flat_x"], 1.0), (L - gd["flat_x"], -1.0)):
        r = _eval(orw, np.array([[xpos, 5.0, 5.0]]), d0, L, kappa)
        assert r["E_ov"] == pytest.approx(gd["flat_E"], rel=1e-15)
        assert r["g"][0] == pytest.approx([sgn * gd["flat_dEdx"], 0.0, 0.0], abs=1e-15)
        assert r["gk_ov"] == pytest.approx(gd["flat_dEdkappa"], rel=1e-15)
        assert r["max_delta"] == pytest.approx(0.25, rel=1e-15)
        assert r["n_overlap"] == 1
    # the same sphere in the middle touches nothing; without walls the
    # sphere at 0.75 touches nothing either (periodic axis, no image pair)
    r = _eval(orw, np.array([[5.0, 5.0, 5.0]]), d0, L, kappa)
    assert r["E_ov"] == 0.0 and r["n_overlap"] == 0 and not np.any(r["g"])
    orw.set_boundary(0, 0)
    r = _eval(orw, np.array([[0.75, 5.0, 5.0]]), d0, L, kappa)
    assert r["E_ov"] == 0.0 and r["n_overlap"] == 0


def test_one_sphere_corner_hand_values(orw):
    gd = _golden("one_sphere_walls.txt")
    orw.set_boundary(walls=X | Y)
    r = _eval(orw, np.array([[gd["corner_x"], gd["corner_y"], 5.0]]), np.ones(1), 10.0, 2.0)
    assert r["E_ov"] == pytest.approx(gd["corner_E"], rel=1e-15)
    assert r["g"][0] == pytest.approx([gd["corner_dEdx"], gd["corner_dEdy"], 0.0], abs=1e-15)
    assert r["gk_ov"] == pytest.approx(gd["corner_dEdkappa"], rel=1e-15)
    assert r["max_delta"] == 0.25 and r["n_overlap"] == 2


@pytest.mark.parametrize("round_axes,zpos", [(X | Y | Z, 5.0), (X | Y, 1.234)])
def test_one_sphere_round_wall_hand_values(orw, round_axes, zpos):
    # a ball, and a cylinder along z (z periodic): the same radial contact
    gd = _golden("one_sphere_walls.txt")
    orw.set_boundary(round=round_axes)
    rho = gd["ball_rho"]
    p = np.array([[5.0 + rho * 0.6, 5.0 + rho * 0.8, zpos]])
    r = _eval(orw, p, np.ones(1), 10.0, 2.0)
    assert r["E_ov"] == pytest.approx(gd["ball_E"], rel=1e-12)
    assert r["g"][0] == pytest.approx([gd["ball_dEdx"], gd["ball_dEdy"], 0.0], rel=1e-12, abs=1e-15)
    assert r["gk_ov"] == pytest.approx(gd["ball_dEdkappa"], rel=1e-12)
    assert r["n_overlap"] == 1


def test_container_volume_closed_form(orw):
    gd = _golden("one_sphere_walls.txt")
    orw.set_boundary(round=X | Y)
    assert orw.phi(np.ones(1), 2.0, 1.0) == pytest.approx(gd["cylinder_phi"], rel=1e-15)
    orw.set_boundary(round=X | Y | Z)   # ball of diameter L: phi = (D / L)^3
    assert orw.phi(np.ones(1), 2.0, 1.0) == pytest.approx(1.0 / 8.0, rel=1e-15)
    orw.set_boundary(walls=X | Y | Z)   # flat walls: the cube, as periodic
    assert orw.phi(np.ones(1), 2.0, 1.0) == pytest.approx(math.pi / 48.0, rel=1e-15)
    orw.set_dim(2)
    orw.set_boundary(round=X | Y)       # circle of diameter L: phi = (D / L)^2
    assert orw.phi(np.ones(1), 2.0, 1.0) == pytest.approx(0.25, rel=1e-15)


# ------------------------------------------------------ derivatives, symmetry
def _dense_config(n, L, seed, inset=0.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(inset, L - inset, (n, 3))
    d0 = rng.uniform(0.8, 1.6, n)
    return x, d0


@pytest.mark.parametrize("walls,round_axes", [(X | Y | Z, 0), (X, 0), (0, X | Y | Z),
                                               (Z, X | Y)])
def test_wall_gradient_finite_differences(orw, walls, round_axes):
    orw.set_boundary(walls, round_axes)
    L, kappa, mu = 6.0, 1.1, 3e-3
    x, d0 = _dense_config(60, L, seed=walls * 8 + round_axes)
    r = _eval(orw, x, d0, L, kappa, mu)
    assert r["n_overlap"] > 20

    def etot(xx, k):
        q = _eval(orw, xx, d0, L, k, mu)
        return q["E_ov"] + q["E_growth"]

    h = 1e-6
    rng = np.random.default_rng(1)
    for i in rng.choice(60, 12, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (etot(xp, kappa) - etot(xm, kappa)) / (2 * h)
            assert r["g"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    fdk = (etot(x, kappa + h) - etot(x, kappa - h)) / (2 * h)
    assert r["gk_ov"] + r["gk_growth"] == pytest.approx(fdk, rel=1e-6, abs=1e-8)


def test_reflection_across_flat_walls(orw):
    # x -> L - x on a walled axis swaps the two walls: the energy is
    # unchanged and that gradient component changes sign
    orw.set_boundary(walls=X | Y | Z)
    L, kappa = 6.0, 1.1
    x, d0 = _dense_config(80, L, seed=3)
    r = _eval(orw, x, d0, L, kappa)
    xr = x.copy()
    xr[:, 1] = L - xr[:, 1]
    q = _eval(orw, xr, d0, L, kappa)
    assert q["E_ov"] == pytest.approx(r["E_ov"], rel=1e-12)
    assert q["gk_ov"] == pytest.approx(r["gk_ov"], rel=1e-12)
    assert np.allclose(q["g"][:, 1], -r["g"][:, 1], rtol=1e-9, atol=1e-12)
    assert np.allclose(q["g"][:, [0, 2]], r["g"][:, [0, 2]], rtol=1e-9, atol=1e-12)


def test_rotation_of_a_round_container(orw):
    # a quarter turn about the ball's centre: (u, v) -> (-v, u) in the xy
    # plane; the energy is unchanged and the gradient turns with it
    orw.set_boundary(round=X | Y | Z)
    L, kappa = 6.0, 1.1
    x, d0 = _dense_config(80, L, seed=4)
    r = _eval(orw, x, d0, L, kappa)
    assert r["n_overlap"] > 30
    c = 0.5 * L
    xr = x.copy()
    xr[:, 0] = c - (x[:, 1] - c)
    xr[:, 1] = x[:, 0]
    q = _eval(orw, xr, d0, L, kappa)
    assert q["E_ov"] == pytest.approx(r["E_ov"], rel=1e-12)
    assert np.allclose(q["g"][:, 0], -r["g"][:, 1], rtol=1e-9, atol=1e-12)
    assert np.allclose(q["g"][:, 1], r["g"][:, 0], rtol=1e-9, atol=1e-12)
    assert np.allclose(q["g"][:, 2], r["g"][:, 2], rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------- shrink
@pytest.mark.parametrize("walls", [X | Y | Z, X])
def test_cubic_lattice_in_a_walled_box_shrinks_to_touching(orw, walls):
    # n^3 unit spheres on the cubic lattice (i + 1/2) in a box of side n:
    # neighbours and walls are both touched at kappa' = 1, phi = pi / 6
    orw.set_boundary(walls=walls)
    n = 4
    g = np.arange(n) + 0.5
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    d0 = np.ones(n ** 3)
    pi, pj = orw.pairs_brute(x, d0, float(n), 1.3, 0.0, 0.0)
    kp = orw.shrink(x, d0, float(n), 1.3, pi, pj)
    assert kp == 1.0
    assert orw.phi(d0, float(n), kp) == pytest.approx(math.pi / 6.0, rel=1e-15)
    # an extra margin at one wall only: the walls bind no more, the
    # lattice still does
    x2 = x.copy()
    x2[:, 0] += 0.25
    kp2 = orw.shrink(x2, d0, float(n) + 0.5, 1.3, *orw.pairs_brute(x2, d0, float(n) + 0.5,
                                                                   1.3, 0.0, 0.0))
    assert kp2 == 1.0


def test_one_sphere_fills_the_ball(orw):
    orw.set_boundary(round=X | Y | Z)
    x = np.array([[5.0, 5.0, 5.0]])
    kp = orw.shrink(x, np.ones(1), 10.0, 20.0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert kp == 10.0
    assert orw.phi(np.ones(1), 10.0, kp) == 1.0


def test_seven_disks_in_a_circle(orw):
    # the hexagonal seven: a central disk and six around it at unit distance
    # fill a circle of diameter 3 (every disk touches its neighbours and the
    # outer ones the wall); phi = 7 / 9
    orw.set_dim(2)
    orw.set_boundary(round=X | Y)
    t = np.arange(6) * math.pi / 3.0
    x = np.zeros((7, 3))
    x[:, :2] = 1.5
    x[1:, 0] += np.cos(t)
    x[1:, 1] += np.sin(t)
    d0 = np.ones(7)
    pi, pj = orw.pairs_brute(x, d0, 3.0, 1.2, 0.0, 0.0)
    kp = orw.shrink(x, d0, 3.0, 1.2, pi, pj)
    assert kp == pytest.approx(1.0, abs=4e-16)
    assert orw.phi(d0, 3.0, kp) == pytest.approx(7.0 / 9.0, rel=1e-15)


# ---------------------------------------------------------- placement
def _clear_of_walls(x, sig, L, walls, round_axes, tol=0.0):
    ok = np.ones(x.shape[0], bool)
    for a in range(3):
        if walls >> a & 1:
            ok &= (x[:, a] >= 0.5 * sig - tol) & (x[:, a] <= L - 0.5 * sig + tol)
    if round_axes:
        ax = [a for a in range(3) if round_axes >> a & 1]
        rho = np.sqrt(np.sum((x[:, ax] - 0.5 * L) ** 2, axis=1))
        ok &= rho <= 0.5 * (L - sig) + tol
    return ok


def _no_pair_overlap(x, sig, L, periodic):
    dx = x[None, :, :] - x[:, None, :]
    for a in range(3):
        if periodic[a]:
            dx[:, :, a] -= L * np.round(dx[:, :, a] / L)
    r = np.sqrt(np.sum(dx ** 2, -1))
    d = 0.5 * (sig[None, :] + sig[:, None])
    np.fill_diagonal(r, np.inf)
    return np.all(r >= d * (1 - 1e-12))


@pytest.mark.parametrize("walls,round_axes", [(X | Y | Z, 0), (Y, 0), (0, X | Y | Z),
                                               (Z, X | Y)])
def test_rsa_inside_walls(orw, walls, round_axes):
    orw.set_boundary(walls, round_axes)
    rng = np.random.default_rng(5)
    d0 = rng.uniform(0.5, 2.0, 400)
    L = 14.0
    x = orw.rsa(d0, L, 1.0, 17)
    assert np.all(_clear_of_walls(x, d0, L, walls, round_axes))
    per = [not ((walls | round_axes) >> a & 1) for a in range(3)]
    assert _no_pair_overlap(x, d0, L, per)
    # the proposals that land close to a wall are rejected, not moved: a
    # few spheres must sit close to the walls
    near = ~_clear_of_walls(x, d0 + 0.6, L, walls, round_axes)
    assert near.sum() > 5
    # rounds of one proposal are the sequential procedure, attempt for attempt
    xr, _ = orw.rsa_rounds(d0, L, 1.0, 17, 1)
    assert np.array_equal(x, xr)


def test_rsa_fills_the_ball_uniformly(orw):
    # tiny spheres at phi ~ 0.002: the centres are uniform in the ball of
    # radius R' = (L - sigma) / 2, so (rho / R')^3 is uniform on [0, 1]
    orw.set_boundary(round=X | Y | Z)
    d0 = np.full(3000, 0.1)
    L = 10.0
    x = orw.rsa(d0, L, 1.0, 3)
    u = (np.sqrt(np.sum((x - 5.0) ** 2, 1)) / (0.5 * (L - 0.1))) ** 3
    assert u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 4.0 * math.sqrt(1.0 / 12.0 / 3000)
    assert abs(np.mean(u < 0.25) - 0.25) < 4.0 * math.sqrt(0.25 * 0.75 / 3000)


# -------------------------------------------------------------- whole runs
@pytest.mark.parametrize("walls,round_axes", [(X | Y | Z, 0), (0, X | Y | Z)])
def test_whole_run_in_a_container_ends_clear_of_the_walls(orw, walls, round_axes):
    orw.set_boundary(walls, round_axes)
    n = 256
    d0 = np.where(np.arange(n) % 2 == 0, 1.0, 1.4)
    vol = math.pi / 6.0 * np.sum(d0 ** 3) / 0.1
    # the domain's volume at side L: L^3 for the cube, pi/6 L^3 for the ball
    L = float((vol / (1.0 if round_axes == 0 else math.pi / 6.0)) ** (1.0 / 3.0))
    st = orw.RunState(orw.rsa(d0, L, 1.0, 2), d0, L, 1.0)
    status, res, _ = orw.run(st, orw.default_params(d0), orw.default_schedule(n, S=1.4))
    assert status == 0 and res.max_overlap < 5e-4
    sig = res.kappa_shrunk * d0
    assert np.all(_clear_of_walls(st.x, sig, L, walls, round_axes, tol=1e-12))
    assert _no_pair_overlap(st.x, sig, L, [False] * 3)
    # confinement leaves a looser layer at the walls than the periodic
    # packing of the same spheres (about 0.64 at this size)
    assert 0.50 < res.phi < 0.635, res.phi


@pytest.mark.parametrize("walls,round_axes", [(X, 0), (0, X | Y | Z), (Z, X | Y)])
def test_no_image_across_a_bounded_axis(orw, walls, round_axes):
    # two spheres pressed into opposite walls along x: 0.6 apart through the
    # periodic image, 9.4 apart inside the container; only the two wall
    # contacts count (delta = 1 - 0.6 / 1 each)
    orw.set_boundary(walls, round_axes)
    x = np.array([[0.3, 5.0, 5.0], [9.7, 5.0, 5.0]])
    r = _eval(orw, x, np.ones(2), 10.0, 1.0)
    assert r["n_overlap"] == 2
    assert r["E_ov"] == pytest.approx(0.16, rel=1e-14)
    assert r["g"][0, 0] < 0.0 < r["g"][1, 0]


def test_shrink_takes_each_wall(orw):
    # one sphere near the lower and one near the upper wall of x: each wall
    # sets the contact scale of its own sphere
    orw.set_boundary(walls=X)
    e = np.zeros(0, np.int32)
    for xpos in (0.5, 9.5):
        kp = orw.shrink(np.array([[xpos, 5.0, 5.0]]), np.ones(1), 10.0, 3.0, e, e)
        assert kp == 1.0
    kp = orw.shrink(np.array([[0.75, 5.0, 5.0], [9.6, 2.0, 2.0]]), np.ones(2), 10.0, 3.0, e, e)
    assert kp == pytest.approx(0.8, rel=1e-15)


def test_adam_does_not_wrap_across_a_wall(orw):
    # a sphere whose centre has crossed the lower wall takes one small Adam
    # step inwards and stays on the far side (no wrap to x + L)
    orw.set_boundary(walls=X)
    d0 = np.ones(1)
    st = orw.RunState(np.array([[-0.1, 5.0, 5.0]]), d0, 10.0, 1.0)
    orw.run(st, orw.default_params(d0), orw.oracle.absolute_schedule(0.0, 0.01, 0.0, 1))
    assert st.x[0, 0] == pytest.approx(-0.09, rel=1e-9)
    orw.set_boundary(0, 0)   # periodic: the same step wraps (no wall force)
    st = orw.RunState(np.array([[-0.1, 5.0, 5.0]]), d0, 10.0, 1.0)
    orw.run(st, orw.default_params(d0), orw.oracle.absolute_schedule(0.0, 0.01, 0.0, 1))
    assert st.x[0, 0] == pytest.approx(9.9, rel=1e-12)


@pytest.mark.parametrize("walls,round_axes", [(X | Y, 0), (0, X | Y), (X, 0)])
def test_wall_gradient_finite_differences_2d(orw, walls, round_axes):
    # disks (z = 0) against flat walls and a circle: central differences of
    # E in x, y and kappa; the z gradient stays exactly zero
    orw.set_dim(2)
    orw.set_boundary(walls, round_axes)
    L, kappa, mu = 8.0, 1.1, 3e-3
    rng = np.random.default_rng(walls + 4 * round_axes)
    x = np.column_stack([rng.uniform(0, L, (70, 2)), np.zeros(70)])
    d0 = rng.uniform(0.8, 1.6, 70)
    r = _eval(orw, x, d0, L, kappa, mu)
    assert r["n_overlap"] > 20 and np.all(r["g"][:, 2] == 0.0)

    def etot(xx, k):
        q = _eval(orw, xx, d0, L, k, mu)
        return q["E_ov"] + q["E_growth"]

    h = 1e-6
    for i in rng.choice(70, 12, replace=False):
        for a in range(2):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (etot(xp, kappa) - etot(xm, kappa)) / (2 * h)
            assert r["g"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    fdk = (etot(x, kappa + h) - etot(x, kappa - h)) / (2 * h)
    assert r["gk_ov"] + r["gk_growth"] == pytest.approx(fdk, rel=1e-6, abs=1e-8)
