"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test states what fixes the expected value: a hand-worked case from
Eq. (energy) (tests/golden), a library routine (scipy distributions,
torch.optim.Adam with autograd), a closed form (Eq. (trigger), Eq. (eps3)),
an invariant of the energy, or brute force.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import rcp_inputs as ri

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = [float(t) for t in v] if len(v) > 1 else float(v[0])
    return out


# --------------------------------------------------------------- generator
def test_splitmix64_published_vectors(orc):
    for line in open(os.path.join(GOLD, "splitmix64_seed0.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, want = line.split()
        assert orc.splitmix64(0, int(k)) == int(want, 16)
        assert int(ri.splitmix64(0, int(k))) == int(want, 16)


def test_u01_python_matches_c(orc):
    for (s, i, a, ax) in [(0, 0, 0, 0), (7, 123, 5, 2), (2 ** 40 + 3, 99999, 17, 1)]:
        assert float(ri.u01(s, i, a, ax)) == orc.u01(s, i, a, ax)


# ------------------------------------------------------ two spheres by hand
@pytest.mark.parametrize("wrap", [False, True])
def test_two_sphere_hand_values(orc, wrap):
    gd = _golden("two_sphere.txt")
    d0 = np.array(gd["D0"])
    L = 20.0
    if wrap:   # the pair straddles the periodic boundary
        x = np.array([[0.5, 7.0, 9.0], [L - 2.5, 7.0, 9.0]])
        sgn = -1.0
    else:
        x = np.array([[10.0, 7.0, 9.0], [13.0, 7.0, 9.0]])
        sgn = 1.0
    pi, pj = np.array([0], np.int32), np.array([1], np.int32)
    r = orc.energy_grad(x, d0, L, gd["kappa"], gd["mu"], pi, pj)
    assert r["E_ov"] == pytest.approx(gd["E_overlap"], rel=1e-15)
    assert r["gk_ov"] == pytest.approx(gd["dEdkappa_overlap"], rel=1e-15)
    assert r["E_growth"] == pytest.approx(gd["E_growth"], rel=1e-15)
    assert r["gk_growth"] == pytest.approx(gd["dEdkappa_growth"], rel=1e-15)
    assert r["max_delta"] == pytest.approx(0.25, rel=1e-15)
    g = r["g"]
    assert g[0, 0] == pytest.approx(sgn * gd["grad_along_line"], rel=1e-15)
    assert g[1, 0] == pytest.approx(-sgn * gd["grad_along_line"], rel=1e-15)
    assert np.all(g[:, 1:] == 0.0)


def test_separated_spheres_exactly_zero(orc):
    d0 = np.array([1.0, 3.0])
    x = np.array([[10.0, 7.0, 9.0], [14.0, 7.0, 9.0]])  # touching: r = d
    r = orc.energy_grad(x, d0, 20.0, 2.0, 0.0, [0], [1])
    assert r["E_ov"] == 0.0 and r["gk_ov"] == 0.0 and np.all(r["g"] == 0.0)
    x[1, 0] = 17.0
    r = orc.energy_grad(x, d0, 20.0, 2.0, 0.0, [0], [1])
    assert r["E_ov"] == 0.0 and np.all(r["g"] == 0.0)


# ------------------------------------------------------------ invariants
def _overlapping_case(n=300, phi=0.45, S=4.0, seed=3):
    w = ri.small_polydisperse(n, S, phi, seed)
    return w.x.copy(), w.d0, w.L


def _all_overlaps(orc, x, d0, L, kappa):
    return orc.pairs_brute(x, d0, L, kappa, 0.0, 0.0)


def test_forces_sum_to_zero(orc):
    x, d0, L = _overlapping_case()
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    r = orc.energy_grad(x, d0, L, 1.0, 0.0, pi, pj)
    assert r["n_overlap"] > 50
    tot = r["g"].sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-12 * np.abs(r["g"]).sum(axis=0))


def test_translation_invariance(orc):
    x, d0, L = _overlapping_case()
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    r0 = orc.energy_grad(x, d0, L, 1.0, 0.0, pi, pj)
    xs = (x + np.array([0.37 * L, -0.21 * L, 0.73 * L])) % L
    pi2, pj2 = _all_overlaps(orc, xs, d0, L, 1.0)
    assert np.array_equal(pi, pi2) and np.array_equal(pj, pj2)
    r1 = orc.energy_grad(xs, d0, L, 1.0, 0.0, pi2, pj2)
    assert r1["E_ov"] == pytest.approx(r0["E_ov"], rel=1e-12)
    assert np.allclose(r1["g"], r0["g"], rtol=0, atol=1e-10 * np.abs(r0["g"]).max())


def test_joint_scaling_invariance(orc):
    x, d0, L = _overlapping_case()
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    r0 = orc.energy_grad(x, d0, L, 1.0, 0.0, pi, pj)
    lam = 2.0 ** 0.5
    r1 = orc.energy_grad(x * lam, d0, L * lam, lam, 0.0, pi, pj)
    assert r1["E_ov"] == pytest.approx(r0["E_ov"], rel=1e-12)
    assert np.allclose(r1["g"] * lam, r0["g"], rtol=1e-11, atol=1e-14)


def test_virial_identity_links_kappa_and_position_gradients(orc):
    # A cluster far from the box faces: sum_i x_i . dE/dx_i = -kappa dE/dkappa
    # (overlap part), because E_ov depends only on r/(kappa d0).
    rng = np.random.default_rng(5)
    n = 80
    d0 = np.exp(rng.uniform(0, np.log(3.0), n))
    x = 50.0 + rng.uniform(-4, 4, (n, 3))
    L = 200.0
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    r = orc.energy_grad(x, d0, L, 1.0, 0.0, pi, pj)
    assert r["n_overlap"] > 100
    lhs = float(np.sum(x * r["g"]))
    assert lhs == pytest.approx(-1.0 * r["gk_ov"], rel=1e-10)


def test_central_finite_differences(orc):
    x, d0, L = _overlapping_case(n=120, phi=0.5)
    kappa = 1.0

    def E(xx, kk, only=None):
        pi, pj = _all_overlaps(orc, xx, d0, L, kk)
        if only is not None:   # local energy: the pairs of one particle
            keep = (pi == only) | (pj == only)
            pi, pj = pi[keep], pj[keep]
        return orc.energy_grad(xx, d0, L, kk, 0.3, pi, pj)

    r = E(x, kappa)
    h = 1e-7 * d0.min()
    rng = np.random.default_rng(0)
    checked = 0
    for i in rng.choice(x.shape[0], 40, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = (E(xp, kappa, i)["E_ov"] - E(xm, kappa, i)["E_ov"]) / (2 * h)
            sc = r["gscale"][i, a]
            if sc == 0:
                assert fd == 0.0
                continue
            assert abs(fd - r["g"][i, a]) <= 1e-6 * sc
            checked += 1
    assert checked > 30
    hk = 1e-7 * kappa
    Ep, Em = E(x, kappa + hk), E(x, kappa - hk)
    fdk = ((Ep["E_ov"] + Ep["E_growth"]) - (Em["E_ov"] + Em["E_growth"])) / (2 * hk)
    assert fdk == pytest.approx(r["gk_ov"] + r["gk_growth"], rel=1e-6)


# ---------------------------------------------------------------- Adam
def test_adam_first_step_closed_form(orc):
    gd = _golden("two_sphere.txt")
    d0 = np.array(gd["D0"])
    x = np.array([[10.0, 7.0, 9.0], [13.0, 7.0, 9.0]])
    P = orc.default_params(d0, kappa0=2.0, s=0.1, g=0.02)
    eta_x, eta_k = 1e-3, 1e-4
    S = orc.oracle.absolute_schedule(gd["mu"], eta_x, eta_k, 1)
    st = orc.RunState(x, d0, 20.0, gd["kappa"])
    status, res, _ = orc.run(st, P, S)
    assert status == 1 and res.iterations == 1
    # bias-corrected first step: m_hat = g, v_hat = g^2 => step = eta g/(|g|+eps)
    g = gd["grad_along_line"]
    assert st.x[0, 0] == pytest.approx(10.0 - eta_x * g / (g + P.eps_x), rel=1e-15)
    assert st.x[1, 0] == pytest.approx(13.0 + eta_x * g / (g + P.eps_x), rel=1e-15)
    assert np.all(st.x[:, 1:] == x[:, 1:])
    gk = gd["dEdkappa_overlap"] + gd["dEdkappa_growth"]
    assert st.kappa[0] == pytest.approx(2.0 - eta_k * gk / (abs(gk) + P.eps_k), rel=1e-15)


def test_adam_trajectory_matches_torch_adam_with_autograd(orc):
    torch = pytest.importorskip("torch")
    x, d0, L = _overlapping_case(n=64, phi=0.5, S=3.0, seed=11)
    mu, eta_x, eta_k, steps = 2e-3, 5e-3, 1e-3, 12
    P = orc.default_params(d0, s=0.3, g=0.05)
    st = orc.RunState(x, d0, L, 1.0)
    S = orc.oracle.absolute_schedule(mu, eta_x, eta_k, steps)
    status, res, _ = orc.run(st, P, S)
    assert status == 1 and res.iterations == steps

    tx = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    tk = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    td = torch.tensor(d0, dtype=torch.float64)
    iu = torch.triu_indices(64, 64, 1)
    opt = torch.optim.Adam([{"params": [tx], "lr": eta_x, "eps": P.eps_x},
                            {"params": [tk], "lr": eta_k, "eps": P.eps_k}],
                           betas=(0.9, 0.999))
    for _ in range(steps):
        opt.zero_grad()
        dx = tx[iu[1]] - tx[iu[0]]
        dx = torch.where(dx > L / 2, dx - L, torch.where(dx < -L / 2, dx + L, dx))
        r = torch.sqrt((dx * dx).sum(1))
        d = tk * 0.5 * (td[iu[0]] + td[iu[1]])
        delta = torch.clamp(1 - r / d, min=0)
        E = 0.5 * (delta ** 2).sum() - mu * tk * td.sum()
        E.backward()
        opt.step()
        with torch.no_grad():
            tx[tx < 0] += L
            tx[tx >= L] -= L
    assert np.allclose(st.x, tx.detach().numpy(), rtol=0, atol=1e-9 * eta_x)
    assert st.kappa[0] == pytest.approx(tk.item(), rel=1e-12)


# ------------------------------------------------------------- schedule
def test_n_trig_matches_eq_trigger():
    from oracle import n_trig
    # ceil(4000 Y + X sqrt(N d) - 2000), hand-evaluated
    assert n_trig(512) == 6353          # 6000 + 9 sqrt(1536) = 6352.73
    assert n_trig(100_000) == 10930     # 6000 + 9 sqrt(3e5) = 10929.5
    assert n_trig(1_000_000) == 21589   # 6000 + 9 sqrt(3e6) = 21588.5
    assert n_trig(3_000_000) == 33000   # 6000 + 9 * 3000 = 33000 exactly
    assert n_trig(512, Y=3, X=24) == 10000 + math.ceil(24 * math.sqrt(1536))


# ------------------------------------------------------------ generators
@pytest.mark.parametrize("alpha,S", [(0.3, 4.0), (1.0, 1e3), (2.5, 5e5)])
def test_lognormal_quantiles_follow_truncnorm_cdf(alpha, S):
    n = 4000
    d = ri.lognormal_quantiles(n, alpha, S)
    a = math.log(S) / (2 * alpha)
    z = np.log(d) / alpha - a
    F = stats.truncnorm(-a, a).cdf(z)
    assert np.max(np.abs(F - (np.arange(n) + 0.5) / n)) < 1e-9
    assert d.min() >= 1.0 and d.max() <= S * (1 + 1e-12)
    assert np.all(np.diff(d) >= 0)


def test_powerlaw_quantiles_follow_truncpareto_cdf():
    n, S = 5000, 20.0
    d = ri.powerlaw_quantiles(n, -3.0, S)
    F = stats.truncpareto(2.0, S).cdf(d)   # pdf ~ D^-3 on [1, S]
    assert np.max(np.abs(F - (np.arange(n) + 0.5) / n)) < 1e-10


def test_weibull_quantiles_follow_truncated_weibull_cdf():
    n, S, k = 5000, 300.0, 1.3
    d = ri.weibull_quantiles(n, k, S)
    lo, hi, lam = S ** -0.5, S ** 0.5, S ** 0.5
    W = stats.weibull_min(k, scale=lam)
    F = (W.cdf(d * lo) - W.cdf(lo)) / (W.cdf(hi) - W.cdf(lo))
    assert np.max(np.abs(F - (np.arange(n) + 0.5) / n)) < 1e-9


@pytest.mark.parametrize("alpha,a", [(0.3, 2.3105), (1.0, 3.4539), (0.7, 4.5)])
def test_third_moment_matches_eq_eps3(alpha, a):
    # Eq. (eps3): <D^3> of the truncated law is exp(9 alpha^2 / 2)(1 - eps3)
    S = math.exp(2 * a * alpha)
    d = ri.lognormal_quantiles(200_000, alpha, S) * math.exp(-alpha * a)
    m3 = np.mean(d ** 3)
    want = math.exp(4.5 * alpha ** 2) * (1 - ri.eps3_lognormal(alpha, a))
    assert m3 == pytest.approx(want, rel=2e-4)


def test_box_gives_initial_phi(orc):
    w = ri.c1_lognormal()
    assert orc.phi(w.d0, w.L, 1.0) == pytest.approx(0.1, rel=1e-14)
    w2 = ri.c2_powerlaw(n=5000)
    assert orc.phi(w2.d0, w2.L, 1.0) == pytest.approx(0.05, rel=1e-14)


# -------------------------------------------------------------- pair sets
def _cut_ok(d0, L, kb, s, g):
    return kb * ((1 + g) * d0.max() + 2 * s * d0.min()) < L / 2


PAIR_CASES = [
    ("lognormal", 100.0, 0.5, 1.0, 0.1, 0.02),
    ("powerlaw", 20.0, 0.4, 1.0, 0.3, 0.02),
    ("powerlaw", 300.0, 0.02, 1.0, 0.3, 0.02),
    ("weibull", 300.0, 0.5, 1.1, 0.1, 0.002),
    ("lognormal", 8.0, 0.6, 1.0, 2.0, 0.0),
]


@pytest.mark.parametrize("fam,S,phi,kb,s,g", PAIR_CASES)
def test_cell_list_equals_brute_force(orc, fam, S, phi, kb, s, g):
    w = ri.small_polydisperse(4096, S, phi, seed=17, family=fam)
    assert _cut_ok(w.d0, w.L, kb, s, g)
    a = orc.pairs_brute(w.x, w.d0, w.L, kb, s, g)
    b = orc.pairs_cells(w.x, w.d0, w.L, kb, s, g)
    assert len(a[0]) > 100
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rows_pairs_symmetric_and_equal_to_half_set(orc):
    w = ri.small_polydisperse(1500, 50.0, 0.5, seed=4, family="powerlaw")
    pi, pj = orc.pairs_brute(w.x, w.d0, w.L, 1.0, 0.2, 0.02)
    rows = np.arange(w.n)
    nb = orc.rows_pairs(w.x, w.d0, w.L, 1.0, rows, 0.2, 0.02)
    full = set()
    for i, lst in enumerate(nb):
        for j in lst:
            full.add((i, int(j)))
    half = set(zip(pi.tolist(), pj.tolist()))
    assert all((j, i) in full for (i, j) in full)
    assert {(i, j) for (i, j) in full if i < j} == half


def test_c1_cell_list_equals_brute_force(orc):
    w = ri.c1_lognormal(0)
    x = orc.rsa(w.d0, w.L, 1.0, w.seed)
    a = orc.pairs_brute(x, w.d0, w.L, 1.0, 0.1, 0.02)
    b = orc.pairs_cells(x, w.d0, w.L, 1.0, 0.1, 0.02)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- RSA
def test_rsa_non_overlapping_uniform_and_deterministic(orc):
    w = ri.c1_lognormal(3)
    x = orc.rsa(w.d0, w.L, 1.0, w.seed)
    x2 = orc.rsa(w.d0, w.L, 1.0, w.seed)
    assert np.array_equal(x, x2)
    assert np.all((x >= 0) & (x < w.L))
    pi, _ = orc.pairs_brute(x, w.d0, w.L, 1.0, 0.0, 0.0)
    assert len(pi) == 0
    for a in range(3):
        assert stats.kstest(x[:, a] / w.L, "uniform").pvalue > 1e-3
    # the largest sphere is placed first, at attempt 0
    i = int(np.argmax(w.d0))
    assert x[i, 0] == orc.u01(w.seed, i, 0, 0) * w.L


# -------------------------------------------------------------- shrink
def test_shrink_is_the_largest_contact_scale(orc):
    x, d0, L = _overlapping_case(n=400, phi=0.4, S=4.0, seed=8)
    kappa = 1.0
    pi, pj = _all_overlaps(orc, x, d0, L, kappa)
    assert len(pi) > 10
    kp = orc.shrink(x, d0, L, kappa, pi, pj)
    assert kp < kappa
    none, _ = orc.pairs_brute(x, d0, L, kp, 0.0, 0.0)
    assert len(none) == 0
    up = np.nextafter(kp, np.inf)
    some, _ = orc.pairs_brute(x, d0, L, up, 0.0, 0.0)
    assert len(some) >= 1
    # the touching pair is at contact to a few ulp
    pi2, pj2 = orc.pairs_brute(x, d0, L, kappa, 0.0, 0.0)
    dx = x[pj2] - x[pi2]
    dx -= L * np.round(dx / L)
    r = np.sqrt((dx ** 2).sum(1))
    ratio = r / (kp * 0.5 * (d0[pi2] + d0[pj2]))
    assert ratio.min() >= 1.0 - 4e-16 and ratio.min() - 1.0 <= 4 * 2.2e-16


def test_shrink_keeps_kappa_without_overlap(orc):
    w = ri.c1_lognormal(1)
    x = orc.rsa(w.d0, w.L, 1.0, w.seed)
    pi, pj = orc.pairs_brute(x, w.d0, w.L, 1.0, 0.5, 0.0)
    assert orc.shrink(x, w.d0, w.L, 1.0, pi, pj) == 1.0


# ----------------------------------------------------------- whole run
def test_c1_run_reaches_stop_criterion(orc):
    w = ri.c1_lognormal(0)
    x = orc.rsa(w.d0, w.L, 1.0, w.seed)
    st = orc.RunState(x, w.d0, w.L, 1.0)
    status, res, _ = orc.run(st, orc.default_params(w.d0), orc.default_schedule(w.n))
    assert status == 0
    assert res.max_overlap < 5e-4
    # independent check of the stop test on the returned state
    pi, pj = orc.pairs_brute(st.x, w.d0, w.L, st.kappa[0], 0.0, 0.0)
    r = orc.energy_grad(st.x, w.d0, w.L, st.kappa[0], 0.0, pi, pj)
    assert r["max_delta"] == res.max_overlap
    # zero overlap after the shrink
    none, _ = orc.pairs_brute(st.x, w.d0, w.L, res.kappa_shrunk, 0.0, 0.0)
    assert len(none) == 0
    assert res.phi == pytest.approx(orc.phi(w.d0, w.L, res.kappa_shrunk), rel=1e-15)
    # sanity only (protocol dependent): between the paper's alpha = 0.1 and 0.5
    # rows of Table (tab:cap) at N = 2000, 0.641 and 0.698
    assert 0.63 < res.phi < 0.70


@pytest.mark.slow
@pytest.mark.parametrize("alpha,S,phi_paper", [(0.10, 3.0, 0.641), (0.50, 116.0, 0.698)])
def test_table_cap_sanity(orc, alpha, S, phi_paper):
    # Table (tab:cap), N = 2000 rows.  The rung values are our reading, so
    # the paper's phi is matched only to within 0.03.
    d0 = ri.lognormal_quantiles(2000, alpha, S)
    L = ri.box_for_phi(d0, 0.1)
    x = orc.rsa(d0, L, 1.0, 1)
    st = orc.RunState(x, d0, L, 1.0)
    S = float(d0.max() / d0.min())
    status, res, _ = orc.run(st, orc.default_params(d0, s=1.0), orc.default_schedule(2000, S=S))
    assert status == 0
    assert abs(res.phi - phi_paper) < 0.03


# ------------------------------------------------- schedule machinery, by hand
def _separated_pair_schedule(orc, rungs, tol, eps_k):
    d0 = np.array([1.0, 2.0])
    x = np.array([[5.0, 5.0, 5.0], [25.0, 5.0, 5.0]])   # 20 apart: never touching
    P = orc.Params()
    P.beta1, P.beta2, P.eps_x, P.eps_k, P.skin_s, P.skin_g = 0.0, 0.0, 1e-12, eps_k, 0.1, 0.02
    S = orc.Schedule()
    S.n_rungs, S.absolute, S.tol = len(rungs), 0, tol
    for r, (mu, ex, ek, dc, b) in enumerate(rungs):
        S.mu[r], S.eta_x[r], S.eta_k[r], S.decay[r], S.budget[r] = mu, ex, ek, dc, b
    st = orc.RunState(x, d0, 50.0, 1.0)
    status, res, tr = orc.run(st, P, S, trace_cap=64)
    return d0, x, st, status, res, tr


RUNGS3 = [(0.6, 1e-2, 0.05, 1.0, 3), (0.2, 4e-3, 0.02, 0.5, 2), (0.1, 2e-3, 0.03, 0.8, 4)]


def _kappa_by_hand(rungs, eps_k, n_iters, stop_in_final):
    """The schedule of App. A as a table of rungs, worked in exact rational
    arithmetic for two spheres that never touch (D0 = 1, 2): the overlap
    terms vanish, so dE/dkappa = -mu sum D0 = -3 mu, and with beta1 = beta2
    = 0 Adam's bias-corrected step is eta g / (|g| + eps) (m_hat = g,
    v_hat = g^2).  At a rung start mu = mu~ N_v / (kappa sum D0) with N_v =
    (sum D0^3)^2 / sum D0^6 = 81/65, eta_k = eta~_k kappa, eta_x = eta~_x
    kappa D0_min; every iteration of rung r multiplies mu and both step
    sizes by decay[r]."""
    from fractions import Fraction as F
    nv = F(81, 65)
    kap = F(1)
    ks = []
    r, itr = 0, 0

    def start(r, kap):
        mu_t, ex_t, ek_t = (F(v) for v in rungs[r][:3])
        return mu_t * nv / (kap * 3), ex_t * kap, ek_t * kap

    mu, ex, ek = start(0, kap)
    iters = 0
    while iters < n_iters:
        if stop_in_final and r == len(rungs) - 1:
            break                                  # max delta = 0 < tol
        ks.append(kap)
        g = -3 * mu
        kap = kap - ek * g / (abs(g) + F(eps_k))
        dc = F(rungs[r][3])
        mu, ex, ek = mu * dc, ex * dc, ek * dc
        itr += 1
        iters += 1
        if itr >= rungs[r][4]:
            if r == len(rungs) - 1:
                break
            r, itr = r + 1, 0
            mu, ex, ek = start(r, kap)
    return ks, kap, iters, r, (mu, ex, ek)


@pytest.mark.parametrize("eps_k", [0.7, 1e-12])
def test_schedule_machinery_hand_worked_stop(orc, eps_k):
    # the final rung's stop test (max delta < tol) ends the run before its
    # first update: 3 + 2 iterations, kappa grown by the hand-worked steps
    d0, x, st, status, res, tr = _separated_pair_schedule(orc, RUNGS3, 1e-3, eps_k)
    ks, kap, iters, r, etas = _kappa_by_hand(RUNGS3, eps_k, 100, True)
    assert status == 0 and res.iterations == iters == 5 and res.rung == r == 2
    assert np.array_equal(st.x, x)          # zero gradient: positions never move
    assert st.kappa[0] == pytest.approx(float(kap), rel=1e-14)
    for it, k in enumerate(ks):
        assert tr[it, 1] == pytest.approx(float(k), rel=1e-14)
    # rung 2 started with its own values at the kappa reached then
    assert st.etas[0] == pytest.approx(float(etas[0]), rel=1e-14)
    assert st.etas[1] == pytest.approx(float(etas[1]), rel=1e-14)
    assert st.etas[2] == pytest.approx(float(etas[2]), rel=1e-14)
    assert list(st.ctl) == [5, 2, 0, 0]


def test_schedule_machinery_hand_worked_cap(orc):
    # no stop (tol < 0): the final rung runs to its budget (status 1), with
    # mu and the steps decaying by 0.8 per iteration in it
    eps_k = 0.7
    d0, x, st, status, res, tr = _separated_pair_schedule(orc, RUNGS3, -1.0, eps_k)
    ks, kap, iters, r, etas = _kappa_by_hand(RUNGS3, eps_k, 100, False)
    assert status == 1 and res.iterations == iters == 9 and res.rung == 2
    assert st.kappa[0] == pytest.approx(float(kap), rel=1e-14)
    for it, k in enumerate(ks):
        assert tr[it, 1] == pytest.approx(float(k), rel=1e-14)
    assert st.etas[0] == pytest.approx(float(etas[0]), rel=1e-14)
    assert st.etas[2] == pytest.approx(float(etas[2]), rel=1e-14)
    assert list(st.ctl) == [9, 2, 4, 0]


# ------------------------------------------------------ list validity
def _dense_state(orc, iters=1500, seed=0):
    w = ri.c1_lognormal(seed)
    x0 = orc.rsa(w.d0, w.L, 1.0, w.seed)
    st = orc.RunState(x0, w.d0, w.L, 1.0)
    orc.run(st, orc.default_params(w.d0, s=0.3, g=0.02), orc.default_schedule(w.n),
            max_iters=iters)
    return w, st.x.copy(), float(st.kappa[0])


def test_rebuild_trigger_keeps_every_contact_listed(orc):
    # App. A rebuilds on accumulated displacement; with the rule as stated
    # every overlapping pair is in the list at every gradient evaluation
    w, x, k = _dense_state(orc)
    P = orc.default_params(w.d0, s=0.05, g=0.01)
    st = orc.RunState(x, w.d0, w.L, k)
    try:
        orc.set_list_check(True)
        status, res, _ = orc.run(st, P, orc.default_schedule(w.n), max_iters=400)
        assert orc.list_misses() == 0
        assert res.rebuilds > 5
        # a planted mistake (ten times the displacement allowance) is caught
        st2 = orc.RunState(x, w.d0, w.L, k)
        orc.set_list_check(True, trigger_scale=10.0)
        orc.run(st2, P, orc.default_schedule(w.n), max_iters=400)
        assert orc.list_misses() > 0
    finally:
        orc.set_list_check(False)


def test_skin_changes_only_the_summation_order(orc):
    # a run that rebuilds at every step (skin 0: any motion invalidates the
    # list) and one with a skin follow the same trajectory up to rounding
    w, x, k = _dense_state(orc)
    mu, ex, ek, steps = 2e-3, 2e-3, 2e-4, 30
    out = []
    for s, g in ((0.0, 0.0), (0.5, 0.05)):
        st = orc.RunState(x, w.d0, w.L, k)
        _, res, _ = orc.run(st, orc.default_params(w.d0, s=s, g=g),
                            orc.oracle.absolute_schedule(mu, ex, ek, steps))
        out.append((st.x.copy(), float(st.kappa[0]), res.rebuilds))
    assert out[0][2] >= steps and out[1][2] < steps / 3
    d = np.abs(out[0][0] - out[1][0])
    d = np.minimum(d, w.L - d)
    assert d.max() <= 1e-10 * ex * steps
    assert out[0][1] == pytest.approx(out[1][1], rel=1e-13)


# ------------------------------------------- per-row gradient, brute force
def test_rows_grad_equals_pair_gradient(orc):
    x, d0, L = _overlapping_case(n=600, phi=0.5, S=6.0, seed=21)
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    r = orc.energy_grad(x, d0, L, 1.0, 0.0, pi, pj)
    rows = np.arange(0, 600, 7)
    g, gs, st = orc.rows_grad(x, d0, L, 1.0, rows)
    assert np.all(np.abs(g - r["g"][rows]) <= 1e-13 * r["gscale"][rows])
    assert np.allclose(gs, r["gscale"][rows], rtol=1e-13, atol=0)
    gall, _, stall = orc.rows_grad(x, d0, L, 1.0, np.arange(600))
    # each pair's energy is counted in both of its rows
    assert stall[:, 0].sum() == pytest.approx(2 * r["E_ov"], rel=1e-12)
    assert stall[:, 1].sum() == pytest.approx(2 * r["gk_ov"], rel=1e-12)
    assert stall[:, 2].max() == r["max_delta"]
    assert np.all(np.abs(gall - r["g"]) <= 1e-13 * r["gscale"])


# -------------------------------------- skin predicate, independent numpy
@pytest.mark.parametrize("S,phi,kb,s,g", [(30.0, 0.4, 1.3, 0.7, 0.05), (4.0, 0.6, 0.9, 0.25, 0.1),
                                         (200.0, 0.2, 1.0, 2.0, 0.02)])
def test_skin_predicate_against_numpy(orc, S, phi, kb, s, g):
    # the listing rule written out directly (same operation order, no
    # contraction: numpy rounds every operation): minimum image with one
    # shift beyond +-L/2, r^2 = (dx^2 + dy^2) + dz^2,
    # c = kb ((1 + g) (D0_i + D0_j)/2 + 2 s D0_min), listed iff r^2 < c^2
    w = ri.small_polydisperse(1500, S, phi, seed=31, family="powerlaw")
    x, d0, L = w.x, w.d0, w.L
    hL = 0.5 * L
    i, j = np.triu_indices(len(d0), 1)
    sep = []
    for a in range(3):
        t = x[j, a] - x[i, a]
        sep.append(np.where(t > hL, t - L, np.where(t < -hL, t + L, t)))
    r2 = (sep[0] * sep[0] + sep[1] * sep[1]) + sep[2] * sep[2]
    c = kb * ((1.0 + g) * (0.5 * (d0[i] + d0[j])) + (2.0 * s) * d0.min())
    keep = r2 < c * c
    oi, oj = orc.pairs_brute(x, d0, L, kb, s, g)
    assert keep.sum() > 1000
    assert np.array_equal(oi, i[keep]) and np.array_equal(oj, j[keep])


# ------------------------------------------ coincident centres, +-L/2 image
def test_coincident_centres_hand_values(orc):
    # r = 0: delta = 1, the pair counts in E (1/2) and in max delta but adds
    # nothing to dE/dkappa (delta r / (kappa d) = 0) and nothing to the
    # position gradient (the subgradient 0 is taken)
    d0 = np.array([1.0, 3.0])
    x = np.array([[4.0, 5.0, 6.0], [4.0, 5.0, 6.0]])
    r = orc.energy_grad(x, d0, 20.0, 2.0, 0.0, [0], [1])
    assert r["E_ov"] == 0.5 and r["gk_ov"] == 0.0 and r["max_delta"] == 1.0
    assert r["n_overlap"] == 1 and np.all(r["g"] == 0.0)


@pytest.mark.parametrize("flip", [False, True])
def test_half_box_separation_takes_no_shift(orc, flip):
    # a separation of exactly L/2 (or -L/2) is not shifted: with L = 10, D0 =
    # (4, 8), kappa = 1: d = 6, r = 5, delta = 1/6; E = 1/72; dE/dkappa =
    # delta r / (kappa d) = 5/36; dE/dx_i = delta / (d r) (x_j - x_i) = +-1/36
    d0 = np.array([4.0, 8.0])
    xa, xb = (6.0, 1.0) if flip else (1.0, 6.0)
    x = np.array([[xa, 2.0, 3.0], [xb, 2.0, 3.0]])
    r = orc.energy_grad(x, d0, 10.0, 1.0, 0.0, [0], [1])
    sgn = -1.0 if flip else 1.0
    assert r["E_ov"] == pytest.approx(1.0 / 72.0, rel=1e-15)
    assert r["gk_ov"] == pytest.approx(5.0 / 36.0, rel=1e-15)
    assert r["g"][0, 0] == pytest.approx(sgn / 36.0, rel=1e-15)
    assert r["g"][1, 0] == pytest.approx(-sgn / 36.0, rel=1e-15)
    assert np.all(r["g"][:, 1:] == 0.0)
    # the listing rule uses the same unshifted separation
    pi, pj = orc.pairs_brute(x, d0, 10.0, 1.0, 0.0, 0.0)
    assert list(pi) == [0] and list(pj) == [1]


# ------------------------------------------------- stored oracle whole runs
def test_stored_census_runs_come_from_the_oracle(orc):
    # the stored whole-run results are the oracle's: its smallest case, rerun,
    # gives the stored phi to the last bit
    import json
    with open(os.path.join(GOLD, "census8_phi_oracle.json")) as fh:
        runs = json.load(fh)["runs"]
    w = sorted(ri.census_draw(64), key=lambda w: w.n)[0]
    g = runs[0]
    assert (g["n"], g["seed"]) == (w.n, 1000)
    st = orc.RunState(orc.rsa(w.d0, w.L, 1.0, 1000), w.d0, w.L, 1.0)
    S = float(w.d0.max() / w.d0.min())
    status, res, _ = orc.run(st, orc.default_params(w.d0, s=0.5), orc.default_schedule(w.n, S=S))
    assert status == g["status"] == 0
    assert res.iterations == g["iterations"]
    assert res.phi == g["phi"]


# ------------------------------------------------ placement in rounds
@pytest.mark.parametrize("seed", [0, 3])
def test_rsa_rounds_of_one_is_sequential_rsa(orc, seed):
    # a round of one proposal is the sequential procedure, attempt for
    # attempt (an independent implementation with a single grid)
    w = ri.c1_lognormal(seed)
    x1 = orc.rsa(w.d0, w.L, 1.0, w.seed)
    x2, nr = orc.rsa_rounds(w.d0, w.L, 1.0, w.seed, 1)
    assert np.array_equal(x1, x2) and nr >= w.n
    d0 = ri.lognormal_quantiles(1500, 0.7, 60.0)
    L = ri.box_for_phi(d0, 0.08)
    assert np.array_equal(orc.rsa(d0, L, 1.0, 11), orc.rsa_rounds(d0, L, 1.0, 11, 1)[0])


@pytest.mark.parametrize("window", [16, 256, 1 << 16])
def test_rsa_rounds_non_overlapping_uniform_deterministic(orc, window):
    d0 = ri.lognormal_quantiles(3000, 0.7, 60.0)
    L = ri.box_for_phi(d0, 0.08)
    x, nr = orc.rsa_rounds(d0, L, 1.0, 5, window)
    x2, nr2 = orc.rsa_rounds(d0, L, 1.0, 5, window)
    assert np.array_equal(x, x2) and nr == nr2
    assert np.all((x >= 0) & (x < L))
    pi, _ = orc.pairs_brute(x, d0, L, 1.0, 0.0, 0.0)
    assert len(pi) == 0
    for a in range(3):
        assert stats.kstest(x[:, a] / L, "uniform").pvalue > 1e-3
    # fewer rounds than spheres once a round holds several proposals
    assert nr < 3000 or window == 1


# ------------------------------------------ frozen spheres (cascade stages)
def test_frozen_two_sphere_hand_values(orc):
    # a frozen sphere against a growing one (tests/golden/two_sphere_frozen.txt)
    gd = _golden("two_sphere_frozen.txt")
    d0 = np.array(gd["D0"])
    L = 20.0
    x = np.array([[10.0, 7.0, 9.0], [10.0 + gd["r"], 7.0, 9.0]])
    pi, pj = np.array([0], np.int32), np.array([1], np.int32)
    orc.set_frozen(np.array([1, 0], np.uint8))
    try:
        r = orc.energy_grad(x, d0, L, gd["kappa"], gd["mu"], pi, pj)
        assert r["E_ov"] == pytest.approx(gd["E_overlap"], rel=1e-15)
        assert r["gk_ov"] == pytest.approx(gd["dEdkappa_overlap"], rel=1e-15)
        assert r["E_growth"] == pytest.approx(gd["E_growth"], rel=1e-15)
        assert r["gk_growth"] == pytest.approx(gd["dEdkappa_growth"], rel=1e-15)
        assert r["max_delta"] == pytest.approx(0.25, rel=1e-15)
        assert r["g"][0, 0] == pytest.approx(gd["grad_along_line"], rel=1e-15)
        assert r["g"][1, 0] == pytest.approx(-gd["grad_along_line"], rel=1e-15)
        assert np.all(r["g"][:, 1:] == 0.0)
        touch = orc.energy_grad(x, d0, L, 1.0, gd["mu"], pi, pj)
        assert touch["E_ov"] == 0.0 and touch["n_overlap"] == 0
        # the frozen sphere's diameter does not follow kappa: with the mask
        # cleared the same numbers give the plain two-sphere case
        orc.set_frozen(None)
        plain = orc.energy_grad(x, d0, L, gd["kappa"], gd["mu"], pi, pj)
        assert plain["E_ov"] != pytest.approx(gd["E_overlap"])
    finally:
        orc.set_frozen(None)


def test_frozen_mask_of_zeros_is_the_plain_protocol(orc):
    x, d0, L = _overlapping_case(n=120, phi=0.5)
    pi, pj = _all_overlaps(orc, x, d0, L, 1.0)
    ref = orc.energy_grad(x, d0, L, 1.0, 0.3, pi, pj)
    orc.set_frozen(np.zeros(d0.shape[0], np.uint8))
    try:
        got = orc.energy_grad(x, d0, L, 1.0, 0.3, pi, pj)
    finally:
        orc.set_frozen(None)
    for k in ("E_ov", "gk_ov", "E_growth", "gk_growth", "max_delta"):
        assert got[k] == pytest.approx(ref[k], rel=1e-13, abs=1e-300), k
    assert np.allclose(got["g"], ref["g"], rtol=1e-13, atol=1e-15)


def test_frozen_energy_central_finite_differences(orc):
    # dE/dkappa and dE/dx with a third of the spheres frozen (absolute
    # diameters), against central differences of the energy
    x, d0, L = _overlapping_case(n=150, phi=0.5)
    rng = np.random.default_rng(5)
    mask = (rng.random(d0.shape[0]) < 0.33).astype(np.uint8)
    kappa = 1.0
    d = d0.copy()
    d[mask == 1] *= kappa   # the frozen ones at their size for kappa = 1
    orc.set_frozen(mask)
    try:
        def E(xx, kk):
            pi, pj = orc.pairs_brute(xx, np.where(mask == 1, d, d * kk), L, 1.0)
            return orc.energy_grad(xx, d, L, kk, 0.3, pi, pj)
        r = E(x, kappa)
        assert r["n_overlap"] > 50
        hk = 1e-7
        Ep, Em = E(x, kappa + hk), E(x, kappa - hk)
        fdk = ((Ep["E_ov"] + Ep["E_growth"]) - (Em["E_ov"] + Em["E_growth"])) / (2 * hk)
        assert fdk == pytest.approx(r["gk_ov"] + r["gk_growth"], rel=1e-6)
        h = 1e-7 * d0.min()
        checked = 0
        for i in rng.choice(x.shape[0], 30, replace=False):
            for a in range(3):
                xp, xm = x.copy(), x.copy()
                xp[i, a] += h
                xm[i, a] -= h
                fd = (E(xp, kappa)["E_ov"] - E(xm, kappa)["E_ov"]) / (2 * h)
                sc = r["gscale"][i, a]
                if sc == 0:
                    continue
                assert abs(fd - r["g"][i, a]) <= 1e-6 * max(sc, abs(r["E_ov"]) * 1e-3)
                checked += 1
        assert checked > 20
    finally:
        orc.set_frozen(None)


def test_frozen_spheres_hold_still_while_the_others_inflate(orc):
    # a cascade stage in miniature: 10 frozen spheres, 300 small ones seated
    # in their voids and inflated until the stop criterion
    d = np.ones(10)
    L = float((np.pi / 6.0 * 10 / 0.3) ** (1.0 / 3.0))
    xb = orc.rsa(d, L, 1.0, 4)
    d0 = np.concatenate([d, np.full(300, 0.2)])
    mask = np.concatenate([np.ones(10, np.uint8), np.zeros(300, np.uint8)])
    orc.set_frozen(mask)
    try:
        xs = orc.seat(np.concatenate([xb, np.zeros((300, 3))]), d0, L, 0.4, 4)
        assert np.array_equal(xs[:10], xb)
        st = orc.RunState(xs, d0, L, 0.4)
        status, res, _ = orc.run(st, orc.default_params(d0[10:], 0.4),
                                 orc.default_schedule(300, S=1.0))
        assert status == 0 and res.max_overlap < 5e-4
        assert np.array_equal(st.x[:10], xb)            # positions held
        assert np.all(st.m[:10] == 0) and np.all(st.v[:10] == 0)
        assert st.kappa[0] > 0.4                        # the small ones grew
        phi_f = orc.phi_frozen(d0, L, st.kappa[0])
        big = np.pi / 6.0 * 10 / L ** 3
        assert phi_f == pytest.approx(big + np.pi / 6.0 * 300 * (0.2 * st.kappa[0]) ** 3 / L ** 3,
                                      rel=1e-12)
        assert res.phi == pytest.approx(phi_f, rel=1e-15)
    finally:
        orc.set_frozen(None)


def test_seating_is_the_first_free_proposal(orc):
    # every seated sphere sits at its first proposal that overlaps no frozen
    # sphere (checked by brute force in numpy), whatever the thread count
    d = np.ones(12)
    L = float((np.pi / 6.0 * 12 / 0.3) ** (1.0 / 3.0))
    xb = orc.rsa(d, L, 1.0, 9)
    n = 200
    d0 = np.concatenate([d, np.full(n, 0.3)])
    mask = np.concatenate([np.ones(12, np.uint8), np.zeros(n, np.uint8)])
    k0 = 0.5
    orc.set_frozen(mask)
    try:
        xs = orc.seat(np.concatenate([xb, np.zeros((n, 3))]), d0, L, k0, 9)
        orc.set_threads(1)
        xs1 = orc.seat(np.concatenate([xb, np.zeros((n, 3))]), d0, L, k0, 9)
    finally:
        orc.set_threads(0)
        orc.set_frozen(None)
    assert np.array_equal(xs, xs1)
    hL = 0.5 * L
    for i in range(12, 12 + n):
        for a in range(1 << 12):
            p = np.array([orc.u01(9, i, a, ax) * L for ax in range(3)])
            p[p >= L] -= L
            sep = xb - p
            sep = np.where(sep > hL, sep - L, np.where(sep < -hL, sep + L, sep))
            r2 = (sep[:, 0] * sep[:, 0] + sep[:, 1] * sep[:, 1]) + sep[:, 2] * sep[:, 2]
            dd = 0.5 * (d + k0 * 0.3)
            if np.all(r2 >= dd * dd):
                assert np.array_equal(xs[i], p), i
                break
        else:
            raise AssertionError("no free proposal for %d" % i)


def test_cascade_counts_give_eq_cascade():
    # with every class filling its voids at phi1 (nominal diameters
    # rho^-c), the counts give the ideal phi_n = 1 - (1 - phi1)^n of
    # Eq. (cascade)
    from oracle import cascade_counts
    phi1, rho = 0.6435, 7.0
    n1 = 1000
    counts = cascade_counts(n1, rho, 4, phi1)
    V = n1 / phi1   # box volume in units of one class-1 sphere
    for n in range(1, 5):
        vol = sum(counts[c] * rho ** (-3 * c) for c in range(n))
        assert vol / V == pytest.approx(1.0 - (1.0 - phi1) ** n, rel=2e-3)


@pytest.mark.slow
def test_binary_cascade_fills_the_voids(orc):
    # Table (tab:cascade): one class packs near 0.62-0.64, two classes at a
    # diameter ratio of about 7 near 0.80 (0.800 printed for 30-60 coarse
    # spheres); a cascade of 8 coarse spheres lands in the same range, and
    # the second class raises phi by far more than a monodisperse packing's
    # finite-size scatter
    phis, counts = orc.cascade(8, 7.0, 2, seed=0)
    assert counts == [8, 978]
    assert 0.58 < phis[0] < 0.70
    assert 0.74 < phis[1] < 0.85
    assert phis[1] - phis[0] > 0.1


# ------------------------------------------------- two dimensions (Sec. 2)
@pytest.fixture
def orc2(orc):
    orc.set_dim(2)
    yield orc
    orc.set_dim(3)


def test_2d_square_lattice_shrinks_to_touching(orc2):
    # n x n equal disks on a square lattice of spacing 1 in a periodic box
    # of side n: at kappa = 1.3 every lattice neighbour overlaps; the
    # shrink lands on touching, kappa' = 1, and the area fraction is then
    # pi / 4 (closed form); gradients vanish by symmetry
    n = 6
    g = np.arange(n) + 0.5
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), np.zeros(n * n)], axis=1)
    d0 = np.ones(n * n)
    L = float(n)
    pi, pj = orc2.pairs_brute(x, d0, L, 1.3, 0.0, 0.0)
    assert pi.shape[0] == 2 * n * n        # 4 neighbours each, pairs counted once
    r = orc2.energy_grad(x, d0, L, 1.3, 0.0, pi, pj)
    delta = 1.0 - 1.0 / 1.3
    assert r["E_ov"] == pytest.approx(2 * n * n * 0.5 * delta ** 2, rel=1e-13)
    assert np.abs(r["g"]).max() <= 1e-13
    kp = orc2.shrink(x, d0, L, 1.3, pi, pj)
    assert kp == 1.0
    assert orc2.phi(d0, L, kp) == pytest.approx(np.pi / 4.0, rel=1e-15)


def test_2d_rsa_stays_in_the_plane(orc2):
    w = ri.small_polydisperse(400, 3.0, 0.3, seed=5)
    L = float(np.sqrt(np.pi / 4.0 * np.sum(w.d0 ** 2) / 0.3))
    x = orc2.rsa(w.d0, L, 1.0, 8)
    assert np.all(x[:, 2] == 0.0)
    pi, pj = orc2.pairs_brute(x, w.d0, L, 1.0, 0.0, 0.0)
    assert pi.shape[0] == 0
    for ax in range(2):
        assert stats.kstest(x[:, ax] / L, "uniform").pvalue > 1e-3
    assert np.array_equal(x, orc2.rsa(w.d0, L, 1.0, 8))


def test_2d_area_participation_number_sets_mu(orc2):
    # two disks, D0 = 1 and 2: N_v = (1 + 4)^2 / (1 + 16) = 25/17 in 2-D
    # (against (1 + 8)^2 / (1 + 64) = 81/65 in 3-D); the rung start sets
    # mu = mu~ N_v / (kappa sum D0)
    d0 = np.array([1.0, 2.0])
    x = np.array([[1.0, 1.0, 0.0], [5.0, 5.0, 0.0]])
    sc = orc2.default_schedule(2, d=2)
    st = orc2.RunState(x, d0, 10.0, 1.0)
    orc2.run(st, orc2.default_params(d0), sc, max_iters=1)
    assert st.etas[0] == pytest.approx(sc.mu[0] * (25.0 / 17.0) / 3.0, rel=1e-14)


def test_2d_bidisperse_run_jams_in_the_plane(orc2):
    # 50:50 disks of diameter ratio 1.4 (the usual 2-D glass former): the
    # protocol stops with z untouched, at an area fraction in the range
    # reported for random close packing of such mixtures (about 0.84)
    n = 512
    d0 = np.where(np.arange(n) % 2 == 0, 1.0, 1.4)
    L = float(np.sqrt(np.pi / 4.0 * np.sum(d0 ** 2) / 0.1))
    x = orc2.rsa(d0, L, 1.0, 2)
    st = orc2.RunState(x, d0, L, 1.0)
    status, res, _ = orc2.run(st, orc2.default_params(d0), orc2.default_schedule(n, d=2, S=1.4))
    assert status == 0 and res.max_overlap < 5e-4
    assert np.all(st.x[:, 2] == 0.0)
    assert 0.80 < res.phi < 0.88


# ------------------------------------- close-packed lattices (closed forms)
def _lattice(kind, n):
    # n^3 cubic cells of side 1 in a periodic cube of side n: face-centred
    # (4 sites a cell, nearest neighbours at 1/sqrt(2), 12 of them) or
    # body-centred (2 sites, nearest at sqrt(3)/2 along the body diagonals,
    # 8 of them); sites offset by a quarter cell so that no coordinate sits
    # on the wrap point
    basis = {"fcc": [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)],
             "bcc": [(0, 0, 0), (0.5, 0.5, 0.5)]}[kind]
    c = np.stack(np.meshgrid(*(np.arange(n),) * 3, indexing="ij"), -1).reshape(-1, 3)
    x = (c[:, None, :] + np.array(basis)[None, :, :] + 0.25).reshape(-1, 3)
    contact, z, phi = {"fcc": (np.sqrt(0.5), 12, np.pi / (3.0 * np.sqrt(2.0))),
                       "bcc": (np.sqrt(0.75), 8, np.pi * np.sqrt(3.0) / 8.0)}[kind]
    return x.astype(np.float64), contact, z, phi, float(n)


@pytest.mark.parametrize("kind", ["fcc", "bcc"])
def test_close_packed_lattices_closed_forms(orc, kind):
    # equal spheres of diameter the nearest-neighbour distance: at kappa > 1
    # exactly the z nearest neighbours of each site overlap, each pair by
    # delta = 1 - 1/kappa (r = D0, d = kappa D0), so E = (z N / 2) delta^2 / 2
    # and dE/dkappa = (z N / 2) delta / kappa^2; every gradient vanishes by
    # the lattice's inversion symmetry; the shrink lands on touching,
    # kappa' = 1, and phi is the lattice's packing fraction
    x, D, z, phi_lat, L = _lattice(kind, 3)
    n = x.shape[0]
    d0 = np.full(n, D)
    kappa = 1.15
    pi, pj = orc.pairs_brute(x, d0, L, kappa, 0.0, 0.0)
    assert pi.shape[0] == z * n // 2
    assert np.all(np.bincount(np.concatenate([pi, pj]), minlength=n) == z)
    r = orc.energy_grad(x, d0, L, kappa, 0.0, pi, pj)
    delta = 1.0 - 1.0 / kappa
    P = z * n / 2
    assert r["n_overlap"] == P
    assert r["E_ov"] == pytest.approx(P * 0.5 * delta ** 2, rel=1e-12)
    assert r["gk_ov"] == pytest.approx(P * delta / kappa ** 2, rel=1e-12)
    assert r["max_delta"] == pytest.approx(delta, rel=1e-12)
    assert np.abs(r["g"]).max() <= 1e-12
    kp = orc.shrink(x, d0, L, kappa, pi, pj)
    assert kp == pytest.approx(1.0, rel=1e-15)
    assert orc.phi(d0, L, kp) == pytest.approx(phi_lat, rel=1e-14)
    # at kappa just below touching no pair overlaps and the shrink keeps kappa
    pi0, pj0 = orc.pairs_brute(x, d0, L, 0.999, 0.0, 0.0)
    assert pi0.shape[0] == 0
    assert orc.energy_grad(x, d0, L, 0.999, 0.0, pi, pj)["E_ov"] == 0.0


def test_fcc_site_displacement_restoring_force(orc):
    # one site of the face-centred lattice moved by e along x, at kappa =
    # 1.2 (every nearest-neighbour pair overlapping by delta = 1/6): its
    # gradient is dE/de = sum_j delta_j (a_jx - e) / (kappa D r_j) over its
    # 12 neighbours a_j (|a_j| = D = 1/sqrt(2)); to first order in e that
    # is k e with k = c (12 c - 12 / D + sum_j a_jx^2 / D^3), c = 1 / (kappa
    # D), and sum_j a_jx^2 = 2 (8 neighbours with a_jx = +-1/2): k = (2 /
    # kappa) (12 / kappa - 8) = 10/3.  Checked by the central difference of
    # the oracle's gradient and against a brute-force sum over every site
    x, D, z, _, L = _lattice("fcc", 3)
    n = x.shape[0]
    d0 = np.full(n, D)
    kappa = 1.2
    pi, pj = orc.pairs_brute(x, d0, L, kappa + 0.05, 0.0, 0.0)
    site = 13

    def g(e):
        y = x.copy()
        y[site, 0] += e
        return orc.energy_grad(y, d0, L, kappa, 0.0, pi, pj)["g"][site]

    def brute(e):
        p = x[site] + np.array([e, 0.0, 0.0])
        out = np.zeros(3)
        for j in range(n):
            if j == site:
                continue
            dv = x[j] - p
            dv -= L * np.round(dv / L)
            rj = np.linalg.norm(dv)
            dl = 1.0 - rj / (kappa * D)
            if dl > 0:
                out += dl / (kappa * D) * dv / rj
        return out      # dE/dx of the displaced site (d delta / dp = dv / (kappa D r))

    k = (2.0 / kappa) * (12.0 / kappa - 8.0)
    h = 1e-6
    assert (g(h)[0] - g(-h)[0]) / (2 * h) == pytest.approx(k, rel=1e-8)
    for e in (1e-3, -2e-3, 0.01):
        np.testing.assert_allclose(g(e), brute(e), rtol=1e-11, atol=1e-14)
        assert g(e)[0] * e > 0   # the energy rises as the site leaves its cage
        assert abs(g(e)[1]) <= 1e-14 and abs(g(e)[2]) <= 1e-14


@pytest.mark.parametrize("kind", ["fcc", "bcc"])
def test_lattice_kappa_adam_is_the_scalar_recurrence(orc, kind):
    # with the position step zero the sites stay on the lattice and every
    # iteration sees E(kappa) = (z N / 2) (1 - 1/kappa)^2 / 2 exactly, so
    # Adam on kappa (App. A; Kingma and Ba, bias-corrected) is the scalar
    # recurrence on dE/dkappa = (z N / 2) (1 - 1/kappa) / kappa^2
    x, D, z, _, L = _lattice(kind, 4)
    n = x.shape[0]
    d0 = np.full(n, D)
    kappa, eta_k, steps = 1.1, 2e-3, 12
    P = orc.default_params(d0, s=0.2, g=0.02)
    st = orc.RunState(x, d0, L, kappa)
    status, res, _ = orc.run(st, P, orc.absolute_schedule(0.0, 0.0, eta_k, steps))
    assert status == 1 and res.iterations == steps
    m = v = 0.0
    b1t = b2t = 1.0
    k = kappa
    for _ in range(steps):
        g = (z * n / 2) * (1.0 - 1.0 / k) / k ** 2
        b1t *= P.beta1
        b2t *= P.beta2
        m = P.beta1 * m + (1.0 - P.beta1) * g
        v = P.beta2 * v + (1.0 - P.beta2) * g * g
        k = k - eta_k * (m / (1.0 - b1t)) / (np.sqrt(v / (1.0 - b2t)) + P.eps_k)
    assert st.kappa[0] == pytest.approx(k, rel=1e-13)
    assert np.array_equal(st.x, x)
