"""Differentiation path: the energy kernel and its hand-written adjoint
behind torch.autograd.Function, against torch's gradcheck (finite
differences on a small packing), central finite differences with
h = 1e-7 D_min on the dense C3 state, and the FP64 oracle on a 1e4-sphere
subset of C3 (1e-10 per component relative to the sum of absolute pair
contributions)."""
import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2608_12235_amd as m
    m.lib()
    return torch, m


@pytest.fixture(scope="module")
def c3(env):
    torch, m = env
    w = ri.c3_lognormal_dense(seed=0)
    p = m.Packing(w.d0, w.L, 1.0, 0, init="none", params=m.make_params(skin_s=2.0, skin_g=0.02))
    x = torch.tensor(w.x, dtype=torch.float64, device="cuda")
    return w, p, x


def _far_from_contact(orc, x, d0, L, kappa, margin):
    pi, pj = orc.pairs_brute(x, d0, L, kappa, 0.0, 0.02)
    dx = x[pj] - x[pi]
    dx -= L * np.round(dx / L)
    r = np.sqrt((dx * dx).sum(1))
    d = kappa * 0.5 * (d0[pi] + d0[pj])
    return np.all(np.abs(r / d - 1.0) > margin)


def test_gradcheck_small(env, orc):
    torch, m = env
    # a small overlapping packing whose pairs all stay clear of contact by
    # much more than the finite-difference step
    for seed in range(50):
        w = ri.small_polydisperse(120, 4.0, 0.3, seed=seed)
        if _far_from_contact(orc, w.x, w.d0, w.L, 1.0, 1e-4):
            break
    else:
        pytest.skip("no seed without near-contact pairs")
    _say("gradcheck N=120 seed", seed)
    p = m.Packing(w.d0, w.L, 1.0, 0, init="none", params=m.make_params(skin_s=0.2))
    x = torch.tensor(w.x, dtype=torch.float64, device="cuda", requires_grad=True)
    k = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda xx, kk: m.overlap_energy(xx, kk, p, 3e-3)[0]
    assert torch.autograd.gradcheck(f, (x, k), eps=1e-6, atol=1e-7, rtol=1e-6)


def test_forward_and_adjoint_match_oracle(env, orc):
    torch, m = env
    w = ri.small_polydisperse(3000, 50.0, 0.45, seed=5)
    p = m.Packing(w.d0, w.L, 1.0, 0, init="none", params=m.make_params(skin_s=0.5))
    x = torch.tensor(w.x, dtype=torch.float64, device="cuda", requires_grad=True)
    k = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    mu = 2e-3
    E, mx = m.overlap_energy(x, k, p, mu)
    E.backward()
    pi, pj = orc.pairs_brute(w.x, w.d0, w.L, 1.0, 0.0, 0.0)
    r = orc.energy_grad(w.x, w.d0, w.L, 1.0, mu, pi, pj)
    assert abs(E.item() - (r["E_ov"] + r["E_growth"])) <= TOL * (r["E_ov"] + abs(r["E_growth"]))
    assert mx.item() == pytest.approx(r["max_delta"], rel=1e-13)
    g = x.grad.cpu().numpy()
    err = np.abs(g - r["g"])
    assert np.all(err <= TOL * r["gscale"]), float(np.max(err / (r["gscale"] + 1e-300)))
    gk = k.grad.item()
    want = r["gk_ov"] + r["gk_growth"]
    assert abs(gk - want) <= TOL * (abs(r["gk_ov"]) + abs(r["gk_growth"]))


def test_c3_adjoint_matches_oracle_on_subset(env, orc, c3):
    torch, m = env
    w, p, x0 = c3
    _say("C3 adjoint vs oracle rows")
    x = x0.clone().requires_grad_(True)
    k = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    E, _ = m.overlap_energy(x, k, p, 2e-3)
    E.backward()
    rows = np.sort(np.random.default_rng(7).choice(w.n, 10000, replace=False))
    g, gs, _ = orc.rows_grad(w.x, w.d0, w.L, 1.0, rows)
    got = x.grad[torch.tensor(rows, device="cuda")].cpu().numpy()
    err = np.abs(got - g)
    assert np.all(err <= TOL * gs), float(np.max(err / (gs + 1e-300)))


def test_c3_central_finite_differences(env, c3):
    torch, m = env
    w, p, x0 = c3
    mu = 2e-3
    h = 1e-7 * float(w.d0.min())
    rng = np.random.default_rng(11)
    rows = rng.choice(w.n, 1000, replace=False)
    axes = rng.integers(0, 3, 1000)
    x = x0.clone().requires_grad_(True)
    k = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    E, _ = m.overlap_energy(x, k, p, mu)
    E.backward()
    g = x.grad.cpu().numpy()
    gk = k.grad.item()
    _say("C3 finite differences, 1000 coordinates + kappa")
    kk = torch.tensor(1.0, dtype=torch.float64, device="cuda")
    xs = x0.clone()
    worst = 0.0
    for i, a in zip(rows, axes):
        xs[i, a] += h
        ep = m.overlap_energy(xs, kk, p, mu)[0].item()
        xs[i, a] -= 2 * h
        em = m.overlap_energy(xs, kk, p, mu)[0].item()
        xs[i, a] += h
        fd = (ep - em) / (2 * h)
        # rounding of E (about 1e5 here) over 2h bounds the FD accuracy
        worst = max(worst, abs(fd - g[i, a]) / (1e-3 + 1e-4 * abs(g[i, a])))
    assert worst <= 1.0, worst
    hk = 1e-7
    ep = m.overlap_energy(x0, torch.tensor(1.0 + hk, dtype=torch.float64), p, mu)[0].item()
    em = m.overlap_energy(x0, torch.tensor(1.0 - hk, dtype=torch.float64), p, mu)[0].item()
    fdk = (ep - em) / (2 * hk)
    assert fdk == pytest.approx(gk, rel=1e-6)
