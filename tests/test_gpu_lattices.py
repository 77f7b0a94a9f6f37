"""Close-packed lattices on the GPU, through the C ABI, against closed forms
that do not involve the oracle: equal spheres on face- and body-centred
cubic lattices in a periodic cube, touching at kappa = 1.  Also: the two
read-back paths of the state give the same positions.

At kappa > 1 exactly the z nearest neighbours of every site overlap, each
pair by delta = 1 - 1/kappa (Eq. (energy) with r = D0, d = kappa D0); the
gradient of every site vanishes by inversion symmetry; the shrink lands on
touching and phi is the lattice's packing fraction.  With the position
step set to zero, Adam on kappa alone (App. A) is the scalar recurrence on
E(kappa) = (z N / 2) (1 - 1/kappa)^2 / 2.
"""
import math

import numpy as np
import pytest

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


def _lattice(kind, n):
    # n^3 cubic cells of side 1 in a periodic cube of side n, sites offset by
    # a quarter cell (no coordinate on the wrap point)
    basis = {"fcc": [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)],
             "bcc": [(0, 0, 0), (0.5, 0.5, 0.5)]}[kind]
    c = np.stack(np.meshgrid(*(np.arange(n),) * 3, indexing="ij"), -1).reshape(-1, 3)
    x = (c[:, None, :] + np.array(basis)[None, :, :] + 0.25).reshape(-1, 3)
    contact, z, phi = {"fcc": (math.sqrt(0.5), 12, math.pi / (3.0 * math.sqrt(2.0))),
                       "bcc": (math.sqrt(0.75), 8, math.pi * math.sqrt(3.0) / 8.0)}[kind]
    return x.astype(np.float64), contact, z, phi, float(n)


@pytest.mark.parametrize("kind", ["fcc", "bcc"])
@pytest.mark.parametrize("skin", [0.05, 0.4])
def test_lattice_energy_shrink_closed_forms(rcp, kind, skin):
    x, D, z, phi_lat, L = _lattice(kind, 4)
    n = x.shape[0]
    d0 = np.full(n, D)
    kappa = 1.15
    _say("lattice", kind, "N", n, "skin", skin)
    p = rcp.Packing(d0, L, 1.0, 0, init="none",
                    params=rcp.make_params(skin_s=skin, skin_g=0.02))
    p.set_state(x, kappa)
    e = p.energy_grad(mu=0.0)
    P = z * n // 2
    delta = 1.0 - 1.0 / kappa
    assert e["n_overlap"] == P
    assert e["E_overlap"] == pytest.approx(P * 0.5 * delta ** 2, rel=1e-12)
    assert e["dE_dkappa_overlap"] == pytest.approx(P * delta / kappa ** 2, rel=1e-12)
    assert e["max_overlap"] == pytest.approx(delta, rel=1e-12)
    assert np.abs(e["g"]).max() <= 1e-12
    kp, phi = p.shrink()
    p.close()
    assert kp == pytest.approx(1.0, rel=1e-15)
    assert phi == pytest.approx(phi_lat, rel=1e-14)


@pytest.mark.parametrize("kind", ["fcc", "bcc"])
def test_lattice_adam_on_kappa_is_the_scalar_recurrence(rcp, kind):
    # eta_x = 0 holds the sites where they are: with a position step, Adam
    # would scale the rounding-size gradients of the symmetric sites up to
    # steps of order eta_x, and the compressed lattice would leave its
    # symmetric state (on the oracle as on the GPU, each with its own noise)
    x, D, z, _, L = _lattice(kind, 4)
    n = x.shape[0]
    d0 = np.full(n, D)
    kappa, eta_k, steps = 1.1, 2e-3, 12
    pr = rcp.make_params(skin_s=0.2, skin_g=0.02)
    p = rcp.Packing(d0, L, 1.0, 0, init="none", params=pr)
    p.set_state(x, kappa)
    p.adam_step(0.0, 0.0, eta_k, steps)
    xg, kg = p.get_state()
    p.close()
    # Kingma-Ba with bias correction on the single coordinate kappa
    P = z * n // 2
    m = v = 0.0
    b1t = b2t = 1.0
    k = kappa
    for _ in range(steps):
        g = P * (1.0 - 1.0 / k) / k ** 2
        b1t *= pr.beta1
        b2t *= pr.beta2
        m = pr.beta1 * m + (1.0 - pr.beta1) * g
        v = pr.beta2 * v + (1.0 - pr.beta2) * g * g
        k = k - eta_k * (m / (1.0 - b1t)) / (math.sqrt(v / (1.0 - b2t)) + pr.eps_k)
    _say(kind, "kappa gpu", kg, "recurrence", k)
    assert kg < kappa
    assert kg == pytest.approx(k, rel=1e-12)
    assert np.array_equal(xg, x)


@pytest.mark.parametrize("dim", [3, 2])
def test_state_readback_paths_agree(rcp, dim):
    # positions read back in user order by the device scatter (positions
    # only) and by the host path (with diameters) are the same bits, after
    # a run has permuted the records through list builds; the
    # diameters are kappa D0 in user order
    import rcp_inputs as ri
    w = ri.small_polydisperse(20000, 20.0, 0.3, seed=4)
    d0 = w.d0
    L = w.L if dim == 3 else float(np.sqrt(np.pi / 4.0 * np.sum(d0 ** 2) / 0.3))
    p = rcp.Packing(d0, L, 1.0, 3, init="rsa_device", dim=dim,
                    params=rcp.make_params(skin_s=0.05))
    p.run_start(rcp.default_schedule(len(d0), dim=dim, S=float(d0.max() / d0.min())))
    p.run_continue(600)
    assert p.stats()["rebuilds"] >= 1
    x1, k1 = p.get_state()
    x2, k2, dm = p.get_state(diameters=True)
    p.close()
    assert k1 == k2
    assert x1.shape == (len(d0), dim)
    assert np.array_equal(x1, x2)
    np.testing.assert_allclose(dm, k1 * d0, rtol=1e-15)
