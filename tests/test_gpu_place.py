"""Random sequential addition in rounds on the GPU (rcp_place_device)
against the oracle's plain emulation of the same rounds: positions bit for
bit, the same number of rounds, no overlap."""
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


def _c1():
    w = ri.c1_lognormal(0)
    return w.d0, w.L, w.seed


def _poly():
    d0 = ri.lognormal_quantiles(3000, 0.7, 60.0)
    return d0, ri.box_for_phi(d0, 0.08), 11


def _c5dist():
    # C5's size distribution (lognormal sigma_lnD = 2.5, S = 5e5) at N = 2e4,
    # phi0 = 0.05: 19 size classes
    d0 = ri.lognormal_quantiles(20000, 2.5, 5e5)
    return d0, ri.box_for_phi(d0, 0.05), 3


@pytest.mark.parametrize("case,window", [(_c1, 1), (_c1, 64), (_poly, 256), (_poly, 1 << 16),
                                         (_c5dist, 4096), (_c5dist, 1)])
def test_device_placement_bit_exact(rcp, orc, case, window):
    d0, L, seed = case()
    print("device placement N=%d window=%d" % (len(d0), window), flush=True)
    p = rcp.Packing(d0, L, 1.0, seed, init="none")
    nr = p.place_device(seed, window)
    xg, kg = p.get_state()
    p.close()
    xo, nro = orc.rsa_rounds(d0, L, 1.0, seed, window)
    assert kg == 1.0 and nr == nro
    assert np.array_equal(xg, xo)
    if window == 1:
        assert np.array_equal(xg, orc.rsa(d0, L, 1.0, seed))


def test_device_placement_init_mode(rcp, orc):
    d0, L, seed = _poly()
    p = rcp.Packing(d0, L, 1.0, seed, init="rsa_device")
    xg, _ = p.get_state()
    # the placed state runs like any other: a list builds, no pair overlaps
    p.neighbor_build()
    assert p.energy_grad()["n_overlap"] == 0
    p.close()
    xo, _ = orc.rsa_rounds(d0, L, 1.0, seed, rcp._lib.RCP_PLACE_WINDOW)
    assert np.array_equal(xg, xo)
