"""rcp_energy_dev_static (no device allocation, fixed scratch array) against
rcp_energy_dev, the entry point it is a variant of, through the C ABI.

Both run the same kernels in the same order, so the bar is bit equality
(tighter than the 1e-10 relative bar of the energy); two calls in a row on
one GPU, the second with a smaller input, show that the shared scratch
array's leftover contents from the first call do not leak into the second.
"""
import ctypes as C

import numpy as np
import pytest

import rcp_inputs as ri

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2608_12235_amd as rcp
    rcp.lib()
    return torch, rcp


def _energies(torch, rcp, p, x, kappa, mu):
    lib = rcp.lib()
    xt = torch.tensor(x, dtype=torch.float64, device="cuda")
    e_alloc = torch.full((2,), -1.0, dtype=torch.float64, device="cuda")
    e_static = torch.full((2,), -2.0, dtype=torch.float64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rcp.api.check(lib.rcp_energy_dev(p.handle, C.c_void_p(xt.data_ptr()), kappa, mu,
                                     C.c_void_p(e_alloc.data_ptr()), stream))
    rc = lib.rcp_energy_dev_static(p.handle, C.c_void_p(xt.data_ptr()), kappa, mu,
                                   C.c_void_p(e_static.data_ptr()), stream)
    torch.cuda.synchronize()
    return rc, e_alloc.cpu().numpy(), e_static.cpu().numpy()


def test_static_energy_equals_allocating_entry_point(env):
    torch, rcp = env
    cases = [ri.small_polydisperse(20000, 40.0, 0.5, seed=5, family="powerlaw"),
             ri.small_polydisperse(3000, 10.0, 0.45, seed=6, family="lognormal")]
    for w, mu in zip(cases, (1e-3, 2e-2)):
        print("static energy, N =", w.n, flush=True)
        p = rcp.Packing(w.d0, w.L, 1.0, 0, init="none",
                        params=rcp.make_params(skin_s=0.3, skin_g=0.02))
        p.set_state(w.x, 1.0)
        p.neighbor_build()
        rc, ea, es = _energies(torch, rcp, p, w.x, 1.0, mu)
        assert rc == 0, rcp.lib().rcp_last_error()
        assert ea[0] != 0.0 and ea[1] > 0.0
        assert np.array_equal(ea, es), (ea, es)
        assert abs(es[0] - ea[0]) <= 1e-10 * abs(ea[0])
        p.close()


def test_static_energy_refuses_an_invalid_list_and_oversize(env):
    torch, rcp = env
    lib = rcp.lib()
    w = ri.small_polydisperse(3000, 10.0, 0.45, seed=6, family="lognormal")
    p = rcp.Packing(w.d0, w.L, 1.0, 0, init="none",
                    params=rcp.make_params(skin_s=0.3, skin_g=0.02))
    p.set_state(w.x, 1.0)
    e = torch.zeros(2, dtype=torch.float64, device="cuda")
    xt = torch.tensor(w.x, dtype=torch.float64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # no list built yet
    assert lib.rcp_energy_dev_static(p.handle, C.c_void_p(xt.data_ptr()), 1.0, 0.0,
                                     C.c_void_p(e.data_ptr()), stream) == rcp._lib.RCP_ESTATE
    p.neighbor_build()
    # positions moved beyond the listing skin: the list is not valid there
    xm = torch.tensor(np.mod(w.x + 0.8 * w.d0.min(), w.L), dtype=torch.float64, device="cuda")
    assert lib.rcp_energy_dev_static(p.handle, C.c_void_p(xm.data_ptr()), 1.0, 0.0,
                                     C.c_void_p(e.data_ptr()), stream) == rcp._lib.RCP_ESTATE
    assert b"not valid" in lib.rcp_last_error()
    p.close()
    # more spheres than the fixed scratch holds
    n = (1 << 24) + 1
    big = rcp.Packing(np.ones(n), 1e4, 1.0, 0, init="none")
    xb = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    assert lib.rcp_energy_dev_static(big.handle, C.c_void_p(xb.data_ptr()), 1.0, 0.0,
                                     C.c_void_p(e.data_ptr()), stream) == rcp._lib.RCP_EINVAL
    assert b"fixed scratch" in lib.rcp_last_error()
    big.close()
