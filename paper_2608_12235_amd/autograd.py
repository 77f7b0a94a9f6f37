"""The overlap energy as a differentiable torch function.

E(x, kappa) = E_overlap + E_growth of App. A, Eq. (energy) (eps = 1):
    E_overlap = 1/2 sum_{i<j} (1 - r_ij/d_ij)^2 Theta(1 - r_ij/d_ij),
    d_ij = kappa (D0_i + D0_j) / 2,      E_growth = -mu kappa sum_i D0_i.
The forward value comes from the library's energy kernel and the backward
pass from its hand-written adjoint (rcp_energy_dev / rcp_adjoint_dev):
    dE/dx_i   = sum_j delta_ij / (d_ij r_ij) (x_j - x_i)_mi,
    dE/dkappa = sum_{i<j} delta_ij r_ij / (kappa d_ij) - mu sum_i D0_i,
both evaluated on the device from the tensors' storage on the current
torch stream.  Second derivatives are not provided.
"""
import ctypes as C

import torch

from ._lib import check, lib


def _stream_handle(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class OverlapEnergy(torch.autograd.Function):
    """E(x, kappa) for packing 0 of a Packing; x is (n, 3) float64 on the
    device in the packing's user order, kappa a float64 scalar tensor."""

    @staticmethod
    def forward(ctx, x, kappa, packing, mu):
        if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 2 or x.shape[1] != 3:
            raise TypeError("x must be a float64 (n, 3) tensor on the HIP device")
        if x.shape[0] != packing.n[0]:
            raise ValueError("x has %d rows, the packing %d spheres" % (x.shape[0], packing.n[0]))
        xc = x.detach().contiguous()
        kv = float(kappa)
        out = torch.empty(2, dtype=torch.float64, device=x.device)
        check(lib().rcp_energy_dev(packing.handle, C.c_void_p(xc.data_ptr()), kv, float(mu),
                                   C.c_void_p(out.data_ptr()), _stream_handle(x.device)))
        ctx.save_for_backward(xc)
        ctx.kappa = kv
        ctx.kappa_shape = kappa.shape if torch.is_tensor(kappa) else None
        ctx.kappa_device = kappa.device if torch.is_tensor(kappa) else None
        ctx.packing = packing
        ctx.mu = float(mu)
        ctx.mark_non_differentiable(out)
        return out[0], out[1]

    @staticmethod
    def backward(ctx, g_energy, g_maxov):
        (xc,) = ctx.saved_tensors
        gx = torch.empty_like(xc)
        gk = torch.empty(1, dtype=torch.float64, device=xc.device)
        check(lib().rcp_adjoint_dev(ctx.packing.handle, C.c_void_p(xc.data_ptr()), ctx.kappa,
                                    ctx.mu, C.c_void_p(gx.data_ptr()), C.c_void_p(gk.data_ptr()),
                                    _stream_handle(xc.device)))
        dx = g_energy * gx
        dk = None
        if ctx.kappa_shape is not None and ctx.needs_input_grad[1]:
            dk = (g_energy * gk[0]).reshape(ctx.kappa_shape).to(ctx.kappa_device)
        return dx, dk, None, None


def overlap_energy(x, kappa, packing, mu=0.0):
    """Energy E(x, kappa) (differentiable in x and kappa) and, not
    differentiable, the largest fractional overlap."""
    if not torch.is_tensor(kappa):
        kappa = torch.tensor(float(kappa), dtype=torch.float64)
    return OverlapEnergy.apply(x, kappa, packing, mu)
