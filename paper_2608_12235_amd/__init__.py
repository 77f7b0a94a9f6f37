"""MI355X (gfx950) implementation of the hot path of the Adam-based
inflation protocol for random close packings of polydisperse spheres.

The compute path is librcp.so (hand-written HIP kernels behind the C ABI of
include/rcp.h).  This package is a thin binding: ctypes marshalling
(`api`), a torch.autograd.Function around the energy and its hand-written
adjoint (`autograd`), the batched census driver (`census`) and the launch
autotuner (`autotune`).
"""
from ._lib import lib, RcpError, LIB_PATH
from .api import (Packing, make_params, make_tuning, default_schedule,
                  absolute_schedule, schedule_from_rungs, longer_schedule)


def overlap_energy(x, kappa, packing, mu=0.0):
    """See autograd.overlap_energy (imports torch on first use)."""
    from .autograd import overlap_energy as f
    return f(x, kappa, packing, mu)


__all__ = ["lib", "RcpError", "LIB_PATH", "Packing", "make_params", "make_tuning",
           "default_schedule", "absolute_schedule", "schedule_from_rungs", "longer_schedule",
           "overlap_energy"]
