"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package holds none of the packing method's arithmetic: it only draws
the relative-diameter lists (equal-probability quantiles of the three size
distribution families, Sec. 2 and Eqs. (lognormal), (S), (weibull) of the
paper), the periodic box implied by an initial volume fraction, uniform
random positions from a counter-based SplitMix64 generator, and the census
parameter draw.  Both the CPU oracle and the HIP path consume these arrays
as plain inputs.
"""
from .diameters import (lognormal_quantiles, powerlaw_quantiles,
                        weibull_quantiles, eps3_lognormal, box_for_phi)
from .rng import splitmix64, u01, uniform_positions
from .configs import (Workload, c1_lognormal, c2_powerlaw, c3_lognormal_dense,
                      c5_extreme, census_draw, small_polydisperse)

__all__ = [
    "lognormal_quantiles", "powerlaw_quantiles", "weibull_quantiles",
    "eps3_lognormal", "box_for_phi", "splitmix64", "u01",
    "uniform_positions", "Workload", "c1_lognormal", "c2_powerlaw",
    "c3_lognormal_dense", "c5_extreme", "census_draw", "small_polydisperse",
]
