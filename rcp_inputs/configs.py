"""Synthetic workloads with the shapes of the paper's 3-D periodic studies.

Each workload is a relative-diameter list (quantile rule, Sec. 2), a cube
edge L fixed by the initial volume fraction at kappa = 1, a seed, and
optionally explicit positions (i.i.d. uniform, overlaps allowed).  Runs that
start from a non-overlapping state ask the library / oracle for random
sequential addition with the same seed instead.
"""
from dataclasses import dataclass, field
from typing import Optional
import numpy as np

from .diameters import (lognormal_quantiles, powerlaw_quantiles,
                        weibull_quantiles, box_for_phi)
from .rng import uniform_positions, splitmix64


@dataclass
class Workload:
    name: str
    d0: np.ndarray
    L: float
    phi0: float
    seed: int
    family: str
    params: dict = field(default_factory=dict)
    x: Optional[np.ndarray] = None   # explicit start (uniform, overlapping)

    @property
    def n(self):
        return int(self.d0.shape[0])

    @property
    def S_realised(self):
        return float(self.d0.max() / self.d0.min())


def _wl(name, d0, phi0, seed, family, params, uniform):
    L = box_for_phi(d0, phi0)
    x = uniform_positions(d0.shape[0], L, seed) if uniform else None
    return Workload(name, d0, L, phi0, seed, family, params, x)


def c1_lognormal(seed=0, n=512):
    """Lognormal sigma_lnD = 0.3, nominal S = 4, N = 512, phi0 = 0.1."""
    d0 = lognormal_quantiles(n, 0.3, 4.0)
    return _wl("lognormal a=0.3 S=4 N=%d phi0=0.1" % n, d0, 0.1, seed,
               "lognormal", {"alpha": 0.3, "S": 4.0}, uniform=False)


def c2_powerlaw(seed=0, n=100_000):
    """Power law P(D) ~ D^-3 on [1, 20], N = 1e5, phi0 = 0.05."""
    d0 = powerlaw_quantiles(n, -3.0, 20.0)
    return _wl("powerlaw p=-3 S=20 N=%d phi0=0.05" % n, d0, 0.05, seed,
               "powerlaw", {"p": -3.0, "S": 20.0}, uniform=False)


def c3_lognormal_dense(seed=0, n=1_000_000, phi0=0.6):
    """Lognormal sigma_lnD = 1.0, S = 1e3, N = 1e6, i.i.d. uniform at phi = 0.6."""
    d0 = lognormal_quantiles(n, 1.0, 1e3)
    return _wl("lognormal a=1.0 S=1e3 N=%d phi=%.2g uniform" % (n, phi0), d0,
               phi0, seed, "lognormal", {"alpha": 1.0, "S": 1e3}, uniform=True)


def c5_extreme(seed=0, n=3_000_000, uniform=False):
    """Lognormal sigma_lnD = 2.5, S = 5e5, N = 3e6, phi0 = 0.05."""
    d0 = lognormal_quantiles(n, 2.5, 5e5)
    return _wl("lognormal a=2.5 S=5e5 N=%d phi0=0.05" % n, d0, 0.05, seed,
               "lognormal", {"alpha": 2.5, "S": 5e5}, uniform=uniform)


def small_polydisperse(n, S, phi, seed, family="lognormal", uniform=True):
    """Small random cases used by the pair-set and gradient tests."""
    if family == "lognormal":
        d0 = lognormal_quantiles(n, 1.0, S)
    elif family == "powerlaw":
        d0 = powerlaw_quantiles(n, -3.0, S)
    else:
        d0 = weibull_quantiles(n, 1.0, S)
    return _wl("%s S=%g N=%d phi=%g" % (family, S, n, phi), d0, phi, seed,
               family, {"S": S}, uniform=uniform)


def census_draw(n_prob=64, seed=2026, n_lo=1_000, n_hi=200_000, phi0=0.05, span_max=0.4):
    """Seeded parameter draw over the three families.

    Packing k uses family k mod 3: lognormal alpha ~ U[0.2, 1.5]; power law
    exponent p ~ U[-4, -2]; Weibull modulus k ~ logU[0.5, 3].  S ~ logU[2,
    100] and N ~ logU[n_lo, n_hi]; each packing gets its own placement seed.
    As in the paper's studies, where N is chosen so that the largest sphere
    spans a fixed fraction of the box (Sec. 3), a draw whose largest sphere
    would span more than span_max of the box edge at phi = 0.8 is drawn
    again (attempt a uses counters k * 8 + j + a * 2^20).
    """
    out = []
    for k in range(n_prob):
        for a in range(1000):
            u = lambda j: float((splitmix64(seed, k * 8 + j + a * (1 << 20)) >> np.uint64(11))
                                .astype(np.float64) * 2.0 ** -53)
            S = float(np.exp(np.log(2.0) + u(0) * (np.log(100.0) - np.log(2.0))))
            n = int(np.exp(np.log(n_lo) + u(1) * (np.log(n_hi) - np.log(n_lo))))
            fam = k % 3
            if fam == 0:
                al = 0.2 + 1.3 * u(2)
                d0 = lognormal_quantiles(n, al, S)
                name, params = "lognormal", {"alpha": al, "S": S}
            elif fam == 1:
                p = -4.0 + 2.0 * u(2)
                d0 = powerlaw_quantiles(n, p, S)
                name, params = "powerlaw", {"p": p, "S": S}
            else:
                kk = float(np.exp(np.log(0.5) + u(2) * (np.log(3.0) - np.log(0.5))))
                d0 = weibull_quantiles(n, kk, S)
                name, params = "weibull", {"k": kk, "S": S}
            L = box_for_phi(d0, phi0)
            if (0.8 / phi0) ** (1.0 / 3.0) * float(d0.max()) <= span_max * L:
                break
        else:
            raise RuntimeError("census draw %d: no admissible parameters" % k)
        wseed = int(splitmix64(seed, 10_000 + k) & np.uint64(0xFFFFFFFF))
        out.append(_wl("%s #%d N=%d S=%.3g" % (name, k, n, S), d0, phi0, wseed,
                       name, params, uniform=False))
    return out
