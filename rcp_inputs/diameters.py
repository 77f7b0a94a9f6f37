"""Relative-diameter lists by the equal-probability quantile rule.

Sec. 2 of the paper fixes the sampling: diameter i (0-based) is the inverse
CDF of the chosen distribution at cumulative probability (i + 1/2)/N.  The
lists returned here are ascending and scaled so that the nominal lower
truncation point equals 1, i.e. every entry lies in [1, S].
"""
import numpy as np
from scipy import special


def _u(n):
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def lognormal_quantiles(n, alpha, S):
    """Truncated lognormal, Eq. (lognormal): D = exp(alpha z), |z| <= a.

    The truncation follows from Eq. (S), S = exp(2 a alpha), so
    a = ln S / (2 alpha).  z is the truncated standard-normal quantile;
    the result is divided by exp(-alpha a) so the nominal D_min is 1.
    """
    a = np.log(S) / (2.0 * alpha)
    lo, hi = special.ndtr(-a), special.ndtr(a)
    z = special.ndtri(lo + _u(n) * (hi - lo))
    z = np.clip(z, -a, a)
    return np.exp(alpha * (z + a))


def powerlaw_quantiles(n, p, S):
    """Truncated power law P(D) ~ D^p on [1, S] (Sec. 3.2)."""
    u = _u(n)
    if abs(p + 1.0) < 1e-14:
        return np.power(S, u)
    q = p + 1.0
    d = np.power(1.0 + u * (S ** q - 1.0), 1.0 / q)
    return np.clip(d, 1.0, S)


def weibull_quantiles(n, k, S):
    """Weibull (Rosin-Rammler) law, Eq. (weibull), on [S^-1/2, S^1/2].

    The scale is the largest diameter, lambda = sqrt(S), as the paper
    states.  Quantiles come from the truncated CDF; the list is divided by
    the lower support point so that it spans [1, S].
    """
    lam = np.sqrt(S)
    lo, hi = 1.0 / np.sqrt(S), np.sqrt(S)
    F = lambda d: -np.expm1(-np.power(d / lam, k))
    Flo, Fhi = F(lo), F(hi)
    q = Flo + _u(n) * (Fhi - Flo)
    d = lam * np.power(-np.log1p(-q), 1.0 / k)
    d = np.clip(d, lo, hi)
    return d / lo


def eps3_lognormal(alpha, a):
    """Missing third-moment fraction of the truncated lognormal, Eq. (eps3)."""
    P = special.ndtr
    return 1.0 - (P(a - 3 * alpha) - P(-a - 3 * alpha)) / (P(a) - P(-a))


def box_for_phi(d0, phi0, kappa=1.0):
    """Cube edge L such that sum(pi (kappa D0)^3 / 6) / L^3 = phi0."""
    vol = np.pi / 6.0 * np.sum((kappa * np.asarray(d0, np.float64)) ** 3)
    return float((vol / phi0) ** (1.0 / 3.0))
