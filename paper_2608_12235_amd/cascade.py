"""Sequential multimodal cascade (Sec. 4) on the device.

The coarsest class is packed alone by the plain protocol; then, one class
at a time, the spheres packed so far are frozen at their diameters
(rcp_set_frozen), the next finer class is seated in their voids
(rcp_seat_device) and inflated with them held fixed, and every sphere is
released into the plain protocol (a context of its own, down to the
shrink).  Class counts follow the ideal void-filling cascade of
Eq. (cascade): class c + 1 fills the voids left by classes 1..c, a
fraction (1 - phi1)^c of the volume, at the monodisperse fraction phi1,
with diameters rho^c times smaller.  Readings (the paper gives the recipe
in words only): the new class's nominal diameter is the previous class's
mean diameter / rho; it is seated at kappa0 = (phi0 / phi1)^(1/3) of that,
the dilution the plain protocol starts from (in units of twice the
nominal diameter, see run_cascade); its inflation uses the
default schedule for the new class alone; the release relaxes every
sphere together under the final relaxation rung of the default schedule
for the whole set (mu annealed towards 0, then the stop and the shrink).
"""
import math
import time

import numpy as np

from .api import Packing, default_schedule, longer_schedule, make_params, schedule_from_rungs

PHI1 = 0.6435   # the monodisperse value the paper quotes for Eq. (cascade)


def class_counts(n1, rho, n_classes, phi1=PHI1):
    """n_(c+1) = n1 ((1 - phi1) rho^3)^c."""
    return [int(round(n1 * ((1.0 - phi1) * rho ** 3) ** c)) for c in range(n_classes)]


def ideal_phi(n, phi1=PHI1):
    """Eq. (cascade): phi_n = 1 - (1 - phi1)^n."""
    return 1.0 - (1.0 - phi1) ** n


def release_schedule(n, S):
    """The release (every sphere relaxes together, the numerical analogue
    of vibration): the final relaxation rung of the default schedule for
    the whole set, as one rung (mu annealed towards 0, stop criterion, cap
    2 n_trig)."""
    d = default_schedule(n, S=S)
    r = d.n_rungs - 1
    return schedule_from_rungs([(d.mu[r], d.eta_x[r], d.eta_k[r], d.decay[r], d.budget[r])],
                               tol=d.tol, absolute=0)


def run_cascade(n1, rho, n_classes, seed, phi0=0.05, params=None, tuning=None, counts=None,
                log=None, length=1):
    """Returns a dict: phi after each class (after its release), the class
    counts, the packing's final diameters and positions, per-stage
    iterations and seconds.  The default listing skin is 0.05 D0_min: the
    coarse class of a cascade spans a large part of the box (D / L up to
    about 0.4 at 20 spheres), and the listing cutoff must stay below L / 2.
    length > 1 runs every schedule that many times longer (longer_schedule)."""
    sch = (lambda s: s) if length == 1 else (lambda s: longer_schedule(s, length))
    params = params if params is not None else make_params(skin_s=0.05)
    counts = class_counts(n1, rho, n_classes) if counts is None else list(counts)
    d = np.ones(counts[0])
    L = float((math.pi / 6.0 * np.sum(d ** 3) / phi0) ** (1.0 / 3.0))
    t0 = time.perf_counter()
    p = Packing(d, L, 1.0, seed, init="rsa", params=params, tuning=tuning)
    try:
        r = p.inflate_run(sch(default_schedule(counts[0], S=1.0)))[0]
        x, _ = p.get_state()
    finally:
        p.close()
    stages = [{"class": 1, "n": counts[0], "phi": r["phi"], "iterations": r["iterations"],
               "status": r["status"], "seconds": time.perf_counter() - t0}]
    if log:
        log("cascade class 1: n %d phi %.4f (%d its)" % (counts[0], r["phi"], r["iterations"]))
    sig = d * r["kappa"]
    cls = np.zeros(counts[0], np.int64)
    kappa_seat = (phi0 / PHI1) ** (1.0 / 3.0)
    for c in range(1, n_classes):
        nc, nf = counts[c], sig.shape[0]
        dn = float(np.mean(sig[cls == c - 1])) / rho
        # the new class's D0 is twice its nominal diameter, seated at half
        # the seating scale: the same sizes, but kappa stays below 1 through
        # the stage, so the lists are built at scale 1 and the frozen
        # spheres' cutoffs are not stretched by kappa (the protocol's
        # relative schedule does not depend on this unit)
        d0 = np.concatenate([sig, np.full(nc, 2.0 * dn)])
        mask = np.concatenate([np.ones(nf, np.uint8), np.zeros(nc, np.uint8)])
        t1 = time.perf_counter()
        p = Packing(d0, L, 1.0, seed, init="none", params=params, tuning=tuning)
        try:
            p.set_state(np.concatenate([x, np.zeros((nc, 3))]), 1.0)
            p.set_frozen(mask)
            p.seat(0.5 * kappa_seat, seed)
            rf = p.inflate_run(sch(default_schedule(nc, S=1.0)))[0]
            x, kf = p.get_state()
        finally:
            p.close()
        sig = np.concatenate([sig, kf * d0[nf:]])
        cls = np.concatenate([cls, np.full(nc, c)])
        p = Packing(sig, L, 1.0, seed, init="none", params=params, tuning=tuning)
        try:
            p.set_state(x, 1.0)
            r = p.inflate_run(sch(release_schedule(sig.shape[0], float(sig.max() / sig.min()))))[0]
            x, _ = p.get_state()
        finally:
            p.close()
        sig = sig * r["kappa"]
        stages.append({"class": c + 1, "n": nc, "phi": r["phi"], "phi_frozen_stage": rf["phi"],
                       "iterations_frozen_stage": rf["iterations"],
                       "iterations": r["iterations"], "status": r["status"],
                       "status_frozen_stage": rf["status"],
                       "seconds": time.perf_counter() - t1})
        if log:
            log("cascade class %d: n %d, frozen stage phi %.4f (%d its), released phi %.4f "
                "(%d its)" % (c + 1, nc, rf["phi"], rf["iterations"], r["phi"], r["iterations"]))
    return {"phi": [s["phi"] for s in stages], "counts": counts, "stages": stages,
            "diameters": sig, "x": x, "L": L, "seconds": time.perf_counter() - t0}


def run_one_shot(n1, rho, n_classes, seed, phi0=0.05, params=None, tuning=None, counts=None):
    """The same grading in a single quench (Table (tab:cascade), last row):
    every class at once (diameters 1, 1/rho, 1/rho^2, ..., the counts of
    class_counts), placed by random sequential addition on the device at
    phi0 and run by the plain protocol with the default schedule."""
    params = params if params is not None else make_params(skin_s=0.05)
    counts = class_counts(n1, rho, n_classes) if counts is None else list(counts)
    d0 = np.concatenate([np.full(nc, rho ** (-c)) for c, nc in enumerate(counts)])
    L = float((math.pi / 6.0 * np.sum(d0 ** 3) / phi0) ** (1.0 / 3.0))
    t0 = time.perf_counter()
    p = Packing(d0, L, 1.0, seed, init="rsa_device", params=params, tuning=tuning)
    try:
        r = p.inflate_run(default_schedule(d0.shape[0], S=float(d0.max() / d0.min())))[0]
    finally:
        p.close()
    return {"phi": r["phi"], "counts": counts, "iterations": r["iterations"],
            "status": r["status"], "seconds": time.perf_counter() - t0}
