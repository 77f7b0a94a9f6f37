"""Python view of the C ABI: one Packing object per rcp_ctx (argument marshalling only)."""
import ctypes as C

import numpy as np

from ._lib import (lib, check, Params, Tuning, Schedule, Energy, Result, Stats, Optimizer,
                   RCP_INIT_NONE, RCP_INIT_RSA, RCP_INIT_UNIFORM, RCP_INIT_RSA_DEVICE,
                   RCP_PLACE_WINDOW, RcpError)

_INIT = {"none": RCP_INIT_NONE, "rsa": RCP_INIT_RSA, "uniform": RCP_INIT_UNIFORM,
         "rsa_device": RCP_INIT_RSA_DEVICE}


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(**kw):
    p = Params()
    lib().rcp_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def make_tuning(**kw):
    t = Tuning()
    lib().rcp_tuning_default(C.byref(t))
    for k, v in kw.items():
        if not hasattr(t, k):
            raise KeyError(k)
        setattr(t, k, v)
    return t


def default_schedule(n, dim=3, Y=2, X=9, n_min=5000, S=1.0):
    """Default rung table for n spheres with size ratio S (max D0 / min D0)."""
    s = Schedule()
    check(lib().rcp_schedule_default(n, dim, float(S), Y, X, n_min, C.byref(s)))
    return s


def absolute_schedule(mu, eta_x, eta_k, n_steps, tol=-1.0):
    s = Schedule()
    s.size = C.sizeof(Schedule)
    s.n_rungs, s.absolute, s.tol = 1, 1, tol
    s.mu[0], s.eta_x[0], s.eta_k[0], s.decay[0], s.budget[0] = mu, eta_x, eta_k, 1.0, n_steps
    return s


def schedule_from_rungs(rungs, tol=5e-4, absolute=0):
    """rungs: list of (mu, eta_x, eta_k, decay, budget)."""
    s = Schedule()
    s.size = C.sizeof(Schedule)
    s.n_rungs, s.absolute, s.tol = len(rungs), absolute, tol
    for r, (mu, ex, ek, dc, b) in enumerate(rungs):
        s.mu[r], s.eta_x[r], s.eta_k[r], s.decay[r], s.budget[r] = mu, ex, ek, dc, int(b)
    return s


def longer_schedule(s, f):
    """A copy of schedule s with every rung f times longer and the same
    annealing over each rung (decay^(1/f) per iteration).  The default
    budgets are our reading; broad size distributions need longer ones to
    reach the paper's packing fractions (see the bench's extreme2d leg)."""
    t = Schedule()
    C.memmove(C.byref(t), C.byref(s), C.sizeof(Schedule))
    for r in range(t.n_rungs):
        t.budget[r] = int(t.budget[r]) * int(f)
        if t.decay[r] != 1.0:
            t.decay[r] = t.decay[r] ** (1.0 / f)
    return t


def _result_dict(r):
    return {f: getattr(r, f) for f, _ in Result._fields_}


class Packing:
    """One or several independent packings on the GPU (an rcp_ctx); periodic
    unless `boundary` gives hard walls."""

    def __init__(self, d0, L, kappa0=1.0, seed=0, init="rsa", params=None, stream=None,
                 tuning=None, dim=3, boundary=None):
        """boundary: None (periodic), or (walls, round) axis masks (see
        set_boundary) for every packing, or a list of them, one per packing.
        With walls, init "rsa" and "rsa_device" both place on the device
        after the walls are set (the host placement knows no walls)."""
        d0s = d0 if isinstance(d0, (list, tuple)) else [d0]
        Ls = L if isinstance(L, (list, tuple, np.ndarray)) else [L]
        P = len(d0s)
        k0 = kappa0 if isinstance(kappa0, (list, tuple, np.ndarray)) else [kappa0] * P
        seeds = seed if isinstance(seed, (list, tuple, np.ndarray)) else [seed] * P
        self._d0 = [np.ascontiguousarray(a, np.float64) for a in d0s]
        self.n = [a.shape[0] for a in self._d0]
        self.L = [float(v) for v in Ls]
        ns = (C.c_int64 * P)(*self.n)
        ptrs = (C.POINTER(C.c_double) * P)(*[_dp(a) for a in self._d0])
        box = (C.c_double * P)(*self.L)
        kap = (C.c_double * P)(*[float(v) for v in k0])
        sd = (C.c_uint64 * P)(*[int(v) for v in seeds])
        self.params = params if params is not None else make_params()
        h = C.c_void_p()
        self.dim = int(dim)
        bnd = None
        if boundary is not None:
            bnd = list(boundary) if isinstance(boundary, list) else [tuple(boundary)] * P
            assert len(bnd) == P
        walled = bnd is not None and any(w or r for w, r in bnd)
        mode = _INIT[init]
        if walled and init in ("rsa", "rsa_device"):
            mode = RCP_INIT_NONE
        check(lib().rcp_census_init(self.dim, P, ns, ptrs, box, kap, sd, mode,
                                    C.byref(self.params), stream, C.byref(h)))
        self._h = h
        self.boundary = [(0, 0)] * P
        if bnd is not None:
            for k, (w, r) in enumerate(bnd):
                self.set_boundary(w, r, k)
            if walled and init in ("rsa", "rsa_device"):
                for k in range(P):
                    self.place_device(seeds[k], RCP_PLACE_WINDOW, k)
        self.tuning = make_tuning()
        if tuning is not None:
            self.set_tuning(tuning)

    # ------------------------------------------------------------------
    @property
    def handle(self):
        return self._h

    @property
    def n_packings(self):
        return len(self.n)

    def close(self):
        if self._h:
            lib().rcp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, t):
        check(lib().rcp_set_tuning(self._h, C.byref(t)))
        self.tuning = t

    def set_skin(self, skin_s, skin_g):
        check(lib().rcp_set_skin(self._h, float(skin_s), float(skin_g)))
        self.params.skin_s = float(skin_s)
        self.params.skin_g = float(skin_g)

    def set_state(self, x, kappa, k=0):
        x = np.ascontiguousarray(x, np.float64).reshape(-1, self.dim)
        assert x.shape[0] == self.n[k]
        check(lib().rcp_set_state(self._h, k, x.ctypes.data_as(C.c_void_p), float(kappa), 0))

    def get_state(self, k=0, diameters=False):
        x = np.empty((self.n[k], self.dim))
        kap = C.c_double()
        dm = np.empty(self.n[k]) if diameters else None
        check(lib().rcp_get_state(self._h, k, _dp(x), C.byref(kap),
                                  _dp(dm) if diameters else None))
        return (x, kap.value, dm) if diameters else (x, kap.value)

    def get_optimizer(self, k=0, moments=True):
        """Optimiser state of packing k: (m, v, dict of scalars); m and v are
        (n, 3) arrays in user order (None when moments is False)."""
        o = Optimizer()
        o.size = C.sizeof(Optimizer)
        m = np.empty((self.n[k], self.dim)) if moments else None
        v = np.empty((self.n[k], self.dim)) if moments else None
        check(lib().rcp_get_optimizer(self._h, k, _dp(m) if moments else None,
                                      _dp(v) if moments else None, C.byref(o)))
        return m, v, {f: getattr(o, f) for f, _ in Optimizer._fields_ if f != "size"}

    def set_optimizer(self, opt, m=None, v=None, k=0):
        """Restore the optimiser state of packing k (see get_optimizer)."""
        o = Optimizer()
        o.size = C.sizeof(Optimizer)
        for f, val in opt.items():
            setattr(o, f, val)
        mm = None if m is None else np.ascontiguousarray(m, np.float64).reshape(self.n[k], self.dim)
        vv = None if v is None else np.ascontiguousarray(v, np.float64).reshape(self.n[k], self.dim)
        check(lib().rcp_set_optimizer(self._h, k, _dp(mm) if mm is not None else None,
                                      _dp(vv) if vv is not None else None, C.byref(o)))

    def place_device(self, seed, window, k=0):
        """Random sequential addition of packing k on the GPU in rounds of
        up to `window` proposals; returns the number of rounds."""
        r = C.c_int64()
        check(lib().rcp_place_device(self._h, k, int(seed), int(window), C.byref(r)))
        return r.value

    def neighbor_build(self, k=0):
        npairs = C.c_int64()
        check(lib().rcp_neighbor_build(self._h, k, C.byref(npairs)))
        return npairs.value

    def pairs(self, k=0):
        cnt = C.c_int64()
        check(lib().rcp_get_pairs(self._h, k, None, None, 0, C.byref(cnt)))
        m = cnt.value
        pi = np.empty(max(m, 1), np.int32)
        pj = np.empty(max(m, 1), np.int32)
        check(lib().rcp_get_pairs(self._h, k, pi.ctypes.data_as(C.POINTER(C.c_int32)),
                                  pj.ctypes.data_as(C.POINTER(C.c_int32)), m, C.byref(cnt)))
        return pi[:m], pj[:m]

    def energy_grad(self, mu=0.0, k=0, grad=True):
        e = Energy()
        g = np.empty((self.n[k], self.dim)) if grad else None
        check(lib().rcp_energy_grad(self._h, k, float(mu), C.byref(e),
                                    _dp(g) if grad else None))
        out = {f: getattr(e, f) for f, _ in Energy._fields_}
        out["g"] = g
        return out

    def adam_step(self, mu, eta_x, eta_k, n_steps):
        check(lib().rcp_adam_step(self._h, float(mu), float(eta_x), float(eta_k), int(n_steps)))

    def inflate_run(self, schedule=None, max_iters=0, allow_notconv=True, allow_fail=False):
        P = self.n_packings
        if schedule is None:
            schedule = self.default_schedules()
        per = isinstance(schedule, (list, tuple))
        if per:
            arr = (Schedule * P)(*schedule)
            sp = C.cast(arr, C.POINTER(Schedule))
        else:
            sp = C.byref(schedule)
        res = (Result * P)()
        rc = lib().rcp_inflate_run(self._h, sp, 1 if per else 0, int(max_iters), res)
        if rc != 0 and not (allow_notconv and rc == -5) and not (allow_fail and rc in (-2, -5, -6)):
            check(rc)
        return [_result_dict(r) for r in res]

    def default_schedules(self):
        return [default_schedule(n, dim=self.dim, S=float(d.max() / d.min()))
                for n, d in zip(self.n, self._d0)]

    def run_start(self, schedule=None):
        P = self.n_packings
        if schedule is None:
            schedule = self.default_schedules()
        per = isinstance(schedule, (list, tuple))
        if per:
            arr = (Schedule * P)(*schedule)
            check(lib().rcp_run_start(self._h, C.cast(arr, C.POINTER(Schedule)), 1))
        else:
            check(lib().rcp_run_start(self._h, C.byref(schedule), 0))

    def run_continue(self, n_iters=0):
        act = C.c_int32()
        check(lib().rcp_run_continue(self._h, int(n_iters), C.byref(act)))
        return act.value

    def set_frozen(self, mask, k=0):
        """Freeze spheres (mask[i] != 0) of packing k for a cascade stage:
        their D0 becomes an absolute diameter, they take no step; None frees
        every sphere."""
        if mask is None:
            check(lib().rcp_set_frozen(self._h, k, None))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape[0] == self.n[k]
        check(lib().rcp_set_frozen(self._h, k, m.ctypes.data))

    def set_boundary(self, walls=0, round=0, k=0):
        """Hard walls of packing k: bit a of `walls` = flat walls at 0 and L
        across axis a; `round` = the axes (two or three) of a round container
        of diameter L centred at L/2; (0, 0) = periodic."""
        check(lib().rcp_set_boundary(self._h, k, int(walls), int(round)))
        self.boundary[k] = (int(walls), int(round))

    def seat(self, kappa0, seed, max_attempts=1 << 22, k=0):
        """Seat the spheres that are not frozen in the voids of the frozen
        ones at scale kappa0 (then kappa = kappa0)."""
        check(lib().rcp_seat_device(self._h, k, float(kappa0), int(seed), int(max_attempts)))

    def run_prepare(self):
        """Capture the iteration graph ahead of the next run_continue."""
        check(lib().rcp_run_prepare(self._h))

    def run_result(self, k=0):
        r = Result()
        check(lib().rcp_run_result(self._h, k, C.byref(r)))
        return _result_dict(r)

    def shrink(self, k=0):
        kp, ph = C.c_double(), C.c_double()
        check(lib().rcp_shrink(self._h, k, C.byref(kp), C.byref(ph)))
        return kp.value, ph.value

    def time_iterations(self, n_iters):
        """Mean duration (us) of the gradient + Adam kernel and of the tail
        kernel over up to n_iters further iterations, from HIP events."""
        a, t, d = C.c_double(), C.c_double(), C.c_int64()
        check(lib().rcp_time_iterations(self._h, int(n_iters), C.byref(a), C.byref(t),
                                        C.byref(d)))
        return a.value, t.value, d.value

    def stats(self):
        s = Stats()
        check(lib().rcp_get_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def reset_stats(self):
        check(lib().rcp_reset_stats(self._h))


__all__ = ["Packing", "make_params", "make_tuning", "default_schedule",
           "absolute_schedule", "schedule_from_rungs", "RcpError"]
