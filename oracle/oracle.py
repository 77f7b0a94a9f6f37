"""ctypes binding of the C oracle plus the schedule builder (test infrastructure)."""
import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rcp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAX_RUNGS = 16


def build(force=True):
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_u01.restype = C.c_double
        L.orc_u01.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int]
        pair_args = [C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double,
                     C.c_double, C.c_double, ip, ip, C.c_int64]
        for f in (L.orc_pairs_brute, L.orc_pairs_cells):
            f.restype = C.c_int64
            f.argtypes = pair_args
        L.orc_rows_pairs.restype = None
        L.orc_rows_pairs.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_double, lp,
                                     C.c_int64, lp, lp, ip]
        L.orc_energy_grad.restype = None
        L.orc_energy_grad.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double,
                                      C.c_double, C.c_int64, ip, ip, dp, dp, dp]
        L.orc_rows_grad.restype = None
        L.orc_rows_grad.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double,
                                    lp, C.c_int64, dp, dp, dp]
        L.orc_shrink.restype = C.c_double
        L.orc_shrink.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double,
                                 C.c_int64, ip, ip]
        L.orc_phi.restype = C.c_double
        L.orc_phi.argtypes = [C.c_int64, dp, C.c_double, C.c_double]
        L.orc_rsa.restype = C.c_int
        L.orc_rsa.argtypes = [C.c_int64, dp, C.c_double, C.c_double, C.c_uint64,
                              C.c_int64, dp]
        L.orc_rsa_rounds.restype = C.c_int
        L.orc_rsa_rounds.argtypes = [C.c_int64, dp, C.c_double, C.c_double, C.c_uint64,
                                     C.c_int64, C.c_int64, dp, lp]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [C.c_int64, dp, dp, C.c_double, dp, dp, dp, dp, lp,
                              dp, C.POINTER(Params), C.POINTER(Schedule),
                              C.c_int64, C.POINTER(Result), dp, C.c_int64, dp]
        L.orc_time_iterations.restype = C.c_double
        L.orc_time_iterations.argtypes = [C.c_int64, dp, dp, C.c_double,
                                          C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_double, C.c_int64, lp,
                                          C.c_int]
        L.orc_set_list_check.restype = None
        L.orc_set_list_check.argtypes = [C.c_int, C.c_double]
        L.orc_set_dim.restype = None
        L.orc_set_dim.argtypes = [C.c_int]
        L.orc_set_boundary.restype = None
        L.orc_set_boundary.argtypes = [C.c_uint, C.c_uint]
        L.orc_set_frozen.restype = None
        L.orc_set_frozen.argtypes = [C.c_void_p]
        L.orc_phi_frozen.restype = C.c_double
        L.orc_phi_frozen.argtypes = [C.c_int64, dp, C.c_double, C.c_double]
        L.orc_seat.restype = C.c_int
        L.orc_seat.argtypes = [C.c_int64, dp, C.c_double, C.c_double, C.c_uint64,
                               C.c_int64, dp]
        L.orc_list_misses.restype = C.c_int64
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _pos(x):
    return np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)


def _vec(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Params(C.Structure):
    _fields_ = [("beta1", C.c_double), ("beta2", C.c_double),
                ("eps_x", C.c_double), ("eps_k", C.c_double),
                ("skin_s", C.c_double), ("skin_g", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("n_rungs", C.c_int32), ("absolute", C.c_int32),
                ("tol", C.c_double),
                ("mu", C.c_double * MAX_RUNGS), ("eta_x", C.c_double * MAX_RUNGS),
                ("eta_k", C.c_double * MAX_RUNGS), ("decay", C.c_double * MAX_RUNGS),
                ("budget", C.c_int64 * MAX_RUNGS)]

    def rungs(self):
        return [(self.mu[r], self.eta_x[r], self.eta_k[r], self.decay[r],
                 self.budget[r]) for r in range(self.n_rungs)]


class Result(C.Structure):
    _fields_ = [("phi", C.c_double), ("kappa_shrunk", C.c_double),
                ("kappa", C.c_double), ("max_overlap", C.c_double),
                ("energy", C.c_double), ("iterations", C.c_int64),
                ("rebuilds", C.c_int64), ("status", C.c_int32),
                ("rung", C.c_int32)]


def splitmix64(seed, k):
    return lib().orc_splitmix64(seed, k)


def u01(seed, i, attempt, axis):
    return lib().orc_u01(seed, i, attempt, axis)


def set_list_check(on, trigger_scale=1.0):
    """Debug mode of run(): count overlapping pairs missing from the list
    before each gradient (n <= 4096); trigger_scale widens the rebuild
    test's displacement allowance (1 = as stated)."""
    lib().orc_set_list_check(1 if on else 0, float(trigger_scale))


def list_misses():
    return int(lib().orc_list_misses())


_dim = 3


def set_dim(d):
    """Spatial dimension, 3 (default) or 2 (disks in the plane z = 0; see
    orc_set_dim).  Every later call uses it until changed."""
    global _dim
    assert d in (2, 3)
    _dim = d
    lib().orc_set_dim(int(d))


def get_dim():
    return _dim


_boundary = (0, 0)


def set_boundary(walls=0, round=0):
    """Hard walls (see orc_set_boundary): bit a of walls = flat walls at
    x_a = 0 and x_a = L; round = the axes of a round container (ball of
    diameter L centred at L/2 on them, two or three axes).  (0, 0) is the
    periodic box.  Every later call uses it until changed."""
    global _boundary
    walls, round = int(walls), int(round)
    assert 0 <= walls < 8 and 0 <= round < 8 and not (walls & round)
    assert round == 0 or bin(round).count("1") >= 2
    _boundary = (walls, round)
    lib().orc_set_boundary(walls, round)


def get_boundary():
    return _boundary


_frozen_ref = None


def set_frozen(mask):
    """Frozen spheres (cascade stages, Sec. 4): mask[i] != 0 holds sphere i
    fixed, its D0 an absolute diameter (see orc_set_frozen); None clears.
    Every later energy / run / seat call uses the mask until cleared."""
    global _frozen_ref
    if mask is None:
        _frozen_ref = None
        lib().orc_set_frozen(None)
        return
    _frozen_ref = np.ascontiguousarray(mask, dtype=np.uint8)
    lib().orc_set_frozen(_frozen_ref.ctypes.data)


def phi_frozen(d0, L, kappa):
    d0 = _vec(d0)
    assert _frozen_ref is not None and _frozen_ref.shape[0] == d0.shape[0]
    return lib().orc_phi_frozen(d0.shape[0], _d(d0), L, kappa)


def seat(x, d0, L, kappa0, seed, max_attempts=1 << 20):
    """Seat the spheres that are not frozen in the voids of the frozen ones
    (see orc_seat); x holds the frozen positions; returns the new (n, 3)."""
    d0 = _vec(d0)
    assert _frozen_ref is not None and _frozen_ref.shape[0] == d0.shape[0]
    x = _pos(x).copy()
    rc = lib().orc_seat(d0.shape[0], _d(d0), L, kappa0, seed, max_attempts, _d(x))
    if rc != 0:
        raise RuntimeError("seating failed: a sphere exceeded %d attempts" % max_attempts)
    return x


def set_threads(n):
    lib().orc_set_threads(int(n))


def num_threads():
    return lib().orc_num_threads()


def _pairs(fn, x, d0, L, kb, s, g, d0min):
    x, d0 = _pos(x), _vec(d0)
    n = d0.shape[0]
    cap = max(1024, 8 * n)
    while True:
        pi = np.empty(cap, np.int32)
        pj = np.empty(cap, np.int32)
        np_ = fn(n, _d(x), _d(d0), L, kb, s, g, d0min, _i(pi), _i(pj), cap)
        if np_ <= cap:
            return pi[:np_].copy(), pj[:np_].copy()
        cap = int(np_)


def pairs_brute(x, d0, L, kb, s=0.0, g=0.0, d0min=None):
    """Canonical pair set (i<j, lexicographic) by testing all pairs."""
    d0min = float(np.min(d0)) if d0min is None else d0min
    return _pairs(lib().orc_pairs_brute, x, d0, L, kb, s, g, d0min)


def pairs_cells(x, d0, L, kb, s=0.0, g=0.0, d0min=None):
    """Canonical pair set from the size-class cell list."""
    d0min = float(np.min(d0)) if d0min is None else d0min
    return _pairs(lib().orc_pairs_cells, x, d0, L, kb, s, g, d0min)


def rows_pairs(x, d0, L, kb, rows, s=0.0, g=0.0, d0min=None):
    """List of ascending partner arrays for each row in `rows` (brute force)."""
    x, d0 = _pos(x), _vec(d0)
    rows = np.ascontiguousarray(rows, np.int64)
    d0min = float(np.min(d0)) if d0min is None else d0min
    n = d0.shape[0]
    cnt = np.zeros(rows.shape[0], np.int64)
    lib().orc_rows_pairs(n, _d(x), _d(d0), L, kb, s, g, d0min, _l(rows),
                         rows.shape[0], _l(cnt), None, None)
    offs = np.zeros(rows.shape[0], np.int64)
    offs[1:] = np.cumsum(cnt)[:-1]
    nbr = np.empty(max(1, int(cnt.sum())), np.int32)
    lib().orc_rows_pairs(n, _d(x), _d(d0), L, kb, s, g, d0min, _l(rows),
                         rows.shape[0], _l(cnt), _l(offs), _i(nbr))
    return [nbr[o:o + c].copy() for o, c in zip(offs, cnt)]


def energy_grad(x, d0, L, kappa, mu, pi, pj, want_grad=True):
    """Energy terms and gradient over half pairs (pi, pj).

    Returns dict: E_ov, E_growth, gk_ov, gk_growth, max_delta, n_overlap,
    g (n,3), gscale (n,3).
    """
    x, d0 = _pos(x), _vec(d0)
    n = d0.shape[0]
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    out = np.zeros(6)
    g = np.zeros((n, 3)) if want_grad else None
    gs = np.zeros((n, 3)) if want_grad else None
    lib().orc_energy_grad(n, _d(x), _d(d0), L, kappa, mu, pi.shape[0], _i(pi),
                          _i(pj), _d(out), _d(g) if want_grad else None,
                          _d(gs) if want_grad else None)
    return {"E_ov": out[0], "E_growth": out[1], "gk_ov": out[2],
            "gk_growth": out[3], "max_delta": out[4], "n_overlap": int(out[5]),
            "g": g, "gscale": gs}


def rows_grad(x, d0, L, kappa, rows):
    """Per-row gradient by brute force over all partners (true overlaps)."""
    x, d0 = _pos(x), _vec(d0)
    rows = np.ascontiguousarray(rows, np.int64)
    k = rows.shape[0]
    g = np.zeros((k, 3)); gs = np.zeros((k, 3)); st = np.zeros((k, 3))
    lib().orc_rows_grad(d0.shape[0], _d(x), _d(d0), L, kappa, _l(rows), k,
                        _d(g), _d(gs), _d(st))
    return g, gs, st


def shrink(x, d0, L, kappa, pi, pj):
    x, d0 = _pos(x), _vec(d0)
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    return lib().orc_shrink(d0.shape[0], _d(x), _d(d0), L, kappa, pi.shape[0],
                            _i(pi), _i(pj))


def phi(d0, L, kappa):
    d0 = _vec(d0)
    return lib().orc_phi(d0.shape[0], _d(d0), L, kappa)


def rsa(d0, L, kappa0, seed, max_attempts=1 << 20):
    """Random sequential addition, largest first; returns (n, 3) positions."""
    d0 = _vec(d0)
    x = np.zeros((d0.shape[0], 3))
    rc = lib().orc_rsa(d0.shape[0], _d(d0), L, kappa0, seed, max_attempts, _d(x))
    if rc != 0:
        raise RuntimeError("RSA failed: a sphere exceeded %d attempts" % max_attempts)
    return x


def rsa_rounds(d0, L, kappa0, seed, window, max_attempts=1 << 20):
    """Random sequential addition in rounds of up to `window` proposals
    (see orc_rsa_rounds); returns ((n, 3) positions, number of rounds)."""
    d0 = _vec(d0)
    x = np.zeros((d0.shape[0], 3))
    nr = np.zeros(1, np.int64)
    rc = lib().orc_rsa_rounds(d0.shape[0], _d(d0), L, kappa0, seed, int(window),
                              int(max_attempts), _d(x), _l(nr))
    if rc != 0:
        raise RuntimeError("RSA in rounds failed: a sphere exceeded %d attempts" % max_attempts)
    return x, int(nr[0])


def n_trig(N, d=3, Y=2, X=9):
    """Rung budget of Eq. (trigger): 4000 Y + X sqrt(N d) - 2000, rounded up."""
    return int(math.ceil(4000.0 * Y + X * math.sqrt(N * d) - 2000.0))


# Rung table (our reading of App. A; values are unstated in the paper):
# (mu~, eta_x~, eta_k~, half-life as a fraction of the rung, budget fraction)
# The half-life applies to mu and both step sizes; only the final rung
# decays, so mu is annealed towards 0 there (the dense endpoint of App. A).
# mu = mu~ N_v / (kappa sum D0) sets the equilibrium summed overlap to mu~ N_v,
# N_v = (sum D0^3)^2 / sum D0^6 (volume participation number);
# eta_x = eta_x~ kappa D0_min, eta_k = eta_k~ kappa at the rung start.
DEFAULT_RUNGS = [
    (1e-2, 1e-2, 1e-3, 0.0, 1.0),        # densify
    (1e-3, 5e-3, 5e-4, 0.0, 0.25),
    (1e-4, 2.5e-3, 2.5e-4, 0.0, 0.25),
    (1e-3, 2.5e-3, 2.5e-4, 0.0, 0.125),  # two mu cycles
    (1e-4, 2.5e-3, 2.5e-4, 0.0, 0.125),
    (1e-3, 2.5e-3, 2.5e-4, 0.0, 0.125),
    (1e-4, 2.5e-3, 2.5e-4, 0.0, 0.125),
    (1e-5, 1.25e-3, 1.25e-4, 1.0 / 16, 2.0),  # final relaxation (cap), mu -> 0
]


def size_ratio_factors(S):
    """Step-size and budget factors for a size ratio S = max D0 / min D0.

    Our reading for broad distributions (the paper does not list its rung
    values): a large sphere's radius grows by about eta_k D_max / 2 per
    update, and small spheres must be able to move away from it, so the
    kappa step shrinks as sqrt(160 / S) beyond S = 160, the position step
    grows as sqrt(S / 10), and the densification rung is lengthened by
    1 + log10(S / 10).  All three are 1 for S <= 10.  Beyond S = 1e4 the
    kappa step shrinks by a further (1e4 / S)^(1/4) and the densification
    rung grows by a further 1.7 log10(S / 1e4), so the largest spheres do
    not outrun the smallest ones at S ~ 1e5 (a run at S = 5e5 engulfed
    small spheres and did not converge without it).
    """
    S = max(float(S), 1.0)
    fx = max(1.0, math.sqrt(S / 10.0))
    fk = min(1.0, math.sqrt(160.0 / S)) * min(1.0, (1e4 / S) ** 0.25)
    fb = 1.0 + max(0.0, math.log10(S / 10.0)) + 1.7 * max(0.0, math.log10(S / 1e4))
    return fx, fk, fb


def default_schedule(N, d=3, Y=2, X=9, n_min=5000, tol=5e-4, rungs=None, S=1.0):
    nt = max(n_trig(N, d, Y, X), n_min)
    fx, fk, fb = size_ratio_factors(S)
    Sc = Schedule()
    rungs = DEFAULT_RUNGS if rungs is None else rungs
    Sc.n_rungs = len(rungs)
    Sc.absolute = 0
    Sc.tol = tol
    for r, (mu, ex, ek, hl, bf) in enumerate(rungs):
        Sc.mu[r], Sc.eta_x[r], Sc.eta_k[r] = mu, ex * fx, ek * fk
        Sc.budget[r] = max(1, int(math.ceil(bf * (fb if r == 0 else 1.0) * nt)))
        Sc.decay[r] = 1.0 if hl <= 0 else 2.0 ** (-1.0 / (hl * Sc.budget[r]))
    return Sc


def absolute_schedule(mu, eta_x, eta_k, n_steps):
    """One rung with the given numbers, no stop test, n_steps iterations."""
    S = Schedule()
    S.n_rungs, S.absolute, S.tol = 1, 1, -1.0
    S.mu[0], S.eta_x[0], S.eta_k[0], S.decay[0] = mu, eta_x, eta_k, 1.0
    S.budget[0] = n_steps
    return S


class RunState:
    """Resumable oracle run state (positions, kappa, Adam moments, schedule)."""

    def __init__(self, x, d0, L, kappa):
        self.x = _pos(x).copy()
        self.d0 = _vec(d0)
        self.L = float(L)
        self.kappa = np.array([kappa], np.float64)
        n = self.d0.shape[0]
        self.m = np.zeros((n, 3)); self.v = np.zeros((n, 3))
        self.mkvk = np.zeros(2)
        self.ctl = np.array([0, 0, 0, 1], np.int64)
        self.etas = np.zeros(3)

    def new_schedule(self):
        """Start the next call of run() at rung 0 of its schedule while the
        Adam moments and step counter carry over."""
        self.ctl[1:] = (0, 0, 1)


def default_params(d0, kappa0=1.0, s=0.1, g=0.02):
    P = Params()
    P.beta1, P.beta2 = 0.9, 0.999
    P.eps_x = 1e-12 / (kappa0 * float(np.max(d0)))
    P.eps_k = 1e-12
    P.skin_s, P.skin_g = s, g
    return P


def run(state, params, sched, max_iters=1 << 62, trace_cap=0, gsmax=None):
    """Advance `state` by the schedule; returns (status, Result, trace).
    gsmax (n, 3) float64, optional: raised in place to the largest sum of
    |pair contributions| per component over the gradients evaluated."""
    res = Result()
    tr = np.zeros((max(trace_cap, 1), 3))
    if gsmax is not None:
        assert gsmax.dtype == np.float64 and gsmax.flags.c_contiguous
        assert gsmax.shape == (state.d0.shape[0], 3)
    st = lib().orc_run(state.d0.shape[0], _d(state.x), _d(state.d0), state.L,
                       _d(state.kappa), _d(state.m), _d(state.v), _d(state.mkvk),
                       _l(state.ctl), _d(state.etas), C.byref(params),
                       C.byref(sched), max_iters, C.byref(res),
                       _d(tr) if trace_cap else None, trace_cap,
                       _d(gsmax) if gsmax is not None else None)
    ntr = min(trace_cap, int(res.iterations) + 1)
    return st, res, (tr[:ntr] if trace_cap else None)


def time_iterations(x, d0, L, kappa, eta_x, iters, s=0.1, g=0.02, threads=0):
    """Seconds for `iters` gradient + Adam evaluations on a fixed list
    (timed on `threads` threads, 0 = all)."""
    x = _pos(x).copy()
    d0 = _vec(d0)
    npairs = np.zeros(1, np.int64)
    t = lib().orc_time_iterations(d0.shape[0], _d(x), _d(d0), L, kappa, 0.0,
                                  eta_x, s, g, iters, _l(npairs), int(threads))
    return t, int(npairs[0])


# ---------------------------------------------------------------- cascade
def cascade_counts(n1, rho, n_classes, phi1=0.6435):
    """Class counts of the ideal void-filling cascade (Eq. (cascade)): class
    c + 1 fills the voids left by classes 1..c, a fraction (1 - phi1)^c of
    the volume, at the monodisperse fraction phi1, with spheres rho^c times
    smaller in diameter than class 1, so n_(c+1) = n1 ((1 - phi1) rho^3)^c."""
    return [int(round(n1 * ((1.0 - phi1) * rho ** 3) ** c)) for c in range(n_classes)]


def release_schedule(N, S):
    """The release of a cascade stage (Sec. 4: every sphere relaxes
    together, the numerical analogue of vibration): the final relaxation
    rung of the default schedule for the whole set (mu annealed towards 0,
    the stop criterion, cap 2 n_trig), as one rung."""
    d = default_schedule(N, S=S)
    r = d.n_rungs - 1
    Sc = Schedule()
    Sc.n_rungs, Sc.absolute, Sc.tol = 1, 0, d.tol
    Sc.mu[0], Sc.eta_x[0], Sc.eta_k[0] = d.mu[r], d.eta_x[r], d.eta_k[r]
    Sc.decay[0], Sc.budget[0] = d.decay[r], d.budget[r]
    return Sc


def cascade(n1, rho, n_classes, seed, phi0=0.05, s=0.1, g=0.02, counts=None):
    """The sequential multimodal cascade (Sec. 4) as our reading takes it:
    the coarsest class alone is packed by the plain protocol from a random
    sequential addition at phi0 (D0 = 1); then for each finer class c the
    spheres packed so far are frozen at their diameters, and the new class
    (count from cascade_counts, nominal diameter D0 = the previous class's
    mean diameter / rho) is seated in their voids at the scale kappa0 =
    (phi0 / 0.6435)^(1/3), the dilution of the protocol's own start
    relative to the monodisperse packing, and inflated by the protocol
    (default schedule for the new class alone); then every sphere is
    released: all of them relax together (D0 = their diameters, kappa from
    1) under the final relaxation rung of the default schedule for the
    whole set (release_schedule), down to the stop and the shrink.
    Returns (phi after each class, counts)."""
    counts = cascade_counts(n1, rho, n_classes) if counts is None else counts
    d = np.ones(counts[0])
    L = float((np.pi / 6.0 * np.sum(d ** 3) / phi0) ** (1.0 / 3.0))
    x = rsa(d, L, 1.0, seed)
    st = RunState(x, d, L, 1.0)
    _, res, _ = run(st, default_params(d, 1.0, s, g), default_schedule(counts[0], S=1.0))
    phis = [res.phi]
    sig = d * res.kappa_shrunk
    cls = np.zeros(counts[0], np.int64)
    x = st.x
    kappa_seat = (phi0 / 0.6435) ** (1.0 / 3.0)
    for c in range(1, n_classes):
        nc, nf = counts[c], sig.shape[0]
        dn = float(np.mean(sig[cls == c - 1])) / rho
        d0 = np.concatenate([sig, np.full(nc, dn)])
        mask = np.concatenate([np.ones(nf, np.uint8), np.zeros(nc, np.uint8)])
        set_frozen(mask)
        try:
            xs = seat(np.concatenate([x, np.zeros((nc, 3))]), d0, L, kappa_seat, seed)
            st = RunState(xs, d0, L, kappa_seat)
            run(st, default_params(d0[nf:], kappa_seat, s, g), default_schedule(nc, S=1.0))
            kf = float(st.kappa[0])
        finally:
            set_frozen(None)
        sig = np.concatenate([sig, kf * d0[nf:]])
        cls = np.concatenate([cls, np.full(nc, c)])
        st = RunState(st.x, sig, L, 1.0)
        _, res, _ = run(st, default_params(sig, 1.0, s, g),
                        release_schedule(sig.shape[0], float(sig.max() / sig.min())))
        phis.append(res.phi)
        sig = sig * res.kappa_shrunk
        x = st.x
    return phis, counts
