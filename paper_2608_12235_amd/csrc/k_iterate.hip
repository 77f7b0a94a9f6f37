// One inflation iteration on the device, for every active packing at once.
//
// k_iterate: for each particle i evaluate the overlap gradient of Eq. (energy)
//     dE/dx_i = sum_j delta_ij / (d_ij r_ij) (x_j - x_i)_mi,
//     delta = 1 - r/d,  d = kappa (D0_i + D0_j)/2,
// over the listed partners with delta > 0, apply Adam (Kingma and Ba, bias
// corrected) to the three coordinates, wrap into [0, L), and write the new
// positions into the other ping-pong buffer.  Per block it also forms the
// partial sums the kappa update and the stop / rebuild tests need:
//     E_ov = 1/2 sum delta^2, S = sum delta r/d (each pair once),
//     max delta, max |x_new - x_ref|^2.
// k_tail (one block per packing) reduces those partials in a fixed order
// (so runs are bit-reproducible), forms dE/dkappa = S/kappa - mu sum D0,
// applies the stop test of App. A (final rung, max delta < tol, evaluated
// before the update), Adam on kappa, the decay of mu and the step sizes, the rung
// advance, and the list-validity test that requests a rebuild.
#include "rcp_kernels.hpp"

namespace rcp {

__device__ __forceinline__ int remap_block(int b, int G)
{
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD
    // a contiguous range of row blocks so neighbour gathers share its L2.
    const int nx = 8, per = G / nx, rem = G % nx;
    const int xcd = b % nx, loc = b / nx;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + loc;
}

// Running sums of pair terms: the gradient of the current row, and the
// energy, kappa-gradient and max-overlap terms (per thread in the iteration
// kernel, per row in the evaluation kernel); c counts overlapping pairs
// (evaluation only).
struct Acc {
    double gx, gy, gz, e, s, m, c;
};

// Minimum image of the separation of a listed pair: the nearest multiple of
// L is removed.  Same value as min_image() whenever the imaged separation
// is below L/2 (true of every listed pair that can be in contact), with
// three instructions instead of two compares and selects.
__device__ __forceinline__ double near_image(double d, double L, double iL)
{
    return fma(-L, rint(d * iL), d);
}

// Reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64, v_rsq_f64), refined by kSteps Newton steps (each doubles the
// correct bits of the estimate): a few units in the last place after one,
// within two after two, at a fraction of the cost of an IEEE division or
// root.
#ifndef RCP_NEWTON_STEPS
#define RCP_NEWTON_STEPS 1
#endif
template <int kSteps = RCP_NEWTON_STEPS>
__device__ __forceinline__ double fast_rcp(double d)
{
    double y = __builtin_amdgcn_rcp(d);
#pragma unroll
    for (int k = 0; k < kSteps; ++k) {
        const double e = fma(-d, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

template <int kSteps = RCP_NEWTON_STEPS>
__device__ __forceinline__ double fast_rsq(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
#pragma unroll
    for (int k = 0; k < kSteps; ++k) {
        const double t = fma(-(h * y), y, 0.5);
        y = fma(y, t, y);
    }
    return y;
}

// Squared distances below this use the IEEE root (the estimates lose range
// near the bottom of the exponent range).
constexpr double kTinyR2 = 1e-200;
// Overlaps shallower than this take the definition's own rounding (below).
constexpr double kShallow = 0x1p-10;
// Pairs with r^2 below d^2 (1 + 2^-50) are examined: every pair whose
// correctly rounded r can be below d passes this filter.
constexpr double kLoose = 1.0 + 0x1p-50;

// One listed partner's terms (Eq. energy): with q = r/d and delta = 1 - q,
// E += delta^2 / 4 and S += delta q / 2 (each pair is seen from both ends),
// and the gradient on x_i gains delta / (d r) (x_j - x_i); a pair counts
// when r < d.  r^2 is formed without contraction.  r and q come from the
// hardware estimates refined by Newton steps (a few ulp); that is far inside
// the 1e-10 bar while delta is not small, but delta = 1 - q cancels for
// shallow overlaps (a small sphere grazing one 10^5 times larger has delta ~
// 1e-6), so below kShallow r and q are recomputed as the plain definition
// rounds them (IEEE root and quotient): then delta and the test r < d are
// exactly the definition's, which also makes the stop test (max delta below
// the tolerance) exact.  The factor delta / (d r) is well conditioned.
//
// kMixed: some spheres are frozen (a cascade stage, Sec. 4): a record with a
// negative D0 holds a frozen sphere whose diameter is -D0 in absolute
// units, the others have D = kappa D0.  Then d = (sigma_i + sigma_j) / 2 and
// the pair's dE/dkappa is delta (r / d^2) dd/dkappa with dd/dkappa = (g_i D0_i
// + g_j D0_j) / 2 (g = 0 for a frozen sphere); S gains delta q (kappa dd/dkappa
// / d) / 2, so that S / kappa in the tail is that derivative summed.
//
// iLa[a] is 1 / L on a periodic axis and 0 on an axis bounded by walls
// (no image: near_image then returns the plain difference).
//
// kDim = 2: disks in the plane z = 0 (every z is 0, so dz = 0 and r^2 is
// dx^2 + dy^2 exactly as the three-term sum rounds it); the z terms are
// left out.
template <bool kCount = true, bool kMixed = false, int kDim = 3>
__device__ __forceinline__ void pair_term(Acc &a, const P4 &qi, const P4 &qj, double kappa,
                                          double L, const double (&iLa)[3])
{
#pragma clang fp contract(off)
    const double dx = near_image(qj.x - qi.x, L, iLa[0]);
    const double dy = near_image(qj.y - qi.y, L, iLa[1]);
    const double dz = kDim == 3 ? near_image(qj.z - qi.z, L, iLa[2]) : 0.0;
    const double r2 = kDim == 3 ? (dx * dx + dy * dy) + dz * dz : dx * dx + dy * dy;
    const double d = kMixed ? 0.5 * ((qi.d > 0.0 ? kappa * qi.d : -qi.d) +
                                     (qj.d > 0.0 ? kappa * qj.d : -qj.d))
                            : kappa * (0.5 * (qi.d + qj.d));
    if (r2 < (d * d) * kLoose) {
        const double id = fast_rcp(d);
        double r, ir;
        if (r2 >= kTinyR2) {
            ir = fast_rsq(r2);
            r = r2 * ir;
        } else {
            r = sqrt(r2);
            ir = r > 0.0 ? 1.0 / r : 0.0;
        }
        double q = r * id;
        double delta = 1.0 - q;
        if (delta < kShallow) {
            r = sqrt(r2);
            q = r / d;
            delta = 1.0 - q;
        }
        if (r < d) {
            a.e += 0.25 * (delta * delta);
            if (kMixed)
                a.s += 0.5 * (delta * q) *
                       ((kappa * (0.5 * (fmax(qi.d, 0.0) + fmax(qj.d, 0.0)))) * id);
            else
                a.s += 0.5 * (delta * q);
            a.m = fmax(a.m, delta);
            if (kCount) a.c += 0.5;
            if (r > 0.0) {
                const double f = (delta * id) * ir;
                a.gx += f * dx;
                a.gy += f * dy;
                if (kDim == 3) a.gz += f * dz;
            }
        }
    }
}

// Adam on one coordinate (Kingma and Ba, bias corrected; ib1 = 1 / (1 -
// beta1^t), ib2 = 1 / (1 - beta2^t)), then wrapped into [0, L) (L = 0 on an
// axis bounded by walls leaves the coordinate as it is).
__device__ __forceinline__ double adam_coord(double th, double g, double &m, double &v,
                                             double b1, double b2, double ib1, double ib2,
                                             double eta, double eps, double L)
{
    m = b1 * m + (1.0 - b1) * g;
    v = b2 * v + (1.0 - b2) * (g * g);
    const double mh = m * ib1, vh = v * ib2;
    // sqrt(vh) as vh / sqrt(vh); below 1e-200 (where the estimate loses
    // range, a rarely taken branch) the IEEE root
    double sv = vh * fast_rsq(fmax(vh, 1e-200));
    if (vh < 1e-200) sv = sqrt(vh);
    double t = th - (eta * mh) * fast_rcp(sv + eps);
    if (t < 0.0) t += L;
    if (t >= L) t -= L;
    return t;
}

struct IterScalars {
    double kappa, L, hL, iL, b1, b2, ib1, ib2, eta, eps;
    // per axis: 1 / L and the wrap period L, both 0 on an axis bounded by
    // walls; the walls themselves (see wall_terms)
    double iLa[3], Pa[3];
    int32_t walls, round;
};

// Pointers of one segment with the ping-pong buffers already selected
// (uniform selects keep them in scalar registers; indexing the pointer
// table with the runtime buffer index would spill it to scratch).
struct IterPtrs {
    const P4 *q;        // current (x, y, z, D0)
    P4 *qo;             // next positions
    double *m0, *m1, *m2, *v0, *v1, *v2;
    const float *r0, *r1, *r2;
    const int32_t *rp, *col;
};

__device__ __forceinline__ IterPtrs select_ptrs(const SegPtrs *__restrict__ P, int seg, int cur)
{
    const SegPtrs &s = P[seg];
    IterPtrs p;
    p.q = cur ? s.p[1] : s.p[0];
    p.qo = cur ? s.p[0] : s.p[1];
    p.m0 = s.m[0];
    p.m1 = s.m[1];
    p.m2 = s.m[2];
    p.v0 = s.v[0];
    p.v1 = s.v[1];
    p.v2 = s.v[2];
    p.r0 = s.xref[0];
    p.r1 = s.xref[1];
    p.r2 = s.xref[2];
    p.rp = s.rp;
    p.col = s.col;
    return p;
}

// One coordinate's Adam update from preloaded operands; returns the new
// coordinate and adds its squared (minimum image) displacement from the
// list reference to d2.
__device__ __forceinline__ double update_coord(double xi, double g, double m, double v, double r,
                                               double *mm, double *vv, const IterScalars &c,
                                               int64_t i, double &d2, double period)
{
    const double xn = adam_coord(xi, g, m, v, c.b1, c.b2, c.ib1, c.ib2, c.eta, c.eps, period);
    gstore(mm, i, m);
    gstore(vv, i, v);
    const double dd = min_image(xn - r, c.L, c.hL);
    d2 += dd * dd;
    return xn;
}

struct Pre {
    double m0, m1, m2, v0, v1, v2;
    float r0, r1, r2;
};

// Streamed operands of row i (read once per iteration); in two dimensions
// the z moments and reference are not read.
template <int kDim = 3>
__device__ __forceinline__ Pre preload(const IterPtrs &p, int64_t i)
{
    Pre q;
    q.m0 = gload(p.m0, i);
    q.m1 = gload(p.m1, i);
    q.m2 = kDim == 3 ? gload(p.m2, i) : 0.0;
    q.v0 = gload(p.v0, i);
    q.v1 = gload(p.v1, i);
    q.v2 = kDim == 3 ? gload(p.v2, i) : 0.0;
    q.r0 = gload(p.r0, i);
    q.r1 = gload(p.r1, i);
    q.r2 = kDim == 3 ? gload(p.r2, i) : 0.0f;
    return q;
}

// Adam on particle i's coordinates, new position stored (the three
// coordinates: the record's D0 in the output buffer is already in place,
// written when the list order was set; with `full` the whole record);
// returns |x_new - x_ref|^2 (min image).  kDim = 2: z stays 0 and its
// moments are neither read nor written (they stay 0, as its gradient is 0).
template <bool kMixed = false, int kDim = 3>
__device__ __forceinline__ double update_particle(const IterPtrs &p, const IterScalars &c,
                                                  int64_t i, const P4 &qi, const Pre &q,
                                                  double gx, double gy, double gz, bool full)
{
    if (kMixed && qi.d < 0.0) {
        // a frozen sphere: no step, its record carried to the other buffer
        store_p4(p.qo, (int32_t)i, qi);
        return 0.0;
    }
    double d2 = 0.0;
    P4 o;
    o.x = update_coord(qi.x, gx, q.m0, q.v0, q.r0, p.m0, p.v0, c, i, d2, c.Pa[0]);
    o.y = update_coord(qi.y, gy, q.m1, q.v1, q.r1, p.m1, p.v1, c, i, d2, c.Pa[1]);
    o.z = kDim == 3 ? update_coord(qi.z, gz, q.m2, q.v2, q.r2, p.m2, p.v2, c, i, d2, c.Pa[2])
                    : qi.z;
    o.d = qi.d;
    if (full) store_p4(p.qo, (int32_t)i, o);
    else store_xyz(p.qo, (int32_t)i, o.x, o.y, o.z);
    return d2;
}

// floor(n / d) for 0 <= n < 2^31 and 1 <= d < 2^31 with rd = 1 / d: the
// truncated product is the quotient or one less (never more), one upward
// correction settles it; (q + 1) d <= n + d < 2^32.
__device__ __forceinline__ int32_t div_by(int32_t n, uint32_t d, double rd)
{
    uint32_t q = (uint32_t)((double)n * rd);
    if ((q + 1u) * d <= (uint32_t)n) ++q;
    return (int32_t)q;
}

// The values a rung starts from: given, or scaled from the relative ones
// by the current kappa (mu by N_v / (kappa sum D0), eta_x by kappa D0_min,
// eta_k by kappa).
__device__ __forceinline__ void rung_values(const SchedDev &q, int r, double kappa, double nvol,
                                            double sumd0, double d0min, double &mu,
                                            double &eta_x, double &eta_k)
{
    if (q.absolute) {
        mu = q.mu[r];
        eta_x = q.eta_x[r];
        eta_k = q.eta_k[r];
    } else {
        mu = (q.mu[r] * nvol) / (kappa * sumd0);
        eta_x = q.eta_x[r] * (kappa * d0min);
        eta_k = q.eta_k[r] * kappa;
    }
}

__device__ __forceinline__ void rung_start(SegState *s, int r)
{
    rung_values(s->sched, r, s->kappa, s->nvol, s->sumd0, s->d0min, s->mu, s->eta_x, s->eta_k);
}

// The serial end of one iteration: store the reduced sums, run the stop
// tests, take the Adam step on kappa, decay the rung's values, advance the
// rung and set the list-validity flag.  Every field it reads is loaded
// before any is stored and the results are stored once at the end, so the
// stores force no reloads: the step is one dependent chain of arithmetic,
// not of memory (or LDS) round trips.
__device__ void tail_logic(SegState *s, double E, double S, double md, double mdisp2)
{
    const SchedDev &q = s->sched;
    const int r = s->rung, last = q.n_rungs - 1;
    const double kappa = s->kappa, mu = s->mu, sumd0 = s->sumd0, tol = q.tol;
    const double beta1 = s->beta1, beta2 = s->beta2, eps_k = s->eps_k;
    const double b1t0 = s->b1t, b2t0 = s->b2t, mk0 = s->mk, vk0 = s->vk;
    const double eta_x0 = s->eta_x, eta_k0 = s->eta_k, dec = q.decay[r];
    const double kappa_lim = s->kappa_lim, d0max_k = s->d0max_k, disp_lim = s->disp_lim;
    const int64_t t = s->t, it_rung0 = s->it_rung, iters0 = s->iters;
    const int64_t iter_limit = s->iter_limit, budget = q.budget[r];
    const int32_t cur = s->cur;
    int32_t flags = s->flags;
    s->E_ov = E;
    s->S_drd = S;
    s->max_delta = md;
    s->max_disp2 = mdisp2;
    const double gk = S / kappa - mu * sumd0;
    if (!isfinite(E) || !isfinite(gk) || !isfinite(mdisp2)) {
        s->flags = flags | F_NONFINITE;
        return;
    }
    if (r == last && md < tol) {
        s->flags = flags | F_STOP;
        return;
    }
    const double b1t = b1t0 * beta1, b2t = b2t0 * beta2;
    const double mk = beta1 * mk0 + (1.0 - beta1) * gk;
    const double vk = beta2 * vk0 + (1.0 - beta2) * (gk * gk);
    const double mh = mk / (1.0 - b1t), vh = vk / (1.0 - b2t);
    const double kappa1 = kappa - eta_k0 * mh / (sqrt(vh) + eps_k);
    double mu1 = mu * dec, eta_x1 = eta_x0 * dec, eta_k1 = eta_k0 * dec;
    int64_t it_rung = it_rung0 + 1;
    const int64_t iters = iters0 + 1;
    int rung = r;
    if (it_rung >= budget) {
        if (r == last) {
            flags |= F_CAP;
        } else {
            rung = r + 1;
            it_rung = 0;
            rung_values(q, r + 1, kappa1, s->nvol, sumd0, s->d0min, mu1, eta_x1, eta_k1);
        }
    }
    if (!(kappa1 > 0.0) || !isfinite(kappa1)) flags |= F_NONFINITE;
    // list validity: an unlisted pair had r >= kb ((1 + g) d0_ij + 2 s D0_min)
    // at the build, so it cannot touch while 2 max|dx| + max(0, kappa - (1 +
    // g) kb) D0_max <= 2 s kb D0_min (growth beyond the g allowance is paid
    // from the displacement skin)
    const double excess = fmax(0.0, kappa1 - kappa_lim);
    if (!(2.0 * sqrt(mdisp2) + excess * d0max_k <= 2.0 * disp_lim)) flags |= F_REBUILD;
    if (iter_limit > 0 && iters >= iter_limit) flags |= F_HOLD;
    s->t = t + 1;
    s->b1t = b1t;
    s->b2t = b2t;
    s->ib1n = 1.0 / (1.0 - b1t * beta1);
    s->ib2n = 1.0 / (1.0 - b2t * beta2);
    s->mk = mk;
    s->vk = vk;
    s->kappa = kappa1;
    s->cur = cur ^ 1;
    s->mu = mu1;
    s->eta_x = eta_x1;
    s->eta_k = eta_k1;
    s->it_rung = it_rung;
    s->iters = iters;
    s->rung = rung;
    s->flags = flags;
}

// Per-block partial sums of one iteration: E_ov, S, max delta, max disp^2.
struct alignas(32) Part4 {
    double e, s, m, d;
};

// Deterministic reduction of a segment's block partials by one block of
// kT threads (fixed assignment of partials to threads, fixed combining
// order); thread 0 then runs the tail.  Every thread of the block must call
// it.
// A block partial read at the device's coherence point (agent-scope relaxed
// atomic loads, which bypass the reading XCD's L2): used when the partials
// were written in the same kernel by other XCDs (with agent-scope stores).
__device__ __forceinline__ Part4 load_part_coherent(const Part4 *p)
{
    Part4 r;
    r.e = __hip_atomic_load(&p->e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.s = __hip_atomic_load(&p->s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.m = __hip_atomic_load(&p->m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.d = __hip_atomic_load(&p->d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return r;
}

template <bool kCoherent>
__device__ __forceinline__ Part4 load_part(const Part4 *p)
{
    return kCoherent ? load_part_coherent(p) : *p;
}

// This thread's share of a packing's block partials: partials t, t + kT,
// t + 2 kT, ... in rounds of eight whose loads are all in flight together,
// combined in a fixed order.
template <int kT, bool kCoherent>
__device__ __forceinline__ Part4 thread_partials(int64_t nb, int64_t b0, const double *partials)
{
    const Part4 *P = reinterpret_cast<const Part4 *>(partials) + b0;
    Part4 a = {0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nb; b += 8 * kT) {
        Part4 p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            p[k] = b + k * kT < nb ? load_part<kCoherent>(P + b + k * kT) : Part4{0, 0, 0, 0};
        a.e += ((p[0].e + p[1].e) + (p[2].e + p[3].e)) + ((p[4].e + p[5].e) + (p[6].e + p[7].e));
        a.s += ((p[0].s + p[1].s) + (p[2].s + p[3].s)) + ((p[4].s + p[5].s) + (p[6].s + p[7].s));
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a.m = fmax(a.m, p[k].m);
            a.d = fmax(a.d, p[k].d);
        }
    }
    return a;
}

// Block reduction of the threads' shares (DPP within waves, then the
// waves' sums by a second DPP pass in wave 0), then thread 0 runs the tail.
// Every thread of the block must call it.
template <int kT>
__device__ __forceinline__ void block_tail(SegState *s, const Part4 &mine)
{
    constexpr int kW = kT / kWave;
    static_assert(kW <= kWave, "one wave combines the waves' sums");
    const double e = wave_sum_dpp(mine.e), sd = wave_sum_dpp(mine.s);
    const double m = wave_max_dpp(mine.m), d = wave_max_dpp(mine.d);
    __shared__ Part4 red[kW];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) red[wv] = Part4{e, sd, m, d};
    __syncthreads();
    if (wv == 0) {
        // lanes past the waves contribute zeros (the maxima are of values
        // >= 0, as the per-thread shares start from 0)
        const Part4 w = lane < kW ? red[lane] : Part4{0, 0, 0, 0};
        const double te = wave_sum_dpp(w.e), ts = wave_sum_dpp(w.s);
        const double tm = wave_max_dpp(w.m), td = wave_max_dpp(w.d);
        if (lane == 0) tail_logic(s, te, ts, tm, td);
    }
}

// Deterministic reduction of a segment's block partials by one block of kT
// threads, then the tail (see thread_partials, block_tail).
template <int kT, bool kCoherent = false>
__device__ void reduce_and_tail(SegState *s, const double *partials)
{
    block_tail<kT>(s, thread_partials<kT, kCoherent>(s->nblocks, s->bfirst, partials));
}

// Partner indices of a work item, staged in LDS at the start of the item
// (entries past the stage are read from global memory).
constexpr int kColStage = 2048;

#ifndef RCP_ITEM_PREFETCH
#define RCP_ITEM_PREFETCH 1
#endif

// Where a thread's partner indices come from: the LDS stage (kStage), else
// global memory, with the first two entries of the thread's chunk [cs, ..)
// already in registers (requested together with the row pointers, so the
// first gathers need no second dependent load).
template <bool kStage>
struct ColSrc {
    const int32_t *__restrict__ col;
    const int32_t *__restrict__ scol;
    int32_t e0, cs, j0, j1;
    __device__ __forceinline__ int32_t at(int32_t q) const
    {
        if (kStage) {
            const int32_t k = q - e0;
            return k < kColStage ? scol[k] : gload(col, q);
        }
        if (RCP_ITEM_PREFETCH && q == cs) return j0;
        if (RCP_ITEM_PREFETCH && q == cs + 1) return j1;
        return gload(col, q);
    }
};

// Entry loop of one row segment [q, qe): kU partners per step so that
// their gathers are in flight together (kU = 2 or 4); the next step's
// partner indices are requested before this step's terms are evaluated, so
// their latency hides behind the arithmetic.
template <int kU, bool kStage, bool kMixed = false, int kDim = 3>
__device__ __forceinline__ void segment_terms(Acc &a, const ColSrc<kStage> &cols,
                                              const P4 *__restrict__ Q, int32_t q, int32_t qe,
                                              const P4 &qi, const IterScalars &c)
{
    if (kU == 4 && q + 4 <= qe) {
        int32_t j0 = cols.at(q), j1 = cols.at(q + 1),
                j2 = cols.at(q + 2), j3 = cols.at(q + 3);
        for (;;) {
            const P4 q0 = load_p4(Q, j0), q1 = load_p4(Q, j1), q2 = load_p4(Q, j2),
                     q3 = load_p4(Q, j3);
            q += 4;
            const bool more = q + 4 <= qe;
            if (more) {
                j0 = cols.at(q);
                j1 = cols.at(q + 1);
                j2 = cols.at(q + 2);
                j3 = cols.at(q + 3);
            }
            pair_term<false, kMixed, kDim>(a, qi, q0, c.kappa, c.L, c.iLa);
            pair_term<false, kMixed, kDim>(a, qi, q1, c.kappa, c.L, c.iLa);
            pair_term<false, kMixed, kDim>(a, qi, q2, c.kappa, c.L, c.iLa);
            pair_term<false, kMixed, kDim>(a, qi, q3, c.kappa, c.L, c.iLa);
            if (!more) break;
        }
    }
    if (kU == 2 && q + 2 <= qe) {
        int32_t j0 = cols.at(q), j1 = cols.at(q + 1);
        for (;;) {
            const P4 q0 = load_p4(Q, j0), q1 = load_p4(Q, j1);
            q += 2;
            const bool more = q + 2 <= qe;
            if (more) {
                j0 = cols.at(q);
                j1 = cols.at(q + 1);
            }
            pair_term<false, kMixed, kDim>(a, qi, q0, c.kappa, c.L, c.iLa);
            pair_term<false, kMixed, kDim>(a, qi, q1, c.kappa, c.L, c.iLa);
            if (!more) break;
        }
    }
    for (; q + 2 <= qe; q += 2) {
        const int32_t j0 = cols.at(q),
                      j1 = cols.at(q + 1);
        const P4 q0 = load_p4(Q, j0), q1 = load_p4(Q, j1);
        pair_term<false, kMixed, kDim>(a, qi, q0, c.kappa, c.L, c.iLa);
        pair_term<false, kMixed, kDim>(a, qi, q1, c.kappa, c.L, c.iLa);
    }
    if (q < qe)
        pair_term<false, kMixed, kDim>(a, qi, load_p4(Q, cols.at(q)), c.kappa, c.L, c.iLa);
}

template <int kN>
__device__ __forceinline__ void store3(double (*M)[kN], int k, const Acc &a)
{
    M[0][k] = a.gx;
    M[1][k] = a.gy;
    M[2][k] = a.gz;
}

// LDS of one work item.
template <int kR>
struct ItemLdsR {
    int32_t srp[kR + 1];
    double G[3][kR];       // gradient of complete rows
    double A[3][kBlock];   // leading piece of chunk t (row began earlier)
    double B[3][kBlock];   // trailing piece of chunk t (row goes on)
    double red[kWavesPerBlock][4];
};
using ItemLds = ItemLdsR<kBlock>;

struct NoHook {
    __device__ void operator()() const {}
};

// One work item: up to kR (256 or 512) consecutive rows [r0, r0 + nrow) of
// one packing; rp_own[k] = rp[r0 + t + 256 k] for the rows this thread owns
// and rp_end = rp[r0 + nrow] are given.
// Phase 1: the item's partner entries (contiguous in the CSR) are split in
// equal chunks over the 256 threads, so a row with thousands of partners is
// shared by many threads instead of serialising one.  A row lying inside one
// chunk is summed by that thread alone; a row spanning chunks is summed as
// (its piece in the chunk where it starts) + (the leading piece of every
// later chunk it covers), in chunk order, so the result does not depend on
// timing.  Phase 2: one thread per row applies Adam (coalesced).  hook() runs
// between the phases (the persistent kernel prefetches there).  Thread 0
// writes the item's partial sums to *out.  Every thread must call it.
template <int kU, bool kEarly, bool kStage, int kR, class Hook, bool kCoherentOut = false,
          bool kMixed = false, bool kWalls = false, int kDim = 3>
__device__ __forceinline__ void item_body(const IterPtrs &p, const IterScalars &c, int64_t r0,
                                          int nrow, int32_t e0, int32_t e1,
                                          const int32_t *rp_own, int32_t rp_end,
                                          ItemLdsR<kR> &L, int32_t *scol, Part4 *out, Hook hook,
                                          bool full)
{
    static_assert(kR == kBlock || (kR == 2 * kBlock && !kEarly), "rows per item");
    constexpr int kOwn = kR / kBlock;
    const P4 *Q = p.q;
    const int t = threadIdx.x;
    // this thread's chunk of the item's entries [e0, e1), and its first two
    // partner indices, requested alongside the row pointers
    const int32_t chunk = max(1, (e1 - e0 + kBlock - 1) / kBlock);
    const int32_t cs = e0 + t * chunk, ce = min(cs + chunk, e1);
    ColSrc<kStage> cols = {p.col, scol, e0, cs, 0, 0};
    if (!kStage && RCP_ITEM_PREFETCH) {
        if (cs < ce) cols.j0 = gload(p.col, cs);
        if (cs + 1 < ce) cols.j1 = gload(p.col, cs + 1);
    }
    // phase-2 operands either first (their latency hides behind phase 1)
    // or after it (fewer registers live through phase 1)
    P4 oq = {0, 0, 0, 0};
    Pre pre = {0, 0, 0, 0, 0, 0, 0.f, 0.f, 0.f};
    if (kEarly && t < nrow) {
        oq = load_p4(Q, (int32_t)(r0 + t));
        pre = preload<kDim>(p, r0 + t);
    }
#pragma unroll
    for (int k = 0; k < kOwn; ++k)
        if (t + k * kBlock < nrow) L.srp[t + k * kBlock] = rp_own[k];
    if (t == 0) L.srp[nrow] = rp_end;
    if (kStage) {
        // the item's partner indices, one coalesced pass
        const int32_t nst = min(e1 - e0, (int32_t)kColStage);
        for (int k = t; k < nst; k += kBlock) scol[k] = gload(p.col, (int64_t)e0 + k);
    }
    __syncthreads();

    // energy, kappa-gradient and max-overlap terms are block totals: each
    // thread keeps its own sums over its chunk (fixed assignment, so fixed
    // order); only the gradient needs per-row bookkeeping
    Acc a = {0, 0, 0, 0, 0, 0, 0};   // e, s, m: this thread's totals
    double bd = 0;
    const double rchunk = 1.0 / (double)chunk;   // block-uniform
    // the partner loop's waves take issue priority over the waves of other
    // blocks in their streaming phase (its dependent gathers are the longer
    // chain; measured 0.7-1.2 us faster per launch on the C3 state, priority
    // 1 and 3 less, priority in the Adam phase as well slower)
    __builtin_amdgcn_s_setprio(2);
    if (cs < ce) {
        int lo = 0, hi = nrow - 1;   // the row holding entry cs
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.srp[mid] <= cs) lo = mid;
            else hi = mid - 1;
        }
        int r = lo;
        int32_t q = cs;
        for (;;) {
            const P4 qi = load_p4(Q, (int32_t)(r0 + r));
            const int32_t rend = L.srp[r + 1], qe = min(rend, ce);
            a.gx = a.gy = a.gz = 0.0;
            segment_terms<kU, kStage, kMixed, kDim>(a, cols, Q, q, qe, qi, c);
            const bool began_before = L.srp[r] < cs, goes_on = rend > ce;
            if (began_before) store3<kBlock>(L.A, t, a);
            else if (goes_on) store3<kBlock>(L.B, t, a);
            else store3<kR>(L.G, r, a);
            q = qe;
            if (q >= ce) break;
            do {
                ++r;
            } while (L.srp[r + 1] <= q);   // skip rows without partners
        }
    }
    hook();
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();

#pragma unroll
    for (int k = 0; k < kOwn; ++k) {
        const int row = t + k * kBlock;
        if (row >= nrow) break;
        const int64_t io = r0 + row;
        if (!kEarly) {
            oq = load_p4(Q, (int32_t)io);
            pre = preload<kDim>(p, io);
        }
        const int32_t qb = L.srp[row], qe = L.srp[row + 1];
        double g[3] = {0, 0, 0};
        if (qb < qe) {
            const int tf = div_by(qb - e0, (uint32_t)chunk, rchunk),
                      tl = div_by(qe - 1 - e0, (uint32_t)chunk, rchunk);
            if (tf == tl) {
#pragma unroll
                for (int d = 0; d < 3; ++d) g[d] = L.G[d][row];
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) g[d] = L.B[d][tf];
                for (int u = tf + 1; u <= tl; ++u) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) g[d] += L.A[d][u];
                }
            }
        }
        if (kWalls) {
            // the row's wall terms (a sphere against the walls, in full)
            WallAcc w = {{0.0, 0.0, 0.0}, 0.0, 0.0, 0.0, 0.0};
            const double px[3] = {oq.x, oq.y, oq.z};
            wall_terms(px, c.kappa * oq.d, c.L, c.walls, c.round, w);
#pragma unroll
            for (int d = 0; d < 3; ++d) g[d] += w.g[d];
            a.e += w.e;
            a.s += w.s;
            a.m = fmax(a.m, w.m);
        }
        bd = fmax(bd, update_particle<kMixed, kDim>(p, c, io, oq, pre, g[0], g[1], g[2], full));
    }
    // block reduction of the four partials
    const int lane = t & (kWave - 1);
    const double be = wave_sum_dpp(a.e);
    const double bs = wave_sum_dpp(a.s);
    const double bm = wave_max_dpp(a.m);
    bd = wave_max_dpp(bd);
    const int wv = t / kWave;
    if (lane == 0) {
        L.red[wv][0] = be;
        L.red[wv][1] = bs;
        L.red[wv][2] = bm;
        L.red[wv][3] = bd;
    }
    __syncthreads();
    if (t == 0) {
        double e = 0, sd = 0, m = 0, d = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            e += L.red[k][0];
            sd += L.red[k][1];
            m = fmax(m, L.red[k][2]);
            d = fmax(d, L.red[k][3]);
        }
        if (kCoherentOut) {
            // agent-scope stores reach the device's coherence point: the
            // tail may run on another XCD
            __hip_atomic_store(&out->e, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&out->s, sd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&out->m, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&out->d, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            Part4 o;
            o.e = e;
            o.s = sd;
            o.m = m;
            o.d = d;
            *out = o;
        }
    }
}

template <bool kWalls = false>
__device__ __forceinline__ void load_scalars(const SegState *s, IterScalars &c)
{
    c.kappa = s->kappa;
    c.L = s->L;
    c.hL = s->hL;
    c.b1 = s->beta1;
    c.b2 = s->beta2;
    c.iL = s->iL;
    c.ib1 = s->ib1n;
    c.ib2 = s->ib2n;
    c.eta = s->eta_x;
    c.eps = s->eps_x;
    const int32_t bounded = kWalls ? (s->walls | s->round) : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool b = (bounded >> a) & 1;
        c.iLa[a] = b ? 0.0 : c.iL;
        c.Pa[a] = b ? 0.0 : c.L;
    }
    c.walls = kWalls ? s->walls : 0;
    c.round = kWalls ? s->round : 0;
}

// One block per work item; kWaves > 1 asks the compiler for that many
// waves per SIMD (fewer registers, a little spilling).
template <bool kFusedTail, int kU, bool kEarly, bool kStage, int kWaves, bool kMixed = false,
          bool kWalls = false, int kDim = 3>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWaves))) void k_iterate(const SegPtrs *__restrict__ P,
                                                   SegState *__restrict__ S,
                                                   const WorkItem *__restrict__ W,
                                                   double *__restrict__ partials, int flags)
{
    const int b = (flags & 1) ? remap_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const WorkItem w = W[b];
    SegState *s = S + w.seg;
    if (s->flags & F_IDLE) return;
    IterScalars c;
    load_scalars<kWalls>(s, c);
    const IterPtrs p = select_ptrs(P, w.seg, s->cur);
    __shared__ ItemLds L;
    __shared__ int32_t scol[kStage ? kColStage : 1];
    const int t = threadIdx.x;
    const int64_t r0 = w.begin;
    const int nrow = (int)(w.end - w.begin);
    const int32_t rp_t = t < nrow ? gload(p.rp, r0 + t) : 0;
    const int32_t rp_end = gload(p.rp, r0 + nrow);
    item_body<kU, kEarly, kStage, kBlock, NoHook, kFusedTail, kMixed, kWalls, kDim>(
        p, c, r0, nrow, w.e0, w.e1, &rp_t, rp_end, L, scol,
        reinterpret_cast<Part4 *>(partials) + b, NoHook(), (flags & 4) != 0);
    if (kFusedTail) {
        // the last block of the packing to finish reduces the partials and
        // runs the tail.  Partials are written and read with agent-scope
        // atomics (at the device's coherence point, past the XCDs' L2s); the
        // ticket is taken only after this block's partial stores have
        // completed (no release fence: on this part a fence writes back the
        // whole L2 of the XCD).
        __shared__ int last;
        if (t == 0) {
            __builtin_amdgcn_s_waitcnt(0);
            const uint32_t prev = __hip_atomic_fetch_add(&s->ticket, 1u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            last = (prev == (uint32_t)s->nblocks - 1u);
        }
        __syncthreads();
        if (last) {
            reduce_and_tail<kBlock, true>(s, partials);
            if (t == 0) __hip_atomic_store(&s->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Items of up to 512 rows: two rows per thread in the Adam phase, so half as
// many blocks carry the per-item set-up, synchronisation and reduction.
template <int kU>
__global__ __launch_bounds__(kBlock) void k_iterate512(const SegPtrs *__restrict__ P,
                                                      SegState *__restrict__ S,
                                                      const WorkItem *__restrict__ W,
                                                      double *__restrict__ partials, int flags)
{
    const int b = (flags & 1) ? remap_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const WorkItem w = W[b];
    SegState *s = S + w.seg;
    if (s->flags & F_IDLE) return;
    IterScalars c;
    load_scalars(s, c);
    const IterPtrs p = select_ptrs(P, w.seg, s->cur);
    __shared__ ItemLdsR<2 * kBlock> L;
    const int t = threadIdx.x;
    const int64_t r0 = w.begin;
    const int nrow = (int)(w.end - w.begin);
    int32_t rp_own[2];
    rp_own[0] = t < nrow ? gload(p.rp, r0 + t) : 0;
    rp_own[1] = t + kBlock < nrow ? gload(p.rp, r0 + t + kBlock) : 0;
    const int32_t rp_end = gload(p.rp, r0 + nrow);
    item_body<kU, false, false, 2 * kBlock>(p, c, r0, nrow, w.e0, w.e1, rp_own, rp_end, L,
                                            nullptr,
                                            reinterpret_cast<Part4 *>(partials) + b, NoHook(),
                                            (flags & 4) != 0);
}

// resident blocks of the persistent form: 256 CUs x 5 blocks (the occupancy
// of the two-gather variant)
constexpr int kPersistBlocks = 256 * 5;

// Persistent form: a grid of resident blocks, each taking the work items
// lo + slot, lo + slot + nbx, ... of its XCD's contiguous range (blocks are
// dispatched round-robin over the 8 XCDs).  The next item's descriptor is
// requested at the top of an item and its row pointers between the item's
// two phases, so they are in registers when the item starts.
template <int kU>
__global__ __launch_bounds__(kBlock) void k_iterate_persist(const SegPtrs *__restrict__ P,
                                                           SegState *__restrict__ S,
                                                           const WorkItem *__restrict__ W,
                                                           double *__restrict__ partials,
                                                           int nitems, int flags)
{
    constexpr int nx = 8;
    const int G = (int)gridDim.x;
    int lo = 0, hi = nitems, slot = (int)blockIdx.x, nbx = G;
    if ((flags & 1) && G >= nx) {
        const int xcd = (int)blockIdx.x % nx;
        slot = (int)blockIdx.x / nx;
        nbx = (G - xcd + nx - 1) / nx;
        const int per = nitems / nx, rem = nitems % nx;
        lo = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
        hi = lo + per + (xcd < rem ? 1 : 0);
    }
    int item = lo + slot;
    if (item >= hi) return;
    __shared__ ItemLds L;
    const int t = threadIdx.x;
    WorkItem wn = W[item];
    int cseg = -1;
    bool idle = true;
    IterScalars c;
    IterPtrs p;
    int32_t rpn_t = 0, rpn_e = 0;
    bool have = false;
    for (;;) {
        const WorkItem w = wn;
        const int next = item + nbx;
        if (next < hi) wn = W[next];
        if (w.seg != cseg) {
            cseg = w.seg;
            const SegState *s = S + cseg;
            idle = (s->flags & F_IDLE) != 0;
            if (!idle) {
                load_scalars(s, c);
                p = select_ptrs(P, cseg, s->cur);
            }
            have = false;
        }
        if (!idle) {
            const int nrow = (int)(w.end - w.begin);
            int32_t rp_t, rp_end;
            if (have) {
                rp_t = rpn_t;
                rp_end = rpn_e;
            } else {
                rp_t = t < nrow ? gload(p.rp, w.begin + t) : 0;
                rp_end = gload(p.rp, w.begin + nrow);
            }
            have = false;
            auto hook = [&]() {
                if (next < hi && wn.seg == cseg) {
                    const int nr = (int)(wn.end - wn.begin);
                    rpn_t = t < nr ? gload(p.rp, wn.begin + t) : 0;
                    rpn_e = gload(p.rp, wn.begin + nr);
                    have = true;
                }
            };
            item_body<kU, false, false, kBlock>(p, c, w.begin, nrow, w.e0, w.e1, &rp_t, rp_end,
                                                L, nullptr,
                                                reinterpret_cast<Part4 *>(partials) + item,
                                                hook, (flags & 4) != 0);
        }
        item = next;
        if (item >= hi) break;
        __syncthreads();   // the item's LDS is reused
    }
}

template <bool kF, int kU, bool kE, bool kNT, int kW, bool kMixed = false, bool kWalls = false,
          int kDim = 3>
static void launch_one(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                       int nitems, int f, hipStream_t st)
{
    hipLaunchKernelGGL((k_iterate<kF, kU, kE, kNT, kW, kMixed, kWalls, kDim>), dim3(nitems),
                       dim3(kBlock), 0, st, P, S, W, partials, f);
}

template <bool kF, int kW>
static void launch_basic(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                         int nitems, int f, int variant, hipStream_t st)
{
    switch (variant & 7) {
    case 0: launch_one<kF, 2, false, false, kW>(P, S, W, partials, nitems, f, st); break;
    case 1: launch_one<kF, 4, false, false, kW>(P, S, W, partials, nitems, f, st); break;
    case 2: launch_one<kF, 2, true, false, kW>(P, S, W, partials, nitems, f, st); break;
    case 3: launch_one<kF, 4, true, false, kW>(P, S, W, partials, nitems, f, st); break;
    case 4: launch_one<kF, 2, false, true, kW>(P, S, W, partials, nitems, f, st); break;
    case 5: launch_one<kF, 4, false, true, kW>(P, S, W, partials, nitems, f, st); break;
    case 6: launch_one<kF, 2, true, true, kW>(P, S, W, partials, nitems, f, st); break;
    default: launch_one<kF, 4, true, true, kW>(P, S, W, partials, nitems, f, st); break;
    }
}

template <bool kF>
static void launch_variant(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                           int nitems, int f, int variant, hipStream_t st)
{
    // bit 0: four gathers in flight; bit 1: early Adam operands; bit 2:
    // partner indices staged in LDS; bit 3: persistent blocks (bits 1, 2 and
    // the fused tail do not apply to it); bit 4: seven waves per SIMD asked
    // of the compiler; bit 5: items of up to 512 rows (bits 1-4 and the
    // fused tail do not apply)
    if (variant & 8) {
        const int grid = std::min(nitems, kPersistBlocks);
        if (variant & 1)
            hipLaunchKernelGGL(k_iterate_persist<4>, dim3(grid), dim3(kBlock), 0, st, P, S, W,
                               partials, nitems, f);
        else
            hipLaunchKernelGGL(k_iterate_persist<2>, dim3(grid), dim3(kBlock), 0, st, P, S, W,
                               partials, nitems, f);
        return;
    }
    if (variant & 32) {
        if (variant & 1)
            hipLaunchKernelGGL(k_iterate512<4>, dim3(nitems), dim3(kBlock), 0, st, P, S, W,
                               partials, f);
        else
            hipLaunchKernelGGL(k_iterate512<2>, dim3(nitems), dim3(kBlock), 0, st, P, S, W,
                               partials, f);
        return;
    }
    if (variant & 16) launch_basic<kF, 7>(P, S, W, partials, nitems, f, variant, st);
    else launch_basic<kF, 1>(P, S, W, partials, nitems, f, variant, st);
}

void launch_iterate(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                    int nitems, int flags, hipStream_t st)
{
    // bit 0: XCD-aware order; bit 1: fused tail; bit 2: whole 32-byte
    // records written; bit 4: some packing has frozen spheres (then the
    // two-gather kernel with the mixed pair terms runs, whatever the
    // variant); bit 5: some packing has walls (then the two-gather kernel
    // with the wall terms runs, whatever the variant; never together with
    // bit 4); bit 6: two dimensions (the two-gather kernel for two
    // coordinates, whatever the variant); bits 8-13: kernel variant (see
    // launch_variant)
    const int f = flags & 5, variant = (flags >> 8) & 63;
    if (flags & 64) {
        if (flags & 32)
            launch_one<false, 2, false, false, 1, false, true, 2>(P, S, W, partials, nitems, f, st);
        else if (flags & 16)
            launch_one<false, 2, false, false, 1, true, false, 2>(P, S, W, partials, nitems, f, st);
        else
            launch_one<false, 2, false, false, 1, false, false, 2>(P, S, W, partials, nitems, f,
                                                                   st);
    } else if (flags & 32)
        launch_one<false, 2, false, false, 1, false, true>(P, S, W, partials, nitems, f, st);
    else if (flags & 16)
        launch_one<false, 2, false, false, 1, true>(P, S, W, partials, nitems, f, st);
    else if (variant & 40) launch_variant<false>(P, S, W, partials, nitems, f, variant, st);
    else if (flags & 2) launch_variant<true>(P, S, W, partials, nitems, f, variant, st);
    else launch_variant<false>(P, S, W, partials, nitems, f, variant, st);
}

constexpr int kTailBlock = 1024;

// One block per packing.  The packing's record is copied to LDS in one
// parallel pass, the tail works on the copy (its many dependent reads and
// writes then cost LDS latency, not memory latency) and the block writes the
// record back.
__global__ __launch_bounds__(kTailBlock) void k_tail(SegState *__restrict__ S,
                                                    const double *__restrict__ partials,
                                                    int64_t b0, int64_t nb)
{
    static_assert(sizeof(SegState) % 8 == 0, "SegState is copied in 8-byte words");
    constexpr int kWords = (int)(sizeof(SegState) / 8);
    __shared__ SegState ls;
    SegState *gs = S + blockIdx.x;
    // the partials are loaded before the record is copied, so the two
    // latencies overlap (an idle packing's stale partials are then dropped);
    // with one packing their range comes with the launch (nb >= 0), so the
    // loads need not wait for the record
    if (nb < 0) {
        nb = gs->nblocks;
        b0 = gs->bfirst;
    }
    const Part4 mine = thread_partials<kTailBlock, false>(nb, b0, partials);
    uint64_t *src = reinterpret_cast<uint64_t *>(gs);
    uint64_t *dst = reinterpret_cast<uint64_t *>(&ls);
    for (int k = threadIdx.x; k < kWords; k += kTailBlock) dst[k] = src[k];
    __syncthreads();
    if (ls.flags & F_IDLE) return;
    block_tail<kTailBlock>(&ls, mine);
    __syncthreads();
    for (int k = threadIdx.x; k < kWords; k += kTailBlock) src[k] = dst[k];
}

// Work items.  Row i of a packing has work coordinate w(i) = rc * i + rp[i]
// (strictly increasing, w(0) = 0); item b holds the rows with w(i) in
// [b * wk, (b + 1) * wk), i.e. it begins at the first row with w(i) >= b * wk.
// Row i is that first row for the items b with w(i - 1) < b * wk <= w(i),
// so one thread per row writes every boundary exactly once; items past the
// last row keep begin = end = n from the fill.  With wk <= 256 rc no item
// holds more than 256 rows.
__global__ __launch_bounds__(kBlock) void k_items_fill(WorkItem *__restrict__ W, int64_t nslots,
                                                      int seg, const int32_t *__restrict__ rp,
                                                      int64_t n)
{
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nslots) return;
    WorkItem w;
    w.seg = seg;
    w.e0 = w.e1 = rp ? rp[n] : 0;
    w.pad = 0;
    w.begin = n;
    w.end = n;
    W[b] = w;
}

__global__ __launch_bounds__(kBlock) void k_items(const int32_t *__restrict__ rp, int64_t n,
                                                 int64_t rc, int64_t wk,
                                                 WorkItem *__restrict__ W, int64_t nslots)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t hi = rc * i + (int64_t)rp[i];
    const int64_t bl = i == 0 ? 0 : (rc * (i - 1) + (int64_t)rp[i - 1]) / wk + 1;
    const int64_t bh = min(hi / wk, nslots - 1);
    for (int64_t b = bl; b <= bh; ++b) {
        W[b].begin = i;
        W[b].e0 = rp[i];
        if (b > 0) {
            W[b - 1].end = i;
            W[b - 1].e1 = rp[i];
        }
    }
}

void launch_items(const int32_t *rp, int64_t n, int seg, int row_cost, int item_work,
                  WorkItem *W, int64_t nslots, hipStream_t st)
{
    if (nslots <= 0) return;
    const unsigned gf = (unsigned)((nslots + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_items_fill, dim3(gf), dim3(kBlock), 0, st, W, nslots, seg, rp,
                       rp ? n : (int64_t)0);
    if (!rp || n <= 0) return;
    const unsigned gi = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_items, dim3(gi), dim3(kBlock), 0, st, rp, n, (int64_t)row_cost,
                       (int64_t)item_work, W, nslots);
}

// Segmented forms for a batch of list builds: block b of a grid belongs
// to the last job whose first block is <= b.
__device__ __forceinline__ int back_job_of(const BackJob *__restrict__ jobs, int J, int64_t b,
                                           int64_t BackJob::*first)
{
    int lo = 0, hi = J - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*first <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_items_fill_seg(const BackJob *__restrict__ jobs, int J)
{
    const BackJob &B = jobs[back_job_of(jobs, J, blockIdx.x, &BackJob::bs0)];
    const int64_t b = ((int64_t)blockIdx.x - B.bs0) * kBlock + threadIdx.x;
    if (!B.fill || b >= B.nslots) return;
    WorkItem w;
    w.seg = B.seg;
    w.e0 = w.e1 = B.rp ? B.rp[B.n] : 0;
    w.pad = 0;
    w.begin = B.n;
    w.end = B.n;
    B.W[b] = w;
}

__global__ __launch_bounds__(kBlock) void k_items_seg(const BackJob *__restrict__ jobs, int J)
{
    const BackJob &B = jobs[back_job_of(jobs, J, blockIdx.x, &BackJob::br0)];
    const int64_t i = ((int64_t)blockIdx.x - B.br0) * kBlock + threadIdx.x;
    if (!B.fill || i >= B.n) return;
    const int64_t rc = B.row_cost, wk = B.item_work;
    const int64_t hi = rc * i + (int64_t)B.rp[i];
    const int64_t bl = i == 0 ? 0 : (rc * (i - 1) + (int64_t)B.rp[i - 1]) / wk + 1;
    const int64_t bh = min(hi / wk, B.nslots - 1);
    for (int64_t b = bl; b <= bh; ++b) {
        B.W[b].begin = i;
        B.W[b].e0 = B.rp[i];
        if (b > 0) {
            B.W[b - 1].end = i;
            B.W[b - 1].e1 = B.rp[i];
        }
    }
}

__global__ void k_after_seg(const BackJob *__restrict__ jobs, int J, SegState *S, SegPtrs *P)
{
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= J) return;
    const BackJob &B = jobs[j];
    SegState *s = S + B.seg;
    s->kb = B.kb;
    s->disp_lim = B.disp_lim;
    s->kappa_lim = B.kappa_lim;
    s->cur = B.cur;
    s->flags &= ~(F_REBUILD | F_STALE);
    P[B.seg] = B.ptrs;
}

void launch_items_seg(const BackJob *jobs, int J, int64_t nbs, int64_t nbr, hipStream_t st)
{
    if (nbs > 0)
        hipLaunchKernelGGL(k_items_fill_seg, dim3((unsigned)nbs), dim3(kBlock), 0, st, jobs, J);
    if (nbr > 0)
        hipLaunchKernelGGL(k_items_seg, dim3((unsigned)nbr), dim3(kBlock), 0, st, jobs, J);
}

void launch_after_seg(const BackJob *jobs, int J, SegState *S, SegPtrs *P, hipStream_t st)
{
    if (J > 0)
        hipLaunchKernelGGL(k_after_seg, dim3((unsigned)((J + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           st, jobs, J, S, P);
}

// Work-table layout of every packing: lay[2k] blocks, lay[2k + 1] first item.
__global__ void k_set_layout(SegState *S, int nseg, const int64_t *__restrict__ lay)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= nseg) return;
    S[k].nblocks = (int32_t)lay[2 * k];
    S[k].bfirst = lay[2 * k + 1];
}

void launch_set_layout(SegState *S, int nseg, const int64_t *lay, hipStream_t st)
{
    if (nseg > 0)
        hipLaunchKernelGGL(k_set_layout, dim3((unsigned)((nseg + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, S, nseg, lay);
}

void launch_tail(SegState *S, const double *partials, int nseg, int64_t b0, int64_t nb,
                 hipStream_t st)
{
    if (nseg != 1) b0 = 0, nb = -1;
    hipLaunchKernelGGL(k_tail, dim3(nseg), dim3(kTailBlock), 0, st, S, partials, b0, nb);
}

__global__ void k_sched_start(SegState *S, int seg, SchedDev q, int reset_adam,
                              int64_t iter_limit)
{
    SegState *s = S + seg;
    s->sched = q;
    s->rung = 0;
    s->it_rung = 0;
    s->iters = 0;
    s->iter_limit = iter_limit;
    if (reset_adam) {
        s->t = 0;
        s->b1t = 1.0;
        s->b2t = 1.0;
        seg_bias_terms(*s);
        s->mk = 0.0;
        s->vk = 0.0;
    }
    s->flags &= ~(F_STOP | F_CAP | F_HOLD | F_NONFINITE | F_ABORT);
    rung_start(s, 0);
}

void launch_sched_start(SegState *S, int seg, const SchedDev &q, int reset_adam,
                        int64_t iter_limit, hipStream_t st)
{
    hipLaunchKernelGGL(k_sched_start, dim3(1), dim3(1), 0, st, S, seg, q, reset_adam,
                       iter_limit);
}

__global__ void k_set_flags(SegState *S, int seg, int32_t clear, int32_t set)
{
    S[seg].flags = (S[seg].flags & ~clear) | set;
}

void launch_set_flags(SegState *S, int seg, int32_t clear, int32_t set, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(1), 0, st, S, seg, clear, set);
}

// ------------------------------------------------------- evaluation
// Thread per row over the whole list (not on the iteration path); positions
// from the user-order array xu (gathered through orig) or from the current
// buffer.  Partials per block: E_ov, S, max delta, overlapping pairs (and
// wall contacts, with walls).
__global__ __launch_bounds__(kBlock) void k_eval(const SegPtrs *__restrict__ P,
                                                const SegState *__restrict__ S, int seg,
                                                int64_t n, const double *__restrict__ xu,
                                                double kappa, double *__restrict__ part,
                                                double *__restrict__ gu)
{
    const SegState *s = S + seg;
    const IterPtrs p = select_ptrs(P, seg, s->cur);
    const int32_t *orig = P[seg].orig;
    const double L = s->L, iL = 1.0 / L;
    const int32_t bounded = s->walls | s->round;
    const double iLa[3] = {(bounded & 1) ? 0.0 : iL, (bounded & 2) ? 0.0 : iL,
                           (bounded & 4) ? 0.0 : iL};
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double be = 0, bs = 0, bm = 0, bn = 0;
    if (i < n) {
        // position from the user-order array when given, D0 from the list
        auto pos = [&](int64_t k) -> P4 {
            P4 q = p.q[k];
            if (xu) {
                const int64_t u = orig[k];
                q.x = xu[3 * u];
                q.y = xu[3 * u + 1];
                q.z = xu[3 * u + 2];
            }
            return q;
        };
        const P4 qi = pos(i);
        Acc a = {0, 0, 0, 0, 0, 0, 0};
        if (s->mixed)
            for (int32_t q = p.rp[i]; q < p.rp[i + 1]; ++q)
                pair_term<true, true>(a, qi, pos(p.col[q]), kappa, L, iLa);
        else
            for (int32_t q = p.rp[i]; q < p.rp[i + 1]; ++q)
                pair_term(a, qi, pos(p.col[q]), kappa, L, iLa);
        if (bounded) {
            WallAcc w = {{0.0, 0.0, 0.0}, 0.0, 0.0, 0.0, 0.0};
            const double px[3] = {qi.x, qi.y, qi.z};
            wall_terms(px, kappa * qi.d, L, s->walls, s->round, w);
            a.gx += w.g[0];
            a.gy += w.g[1];
            a.gz += w.g[2];
            a.e += w.e;
            a.s += w.s;
            a.m = fmax(a.m, w.m);
            a.c += w.c;
        }
        be = a.e;
        bs = a.s;
        bm = a.m;
        bn = a.c;
        if (gu) {
            const int64_t u = orig[i];
            gu[3 * u] = a.gx;
            gu[3 * u + 1] = a.gy;
            gu[3 * u + 2] = a.gz;
        }
    }
    be = wave_sum(be);
    bs = wave_sum(bs);
    bm = wave_max(bm);
    bn = wave_sum(bn);
    __shared__ double red[kWavesPerBlock][4];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) {
        red[wv][0] = be;
        red[wv][1] = bs;
        red[wv][2] = bm;
        red[wv][3] = bn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0, sd = 0, m = 0, c = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            e += red[k][0];
            sd += red[k][1];
            m = fmax(m, red[k][2]);
            c += red[k][3];
        }
        double *o = part + 4 * (int64_t)blockIdx.x;
        o[0] = e;
        o[1] = sd;
        o[2] = m;
        o[3] = c;
    }
}

void launch_eval(const SegPtrs *P, const SegState *S, int seg, int64_t n, const double *xu,
                 double kappa, const EvalOut &o, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_eval, dim3(nblocks), dim3(kBlock), 0, st, P, S, seg, n, xu, kappa,
                       o.part, o.gu);
}

__global__ __launch_bounds__(kWave) void k_eval_finish(const double *__restrict__ part,
                                                      int nblocks, double kappa, double mu,
                                                      const SegState *__restrict__ S, int seg,
                                                      double *__restrict__ out)
{
    const int lane = threadIdx.x;
    double e = 0, sd = 0, m = 0, c = 0;
    for (int b = lane; b < nblocks; b += kWave) {
        e += part[4 * b];
        sd += part[4 * b + 1];
        m = fmax(m, part[4 * b + 2]);
        c += part[4 * b + 3];
    }
    e = wave_sum(e);
    sd = wave_sum(sd);
    m = wave_max(m);
    c = wave_sum(c);
    if (lane == 0) {
        const double sum0 = S[seg].sumd0;
        out[0] = e;
        out[1] = -mu * kappa * sum0;
        out[2] = sd / kappa;
        out[3] = -mu * sum0;
        out[4] = m;
        out[5] = c;
    }
}

void launch_eval_finish(const double *part, int nblocks, double kappa, double mu,
                        const SegState *S, int seg, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_eval_finish, dim3(1), dim3(kWave), 0, st, part, nblocks, kappa, mu, S,
                       seg, out);
}

__global__ __launch_bounds__(kBlock) void k_disp(const SegPtrs *__restrict__ P,
                                                const SegState *__restrict__ S, int seg,
                                                int64_t n, const double *__restrict__ xu,
                                                double *__restrict__ part)
{
    const SegPtrs p = P[seg];
    const double L = S[seg].L, hL = S[seg].hL;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double d2 = 0;
    if (i < n) {
        const int64_t u = p.orig[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double dd = min_image(xu[3 * u + a] - (double)p.xref[a][i], L, hL);
            d2 += dd * dd;
        }
    }
    d2 = wave_max(d2);
    __shared__ double red[kWavesPerBlock];
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) m = fmax(m, red[k]);
        part[blockIdx.x] = m;
    }
}

void launch_disp(const SegPtrs *P, const SegState *S, int seg, int64_t n, const double *xu,
                 double *part, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_disp, dim3(nblocks), dim3(kBlock), 0, st, P, S, seg, n, xu, part);
}

__global__ __launch_bounds__(kBlock) void k_set_frozen(const SegPtrs *__restrict__ P, int seg,
                                                      int64_t n, const uint8_t *__restrict__ mask)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const SegPtrs &p = P[seg];
    const bool f = mask[p.orig[i]] != 0;
    for (int b = 0; b < 2; ++b) {
        const double d = fabs(p.p[b][i].d);
        p.p[b][i].d = f ? -d : d;
    }
}

void launch_set_frozen(const SegPtrs *P, int seg, int64_t n, const uint8_t *mask, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_set_frozen, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, st, P, seg, n, mask);
}

__global__ __launch_bounds__(kBlock) void k_set_positions(const SegPtrs *__restrict__ P,
                                                         int seg, int64_t n,
                                                         const double *__restrict__ xu, int cur)
{
    P4 *Q = cur ? P[seg].p[1] : P[seg].p[0];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t u = P[seg].orig[i];
    P4 q = Q[i];
    q.x = xu[3 * u];
    q.y = xu[3 * u + 1];
    q.z = xu[3 * u + 2];
    Q[i] = q;
}

// Adam moments of packing seg between list order and user order (mu, vu:
// n x 3 row-major): dir 0 copies the list's moments out, dir 1 in.
__global__ __launch_bounds__(kBlock) void k_moments_io(const SegPtrs *__restrict__ P, int seg,
                                                      int64_t n, double *__restrict__ mu,
                                                      double *__restrict__ vu, int dir)
{
    const SegPtrs &p = P[seg];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t u = p.orig[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dir == 0) {
            mu[3 * u + a] = p.m[a][i];
            vu[3 * u + a] = p.v[a][i];
        } else {
            p.m[a][i] = mu[3 * u + a];
            p.v[a][i] = vu[3 * u + a];
        }
    }
}

void launch_moments_io(const SegPtrs *P, int seg, int64_t n, double *mu, double *vu, int dir,
                       hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_moments_io, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, P, seg, n, mu, vu, dir);
}

void launch_set_positions(const SegPtrs *P, SegState *S, int seg, int64_t n, const double *xu,
                          int cur, hipStream_t st)
{
    (void)S;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_set_positions, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, st, P, seg, n, xu, cur);
}

}  // namespace rcp
