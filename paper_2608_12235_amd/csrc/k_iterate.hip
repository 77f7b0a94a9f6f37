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
// before the update), Adam on kappa, the step-size decay and the rung
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

struct Acc {
    double gx, gy, gz, e, s, m, c;
};

__device__ __forceinline__ void pair_term(Acc &a, double xi, double yi, double zi, double di,
                                          double xj, double yj, double zj, double dj,
                                          double kappa, double L, double hL)
{
    const double dx = min_image(xj - xi, L, hL);
    const double dy = min_image(yj - yi, L, hL);
    const double dz = min_image(zj - zi, L, hL);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const double d = kappa * (0.5 * (di + dj));
    if (r2 < d * d) {
        const double r = sqrt(r2);
        const double delta = 1.0 - r / d;
        a.e += 0.25 * (delta * delta);
        a.s += 0.5 * (delta * r / d);
        a.m = fmax(a.m, delta);
        a.c += 0.5;
        if (r > 0.0) {
            const double f = delta / (d * r);
            a.gx += f * dx;
            a.gy += f * dy;
            a.gz += f * dz;
        }
    }
}

__device__ __forceinline__ double adam_coord(double th, double g, double &m, double &v,
                                             double b1, double b2, double bc1, double bc2,
                                             double eta, double eps, double L)
{
    m = b1 * m + (1.0 - b1) * g;
    v = b2 * v + (1.0 - b2) * (g * g);
    const double mh = m / bc1, vh = v / bc2;
    double t = th - eta * mh / (sqrt(vh) + eps);
    if (t < 0.0) t += L;
    if (t >= L) t -= L;
    return t;
}

struct IterScalars {
    double kappa, L, hL, b1, b2, bc1, bc2, eta, eps;
};

// Pointers of one segment with the ping-pong buffers already selected
// (uniform selects keep them in scalar registers; indexing the pointer
// table with the runtime buffer index would spill it to scratch).
struct IterPtrs {
    const double *x, *y, *z, *d0;
    double *xo, *yo, *zo;
    double *m0, *m1, *m2, *v0, *v1, *v2, *r0, *r1, *r2;
    const int32_t *rp, *col;
};

__device__ __forceinline__ IterPtrs select_ptrs(const SegPtrs *__restrict__ P, int seg, int cur)
{
    const SegPtrs &q = P[seg];
    IterPtrs p;
    p.x = cur ? q.x[1][0] : q.x[0][0];
    p.y = cur ? q.x[1][1] : q.x[0][1];
    p.z = cur ? q.x[1][2] : q.x[0][2];
    p.xo = cur ? q.x[0][0] : q.x[1][0];
    p.yo = cur ? q.x[0][1] : q.x[1][1];
    p.zo = cur ? q.x[0][2] : q.x[1][2];
    p.d0 = q.d0;
    p.m0 = q.m[0];
    p.m1 = q.m[1];
    p.m2 = q.m[2];
    p.v0 = q.v[0];
    p.v1 = q.v[1];
    p.v2 = q.v[2];
    p.r0 = q.xref[0];
    p.r1 = q.xref[1];
    p.r2 = q.xref[2];
    p.rp = q.rp;
    p.col = q.col;
    return p;
}

// One coordinate's Adam update from preloaded operands; returns the squared
// (minimum image) displacement from the list reference along that axis.
__device__ __forceinline__ double update_coord(double xi, double g, double m, double v, double r,
                                               double *xout, double *mm, double *vv,
                                               const IterScalars &c, int64_t i)
{
    const double xn = adam_coord(xi, g, m, v, c.b1, c.b2, c.bc1, c.bc2, c.eta, c.eps, c.L);
    xout[i] = xn;
    mm[i] = m;
    vv[i] = v;
    const double dd = min_image(xn - r, c.L, c.hL);
    return dd * dd;
}

struct Pre {
    double m0, m1, m2, v0, v1, v2, r0, r1, r2;
};

__device__ __forceinline__ Pre preload(const IterPtrs &p, int64_t i)
{
    Pre q;
    q.m0 = p.m0[i];
    q.m1 = p.m1[i];
    q.m2 = p.m2[i];
    q.v0 = p.v0[i];
    q.v1 = p.v1[i];
    q.v2 = p.v2[i];
    q.r0 = p.r0[i];
    q.r1 = p.r1[i];
    q.r2 = p.r2[i];
    return q;
}

// Adam on particle i's coordinates; returns |x_new - x_ref|^2 (min image).
__device__ __forceinline__ double update_particle(const IterPtrs &p, const IterScalars &c,
                                                  int64_t i, double xi, double yi, double zi,
                                                  const Pre &q, double gx, double gy, double gz)
{
    double d2 = update_coord(xi, gx, q.m0, q.v0, q.r0, p.xo, p.m0, p.v0, c, i);
    d2 += update_coord(yi, gy, q.m1, q.v1, q.r1, p.yo, p.m1, p.v1, c, i);
    d2 += update_coord(zi, gz, q.m2, q.v2, q.r2, p.zo, p.m2, p.v2, c, i);
    return d2;
}

__device__ __forceinline__ void rung_start(SegState *s, int r)
{
    const SchedDev &q = s->sched;
    if (q.absolute) {
        s->mu = q.mu[r];
        s->eta_x = q.eta_x[r];
        s->eta_k = q.eta_k[r];
    } else {
        s->mu = (q.mu[r] * (double)s->n) / (s->kappa * s->sumd0);
        s->eta_x = q.eta_x[r] * (s->kappa * s->d0min);
        s->eta_k = q.eta_k[r] * s->kappa;
    }
}

__device__ void tail_logic(SegState *s, double E, double S, double md, double mdisp2)
{
    s->E_ov = E;
    s->S_drd = S;
    s->max_delta = md;
    s->max_disp2 = mdisp2;
    const SchedDev &q = s->sched;
    const int r = s->rung, last = q.n_rungs - 1;
    const double kappa = s->kappa;
    const double gk = S / kappa - s->mu * s->sumd0;
    if (!isfinite(E) || !isfinite(gk) || !isfinite(mdisp2)) {
        s->flags |= F_NONFINITE;
        return;
    }
    if (r == last && md < q.tol) {
        s->flags |= F_STOP;
        return;
    }
    s->t += 1;
    s->b1t *= s->beta1;
    s->b2t *= s->beta2;
    double mk = s->mk, vk = s->vk;
    mk = s->beta1 * mk + (1.0 - s->beta1) * gk;
    vk = s->beta2 * vk + (1.0 - s->beta2) * (gk * gk);
    const double mh = mk / (1.0 - s->b1t), vh = vk / (1.0 - s->b2t);
    s->kappa = kappa - s->eta_k * mh / (sqrt(vh) + s->eps_k);
    s->mk = mk;
    s->vk = vk;
    s->cur ^= 1;
    s->eta_x *= q.decay[r];
    s->eta_k *= q.decay[r];
    s->it_rung += 1;
    s->iters += 1;
    if (s->it_rung >= q.budget[r]) {
        if (r == last) {
            s->flags |= F_CAP;
        } else {
            s->rung = r + 1;
            s->it_rung = 0;
            rung_start(s, r + 1);
        }
    }
    if (!(s->kappa > 0.0) || !isfinite(s->kappa)) s->flags |= F_NONFINITE;
    if (mdisp2 > s->disp_lim2 || s->kappa > s->kappa_lim) s->flags |= F_REBUILD;
    if (s->iter_limit > 0 && s->iters >= s->iter_limit) s->flags |= F_HOLD;
}

// Deterministic reduction of a segment's block partials by one block (fixed
// assignment of partials to threads, fixed combining order); thread 0 then
// runs the tail.  Every thread of the block must call it.
__device__ void reduce_and_tail(SegState *s, const double *partials)
{
    double e = 0, sd = 0, m = 0, d = 0;
    const int64_t nb = s->nblocks, b0 = s->bfirst;
    for (int64_t b = threadIdx.x; b < nb; b += kBlock) {
        const double *p = partials + 4 * (b0 + b);
        e += p[0];
        sd += p[1];
        m = fmax(m, p[2]);
        d = fmax(d, p[3]);
    }
    e = wave_sum(e);
    sd = wave_sum(sd);
    m = wave_max(m);
    d = wave_max(d);
    __shared__ double red[kWavesPerBlock][4];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) {
        red[wv][0] = e;
        red[wv][1] = sd;
        red[wv][2] = m;
        red[wv][3] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        e = 0, sd = 0, m = 0, d = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            e += red[k][0];
            sd += red[k][1];
            m = fmax(m, red[k][2]);
            d = fmax(d, red[k][3]);
        }
        tail_logic(s, e, sd, m, d);
    }
}

// Entry loop of one row segment [q, qe): four partners per step so that
// their gathers are in flight together.
__device__ __forceinline__ void segment_terms(Acc &a, const int32_t *__restrict__ col,
                                              const double *__restrict__ X,
                                              const double *__restrict__ Y,
                                              const double *__restrict__ Z,
                                              const double *__restrict__ D, int32_t q, int32_t qe,
                                              double xi, double yi, double zi, double di,
                                              const IterScalars &c)
{
    for (; q + 4 <= qe; q += 4) {
        const int32_t j0 = col[q], j1 = col[q + 1], j2 = col[q + 2], j3 = col[q + 3];
        const double x0 = X[j0], y0 = Y[j0], z0 = Z[j0], e0 = D[j0];
        const double x1 = X[j1], y1 = Y[j1], z1 = Z[j1], e1 = D[j1];
        const double x2 = X[j2], y2 = Y[j2], z2 = Z[j2], e2 = D[j2];
        const double x3 = X[j3], y3 = Y[j3], z3 = Z[j3], e3 = D[j3];
        pair_term(a, xi, yi, zi, di, x0, y0, z0, e0, c.kappa, c.L, c.hL);
        pair_term(a, xi, yi, zi, di, x1, y1, z1, e1, c.kappa, c.L, c.hL);
        pair_term(a, xi, yi, zi, di, x2, y2, z2, e2, c.kappa, c.L, c.hL);
        pair_term(a, xi, yi, zi, di, x3, y3, z3, e3, c.kappa, c.L, c.hL);
    }
    for (; q < qe; ++q) {
        const int32_t j = col[q];
        pair_term(a, xi, yi, zi, di, X[j], Y[j], Z[j], D[j], c.kappa, c.L, c.hL);
    }
}

__device__ __forceinline__ void store6(double (*M)[kBlock], int k, const Acc &a)
{
    M[0][k] = a.gx;
    M[1][k] = a.gy;
    M[2][k] = a.gz;
    M[3][k] = a.e;
    M[4][k] = a.s;
    M[5][k] = a.m;
}

// One iteration for a block of up to 256 consecutive rows of one packing.
// Phase 1: the block's partner entries (contiguous in the CSR) are split in
// equal chunks over the 256 threads, so a row with thousands of partners is
// shared by many threads instead of serialising one.  A row lying inside one
// chunk is summed by that thread alone; a row spanning chunks is summed as
// (its piece in the chunk where it starts) + (the leading piece of every
// later chunk it covers), in chunk order, so the result does not depend on
// timing.  Phase 2: one thread per row applies Adam (coalesced).
template <bool kFusedTail>
__global__ __launch_bounds__(kBlock) void k_iterate(const SegPtrs *__restrict__ P,
                                                   SegState *__restrict__ S,
                                                   const WorkItem *__restrict__ W,
                                                   double *__restrict__ partials, int flags)
{
    int b = (flags & 1) ? remap_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    if (flags & 4) b = (int)gridDim.x - 1 - b;   // largest particles (last rows) first
    const WorkItem w = W[b];
    SegState *s = S + w.seg;
    if (s->flags & F_IDLE) return;
    IterScalars c;
    c.kappa = s->kappa;
    c.L = s->L;
    c.hL = s->hL;
    c.b1 = s->beta1;
    c.b2 = s->beta2;
    c.bc1 = 1.0 - s->b1t * c.b1;
    c.bc2 = 1.0 - s->b2t * c.b2;
    c.eta = s->eta_x;
    c.eps = s->eps_x;
    const IterPtrs p = select_ptrs(P, w.seg, s->cur);
    const double *X = p.x, *Y = p.y, *Z = p.z, *D = p.d0;

    __shared__ int32_t srp[kBlock + 1];
    __shared__ double G[6][kBlock];   // complete rows
    __shared__ double A[6][kBlock];   // leading piece of chunk t (row began earlier)
    __shared__ double B[6][kBlock];   // trailing piece of chunk t (row goes on)
    const int t = threadIdx.x;
    const int64_t r0 = w.begin;
    const int nrow = (int)(w.end - w.begin);
    // phase-2 operands first: their latency hides behind phase 1
    const int64_t io = r0 + t;
    const bool own = t < nrow;
    double oxi = 0, oyi = 0, ozi = 0;
    Pre pre = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (own) {
        oxi = X[io];
        oyi = Y[io];
        ozi = Z[io];
        pre = preload(p, io);
        srp[t] = p.rp[io];
    }
    if (t == 0) srp[nrow] = p.rp[r0 + nrow];
    __syncthreads();

    const int32_t e0 = srp[0], e1 = srp[nrow];
    const int32_t chunk = max(1, (e1 - e0 + kBlock - 1) / kBlock);
    const int32_t cs = e0 + t * chunk, ce = min(cs + chunk, e1);
    if (cs < ce) {
        int lo = 0, hi = nrow - 1;   // the row holding entry cs
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (srp[mid] <= cs) lo = mid;
            else hi = mid - 1;
        }
        int r = lo;
        int32_t q = cs;
        for (;;) {
            const int64_t i = r0 + r;
            const double xi = X[i], yi = Y[i], zi = Z[i], di = D[i];
            const int32_t rend = srp[r + 1], qe = min(rend, ce);
            Acc a = {0, 0, 0, 0, 0, 0, 0};
            segment_terms(a, p.col, X, Y, Z, D, q, qe, xi, yi, zi, di, c);
            const bool began_before = srp[r] < cs, goes_on = rend > ce;
            if (began_before) store6(A, t, a);
            else if (goes_on) store6(B, t, a);
            else store6(G, r, a);
            q = qe;
            if (q >= ce) break;
            do {
                ++r;
            } while (srp[r + 1] <= q);   // skip rows without partners
        }
    }
    __syncthreads();

    double be = 0, bs = 0, bm = 0, bd = 0;
    if (own) {
        const int32_t qb = srp[t], qe = srp[t + 1];
        double g[6] = {0, 0, 0, 0, 0, 0};
        if (qb < qe) {
            const int tf = (qb - e0) / chunk, tl = (qe - 1 - e0) / chunk;
            if (tf == tl) {
#pragma unroll
                for (int k = 0; k < 6; ++k) g[k] = G[k][t];
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) g[k] = B[k][tf];
                for (int u = tf + 1; u <= tl; ++u) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) g[k] += A[k][u];
                    g[5] = fmax(g[5], A[5][u]);
                }
            }
        }
        be = g[3];
        bs = g[4];
        bm = g[5];
        bd = update_particle(p, c, io, oxi, oyi, ozi, pre, g[0], g[1], g[2]);
    }
    // block reduction of the four partials
    const int lane = t & (kWave - 1);
    be = wave_sum(be);
    bs = wave_sum(bs);
    bm = wave_max(bm);
    bd = wave_max(bd);
    __shared__ double red[kWavesPerBlock][4];
    const int wv = t / kWave;
    if (lane == 0) {
        red[wv][0] = be;
        red[wv][1] = bs;
        red[wv][2] = bm;
        red[wv][3] = bd;
    }
    __syncthreads();
    if (t == 0) {
        double e = 0, sd = 0, m = 0, d = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            e += red[k][0];
            sd += red[k][1];
            m = fmax(m, red[k][2]);
            d = fmax(d, red[k][3]);
        }
        double *o = partials + 4 * (int64_t)b;
        o[0] = e;
        o[1] = sd;
        o[2] = m;
        o[3] = d;
    }
    if (kFusedTail) {
        __shared__ int last;
        __threadfence();
        if (t == 0) {
            const uint32_t prev = atomicAdd(&s->ticket, 1u);
            last = (prev == (uint32_t)s->nblocks - 1u);
        }
        __syncthreads();
        if (last) {
            __threadfence();
            reduce_and_tail(s, partials);
            if (t == 0) s->ticket = 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_tail(SegState *__restrict__ S,
                                                const double *__restrict__ partials)
{
    SegState *s = S + blockIdx.x;
    if (s->flags & F_IDLE) return;
    reduce_and_tail(s, partials);
}

void launch_iterate(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                    int nitems, int flags, hipStream_t st)
{
    // bit 0: XCD-aware order; bit 1: fused tail; bit 2: last rows first
    const int f = flags & 5;
    if (flags & 2) {
        hipLaunchKernelGGL(k_iterate<true>, dim3(nitems), dim3(kBlock), 0, st, P, S, W,
                           partials, f);
    } else {
        hipLaunchKernelGGL(k_iterate<false>, dim3(nitems), dim3(kBlock), 0, st, P, S, W,
                           partials, f);
    }
}

void launch_tail(SegState *S, const double *partials, int nseg, hipStream_t st)
{
    hipLaunchKernelGGL(k_tail, dim3(nseg), dim3(kBlock), 0, st, S, partials);
}

// ------------------------------------------------------- small updates
__global__ void k_after_build(SegState *S, int seg, double kb, double disp_lim2,
                              double kappa_lim, int cur, const uint32_t *maxdeg)
{
    SegState *s = S + seg;
    s->kb = kb;
    s->disp_lim2 = disp_lim2;
    s->kappa_lim = kappa_lim;
    s->cur = cur;
    s->maxdeg = (int32_t)*maxdeg;
    s->flags &= ~(F_REBUILD | F_STALE);
}

void launch_after_build(SegState *S, int seg, double kb, double disp_lim2, double kappa_lim,
                        int cur, const uint32_t *maxdeg_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_after_build, dim3(1), dim3(1), 0, st, S, seg, kb, disp_lim2, kappa_lim,
                       cur, maxdeg_dev);
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
        s->mk = 0.0;
        s->vk = 0.0;
    }
    s->flags &= ~(F_STOP | F_CAP | F_HOLD | F_NONFINITE);
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
// buffer.  Partials per block: E_ov, S, max delta, overlapping pairs.
__global__ __launch_bounds__(kBlock) void k_eval(const SegPtrs *__restrict__ P,
                                                const SegState *__restrict__ S, int seg,
                                                int64_t n, const double *__restrict__ xu,
                                                double kappa, double *__restrict__ part,
                                                double *__restrict__ gu)
{
    const SegState *s = S + seg;
    const IterPtrs p = select_ptrs(P, seg, s->cur);
    const int32_t *orig = P[seg].orig;
    const double L = s->L, hL = s->hL;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double be = 0, bs = 0, bm = 0, bn = 0;
    if (i < n) {
        auto pos = [&](int64_t k, int a) -> double {
            return xu ? xu[3 * (int64_t)orig[k] + a] : (a == 0 ? p.x[k] : (a == 1 ? p.y[k] : p.z[k]));
        };
        const double xi = pos(i, 0), yi = pos(i, 1), zi = pos(i, 2), di = p.d0[i];
        Acc a = {0, 0, 0, 0, 0, 0, 0};
        for (int32_t q = p.rp[i]; q < p.rp[i + 1]; ++q) {
            const int32_t j = p.col[q];
            pair_term(a, xi, yi, zi, di, pos(j, 0), pos(j, 1), pos(j, 2), p.d0[j], kappa, L, hL);
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
            const double dd = min_image(xu[3 * u + a] - p.xref[a][i], L, hL);
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

__global__ __launch_bounds__(kBlock) void k_set_positions(const SegPtrs *__restrict__ P,
                                                         int seg, int64_t n,
                                                         const double *__restrict__ xu, int cur)
{
    const IterPtrs p = select_ptrs(P, seg, cur);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t u = P[seg].orig[i];
    double *X = (double *)p.x, *Y = (double *)p.y, *Z = (double *)p.z;
    X[i] = xu[3 * u];
    Y[i] = xu[3 * u + 1];
    Z[i] = xu[3 * u + 2];
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
