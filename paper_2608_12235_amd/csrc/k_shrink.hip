// Shrink to contact (Sec. 2 and App. A: once the stop test holds, kappa is
// lowered uniformly, positions fixed, until the last overlap vanishes).
//
// For a listed pair with separation r^2 and relative mean diameter
// dd = 0.5 (D0_i + D0_j) the admissible scales are the doubles k with
// fl(fl(k dd) * fl(k dd)) <= r^2 (touching allowed).  That map is monotone
// in k, so the admissible set has a unique largest element; it is found
// from sqrt(r^2)/dd by stepping one ulp at a time, which makes the result
// independent of how sqrt and division round.  kappa' is the minimum over
// pairs, capped by the current kappa.  With hard walls (Sec. 2) every sphere
// must also clear them: a flat wall at gap = 2h admits the k with
// fl(k D0) <= gap, the round wall the k with t = fl(L - fl(k D0)) >= 0 and
// fl(t t) >= 4 rho^2 (both monotone in k; found the same way), and kappa'
// is also the minimum over the spheres of those scales.  No contraction:
// the tests must round exactly as written.
#pragma clang fp contract(off)
#include "rcp_kernels.hpp"

namespace rcp {

__device__ __forceinline__ double ulp_up(double k)
{
    return __longlong_as_double(__double_as_longlong(k) + 1);
}

__device__ __forceinline__ double ulp_down(double k)
{
    return __longlong_as_double(__double_as_longlong(k) - 1);
}

__device__ double contact_scale(double r2, double dd)
{
    if (!(r2 > 0.0)) return 0.0;
    double k = sqrt(r2) / dd;
    for (int it = 0; it < 64 && k > 0.0 && (k * dd) * (k * dd) > r2; ++it) k = ulp_down(k);
    for (int it = 0; it < 64; ++it) {
        const double up = ulp_up(k);
        if ((up * dd) * (up * dd) <= r2) k = up;
        else break;
    }
    return k;
}

// Largest k with fl(k d0) <= gap (0 if gap <= 0).
__device__ double flat_scale(double gap, double d0)
{
    if (!(gap > 0.0)) return 0.0;
    double k = gap / d0;
    for (int it = 0; it < 64 && k > 0.0 && k * d0 > gap; ++it) k = ulp_down(k);
    for (int it = 0; it < 64; ++it) {
        const double up = ulp_up(k);
        if (up * d0 <= gap) k = up;
        else break;
    }
    return k;
}

__device__ __forceinline__ bool round_clear(double k, double d0, double L, double q4)
{
    const double t = L - k * d0;
    return t >= 0.0 && t * t >= q4;
}

// Largest k with round_clear (0 if not even k = 0 clears).
__device__ double round_scale(double q4, double d0, double L)
{
    if (!round_clear(0.0, d0, L, q4)) return 0.0;
    double k = (L - sqrt(q4)) / d0;
    if (k < 0.0) k = 0.0;
    for (int it = 0; it < 64 && k > 0.0 && !round_clear(k, d0, L, q4); ++it) k = ulp_down(k);
    for (int it = 0; it < 64; ++it) {
        const double up = ulp_up(k);
        if (round_clear(up, d0, L, q4)) k = up;
        else break;
    }
    return k;
}

// Largest scale at which a sphere of relative diameter d0 at p clears every wall.
__device__ double wall_scale(const double p[3], double d0, double L, int32_t walls,
                             int32_t round)
{
    double k = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (!((walls >> a) & 1)) continue;
        k = fmin(k, flat_scale(2.0 * p[a], d0));
        k = fmin(k, flat_scale(2.0 * (L - p[a]), d0));
    }
    if (round) k = fmin(k, round_scale(4.0 * round_rho2(p[0], p[1], p[2], L, round), d0, L));
    return k;
}

__global__ __launch_bounds__(kBlock) void k_shrink(const SegPtrs *__restrict__ P,
                                                  const SegState *__restrict__ S, int seg,
                                                  int64_t n, double *__restrict__ part)
{
    const SegPtrs p = P[seg];
    const SegState *s = S + seg;
    const double L = s->L, hL = s->hL;
    const int32_t walls = s->walls, round = s->round, bounded = walls | round;
    // no image across an axis bounded by walls
    const double hx = (bounded & 1) ? INFINITY : hL, hy = (bounded & 2) ? INFINITY : hL,
                 hz = (bounded & 4) ? INFINITY : hL;
    const P4 *Q = s->cur ? p.p[1] : p.p[0];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double kmin = INFINITY;
    if (i < n) {
        const P4 qi = Q[i];
        for (int32_t q = p.rp[i]; q < p.rp[i + 1]; ++q) {
            const P4 qj = Q[p.col[q]];
            const double dx = min_image(qj.x - qi.x, L, hx);
            const double dy = min_image(qj.y - qi.y, L, hy);
            const double dz = min_image(qj.z - qi.z, L, hz);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            kmin = fmin(kmin, contact_scale(r2, 0.5 * (qi.d + qj.d)));
        }
        if (bounded) {
            const double px[3] = {qi.x, qi.y, qi.z};
            kmin = fmin(kmin, wall_scale(px, qi.d, L, walls, round));
        }
    }
    kmin = wave_min(kmin);
    __shared__ double red[kWavesPerBlock];
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = kmin;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = INFINITY;
        for (int k = 0; k < kWavesPerBlock; ++k) m = fmin(m, red[k]);
        part[blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(kWave) void k_min_finish(const double *__restrict__ part, int nb,
                                                     double *__restrict__ out)
{
    double m = INFINITY;
    for (int b = threadIdx.x; b < nb; b += kWave) m = fmin(m, part[b]);
    m = wave_min(m);
    if (threadIdx.x == 0) out[0] = m;
}

void launch_shrink(const SegPtrs *P, const SegState *S, int seg, int64_t n, double *part,
                   int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_shrink, dim3(nblocks), dim3(kBlock), 0, st, P, S, seg, n, part);
    hipLaunchKernelGGL(k_min_finish, dim3(1), dim3(kWave), 0, st, part, nblocks,
                       part + nblocks);
}

__global__ __launch_bounds__(kWave) void k_max_finish(const double *__restrict__ part, int nb,
                                                     double *__restrict__ out)
{
    double m = 0.0;
    for (int b = threadIdx.x; b < nb; b += kWave) m = fmax(m, part[b]);
    m = wave_max(m);
    if (threadIdx.x == 0) out[0] = m;
}

void launch_max_finish(const double *part, int nblocks, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(kWave), 0, st, part, nblocks, out);
}

}  // namespace rcp
