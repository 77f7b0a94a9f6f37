// Shrink to contact (Sec. 2 and App. A: once the stop test holds, kappa is
// lowered uniformly, positions fixed, until the last overlap vanishes).
//
// For a listed pair with separation r^2 and relative mean diameter
// dd = 0.5 (D0_i + D0_j) the admissible scales are the doubles k with
// fl(fl(k dd) * fl(k dd)) <= r^2 (touching allowed).  That map is monotone
// in k, so the admissible set has a unique largest element; it is found
// from sqrt(r^2)/dd by stepping one ulp at a time, which makes the result
// independent of how sqrt and division round.  kappa' is the minimum over
// pairs, capped by the current kappa.  No contraction: the test must round
// exactly as written.
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

__global__ __launch_bounds__(kBlock) void k_shrink(const SegPtrs *__restrict__ P,
                                                  const SegState *__restrict__ S, int seg,
                                                  int64_t n, double *__restrict__ part)
{
    const SegPtrs p = P[seg];
    const SegState *s = S + seg;
    const double L = s->L, hL = s->hL;
    const P4 *Q = s->cur ? p.p[1] : p.p[0];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double kmin = INFINITY;
    if (i < n) {
        const P4 qi = Q[i];
        for (int32_t q = p.rp[i]; q < p.rp[i + 1]; ++q) {
            const P4 qj = Q[p.col[q]];
            const double dx = min_image(qj.x - qi.x, L, hL);
            const double dy = min_image(qj.y - qi.y, L, hL);
            const double dz = min_image(qj.z - qi.z, L, hL);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            kmin = fmin(kmin, contact_scale(r2, 0.5 * (qi.d + qj.d)));
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
