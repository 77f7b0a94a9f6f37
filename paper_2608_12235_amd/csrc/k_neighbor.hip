// Neighbour-list build on multilevel (size-class) cell grids.
//
// Particles carry a size class l = floor(log2(D0/D0_min) / p).  Class l has
// its own cubic grid whose cells are at least as wide as the largest listing
// cutoff between a class-l particle and any particle of class <= l, so a
// particle finds every listed partner of class L >= its own in the 27 cells
// around it in grid L; pairs with a smaller partner are found from the
// smaller side.  This keeps a fine-class particle from scanning a cell sized
// for the largest sphere (the size ratio reaches 5e5 in the paper's
// lognormal study, Sec. 1).
//
// Keys are (class << mb) | Morton(cell) so one stable sort orders particles
// by class, then spatially; occupied cells are located through an
// open-addressing hash of their keys.  The listing predicate is evaluated
// with a fixed operation order and no contraction so that the pair set is
// reproducible bit for bit:
//   dx = mi(x_j - x_i) (same for y, z),  r2 = (dx dx + dy dy) + dz dz,
//   c = kb ((1 + g)(0.5 (D0_i + D0_j)) + 2 s D0_min),  listed iff r2 < c c.
#pragma clang fp contract(off)
#include "rcp_kernels.hpp"

namespace rcp {

__device__ __forceinline__ int64_t cell_coord(double v, double w, int32_t nc)
{
    int64_t c = (int64_t)(v / w);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

__global__ __launch_bounds__(kBlock) void k_keys(BuildArgs a, uint64_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const int l = a.lev[i];
    const LevelGrid g = a.lv[l];
    uint64_t cx = cell_coord(a.x[i], g.w, g.nc);
    uint64_t cy = cell_coord(a.y[i], g.w, g.nc);
    uint64_t cz = cell_coord(a.z[i], g.w, g.nc);
    keys[i] = ((uint64_t)l << a.mb) | morton3(cx, cy, cz);
    vals[i] = (uint32_t)i;
}

void launch_keys(const BuildArgs &a, uint64_t *keys, uint32_t *vals, hipStream_t s)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       a, keys, vals);
}

__global__ __launch_bounds__(kBlock) void k_permute(PermArgs p)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= p.n) return;
    const int64_t s = p.perm[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double xv = p.xs[a][s];
        p.xd[a][k] = xv;
        p.xref[a][k] = xv;
        p.md[a][k] = p.ms[a][s];
        p.vd[a][k] = p.vs[a][s];
    }
    p.d0d[k] = p.d0s[s];
    p.od[k] = p.os[s];
    p.ld[k] = p.ls[s];
}

void launch_permute(const PermArgs &p, hipStream_t s)
{
    if (p.n <= 0) return;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((p.n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, p);
}

// ------------------------------------------------------------- hashing
__global__ void k_fill_u64(uint64_t *__restrict__ p, int64_t n, uint64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *__restrict__ p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       p, n, v);
}

void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       p, n, v);
}

__global__ __launch_bounds__(kBlock) void k_hash_starts(BuildArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const uint64_t key = a.skey[i];
    if (i > 0 && a.skey[i - 1] == key) return;
    uint64_t slot = hash64(key) & a.hmask;
    for (;;) {
        unsigned long long prev = atomicCAS((unsigned long long *)&a.hkey[slot],
                                            (unsigned long long)kEmptyKey,
                                            (unsigned long long)key);
        if (prev == kEmptyKey || prev == key) {
            a.hval[slot].x = (int)i;
            return;
        }
        slot = (slot + 1) & a.hmask;
    }
}

__device__ __forceinline__ int2 hash_find(const BuildArgs &a, uint64_t key)
{
    uint64_t slot = hash64(key) & a.hmask;
    for (;;) {
        const uint64_t k = a.hkey[slot];
        if (k == key) return a.hval[slot];
        if (k == kEmptyKey) return make_int2(0, 0);
        slot = (slot + 1) & a.hmask;
    }
}

__global__ __launch_bounds__(kBlock) void k_hash_counts(BuildArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const uint64_t key = a.skey[i];
    if (i + 1 < a.n && a.skey[i + 1] == key) return;
    uint64_t slot = hash64(key) & a.hmask;
    while (a.hkey[slot] != key) slot = (slot + 1) & a.hmask;
    a.hval[slot].y = (int)(i - a.hval[slot].x + 1);
}

void launch_hash_build(const BuildArgs &a, int64_t cap, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cap + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, a.hkey, cap, kEmptyKey);
    if (a.n <= 0) return;
    const dim3 g((unsigned)((a.n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_hash_starts, g, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_hash_counts, g, dim3(kBlock), 0, s, a);
}

// ------------------------------------------------------- pair search
// Half partners of particle i: same class with a larger sorted index, and
// every larger class.  fill == 0 counts, fill == 1 writes.
__global__ __launch_bounds__(kBlock) void k_half(BuildArgs a, uint32_t *__restrict__ cnt,
                                                const uint32_t *__restrict__ ptr,
                                                int32_t *__restrict__ col, int fill)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i], di = a.d0[i];
    const int li = a.lev[i];
    uint32_t c = 0;
    int32_t *out = fill ? col + ptr[i] : nullptr;
    for (int L = li; L < a.nlev; ++L) {
        const LevelGrid g = a.lv[L];
        if (g.count == 0) continue;
        const int64_t nc = g.nc;
        const int64_t cx = cell_coord(xi, g.w, g.nc), cy = cell_coord(yi, g.w, g.nc),
                      cz = cell_coord(zi, g.w, g.nc);
        const int64_t lo = nc >= 3 ? -1 : 0, hi = nc >= 3 ? 1 : nc - 1;
        for (int64_t ox = lo; ox <= hi; ++ox) {
            const int64_t ax = nc >= 3 ? (cx + ox + nc) % nc : ox;
            for (int64_t oy = lo; oy <= hi; ++oy) {
                const int64_t ay = nc >= 3 ? (cy + oy + nc) % nc : oy;
                for (int64_t oz = lo; oz <= hi; ++oz) {
                    const int64_t az = nc >= 3 ? (cz + oz + nc) % nc : oz;
                    const uint64_t key = ((uint64_t)L << a.mb) |
                                         morton3((uint64_t)ax, (uint64_t)ay, (uint64_t)az);
                    const int2 r = hash_find(a, key);
                    for (int64_t j = r.x; j < (int64_t)r.x + r.y; ++j) {
                        if (L == li && j <= i) continue;
                        const double dx = min_image(a.x[j] - xi, a.L, a.hL);
                        const double dy = min_image(a.y[j] - yi, a.L, a.hL);
                        const double dz = min_image(a.z[j] - zi, a.L, a.hL);
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        const double cc = a.kb * (a.opg * (0.5 * (di + a.d0[j])) + a.sk2);
                        if (r2 < cc * cc) {
                            if (fill) out[c] = (int32_t)j;
                            ++c;
                        }
                    }
                }
            }
        }
    }
    if (!fill) cnt[i] = c;
}

void launch_half(const BuildArgs &a, uint32_t *cnt, const uint32_t *ptr, int32_t *col, int fill,
                 hipStream_t s)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_half, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       a, cnt, ptr, col, fill);
}

// ------------------------------------------------------- full rows
__global__ __launch_bounds__(kBlock) void k_in_count(int64_t n, const uint32_t *__restrict__ hp,
                                                    const int32_t *__restrict__ hcol,
                                                    uint32_t *__restrict__ in_cnt)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (uint32_t q = hp[i]; q < hp[i + 1]; ++q) atomicAdd(&in_cnt[hcol[q]], 1u);
}

void launch_in_count(int64_t n, const uint32_t *hp, const int32_t *hcol, uint32_t *in_cnt,
                     hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_in_count, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, hp, hcol, in_cnt);
}

__global__ __launch_bounds__(kBlock) void k_pair_keys(int64_t n, const uint32_t *__restrict__ hp,
                                                     const int32_t *__restrict__ hcol,
                                                     uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (uint32_t q = hp[i]; q < hp[i + 1]; ++q) {
        keys[q] = (uint64_t)(uint32_t)hcol[q];
        vals[q] = (uint32_t)i;
    }
}

void launch_pair_keys(int64_t n, const uint32_t *hp, const int32_t *hcol, uint64_t *keys,
                      uint32_t *vals, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pair_keys, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, hp, hcol, keys, vals);
}

__global__ __launch_bounds__(kBlock) void k_add_counts(int64_t n, const uint32_t *__restrict__ hp,
                                                      const uint32_t *__restrict__ in_cnt,
                                                      uint32_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    out[i] = (hp[i + 1] - hp[i]) + in_cnt[i];
}

void launch_add_counts(int64_t n, const uint32_t *hp, const uint32_t *in_cnt, uint32_t *out,
                       hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_counts, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, hp, in_cnt, out);
}

// Row i = its half partners (search order) followed by the particles that
// listed i (ascending index, from the stable sort by partner).
__global__ __launch_bounds__(kBlock) void k_full_fill(int64_t n, const uint32_t *__restrict__ hp,
                                                     const int32_t *__restrict__ hcol,
                                                     const uint32_t *__restrict__ ip,
                                                     const uint32_t *__restrict__ src,
                                                     const uint32_t *__restrict__ rp,
                                                     int32_t *__restrict__ col)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t o = rp[i];
    for (uint32_t q = hp[i]; q < hp[i + 1]; ++q) col[o++] = hcol[q];
    for (uint32_t q = ip[i]; q < ip[i + 1]; ++q) col[o++] = (int32_t)src[q];
}

void launch_full_fill(int64_t n, const uint32_t *hp, const int32_t *hcol, const uint32_t *ip,
                      const uint32_t *src, const uint32_t *rp, int32_t *col, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_full_fill, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, hp, hcol, ip, src, rp, col);
}

__global__ __launch_bounds__(kBlock) void k_heavy_mark(int64_t n, const uint32_t *__restrict__ rp,
                                                      int32_t T, uint32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    flag[i] = (rp[i + 1] - rp[i]) > (uint32_t)T ? 1u : 0u;
}

void launch_heavy_mark(int64_t n, const uint32_t *rp, int32_t T, uint32_t *flag, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_heavy_mark, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, rp, T, flag);
}

__global__ __launch_bounds__(kBlock) void k_heavy_compact(int64_t n,
                                                         const uint32_t *__restrict__ flag,
                                                         const uint32_t *__restrict__ pos,
                                                         int32_t *__restrict__ heavy)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) heavy[pos[i]] = (int32_t)i;
}

void launch_heavy_compact(int64_t n, const uint32_t *flag, const uint32_t *pos, int32_t *heavy,
                          hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_heavy_compact, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, n, flag, pos, heavy);
}

}  // namespace rcp
