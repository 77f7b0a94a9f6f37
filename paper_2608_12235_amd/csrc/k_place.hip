// Initial placement on the device: random sequential addition in rounds
// (App. A starts from a dilute, non-overlapping configuration placed with a
// cell list; the algorithm is our reading, stated in include/rcp.h).
//
// Spheres are ranked largest first and placed class by class (size class
// floor(log2(D0 / D0_min)), largest class first).  A round takes a window of
// consecutive ranks of one class; every unplaced sphere of the window
// proposes the position of its next attempt, from the SplitMix64 counter
// stream of the host placement; a proposal is valid when it overlaps no
// placed sphere, and a valid proposal is accepted unless a valid proposal of
// a lower rank in the same round overlaps it.  Accepted spheres are placed,
// the others move on to their next attempt.  The result depends on the
// window but not on timing: every decision is a function of the proposals
// and of the spheres placed before the round.
//
// Placed spheres are binned per class on a grid of cells at least as wide
// as kappa0 times the class's largest diameter (a sphere meets only spheres
// of its own class or larger ones, so the 27 cells around it in each
// larger-or-equal class's grid hold every sphere it can overlap), kept as an
// open-addressing hash of occupied cells with a linked list per cell.  The
// proposals of a round are binned the same way in a table of their own.
//
// Compiled without floating-point contraction: the overlap test rounds
// exactly as the host placement's.
#include "rcp_kernels.hpp"

namespace rcp {

constexpr uint64_t kPlaceEmpty = ~0ull;

__device__ __forceinline__ uint64_t sm64(uint64_t seed, uint64_t k)
{
    // SplitMix64 output function (Steele, Lea and Flood 2014) at counter k
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double place_u01(uint64_t seed, uint64_t i, uint64_t attempt, int axis)
{
    const uint64_t k = ((i << 24) | attempt) * 4u + (uint64_t)axis;
    return (double)(sm64(seed, k) >> 11) * 0x1p-53;
}

__device__ __forceinline__ double place_mi(double d, double L, double hL)
{
    return d > hL ? d - L : (d < -hL ? d + L : d);
}

__device__ __forceinline__ int64_t place_cell(double v, double inv_w, int64_t nc)
{
    int64_t c = (int64_t)(v * inv_w);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ uint64_t place_mix(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    return k;
}

// Head of the list of cell `key` (or -1).
__device__ __forceinline__ int32_t place_find(const PlaceSlot *tab, uint64_t mask, uint64_t key)
{
    for (uint64_t s = place_mix(key) & mask;; s = (s + 1) & mask) {
        const uint64_t k = tab[s].key;
        if (k == key) return tab[s].head;
        if (k == kPlaceEmpty) return -1;
    }
}

// Push item v on the list of cell `key`; returns the previous head.
__device__ __forceinline__ int32_t place_push(PlaceSlot *tab, uint64_t mask, uint64_t key, int32_t v)
{
    for (uint64_t s = place_mix(key) & mask;; s = (s + 1) & mask) {
        const unsigned long long prev =
            atomicCAS((unsigned long long *)&tab[s].key, (unsigned long long)kPlaceEmpty,
                      (unsigned long long)key);
        if (prev == kPlaceEmpty || prev == key) return atomicExch(&tab[s].head, v);
    }
}

// hLa[ax] = L / 2, or +inf on an axis bounded by walls (no image).
__device__ __forceinline__ bool place_overlap(double xj, double yj, double zj, const double *p,
                                              double dj, double di, double kappa0, double L,
                                              const double *hLa)
{
#pragma clang fp contract(off)
    const double dx = place_mi(xj - p[0], L, hLa[0]);
    const double dy = place_mi(yj - p[1], L, hLa[1]);
    const double dz = place_mi(zj - p[2], L, hLa[2]);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    const double dd = kappa0 * (0.5 * (di + dj));
    return r2 < dd * dd;
}

// Clear the proposal table (keys) before a round.
__global__ __launch_bounds__(kBlock) void k_place_clear(PlaceSlot *tab, int64_t cap)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s < cap) {
        tab[s].key = kPlaceEmpty;
        tab[s].head = -1;
    }
}

// Proposals of ranks [lo, hi) of class c: position of the next attempt,
// validity (clear of the walls, if any, and of the placed spheres of
// classes c and larger), and the valid ones binned in the proposal table.
__global__ __launch_bounds__(kBlock) void k_place_propose(PlaceArgs a, int c, int64_t lo,
                                                         int64_t hi)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t k = lo + s;
    if (k >= hi) return;
    a.valid[s] = 0;
    if (a.placed[k]) return;
    const int32_t i = a.ord[k];
    const double di = a.d0[i];
    double p[3];
    for (int ax = 0; ax < 3; ++ax) {
        // in two dimensions z = 0 (axis 2 of the stream is not drawn)
        double v = ax < a.dim ? place_u01(a.seed, (uint64_t)i, (uint64_t)a.att[k], ax) * a.L : 0.0;
        if (v >= a.L) v -= a.L;
        p[ax] = v;
        a.prop[3 * s + ax] = v;
    }
    const int32_t bounded = a.walls | a.round;
    const double hLa[3] = {(bounded & 1) ? INFINITY : a.hL, (bounded & 2) ? INFINITY : a.hL,
                           (bounded & 4) ? INFINITY : a.hL};
    bool ok = !bounded || inside_walls(p, a.kappa0 * di, a.L, a.walls, a.round);
    for (int cc = c; cc < a.ncls && ok; ++cc) {
        const PlaceGrid &g = a.grid[cc];
        if (!g.any) continue;
        const int64_t nc = g.nc;
        const int64_t cx = place_cell(p[0], g.inv_w, nc), cy = place_cell(p[1], g.inv_w, nc),
                      cz = place_cell(p[2], g.inv_w, nc);
        const int64_t lo3 = nc >= 3 ? -1 : 0, hi3 = nc >= 3 ? 1 : nc - 1;
        for (int64_t ox = lo3; ox <= hi3 && ok; ++ox)
            for (int64_t oy = lo3; oy <= hi3 && ok; ++oy)
                for (int64_t oz = lo3; oz <= hi3 && ok; ++oz) {
                    int64_t ax = cx + ox, ay = cy + oy, az = cz + oz;
                    if (nc >= 3) {
                        ax = ax < 0 ? ax + nc : (ax >= nc ? ax - nc : ax);
                        ay = ay < 0 ? ay + nc : (ay >= nc ? ay - nc : ay);
                        az = az < 0 ? az + nc : (az >= nc ? az - nc : az);
                    }
                    const uint64_t key = ((uint64_t)ax * (uint64_t)nc + (uint64_t)ay) *
                                             (uint64_t)nc + (uint64_t)az;
                    for (int32_t j = place_find(a.tab + g.off, g.mask, key); j >= 0;
                         j = a.next[j])
                        if (place_overlap(a.x[3 * j], a.x[3 * j + 1], a.x[3 * j + 2], p, a.d0[j],
                                          di, a.kappa0, a.L, hLa)) {
                            ok = false;
                            break;
                        }
                }
    }
    if (!ok) return;
    a.valid[s] = 1;
    const PlaceGrid &g = a.grid[c];
    const uint64_t key = ((uint64_t)place_cell(p[0], g.inv_w, g.nc) * (uint64_t)g.nc +
                          (uint64_t)place_cell(p[1], g.inv_w, g.nc)) * (uint64_t)g.nc +
                         (uint64_t)place_cell(p[2], g.inv_w, g.nc);
    a.pnext[s] = place_push(a.ptab, a.pmask, key, (int32_t)s);
}

// Conflicts among the round's valid proposals (the lower rank wins), then
// the accepted spheres are placed and the others move on to their next
// attempt; *first receives the lowest rank of the window still unplaced.
__global__ __launch_bounds__(kBlock) void k_place_commit(PlaceArgs a, int c, int64_t lo,
                                                        int64_t hi)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t k = lo + s;
    if (k >= hi || a.placed[k]) return;
    const int32_t i = a.ord[k];
    const double di = a.d0[i];
    const double p[3] = {a.prop[3 * s], a.prop[3 * s + 1], a.prop[3 * s + 2]};
    const int32_t bounded = a.walls | a.round;
    const double hLa[3] = {(bounded & 1) ? INFINITY : a.hL, (bounded & 2) ? INFINITY : a.hL,
                           (bounded & 4) ? INFINITY : a.hL};
    bool acc = a.valid[s] != 0;
    if (acc) {
        const PlaceGrid &g = a.grid[c];
        const int64_t nc = g.nc;
        const int64_t cx = place_cell(p[0], g.inv_w, nc), cy = place_cell(p[1], g.inv_w, nc),
                      cz = place_cell(p[2], g.inv_w, nc);
        const int64_t lo3 = nc >= 3 ? -1 : 0, hi3 = nc >= 3 ? 1 : nc - 1;
        for (int64_t ox = lo3; ox <= hi3 && acc; ++ox)
            for (int64_t oy = lo3; oy <= hi3 && acc; ++oy)
                for (int64_t oz = lo3; oz <= hi3 && acc; ++oz) {
                    int64_t ax = cx + ox, ay = cy + oy, az = cz + oz;
                    if (nc >= 3) {
                        ax = ax < 0 ? ax + nc : (ax >= nc ? ax - nc : ax);
                        ay = ay < 0 ? ay + nc : (ay >= nc ? ay - nc : ay);
                        az = az < 0 ? az + nc : (az >= nc ? az - nc : az);
                    }
                    const uint64_t key = ((uint64_t)ax * (uint64_t)nc + (uint64_t)ay) *
                                             (uint64_t)nc + (uint64_t)az;
                    for (int32_t s2 = place_find(a.ptab, a.pmask, key); s2 >= 0; s2 = a.pnext[s2]) {
                        if (s2 >= s) continue;
                        const int32_t j = a.ord[lo + s2];
                        if (place_overlap(a.prop[3 * s2], a.prop[3 * s2 + 1], a.prop[3 * s2 + 2],
                                          p, a.d0[j], di, a.kappa0, a.L, hLa)) {
                            acc = false;
                            break;
                        }
                    }
                }
    }
    if (acc) {
        a.x[3 * i] = p[0];
        a.x[3 * i + 1] = p[1];
        a.x[3 * i + 2] = p[2];
        a.placed[k] = 1;
        const PlaceGrid &g = a.grid[c];
        const uint64_t key = ((uint64_t)place_cell(p[0], g.inv_w, g.nc) * (uint64_t)g.nc +
                              (uint64_t)place_cell(p[1], g.inv_w, g.nc)) * (uint64_t)g.nc +
                             (uint64_t)place_cell(p[2], g.inv_w, g.nc);
        a.next[i] = place_push(a.tab + g.off, g.mask, key, i);
    } else {
        if (++a.att[k] >= a.max_attempts) atomicOr(a.fail, 1);
        atomicMin(a.first, (unsigned long long)k);
    }
}

// Seating (a cascade stage, Sec. 4: the finer class is seated in the voids
// of the coarser ones): each sphere on its own, its first proposal of the
// placement counter stream that overlaps no frozen sphere, r^2 < dd^2 with
// dd = (D_j + kappa0 D0_i) / 2 and the separation x_j - p (minimum image).
__global__ __launch_bounds__(kBlock) void k_seat(SeatArgs a, int64_t ng)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= ng) return;
    const int32_t i = a.gidx[t];
    const double di = a.gd[t];
    const int64_t nc = a.nc;
    const int64_t lo3 = nc >= 3 ? -1 : 0, hi3 = nc >= 3 ? 1 : nc - 1;
    for (int64_t att = 0; att < a.max_attempts; ++att) {
        double p[3];
        for (int ax = 0; ax < 3; ++ax) {
            double v = ax < a.dim ? place_u01(a.seed, (uint64_t)i, (uint64_t)att, ax) * a.L : 0.0;
            if (v >= a.L) v -= a.L;
            p[ax] = v;
        }
        const int64_t cx = place_cell(p[0], a.inv_w, nc), cy = place_cell(p[1], a.inv_w, nc),
                      cz = place_cell(p[2], a.inv_w, nc);
        bool ok = true;
        for (int64_t ox = lo3; ox <= hi3 && ok; ++ox)
            for (int64_t oy = lo3; oy <= hi3 && ok; ++oy)
                for (int64_t oz = lo3; oz <= hi3 && ok; ++oz) {
                    int64_t ax = cx + ox, ay = cy + oy, az = cz + oz;
                    if (nc >= 3) {
                        ax = ax < 0 ? ax + nc : (ax >= nc ? ax - nc : ax);
                        ay = ay < 0 ? ay + nc : (ay >= nc ? ay - nc : ay);
                        az = az < 0 ? az + nc : (az >= nc ? az - nc : az);
                    }
                    const int64_t q = (ax * nc + ay) * nc + az;
                    for (int32_t o = a.start[q]; o < a.start[q + 1]; ++o) {
                        const double dx = place_mi(a.fxd[4 * o] - p[0], a.L, a.hL);
                        const double dy = place_mi(a.fxd[4 * o + 1] - p[1], a.L, a.hL);
                        const double dz = place_mi(a.fxd[4 * o + 2] - p[2], a.L, a.hL);
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        const double dd = 0.5 * (a.fxd[4 * o + 3] + a.kappa0 * di);
                        if (r2 < dd * dd) {
                            ok = false;
                            break;
                        }
                    }
                }
        if (ok) {
            a.x[3 * (int64_t)i] = p[0];
            a.x[3 * (int64_t)i + 1] = p[1];
            a.x[3 * (int64_t)i + 2] = p[2];
            return;
        }
    }
    atomicOr(a.fail, 1);
}

void launch_seat(const SeatArgs &a, int64_t ng, hipStream_t st)
{
    if (ng <= 0) return;
    hipLaunchKernelGGL(k_seat, dim3((unsigned)((ng + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       a, ng);
}

void launch_place_round(const PlaceArgs &a, int c, int64_t lo, int64_t hi, hipStream_t st)
{
    const int64_t w = hi - lo;
    if (w <= 0) return;
    const unsigned gc = (unsigned)((a.pcap + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_place_clear, dim3(gc), dim3(kBlock), 0, st, a.ptab, a.pcap);
    const unsigned g = (unsigned)((w + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_place_propose, dim3(g), dim3(kBlock), 0, st, a, c, lo, hi);
    hipLaunchKernelGGL(k_place_commit, dim3(g), dim3(kBlock), 0, st, a, c, lo, hi);
}

}  // namespace rcp
