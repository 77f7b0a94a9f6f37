// Stable LSD radix sort of (u64 key, u32 value) pairs and of u64 keys, for
// the neighbour-list build (Morton ordering, entry sort), of several arrays
// at once.
//
// Sort: 8-bit digits, tiles of 2048 keys (256 threads x 8 rounds).  Per pass:
// per-tile digit histogram -> per digit, an exclusive scan over the tiles
// and the digit's total (one block per digit) -> stable scatter, which adds
// the totals of the smaller digits and ranks each key among equal digits of
// its tile with wave ballots (a 9-bit match over the digit) and per-wave
// counts in LDS.
#include "rcp_kernels.hpp"

namespace rcp {

constexpr int kTile = kBlock * 8;   // 2048 items per tile

// ---------------------------------------------------------------- scan
// Inclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t ws[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t u = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += u;
    }
    if (lane == kWave - 1) ws[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < kWavesPerBlock; ++k) {
        if (k < w) off += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---------------------------------------------------------------- sort
// Several independent arrays (segments) are sorted by one sequence of
// launches: every launch covers the tiles of all segments, a block finding
// its segment by binary search over the segments' first tiles.  Histograms
// are laid out per segment, digit-major: hist[256 t0 + d nt + t].

// Segment of tile b: the last segment whose first tile is <= b.
__device__ __forceinline__ int seg_of_tile(const SortSeg *__restrict__ sg, int nseg, int64_t b)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sg[mid].t0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const SortSeg *__restrict__ sg, int nseg,
                                                      int par, int shift,
                                                      uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    const int j = seg_of_tile(sg, nseg, blockIdx.x);
    const int64_t n = sg[j].n, t0 = sg[j].t0, nt = sg[j].nt;
    const int64_t t = (int64_t)blockIdx.x - t0;
    // pointers read from memory: global-address-space views keep the loads
    // off the flat path (which would also wait on the LDS atomics)
    const gptr<const uint64_t> keys = (gptr<const uint64_t>)(par ? sg[j].k[1] : sg[j].k[0]);
    // all eight loads in flight together (clamped indices: a tile holds at
    // least one key)
    const int64_t base = t * kTile;
    uint64_t kk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t i = base + k * kBlock + threadIdx.x;
        kk[k] = keys[i < n ? i : n - 1];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(kk[k] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[256 * t0 + (int64_t)threadIdx.x * nt + t] = cnt[threadIdx.x];
}

// Block (j, d): exclusive scan, in place, of digit d's tile counts in
// segment j (tile order), and the digit's total to totals[256 j + d].
__global__ __launch_bounds__(kBlock) void k_radix_rowscan(const SortSeg *__restrict__ sg,
                                                         uint32_t *__restrict__ hist,
                                                         uint32_t *__restrict__ totals)
{
    const int j = (int)(blockIdx.x >> 8), d = (int)(blockIdx.x & 255u);
    const int64_t nt = sg[j].nt;
    uint32_t *row = hist + 256 * sg[j].t0 + (int64_t)d * nt;
    uint32_t carry = 0;
    for (int64_t base = 0; base < nt; base += 4 * kBlock) {
        const int64_t i0 = base + (int64_t)threadIdx.x * 4;
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < nt ? row[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = carry + block_exclusive(sum, &tot);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < nt) row[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <bool kVals>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const SortSeg *__restrict__ sg, int nseg,
                                                         int par, int shift,
                                                         const uint32_t *__restrict__ off,
                                                         const uint32_t *__restrict__ totals)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kWavesPerBlock][257];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int j = seg_of_tile(sg, nseg, blockIdx.x);
    const int64_t n = sg[j].n, t0 = sg[j].t0, nt = sg[j].nt;
    const int64_t t = (int64_t)blockIdx.x - t0;
    const gptr<const uint64_t> kin = (gptr<const uint64_t>)(par ? sg[j].k[1] : sg[j].k[0]);
    const gptr<uint64_t> kout = (gptr<uint64_t>)(par ? sg[j].k[0] : sg[j].k[1]);
    const gptr<const uint32_t> vin = (gptr<const uint32_t>)(par ? sg[j].v[1] : sg[j].v[0]);
    const gptr<uint32_t> vout = (gptr<uint32_t>)(par ? sg[j].v[0] : sg[j].v[1]);
    // the tile's keys (and values) are loaded up front, all in flight
    // together (clamped indices: a tile holds at least one key)
    const int64_t tile = t * kTile;
    uint64_t kk[8];
    uint32_t vv[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int64_t i = tile + r * kBlock + threadIdx.x;
        const int64_t ic = i < n ? i : n - 1;
        kk[r] = kin[ic];
        vv[r] = kVals ? vin[ic] : 0u;
    }
    // first position of digit threadIdx.x: the segment's totals of smaller
    // digits plus this digit's count in its earlier tiles
    uint32_t all;
    const uint32_t dbase = block_exclusive(totals[256 * j + threadIdx.x], &all);
    base[threadIdx.x] = dbase + off[256 * t0 + (int64_t)threadIdx.x * nt + t];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        for (int k = threadIdx.x; k < kWavesPerBlock * 257; k += kBlock)
            (&wcnt[0][0])[k] = 0;
        __syncthreads();
        const int64_t i = tile + r * kBlock + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = kk[r];
        uint32_t val = vv[r];
        uint32_t d = valid ? (uint32_t)((key >> shift) & 255u) : 256u;
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            uint32_t bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int k = 0; k < w; ++k) pos += wcnt[k][d];
            kout[pos] = key;
            if (kVals) vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) add += wcnt[k][threadIdx.x];
        base[threadIdx.x] += add;
        __syncthreads();
    }
}

// Segment descriptors travel as kernel arguments (no copy engine, no host
// staging that must outlive the call), kSegChunk per launch.
constexpr int kSegChunk = 32;
struct SegChunk {
    SortSeg s[kSegChunk];
};

__global__ void k_put_segs(SortSeg *__restrict__ dst, SegChunk c, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.s[threadIdx.x];
}

void launch_put_segs(SortSeg *dst, const SortSeg *src, int nseg, hipStream_t s)
{
    for (int b = 0; b < nseg; b += kSegChunk) {
        SegChunk c;
        const int n = nseg - b < kSegChunk ? nseg - b : kSegChunk;
        for (int q = 0; q < n; ++q) c.s[q] = src[b + q];
        hipLaunchKernelGGL(k_put_segs, dim3(1), dim3(kSegChunk), 0, s, dst + b, c, n);
    }
}

int radix_sort_segs(const SortSeg *sg, int nseg, int64_t ntiles, int nbits, bool vals,
                    uint32_t *hist, uint32_t *totals, hipStream_t s)
{
    if (nseg <= 0 || ntiles <= 0) return 0;
    int par = 0;
    for (int shift = 0; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kBlock), 0, s, sg, nseg,
                           par, shift, hist);
        hipLaunchKernelGGL(k_radix_rowscan, dim3((unsigned)(256 * nseg)), dim3(kBlock), 0, s, sg,
                           hist, totals);
        if (vals)
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)ntiles), dim3(kBlock), 0, s,
                               sg, nseg, par, shift, hist, totals);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)ntiles), dim3(kBlock), 0, s,
                               sg, nseg, par, shift, hist, totals);
        par ^= 1;
    }
    return par;
}

// ------------------------------------------------ positions out of list order
// Positions of packing seg from list order back into user order (xu:
// n x 3 row-major), the reverse of k_set_positions; orig is a permutation
// of [0, n).
__global__ __launch_bounds__(kBlock) void k_get_positions(const SegPtrs *__restrict__ P,
                                                         int seg, int64_t n,
                                                         double *__restrict__ xu, int cur)
{
    const P4 *Q = cur ? P[seg].p[1] : P[seg].p[0];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t u = P[seg].orig[i];
    const P4 q = Q[i];
    xu[3 * u] = q.x;
    xu[3 * u + 1] = q.y;
    xu[3 * u + 2] = q.z;
}

void launch_get_positions(const SegPtrs *P, int seg, int64_t n, double *xu, int cur,
                          hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_get_positions, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, st, P, seg, n, xu, cur);
}

}  // namespace rcp
