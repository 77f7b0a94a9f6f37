// Stable LSD radix sort of (u64 key, u32 value) pairs and of u64 keys, for
// the neighbour-list build (Morton ordering, entry sort).
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
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                      int64_t n, int shift, int64_t nt,
                                                      uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nt + blockIdx.x] = cnt[threadIdx.x];
}

// Block d: exclusive scan, in place, of digit d's tile counts hist[d * nt
// .. d * nt + nt) (tile order), and the digit's total to totals[d].
__global__ __launch_bounds__(kBlock) void k_radix_rowscan(uint32_t *__restrict__ hist, int64_t nt,
                                                         uint32_t *__restrict__ totals)
{
    uint32_t *row = hist + (int64_t)blockIdx.x * nt;
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
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         uint64_t *__restrict__ kout,
                                                         uint32_t *__restrict__ vout,
                                                         int64_t n, int shift, int64_t nt,
                                                         const uint32_t *__restrict__ off,
                                                         const uint32_t *__restrict__ totals)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kWavesPerBlock][257];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    // first position of digit threadIdx.x: the totals of smaller digits plus
    // this digit's count in earlier tiles
    uint32_t all;
    const uint32_t dbase = block_exclusive(totals[threadIdx.x], &all);
    base[threadIdx.x] = dbase + off[(int64_t)threadIdx.x * nt + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t tile = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < 8; ++r) {
        for (int k = threadIdx.x; k < kWavesPerBlock * 257; k += kBlock)
            (&wcnt[0][0])[k] = 0;
        __syncthreads();
        const int64_t i = tile + r * kBlock + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        uint32_t val = (kVals && valid) ? vin[i] : 0u;
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

int radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int nbits,
               uint32_t *hist, uint32_t *totals, hipStream_t s)
{
    if (n <= 1) return 0;
    const int64_t nt = (n + kTile - 1) / kTile;
    int parity = 0;
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint64_t *ki = parity ? k1 : k0;
        const uint32_t *vi = parity ? v1 : v0;
        uint64_t *ko = parity ? k0 : k1;
        uint32_t *vo = parity ? v0 : v1;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kBlock), 0, s, ki, n, shift,
                           nt, hist);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kBlock), 0, s, hist, nt, totals);
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nt), dim3(kBlock), 0, s, ki, vi,
                           ko, vo, n, shift, nt, hist, totals);
        parity ^= 1;
    }
    return parity;
}

int radix_sort_keys(uint64_t *k0, uint64_t *k1, int64_t n, int nbits, uint32_t *hist,
                    uint32_t *totals, hipStream_t s)
{
    if (n <= 1) return 0;
    const int64_t nt = (n + kTile - 1) / kTile;
    int parity = 0;
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint64_t *ki = parity ? k1 : k0;
        uint64_t *ko = parity ? k0 : k1;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kBlock), 0, s, ki, n, shift,
                           nt, hist);
        hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(kBlock), 0, s, hist, nt, totals);
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nt), dim3(kBlock), 0, s, ki,
                           (const uint32_t *)nullptr, ko, (uint32_t *)nullptr, n, shift, nt,
                           hist, totals);
        parity ^= 1;
    }
    return parity;
}

}  // namespace rcp
