// Stable LSD radix sort of (u64 key, u32 value) pairs and an exclusive scan
// of u32 counts, for the neighbour-list build (Morton ordering, pair
// transposition, compaction).
//
// Sort: 8-bit digits, tiles of 2048 keys (256 threads x 8 rounds).  Per pass:
// per-tile digit histogram -> exclusive scan in digit-major order -> stable
// scatter, where each key's rank among equal digits of its tile comes from
// wave ballots (a 9-bit match over the digit) and per-wave counts in LDS.
#include "rcp_kernels.hpp"

namespace rcp {

constexpr int kTile = kBlock * 8;   // 2048 items per tile

// ---------------------------------------------------------------- scan
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const uint32_t *__restrict__ in,
                                                      int64_t n,
                                                      uint32_t *__restrict__ tile_sums)
{
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int64_t i = base + k * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    __shared__ uint32_t ws[kWavesPerBlock];
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += ws[w];
        tile_sums[blockIdx.x] = t;
    }
}

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

// Single block: exclusive scan of the tile sums, total written to total[0].
__global__ __launch_bounds__(kBlock) void k_scan_top(uint32_t *__restrict__ sums, int64_t nt,
                                                    uint32_t *__restrict__ total)
{
    uint32_t carry = 0;
    for (int64_t base = 0; base < nt; base += kBlock) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nt ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive(v, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t n,
                                                      const uint32_t *__restrict__ tile_off)
{
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = tile_off[blockIdx.x] + block_exclusive(s, &tot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

__global__ void k_write_total(uint32_t *__restrict__ out, int64_t n,
                              const uint32_t *__restrict__ total)
{
    out[n] = *total;
}

// One block of 1024 threads scans up to kScanSingle values in rounds of
// 8192 (8 consecutive values a thread), so a short scan is one launch.
constexpr int kScanThreads = 1024;
constexpr int64_t kScanSingle = 32768;

__global__ __launch_bounds__(kScanThreads) void k_scan_single(const uint32_t *__restrict__ in,
                                                             uint32_t *__restrict__ out,
                                                             int64_t n,
                                                             uint32_t *__restrict__ total)
{
    constexpr int kW = kScanThreads / kWave;
    __shared__ uint32_t ws[kW];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (int64_t base = 0; base < n; base += 8 * kScanThreads) {
        const int64_t i0 = base + (int64_t)threadIdx.x * 8;
        uint32_t v[8], sum = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = (i0 + k < n) ? in[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t inc = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += u;
        }
        if (lane == kWave - 1) ws[w] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (int q = 0; q < kW; ++q) {
            if (q < w) off += ws[q];
            tot += ws[q];
        }
        __syncthreads();   // ws is rewritten in the next round
        uint32_t run = carry + off + inc - sum;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (i0 + k < n) out[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        out[n] = carry;
        if (total) *total = carry;
    }
}

void scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tile_tmp,
                    uint32_t *total, hipStream_t s)
{
    if (n <= kScanSingle) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, in, out,
                           n < 0 ? (int64_t)0 : n, total);
        return;
    }
    const int64_t nt = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(kBlock), 0, s, in, n, tile_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tile_tmp, nt, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(kBlock), 0, s, in, out, n, tile_tmp);
    hipLaunchKernelGGL(k_write_total, dim3(1), dim3(1), 0, s, out, n, total);
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

template <bool kVals>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         uint64_t *__restrict__ kout,
                                                         uint32_t *__restrict__ vout,
                                                         int64_t n, int shift, int64_t nt,
                                                         const uint32_t *__restrict__ off)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kWavesPerBlock][257];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    base[threadIdx.x] = off[(int64_t)threadIdx.x * nt + blockIdx.x];
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
               uint32_t *hist, uint32_t *tile_tmp, uint32_t *total, hipStream_t s)
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
        scan_exclusive(hist, hist, 256 * nt, tile_tmp, total, s);
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nt), dim3(kBlock), 0, s, ki, vi,
                           ko, vo, n, shift, nt, hist);
        parity ^= 1;
    }
    return parity;
}

int radix_sort_keys(uint64_t *k0, uint64_t *k1, int64_t n, int nbits, uint32_t *hist,
                    uint32_t *tile_tmp, uint32_t *total, hipStream_t s)
{
    if (n <= 1) return 0;
    const int64_t nt = (n + kTile - 1) / kTile;
    int parity = 0;
    for (int shift = 0; shift < nbits; shift += 8) {
        const uint64_t *ki = parity ? k1 : k0;
        uint64_t *ko = parity ? k0 : k1;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nt), dim3(kBlock), 0, s, ki, n, shift,
                           nt, hist);
        scan_exclusive(hist, hist, 256 * nt, tile_tmp, total, s);
        hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nt), dim3(kBlock), 0, s, ki,
                           (const uint32_t *)nullptr, ko, (uint32_t *)nullptr, n, shift, nt,
                           hist);
        parity ^= 1;
    }
    return parity;
}

}  // namespace rcp
