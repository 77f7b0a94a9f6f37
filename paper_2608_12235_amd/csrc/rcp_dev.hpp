// Device-side data layout and helpers shared by the HIP kernels.
//
// Every packing ("segment") owns its own FP64 SoA arrays in Morton order
// (level-major: size class first, then the Morton code of the particle's
// cell in its class grid).  A per-segment record in device memory holds the
// array pointers (written by the host) and the optimiser / schedule state
// (written by the device), so captured HIP graphs stay valid when arrays are
// swapped or grown.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcp {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxRungs = 16;
constexpr int kMaxLevels = 48;

// segment flags (device-owned; the host clears REBUILD / HOLD / STALE)
enum : int32_t {
    F_STOP = 1,        // stop test met in the final rung
    F_CAP = 2,         // final-rung iteration cap reached
    F_REBUILD = 4,     // list validity test failed; host must rebuild
    F_NONFINITE = 8,   // NaN / Inf met
    F_HOLD = 16,       // iteration limit of the current call reached
    F_STALE = 32,      // no valid list (host has to build one first)
    F_ABORT = 64,      // the host gave up on this packing (census: others go on)
    F_IDLE = F_STOP | F_CAP | F_REBUILD | F_NONFINITE | F_HOLD | F_STALE | F_ABORT,
};

struct SchedDev {
    int32_t n_rungs, absolute;
    double tol;
    double mu[kMaxRungs], eta_x[kMaxRungs], eta_k[kMaxRungs], decay[kMaxRungs];
    int64_t budget[kMaxRungs];
};

// Position and relative diameter of one particle, 32 bytes: a neighbour
// gather touches a single cache line.  A frozen sphere (cascade stage)
// stores -(its absolute diameter) in d; list builds use |d|.
struct alignas(32) P4 {
    double x, y, z, d;
};

// Array pointers of one segment (host-owned; uploaded whole).
struct SegPtrs {
    P4 *p[2];             // ping-pong (x, y, z, D0)
    double *m[3], *v[3];  // Adam moments, SoA
    float *xref[3];       // positions at the last list build, rounded to float
                          // (they serve only the displacement test, whose
                          // limit is reduced by the rounding, see kXrefErr)
    int32_t *orig;        // sorted index -> user index
    uint8_t *lev;         // size class
    int32_t *rp;          // row pointers (n + 1) into col
    int32_t *col;         // partners (segment-local sorted indices)
};

// Scalars of one segment.  "host" fields are set by the host; the rest are
// owned by the device once a run is under way.
struct SegState {
    // host: constants
    int64_t n;
    double L, hL, d0min, sumd0;
    double nvol;          // (sum D0^3)^2 / sum D0^6, the pressure normaliser
    double d0max_k;       // max D0 (1 + 1e-9), for the list-validity test
    double beta1, beta2, eps_x, eps_k;
    int32_t mixed;        // 1: some spheres are frozen (negative D0 in the records:
                          // absolute diameter -D0, no step; a cascade stage)
    int32_t nblocks;      // iteration-grid blocks of this segment
    int64_t bfirst;       // first of them (index into the work table)
    // set at each list build (k_after_seg)
    double kb, disp_lim, kappa_lim;
    // host: hard walls (bit a = axis a): flat walls at 0 and L across the
    // axes of `walls`, a round container (disk or ball of diameter L
    // centred at L/2) over the axes of `round`; other axes are periodic
    int32_t walls, round;
    // reciprocals the iteration kernel would otherwise divide for in every
    // wave: 1 / L, and the bias corrections of the next position step,
    // 1 / (1 - beta1^(t+1)) and 1 / (1 - beta2^(t+1))
    double iL, ib1n, ib2n;
    // optimiser and schedule state
    double kappa, mk, vk, b1t, b2t, mu, eta_x, eta_k;
    int64_t t, it_rung, iters, iter_limit;
    int32_t rung, flags, cur, pad1;
    // outputs of the last evaluation
    double E_ov, S_drd, max_delta, max_disp2;
    uint32_t ticket, pad2;
    SchedDev sched;
};

// Refresh ib1n, ib2n after b1t = beta1^t or b2t = beta2^t changed.
__host__ __device__ inline void seg_bias_terms(SegState &s)
{
    s.ib1n = 1.0 / (1.0 - s.b1t * s.beta1);
    s.ib2n = 1.0 / (1.0 - s.b2t * s.beta2);
}

// One block of the iteration grid: rows [begin, end) of packing seg.
struct WorkItem {
    int32_t seg;
    int32_t e0, e1;       // its CSR entries [e0, e1) = [rp[begin], rp[end])
    int32_t pad;
    int64_t begin, end;   // its rows
};

// ------------------------------------------------- global-memory access
// Array pointers come from a table in device memory, so the compiler cannot
// tell that they address global memory and would emit flat instructions
// (which also wait on LDS traffic).  These views make the accesses global
// loads / stores; sphere records are addressed with a 32-bit byte offset
// from a uniform base (n < 2^27).
template <class T>
using gptr = __attribute__((address_space(1))) T *;
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ P4 load_p4(const P4 *base, int32_t j)
{
    const gptr<const char> b = (gptr<const char>)base;
    const dbl4 v = *(gptr<const dbl4>)(b + ((uint32_t)j << 5));
    P4 r;
    r.x = v.x;
    r.y = v.y;
    r.z = v.z;
    r.d = v.w;
    return r;
}

__device__ __forceinline__ void store_p4(P4 *base, int32_t j, const P4 &r)
{
    const gptr<char> b = (gptr<char>)base;
    dbl4 v;
    v.x = r.x;
    v.y = r.y;
    v.z = r.z;
    v.w = r.d;
    *(gptr<dbl4>)(b + ((uint32_t)j << 5)) = v;
}

// The three coordinates of a record, its D0 left as it is (16 + 8 bytes).
__device__ __forceinline__ void store_xyz(P4 *base, int32_t j, double x, double y, double z)
{
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    const gptr<char> b = (gptr<char>)base + ((uint32_t)j << 5);
    dbl2 v;
    v.x = x;
    v.y = y;
    *(gptr<dbl2>)b = v;
    *(gptr<double>)(b + 16) = z;
}

template <class T>
__device__ __forceinline__ T gload(const T *base, int64_t i)
{
    return ((gptr<const T>)base)[i];
}

template <class T>
__device__ __forceinline__ void gstore(T *base, int64_t i, T v)
{
    ((gptr<T>)base)[i] = v;
}

// ------------------------------------------------------------------ math
// Minimum image of a separation of two coordinates in [0, L): one box
// length is removed when the separation exceeds half a box; exactly at
// +-L/2 no shift is applied.
__device__ __forceinline__ double min_image(double d, double L, double hL)
{
    // d > hL gives d - L and d < -hL gives d - (-L) = d + L exactly: one
    // compare on |d| and one select instead of two of each
    return fabs(d) > hL ? d - copysign(L, d) : d;
}

// ------------------------------------------------------------ hard walls
// Sec. 2: an axis may be bounded by flat hard walls (planes 0 and L) or be
// one of two or three axes of a round container (the disk or ball of
// diameter L centred at L/2).  A sphere of diameter sig at distance h from
// a wall overlaps it when gap = 2h < sig, with delta = 1 - gap / sig (the
// pair term with its mirror image) and energy delta^2 / 2.  gap is 2 x_a
// and 2 (L - x_a) for the flat walls and L - 2 rho for the round one, rho
// the distance from the container's axis or centre.  Every expression is
// evaluated as written (no contraction): the placement and shrink
// predicates must round exactly as stated.

// rho^2 over the round axes, summed in axis order.
__device__ __forceinline__ double round_rho2(double x, double y, double z, double L,
                                             int32_t round)
{
#pragma clang fp contract(off)
    double r2 = 0.0;
    if (round & 1) {
        const double u = x - 0.5 * L;
        r2 = r2 + u * u;
    }
    if (round & 2) {
        const double u = y - 0.5 * L;
        r2 = r2 + u * u;
    }
    if (round & 4) {
        const double u = z - 0.5 * L;
        r2 = r2 + u * u;
    }
    return r2;
}

// Running sums of a sphere's wall terms: gradient, energy, kappa-gradient
// part delta (gap / sig) (dE/dkappa is its sum over kappa), max delta,
// contacts.
struct WallAcc {
    double g[3], e, s, m, c;
};

__device__ __forceinline__ void wall_terms(const double p[3], double sig, double L, int32_t walls,
                                           int32_t round, WallAcc &w)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!((walls >> a) & 1)) continue;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double gap = side == 0 ? 2.0 * p[a] : 2.0 * (L - p[a]);
            if (!(gap < sig)) continue;
            const double delta = 1.0 - gap / sig;
            w.e += 0.5 * delta * delta;
            w.s += delta * (gap / sig);
            w.m = fmax(w.m, delta);
            w.c += 1.0;
            w.g[a] += (side == 0 ? -2.0 : 2.0) * delta / sig;
        }
    }
    if (round) {
        const double rho = sqrt(round_rho2(p[0], p[1], p[2], L, round));
        const double gap = L - 2.0 * rho;
        if (gap < sig) {
            const double delta = 1.0 - gap / sig;
            w.e += 0.5 * delta * delta;
            w.s += delta * (gap / sig);
            w.m = fmax(w.m, delta);
            w.c += 1.0;
            if (rho > 0.0) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    if ((round >> a) & 1) w.g[a] += 2.0 * delta * (p[a] - 0.5 * L) / (sig * rho);
            }
        }
    }
}

// Placement test: a sphere of diameter sig at p touches no wall (touching
// allowed); round: t = L - sig >= 0 and t^2 >= 4 rho^2.
__device__ __forceinline__ bool inside_walls(const double p[3], double sig, double L,
                                             int32_t walls, int32_t round)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if ((walls >> a) & 1)
            if (!(sig <= 2.0 * p[a]) || !(sig <= 2.0 * (L - p[a]))) return false;
    if (round) {
        const double t = L - sig;
        if (!(t >= 0.0 && t * t >= 4.0 * round_rho2(p[0], p[1], p[2], L, round))) return false;
    }
    return true;
}

// ------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// A double moved across lanes by a DPP control (both halves); lanes that
// the row mask leaves out receive `old`.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ double dpp_f64(double old, double v)
{
    union {
        double d;
        int i[2];
    } a, b, r;
    a.d = old;
    b.d = v;
    r.i[0] = __builtin_amdgcn_update_dpp(a.i[0], b.i[0], kCtrl, kRowMask, 0xf, false);
    r.i[1] = __builtin_amdgcn_update_dpp(a.i[1], b.i[1], kCtrl, kRowMask, 0xf, false);
    return r.d;
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    union {
        double d;
        int i[2];
    } a;
    a.d = v;
    a.i[0] = __builtin_amdgcn_readlane(a.i[0], lane);
    a.i[1] = __builtin_amdgcn_readlane(a.i[1], lane);
    return a.d;
}

// Inclusive prefix sum of an int over the 64 lanes with DPP only:
// Kogge-Stone shifts within rows of 16, then the row broadcasts carry the
// totals of rows 0 and 0..1 (2) forward.
__device__ __forceinline__ int32_t wave_scan_incl_dpp(int32_t v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Wave-wide sum / maximum (of values >= 0) with DPP moves only, no LDS
// traffic: quad butterflies, rotations within rows of 16, then the row
// broadcasts; the total ends in lane 63 and is returned to every lane.
// The combining order is fixed.
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_f64<0xb1>(0.0, v);          // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4e>(0.0, v);          // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x124>(0.0, v);         // row_ror:4
    v += dpp_f64<0x128>(0.0, v);         // row_ror:8
    v += dpp_f64<0x142, 0xa>(0.0, v);    // row_bcast:15 into rows 1, 3
    v += dpp_f64<0x143, 0xc>(0.0, v);    // row_bcast:31 into rows 2, 3
    return readlane_f64(v, kWave - 1);
}

__device__ __forceinline__ double wave_max_dpp(double v)
{
    v = fmax(v, dpp_f64<0xb1>(0.0, v));
    v = fmax(v, dpp_f64<0x4e>(0.0, v));
    v = fmax(v, dpp_f64<0x124>(0.0, v));
    v = fmax(v, dpp_f64<0x128>(0.0, v));
    v = fmax(v, dpp_f64<0x142, 0xa>(0.0, v));
    v = fmax(v, dpp_f64<0x143, 0xc>(0.0, v));
    return readlane_f64(v, kWave - 1);
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

// Morton interleave of three 19-bit cell coordinates (57 bits).
__device__ __host__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __host__ __forceinline__ uint64_t morton3(uint64_t cx, uint64_t cy, uint64_t cz)
{
    return spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
}

__device__ __forceinline__ uint64_t hash64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

constexpr uint64_t kEmptyKey = ~0ull;

}  // namespace rcp
