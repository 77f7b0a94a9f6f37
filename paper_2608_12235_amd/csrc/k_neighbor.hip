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
// Keys are (tile << tshift) | (class << mb) | Morton(cell): one stable sort
// orders particles by spatial tile (a T x T x T split of the box, tiles in
// Morton order), then by class, then by cell.  A tile holds every class of
// its region, so the blocks an XCD runs (a contiguous range) cover a compact
// region and the partners they gather, of any class, stay in that XCD's L2.
// A cell's tile is a function of its integer coordinates, so all particles
// of a cell share it.  Occupied cells are located through an
// open-addressing hash of their keys.  The listing predicate is evaluated
// with a fixed operation order and no contraction so that the pair set is
// reproducible bit for bit:
//   dx = mi(x_j - x_i) (same for y, z),  r2 = (dx dx + dy dy) + dz dz,
//   c = kb ((1 + g)(0.5 (D0_i + D0_j)) + 2 s D0_min),  listed iff r2 < c c.
#pragma clang fp contract(off)
#include "rcp_kernels.hpp"

namespace rcp {

// Cell of coordinate v in a class grid; the same expression is used when
// keys are made and when a particle looks up its stencil, so the two agree.
__device__ __forceinline__ int32_t cell_coord(double v, double inv_w, int32_t nc)
{
    int32_t c = (int32_t)(v * inv_w);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

// Tile coordinate of cell c of a grid with nc cells per axis.
__device__ __forceinline__ uint64_t tile_of(int64_t c, int32_t nc, int32_t tiles)
{
    return (uint64_t)((c * tiles) / nc);
}

__device__ __forceinline__ void key_of(const BuildArgs &a, const P4 *__restrict__ pos,
                                       const uint8_t *__restrict__ lev, int64_t i,
                                       uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int l = lev[i];
    const LevelGrid g = a.lv[l];
    const P4 q = pos[i];
    uint64_t cx = (uint64_t)cell_coord(q.x, g.inv_w, g.nc);
    uint64_t cy = (uint64_t)cell_coord(q.y, g.inv_w, g.nc);
    uint64_t cz = (uint64_t)cell_coord(q.z, g.inv_w, g.nc);
    const uint64_t tile = morton3(tile_of(cx, g.nc, a.tiles), tile_of(cy, g.nc, a.tiles),
                                  tile_of(cz, g.nc, a.tiles));
    keys[i] = (tile << a.tshift) | ((uint64_t)l << a.mb) | morton3(cx, cy, cz);
    vals[i] = (uint32_t)i;
}

__device__ __forceinline__ void permute_one(const PermArgs &p, int64_t k)
{
    const int64_t s = p.perm[k];
    const P4 q = p.ps[s];
    p.pd[k] = q;
    p.xref[0][k] = (float)q.x;
    p.xref[1][k] = (float)q.y;
    p.xref[2][k] = (float)q.z;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.md[a][k] = p.ms[a][s];
        p.vd[a][k] = p.vs[a][s];
    }
    p.od[k] = p.os[s];
    p.ld[k] = p.ls[s];
}

// ------------------------------------------------------------- hashing
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

// Home slot of a cell key.  The low three Morton bits (a 2x2x2 block of
// cells) stay together in one 8-slot group (one 128-byte line); the groups
// themselves are scattered by multiplicative (Fibonacci) hashing of the
// remaining bits, the group number being the top bits of the product with
// 2^64 / golden ratio, so a 27-cell stencil touches about eight lines and
// Morton-adjacent particles share them.  The table size is a power of two,
// at least 64 slots.
__device__ __forceinline__ uint64_t hash_slot(uint64_t key, uint64_t mask)
{
    const int gshift = __builtin_clzll(mask) + 3;   // 64 - log2(number of groups)
    return ((((key >> 3) * 0x9e3779b97f4a7c15ull) >> gshift) << 3) | (key & 7ull);
}

__device__ __forceinline__ int2 hash_find(const BuildArgs &a, uint64_t key)
{
    uint64_t slot = hash_slot(key, a.hmask);
    for (;;) {
        const HashSlot e = a.hash[slot];
        if (e.key == key) return make_int2(e.start, e.count);
        if (e.key == kEmptyKey) return make_int2(0, 0);
        slot = (slot + 1) & a.hmask;
    }
}

// Dense cell index of sorted particle i (its level must be dense).
__device__ __forceinline__ int64_t dense_index(const BuildArgs &a, int64_t i)
{
    const LevelGrid g = a.lv[a.lev[i]];
    const P4 q = a.pos[i];
    const int64_t cx = cell_coord(q.x, g.inv_w, g.nc), cy = cell_coord(q.y, g.inv_w, g.nc),
                  cz = cell_coord(q.z, g.inv_w, g.nc);
    return g.dbase + (cx * g.nc + cy) * g.nc + cz;
}

// End of the run of sorted keys equal to key that starts at i (the first
// index past it, at most n).  The eight keys after i are read together
// (most runs end there); a longer run is bracketed by doubling steps and the
// end found by bisection, so a run of c keys costs O(log c) dependent reads.
__device__ __forceinline__ int64_t run_end(const uint64_t *sk, int64_t n, int64_t i, uint64_t key)
{
    uint64_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = i + 1 + k < n ? gload(sk, i + 1 + k) : ~key;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (v[k] != key) return i + 1 + k;
    int64_t lo = i + 9, hi = n, step = 8;   // keys [i, lo) equal key
    for (;;) {
        const int64_t p = lo + step - 1;
        if (p >= n) break;
        if (gload(sk, p) != key) {
            hi = p;
            break;
        }
        lo = p + 1;
        step *= 2;
    }
    while (lo < hi) {   // the first index in [lo, hi] whose key differs (hi: differs, or n)
        const int64_t mid = lo + (hi - lo) / 2;
        if (gload(sk, mid) == key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// A cell's sorted particles are contiguous (same key): the first one finds
// the end of the run and writes (start, count), into the dense table of its
// level or into the hash (inserted by compare-and-swap on the key).
__device__ __forceinline__ void cells_one(const BuildArgs &a, int64_t i)
{
    const uint64_t key = a.skey[i];
    if (i > 0 && a.skey[i - 1] == key) return;
    const int64_t e = run_end(a.skey, a.n, i, key);
    const int32_t start = (int32_t)i, count = (int32_t)(e - i);
    if (a.lv[a.lev[i]].dbase >= 0) {
        a.dense[dense_index(a, i)] = make_int2(start, count);
        return;
    }
    uint64_t slot = hash_slot(key, a.hmask);
    for (;;) {
        const unsigned long long prev = atomicCAS((unsigned long long *)&a.hash[slot].key,
                                                  (unsigned long long)kEmptyKey,
                                                  (unsigned long long)key);
        if (prev == kEmptyKey) {
            a.hash[slot].start = start;
            a.hash[slot].count = count;
            return;
        }
        slot = (slot + 1) & a.hmask;
    }
}

// Block b of a batch grid belongs to the last job whose first block is <= b.
template <class T>
__device__ __forceinline__ int job_of(const T *__restrict__ jobs, int J, int64_t b,
                                      int64_t T::*first)
{
    int lo = 0, hi = J - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*first <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------- pair search
constexpr int kSearchBuf = 3072;   // entries staged per block in LDS (24 KB)

// Half partners of particle i are searched: same class with a larger sorted
// index, and every larger class.  Each listed pair is appended in both
// directions; a block stages its entries in LDS and reserves global space
// with one atomic (entries that do not fit in LDS go straight to global
// memory).  The order of the list is arbitrary; it is sorted afterwards.
__device__ __forceinline__ int remap_xcd(int b, int G)
{
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of particles (one spatial region, tile-major order)
    const int nx = 8, per = G / nx, rem = G % nx;
    const int xcd = b % nx, loc = b / nx;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + loc;
}

__global__ __launch_bounds__(kBlock) void k_search(BuildArgs a, uint64_t *__restrict__ list,
                                                  unsigned long long *__restrict__ counter, int64_t cap,
                                                  int row_bits, int xcd_remap)
{
    __shared__ uint64_t buf[kSearchBuf];
    __shared__ uint32_t nbuf;
    __shared__ unsigned long long gbase;
    if (threadIdx.x == 0) nbuf = 0;
    __syncthreads();
    const int blk = xcd_remap ? remap_xcd((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int64_t i = (int64_t)blk * kBlock + threadIdx.x;
    if (i < a.n) {
        const P4 qi = a.pos[i];
        const double xi = qi.x, yi = qi.y, zi = qi.z, di = fabs(qi.d);
        const int li = a.lev[i];
        const uint64_t rowi = (uint64_t)i << row_bits;
        for (int L = li; L < a.nlev; ++L) {
            const LevelGrid g = a.lv[L];
            if (g.count == 0) continue;
            const int32_t nc = g.nc;
            // Stencil cells.  With nc >= 3 a neighbour cell is searched only
            // if its nearest point is closer to the particle than the largest
            // cutoff the particle can have with a class-L partner (bound in
            // cell units, with a margin far above the rounding of x * inv_w);
            // with nc < 3 every cell is searched once.  Skipping is exact.
            const double cb =
                a.kb * (a.opg * (0.5 * (di + g.dmax)) + a.sk2) * g.inv_w * (1.0 + 1e-9) + 1e-9;
            const bool dense = g.dbase >= 0;
            uint64_t m[3][3];   // [axis][slot]: Morton parts of the lower, own, upper cell
            uint64_t tp[3][3];  // the same for the tile field
            int32_t cc[3][3];   // the cell coordinates themselves (dense levels)
            double gap[3][3];   // distance (cell units) from the particle to that slab
            bool use[3][3];
            const double pos[3] = {xi, yi, zi};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const double fp = pos[ax] * g.inv_w;
                const int32_t c = cell_coord(pos[ax], g.inv_w, nc);
                if (nc >= 3) {
                    const double f = fp - (double)c;
                    const int32_t lo = c == 0 ? nc - 1 : c - 1, hi = c == nc - 1 ? 0 : c + 1;
                    cc[ax][0] = lo;
                    cc[ax][1] = c;
                    cc[ax][2] = hi;
                    m[ax][0] = spread3((uint64_t)lo) << ax;
                    m[ax][1] = spread3((uint64_t)c) << ax;
                    m[ax][2] = spread3((uint64_t)hi) << ax;
                    tp[ax][0] = spread3(tile_of(lo, nc, a.tiles)) << ax;
                    tp[ax][1] = spread3(tile_of(c, nc, a.tiles)) << ax;
                    tp[ax][2] = spread3(tile_of(hi, nc, a.tiles)) << ax;
                    gap[ax][0] = f;
                    gap[ax][1] = 0.0;
                    gap[ax][2] = 1.0 - f;
                    use[ax][0] = f < cb;
                    use[ax][1] = true;
                    use[ax][2] = 1.0 - f < cb;
                } else {
                    cc[ax][0] = 0;
                    cc[ax][1] = 1;
                    cc[ax][2] = 0;
                    m[ax][0] = 0;
                    m[ax][1] = spread3(1) << ax;
                    m[ax][2] = 0;
                    tp[ax][0] = spread3(tile_of(0, nc, a.tiles)) << ax;
                    tp[ax][1] = spread3(tile_of(1, nc, a.tiles)) << ax;
                    tp[ax][2] = 0;
                    gap[ax][0] = gap[ax][1] = gap[ax][2] = 0.0;
                    use[ax][0] = true;
                    use[ax][1] = nc == 2;
                    use[ax][2] = false;
                }
            }
            const uint64_t base = (uint64_t)L << a.mb;
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
#pragma unroll
                    for (int oz = 0; oz < 3; ++oz) {
                        if (!(use[0][ox] && use[1][oy] && use[2][oz])) continue;
                        // a cell whose nearest point is beyond the cutoff bound
                        // cannot hold a partner (corners and edges of the stencil)
                        const double g2 = (gap[0][ox] * gap[0][ox] + gap[1][oy] * gap[1][oy]) +
                                          gap[2][oz] * gap[2][oz];
                        if (!(g2 < cb * cb)) continue;
                        int2 r;
                        if (dense) {
                            r = a.dense[g.dbase + ((int64_t)cc[0][ox] * nc + cc[1][oy]) * nc +
                                        cc[2][oz]];
                        } else {
                            const uint64_t key = base | m[0][ox] | m[1][oy] | m[2][oz] |
                                                 ((tp[0][ox] | tp[1][oy] | tp[2][oz]) << a.tshift);
                            r = hash_find(a, key);
                        }
                        for (int64_t j = r.x; j < (int64_t)r.x + r.y; ++j) {
                            if (L == li && j <= i) continue;
                            const P4 qj = a.pos[j];
                            const double dx = min_image(qj.x - xi, a.L, a.hLa[0]);
                            const double dy = min_image(qj.y - yi, a.L, a.hLa[1]);
                            const double dz = min_image(qj.z - zi, a.L, a.hLa[2]);
                            const double r2 = (dx * dx + dy * dy) + dz * dz;
                            const double cc = a.kb * (a.opg * (0.5 * (di + fabs(qj.d))) + a.sk2);
                            if (r2 < cc * cc) {
                                const uint64_t e0 = rowi | (uint64_t)j;
                                const uint64_t e1 = ((uint64_t)j << row_bits) | (uint64_t)i;
                                const uint32_t k = atomicAdd(&nbuf, 2u);
                                if (k + 1 < (uint32_t)kSearchBuf) {
                                    buf[k] = e0;
                                    buf[k + 1] = e1;
                                } else {
                                    const unsigned long long gi = atomicAdd(counter, 2ull);
                                    if ((int64_t)gi + 1 < cap) {
                                        list[gi] = e0;
                                        list[gi + 1] = e1;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    const uint32_t mm = nbuf < (uint32_t)kSearchBuf ? nbuf : (uint32_t)kSearchBuf;
    if (threadIdx.x == 0) gbase = mm ? atomicAdd(counter, (unsigned long long)mm) : 0ull;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < mm; k += kBlock)
        if ((int64_t)gbase + k < cap) list[gbase + k] = buf[k];
}

// ------------------------------------------------ wave-cooperative search
// The same search with the candidates of a wave flattened: for one level
// and one stencil plane (the nine cells at one x offset), every lane
// contributes the runs [start, start + count) of its nine cells
// (restricted to larger indices in its own level), a wave prefix sum
// numbers all of them as one sequence, and the 64 lanes test consecutive
// candidates together (test_plane).  A particle's candidate set and the
// pair test are those of k_search, so the listed pairs are the same; only
// the order in which entries are appended differs (the list is sorted
// afterwards).

// Loads through global-address-space views (global rather than flat
// instructions, so waiting for LDS results does not also wait for them).
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int2 load_run(const int2 *t, uint64_t k)
{
    const uint64_t v = ((gptr<const uint64_t>)t)[k];
    return make_int2((int32_t)(uint32_t)v, (int32_t)(uint32_t)(v >> 32));
}

__device__ __forceinline__ HashSlot load_hslot(const HashSlot *t, uint64_t k)
{
    const u64x2 v = ((gptr<const u64x2>)t)[k];
    HashSlot h;
    h.key = v.x;
    h.start = (int32_t)(uint32_t)v.y;
    h.count = (int32_t)(uint32_t)(v.y >> 32);
    return h;
}

__device__ __forceinline__ P4 load_pos(const P4 *t, int64_t k)
{
    const dbl4 v = ((gptr<const dbl4>)t)[k];
    P4 r;
    r.x = v.x;
    r.y = v.y;
    r.z = v.z;
    r.d = v.w;
    return r;
}

// A particle's stencil in one level grid, as the cooperative search keeps
// it in registers: a mask of the searched slots (sphere-distance pruning of
// the 27 cells, as in k_search) and, per axis and offset, the part of the
// cell's table position that axis contributes.  For a hashed level the
// parts are the Morton and tile bits of the key; for a dense level they are
// the strides of the (x, y, z) cell index.  The parts of a key occupy
// disjoint bits, so in both cases the position is base + px + py + pz.
struct CoopStencil {
    uint32_t mask;       // bit sl (slot sl = 9 ox + 3 oy + oz) set if searched
    uint64_t p[3][3];    // [axis][lower, own, upper cell]
};

// Two-bit tile coordinate in Morton form (tiles per axis <= 4).
__device__ __forceinline__ uint64_t spread_tile(uint32_t t)
{
    return (uint64_t)((t & 1u) | ((t & 2u) << 2));
}

__device__ __forceinline__ void coop_stencil(const BuildArgs &a, const LevelGrid &g,
                                             const double pos[3], double di, bool act,
                                             CoopStencil &S)
{
    const int32_t nc = g.nc;
    const bool dense = g.dbase >= 0;
    const double cb = a.kb * (a.opg * (0.5 * (di + g.dmax)) + a.sk2) * g.inv_w * (1.0 + 1e-9) + 1e-9;
    uint32_t m = 0;
    if (nc >= 3) {
        int32_t c[3];
        double sq[3][3];
        bool ok[3][3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const double fp = pos[ax] * g.inv_w;
            c[ax] = cell_coord(pos[ax], g.inv_w, nc);
            const double f = fp - (double)c[ax];
            // squared distance (cell units) to the lower and upper slab
            sq[ax][0] = f * f;
            sq[ax][1] = 0.0;
            sq[ax][2] = (1.0 - f) * (1.0 - f);
            ok[ax][0] = f < cb;
            ok[ax][1] = true;
            ok[ax][2] = 1.0 - f < cb;
        }
        // a cell is searched if its nearest point is within the bound; the
        // zero terms of the own-cell axes are left out of the sums (adding
        // +0.0 changes nothing), the order is (x + y) + z as in k_search
        const double cb2 = cb * cb;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const double sxy = ox == 1 ? sq[1][oy]
                                           : (oy == 1 ? sq[0][ox] : sq[0][ox] + sq[1][oy]);
#pragma unroll
                for (int oz = 0; oz < 3; ++oz) {
                    const double s2 = oz == 1 ? sxy
                                              : (ox == 1 && oy == 1 ? sq[2][oz] : sxy + sq[2][oz]);
                    if (ok[0][ox] && ok[1][oy] && ok[2][oz] && s2 < cb2)
                        m |= 1u << (ox * 9 + oy * 3 + oz);
                }
            }
        }
        if (dense) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int64_t stride = ax == 0 ? (int64_t)nc * nc : (ax == 1 ? (int64_t)nc : 1);
                const int32_t lo = c[ax] == 0 ? nc - 1 : c[ax] - 1;
                const int32_t hi = c[ax] == nc - 1 ? 0 : c[ax] + 1;
                S.p[ax][0] = (uint64_t)((int64_t)lo * stride);
                S.p[ax][1] = (uint64_t)((int64_t)c[ax] * stride);
                S.p[ax][2] = (uint64_t)((int64_t)hi * stride);
            }
        } else {
            // Morton parts of the neighbour cells by dilated-integer
            // increment and decrement of the own cell's, and their tiles from
            // the own cell's tile (tiles per axis T = 1, 2 or 4; tile k starts
            // at cell ceil(k nc / T)); the periodic wraps are the level's
            // first and last cell
            const uint32_t T = (uint32_t)a.tiles, lt = (uint32_t)__builtin_ctz(T);
            const uint32_t tlast = ((uint32_t)(nc - 1) * T) / (uint32_t)nc;
            const uint64_t dlast = spread3((uint64_t)(nc - 1));
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const uint64_t M = 0x1249249249249249ull;
                const uint32_t cu = (uint32_t)c[ax];
                const uint64_t d = spread3((uint64_t)cu);
                const uint64_t dhi = cu == (uint32_t)nc - 1 ? 0ull : ((d | ~M) + 1) & M;
                const uint64_t dlo = cu == 0 ? dlast : (d - 1) & M;
                const uint32_t t = (cu * T) / (uint32_t)nc;
                const uint32_t thi =
                    cu == (uint32_t)nc - 1
                        ? 0u
                        : t + (cu + 1 == (((t + 1) * (uint32_t)nc + T - 1) >> lt) ? 1u : 0u);
                const uint32_t tlo =
                    cu == 0 ? tlast : t - (cu == ((t * (uint32_t)nc + T - 1) >> lt) ? 1u : 0u);
                S.p[ax][0] = (dlo << ax) | ((spread_tile(tlo) << ax) << a.tshift);
                S.p[ax][1] = (d << ax) | ((spread_tile(t) << ax) << a.tshift);
                S.p[ax][2] = (dhi << ax) | ((spread_tile(thi) << ax) << a.tshift);
            }
        }
    } else {
        // one or two cells per axis: each distinct cell is searched once
        int32_t cc[3][3];
        bool use[3][3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            cc[ax][0] = 0;
            cc[ax][1] = 1;
            cc[ax][2] = 0;
            use[ax][0] = true;
            use[ax][1] = nc == 2;
            use[ax][2] = false;
            const int64_t stride = ax == 0 ? (int64_t)nc * nc : (ax == 1 ? (int64_t)nc : 1);
#pragma unroll
            for (int o = 0; o < 3; ++o)
                S.p[ax][o] = dense ? (uint64_t)((int64_t)cc[ax][o] * stride)
                                   : (spread3((uint64_t)cc[ax][o]) << ax) |
                                         ((spread3(tile_of(cc[ax][o], nc, a.tiles)) << ax)
                                          << a.tshift);
        }
#pragma unroll
        for (int sl = 0; sl < 27; ++sl)
            if (use[0][sl / 9] && use[1][(sl / 3) % 3] && use[2][sl % 3]) m |= 1u << sl;
    }
    S.mask = act ? m : 0u;
}

// Cell runs (start, count) of the nine slots of stencil plane ox.  Every
// table read of the plane is issued before any is used, so a wave has nine
// lookups in flight instead of one; lanes that do not search a slot read a
// fixed entry (the level's first dense cell, or the hash table's first
// slot: one shared line) and discard it.  A hash probe that meets another
// key (a collision) continues along the probe sequence.
__device__ __forceinline__ void lookup_plane(const BuildArgs &a, const CoopStencil &S,
                                             bool dense, uint64_t base, int ox, int2 r[9])
{
    if (dense) {
        int2 v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const bool u = (S.mask >> (ox * 9 + k)) & 1u;
            const uint64_t at = base + S.p[0][ox] + S.p[1][k / 3] + S.p[2][k % 3];
            v[k] = load_run(a.dense, u ? at : base);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const bool u = (S.mask >> (ox * 9 + k)) & 1u;
            r[k] = u ? v[k] : make_int2(0, 0);
        }
        return;
    }
    HashSlot e[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const bool u = (S.mask >> (ox * 9 + k)) & 1u;
        const uint64_t key = base + S.p[0][ox] + S.p[1][k / 3] + S.p[2][k % 3];
        e[k] = load_hslot(a.hash, u ? hash_slot(key, a.hmask) : 0ull);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const bool u = (S.mask >> (ox * 9 + k)) & 1u;
        const uint64_t key = base + S.p[0][ox] + S.p[1][k / 3] + S.p[2][k % 3];
        r[k] = make_int2(0, 0);
        if (u && e[k].key == key) r[k] = make_int2(e[k].start, e[k].count);
        if (u && e[k].key != key && e[k].key != kEmptyKey) {
            uint64_t slot = hash_slot(key, a.hmask);
            for (;;) {
                slot = (slot + 1) & a.hmask;
                const HashSlot f = load_hslot(a.hash, slot);
                if (f.key == key) {
                    r[k] = make_int2(f.start, f.count);
                    break;
                }
                if (f.key == kEmptyKey) break;
            }
        }
    }
}

// Inclusive running maximum of a non-negative int over the 64 lanes (DPP
// only; the same shifts and row broadcasts as the prefix sum).
__device__ __forceinline__ int32_t wave_scan_max_dpp(int32_t v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return v;
}

// Per-wave LDS table of one stencil plane's runs.  The candidates of the
// plane are numbered lane by lane and, within a lane, slot by slot; row t
// holds, for lane t's nine runs, the end E_k of run k in that numbering and
// the offset J_k with sorted index j = J_k + q for candidate q of the run.
// Row layout (int32, 16-byte rows): E_0..7, J_0..7, E_8, J_8, 2 unused.
constexpr int kTabRow = 20;

// Per-wave state of k_search_coop in LDS: the wave's particles, its plane
// table and owner marks, and its output staging.  Each wave stages its
// entries; when its staging is full it reserves global space with one
// atomic and copies them out without waiting for the other waves, and what
// remains at the end goes out with one reservation for the whole block.
// Only the wave itself reads and writes these arrays, and the LDS executes
// a wave's accesses in order, so no block barrier is needed between a
// write and the reads of other lanes (the compiler keeps a store and a
// later load of the same array in order, as their addresses may alias).
constexpr uint32_t kWaveBuf = 256;   // staged entries per wave (2 KB)

struct SearchOut {
    const P4 *own;      // LDS, this wave's 64 particles
    int32_t *tab;       // LDS, this wave's 64 rows of kTabRow
    int32_t *mark;      // LDS, this wave's 64 owner marks
    uint64_t *wbuf;     // LDS, this wave's kWaveBuf staged entries
    uint64_t *list;
    unsigned long long *counter;
    int64_t cap;
    int row_bits;
};

// Copy the wave's n staged entries to the list (called by the whole wave).
__device__ __forceinline__ void flush_wave(const SearchOut &out, int lane, uint32_t n)
{
    unsigned long long g = 0;
    if (lane == 0) g = atomicAdd(out.counter, (unsigned long long)n);
    g = (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)g) |
        ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(g >> 32))
         << 32);
    for (uint32_t k = (uint32_t)lane; k < n; k += kWave)
        if ((int64_t)g + k < out.cap) gstore(out.list, (int64_t)g + k, out.wbuf[k]);
    __builtin_amdgcn_wave_barrier();
}

// Test, with the whole wave, the candidates of one stencil plane: lane t
// contributes the runs r[0..8] of its nine cells.  A wave prefix sum of
// the lanes' totals numbers the candidates and each round tests 64
// consecutive ones, so a round is full whichever cells the candidates come
// from.  The owner of candidate q is the number of lanes whose prefix is
// <= q: each lane whose prefix ends inside the round's window marks its
// position there (the last such lane of a position), and a running maximum
// over the window gives every candidate its owner.  The owner's table row
// then gives the run and the sorted index.  Listed pairs are staged at the
// wave's count wn (the same on every lane).
__device__ __forceinline__ void test_plane(const BuildArgs &a, const SearchOut &out, int lane,
                                           uint64_t below, int64_t wbase, const int2 r[9],
                                           uint32_t &wn)
{
    int32_t cum[9];
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        c += r[k].y;
        cum[k] = c;
    }
    // candidate numbers are 32-bit: a plane's total is at most 64 lanes x 9
    // cells x the largest cell, which exceeds 2^31 only with more than 3.7
    // million spheres in one cell (their ~10^13 pairs would not fit any
    // list)
    const int32_t inc = wave_scan_incl_dpp(c);
    const int32_t T = __builtin_amdgcn_readlane(inc, kWave - 1);
    if (T == 0) return;
    const int32_t excl = inc - c;
    int32_t *row = out.tab + lane * kTabRow;
    {
        int32_t E[9], J[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            E[k] = excl + cum[k];
            J[k] = r[k].x - (E[k] - r[k].y);
        }
        *(int4 *)(row + 0) = make_int4(E[0], E[1], E[2], E[3]);
        *(int4 *)(row + 4) = make_int4(E[4], E[5], E[6], E[7]);
        *(int4 *)(row + 8) = make_int4(J[0], J[1], J[2], J[3]);
        *(int4 *)(row + 12) = make_int4(J[4], J[5], J[6], J[7]);
        *(int2 *)(row + 16) = make_int2(E[8], J[8]);
    }
    // the next lane's prefix (past the last lane: beyond every window).  The
    // shuffle runs on every lane: a lane outside the active mask would
    // supply 0 instead of its value.
    int32_t nxt = __shfl(inc, (lane + 1) & (kWave - 1), kWave);
    if (lane == kWave - 1) nxt = 0x7fffffff;
    __builtin_amdgcn_wave_barrier();
    for (int32_t r0 = 0; r0 < T; r0 += kWave) {
        const int32_t q = r0 + lane;
        out.mark[lane] = 0;
        const int32_t P = max(inc - r0, 0), Pn = max(nxt - r0, 0);
        if (P < kWave && Pn != P) out.mark[P] = lane + 1;
        __builtin_amdgcn_wave_barrier();
        const bool has = q < T;
        int o = wave_scan_max_dpp(out.mark[lane]);
        o = has ? o : 0;
        // the owner's whole row in one batch of reads; the run is the first
        // whose end exceeds q, its offset picked by selects
        const int32_t *ro = out.tab + o * kTabRow;
        const int4 e0 = *(const int4 *)(ro + 0);
        const int4 e1 = *(const int4 *)(ro + 4);
        const int4 j0 = *(const int4 *)(ro + 8);
        const int4 j1 = *(const int4 *)(ro + 12);
        const int2 ej8 = *(const int2 *)(ro + 16);
        int32_t jb = ej8.y;
        jb = e1.w > q ? j1.w : jb;
        jb = e1.z > q ? j1.z : jb;
        jb = e1.y > q ? j1.y : jb;
        jb = e1.x > q ? j1.x : jb;
        jb = e0.w > q ? j0.w : jb;
        jb = e0.z > q ? j0.z : jb;
        jb = e0.y > q ? j0.y : jb;
        jb = e0.x > q ? j0.x : jb;
        const int64_t j = (int64_t)jb + q;
        __builtin_amdgcn_wave_barrier();
        bool hit = false;
        // (the index check holds by construction; it keeps a wrong owner from
        // reading outside the positions)
        if (has && (uint64_t)j < (uint64_t)a.n) {
            const P4 oq = out.own[o];
            const P4 qj = load_pos(a.pos, j);
            const double dx = min_image(qj.x - oq.x, a.L, a.hLa[0]);
            const double dy = min_image(qj.y - oq.y, a.L, a.hLa[1]);
            const double dz = min_image(qj.z - oq.z, a.L, a.hLa[2]);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            const double cc = a.kb * (a.opg * (0.5 * (fabs(oq.d) + fabs(qj.d))) + a.sk2);
            hit = r2 < cc * cc;
        }
        const uint64_t bal = __ballot(hit);
        if (bal == 0ull) continue;
        const uint32_t cnt = 2u * (uint32_t)__popcll(bal);
        if (wn + cnt > kWaveBuf) {
            flush_wave(out, lane, wn);
            wn = 0;
        }
        if (hit) {
            const int64_t io = wbase + o;
            const uint32_t kk = wn + 2u * (uint32_t)__popcll(bal & below);
            out.wbuf[kk] = ((uint64_t)io << out.row_bits) | (uint64_t)j;
            out.wbuf[kk + 1] = ((uint64_t)j << out.row_bits) | (uint64_t)io;
        }
        wn += cnt;
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
}

// Restrict a cell run to sorted indices above i (a particle's own level:
// each pair is found once; a cell's particles are one contiguous run).
__device__ __forceinline__ int2 above(int2 r, int64_t i)
{
    const int64_t s2 = (int64_t)r.x > i + 1 ? (int64_t)r.x : i + 1;
    const int64_t e = (int64_t)r.x + r.y;
    return make_int2((int32_t)s2, e > s2 ? (int32_t)(e - s2) : 0);
}

// One launch searches every packing of a batch (job table; block ranges
// F.b0 per packing).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_search_coop(const FrontJob *__restrict__ jobs, int J,
                                                       int xcd_remap, int64_t b_base)
{
    __shared__ P4 own[kBlock];
    __shared__ __align__(16) int32_t tab[kBlock * kTabRow];
    __shared__ int32_t mark[kBlock];
    __shared__ uint64_t wbuf[kWavesPerBlock * kWaveBuf];
    __shared__ uint32_t wcount[kWavesPerBlock];
    __shared__ unsigned long long bbase;
    const int64_t gb =
        b_base + (xcd_remap ? remap_xcd((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x);
    const FrontJob &F = jobs[job_of(jobs, J, gb, &FrontJob::b0)];
    const BuildArgs &a = F.a;
    const int64_t blk = (int64_t)gb - F.b0;
    // split grids give every packing 3 * (the batch's deepest) levels; the
    // slices past this packing's levels have nothing to do
    if (gridDim.y > 1 && (int)blockIdx.y / 3 >= a.nlev) return;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int64_t wbase = (int64_t)blk * kBlock + (threadIdx.x & ~(kWave - 1));
    const int64_t i = wbase + lane;
    const bool valid = i < a.n;
    const int wofs = (int)(threadIdx.x & ~(kWave - 1));
    const SearchOut out{own + wofs, tab + wofs * kTabRow, mark + wofs,
                        wbuf + (wofs / kWave) * kWaveBuf, F.list, F.counter, F.lcap, F.row_bits};
    double xi = 0.0, yi = 0.0, zi = 0.0, di = 0.0;
    int li = kMaxLevels;
    if (valid) {
        const P4 qi = load_pos(a.pos, i);
        xi = qi.x;
        yi = qi.y;
        zi = qi.z;
        di = fabs(qi.d);
        li = gload(a.lev, i);
    }
    own[threadIdx.x] = P4{xi, yi, zi, di};
    __builtin_amdgcn_wave_barrier();
    // a grid with gridDim.y > 1 gives each block one level and one plane
    // (fixed x offset) of the stencil: shorter chains of dependent lookups
    // for packings too small to fill the GPU otherwise
    int Lb = 0, Le = a.nlev, plane = -1;
    if (gridDim.y > 1) {
        Lb = (int)blockIdx.y / 3;
        Le = Lb + 1 < a.nlev ? Lb + 1 : a.nlev;
        plane = (int)blockIdx.y % 3;
    }
    uint32_t wn = 0;
    for (int L = Lb; L < Le; ++L) {
        const LevelGrid g = a.lv[L];
        if (g.count == 0) continue;
        const bool act = li <= L;
        if (__ballot(act) == 0ull) continue;
        CoopStencil S;
        const double pos[3] = {xi, yi, zi};
        coop_stencil(a, g, pos, di, act, S);
        const bool same = L == li;
        const bool dense = g.dbase >= 0;
        const uint64_t base = dense ? (uint64_t)g.dbase : (uint64_t)L << a.mb;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
            if (plane >= 0 && ox != plane) continue;
            int2 r[9];
            lookup_plane(a, S, dense, base, ox, r);
            if (same) {
#pragma unroll
                for (int k = 0; k < 9; ++k) r[k] = above(r[k], i);
            }
            test_plane(a, out, lane, below, wbase, r, wn);
        }
    }
    // what the waves still hold goes out with one reservation per block
    const int w = (int)threadIdx.x / kWave;
    if (lane == 0) wcount[w] = wn;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) tot += wcount[k];
        bbase = tot ? atomicAdd(F.counter, (unsigned long long)tot) : 0ull;
    }
    __syncthreads();
    unsigned long long g = bbase;
    for (int k = 0; k < w; ++k) g += wcount[k];
    for (uint32_t k = (uint32_t)lane; k < wn; k += kWave)
        if ((int64_t)g + k < F.lcap) gstore(F.list, (int64_t)g + k, out.wbuf[k]);
}

void launch_search(const BuildArgs &a, uint64_t *list, unsigned long long *counter, int64_t cap,
                   int row_bits, int xcd_remap, hipStream_t s)
{
    if (a.n <= 0) return;
    const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_search, grid, dim3(kBlock), 0, s, a, list, counter, cap, row_bits,
                       xcd_remap);
}

void launch_search_seg(const FrontJob *jobs, int J, int64_t nb, int max_nlev, int xcd_remap,
                       int64_t b_base, hipStream_t s)
{
    if (nb <= 0) return;
    // fewer than 8 blocks per CU: split the work by level and plane
    const unsigned ny = nb < 2048 ? 3u * (unsigned)max_nlev : 1u;
    hipLaunchKernelGGL(k_search_coop, dim3((unsigned)nb, ny), dim3(kBlock), 0, s, jobs, J,
                       xcd_remap, b_base);
}

// Row pointers and partners from the sorted entry list.  Entry q starts row
// r = key >> row_bits; rows between the previous entry's row and r start at
// q (empty rows included).  Thread m closes the rows after the last entry.
__device__ __forceinline__ void csr_one(const uint64_t *__restrict__ srt, int64_t m, int row_bits,
                                        int64_t n, int32_t *__restrict__ rp,
                                        int32_t *__restrict__ col, int64_t q)
{
    const uint64_t mask = (1ull << row_bits) - 1ull;
    const int64_t prev = q == 0 ? -1 : (int64_t)(srt[q - 1] >> row_bits);
    const int64_t r = q == m ? n : (int64_t)(srt[q] >> row_bits);
    if (q < m) col[q] = (int32_t)(srt[q] & mask);
    for (int64_t rr = prev + 1; rr <= r; ++rr) rp[rr] = (int32_t)q;
}

// ------------------------------------------- segmented build steps
__global__ __launch_bounds__(kBlock) void k_keys_seg(const FrontJob *__restrict__ jobs, int J)
{
    const FrontJob &F = jobs[job_of(jobs, J, blockIdx.x, &FrontJob::b0)];
    const int64_t i = ((int64_t)blockIdx.x - F.b0) * kBlock + threadIdx.x;
    if (i < F.a.n) key_of(F.a, F.pos0, F.lev0, i, F.keys, F.vals);
}

__global__ __launch_bounds__(kBlock) void k_permute_seg(const FrontJob *__restrict__ jobs, int J)
{
    const FrontJob &F = jobs[job_of(jobs, J, blockIdx.x, &FrontJob::b0)];
    const int64_t k = ((int64_t)blockIdx.x - F.b0) * kBlock + threadIdx.x;
    if (k < F.pa.n) permute_one(F.pa, k);
}

// After the permutation: the other position buffer (the source of the
// permutation, which the next iteration writes) takes the D0 of the new
// order, so that iterations need to write only the three coordinates.
__global__ __launch_bounds__(kBlock) void k_d0_copy_seg(const FrontJob *__restrict__ jobs, int J)
{
    const FrontJob &F = jobs[job_of(jobs, J, blockIdx.x, &FrontJob::b0)];
    const int64_t k = ((int64_t)blockIdx.x - F.b0) * kBlock + threadIdx.x;
    if (k < F.pa.n) const_cast<P4 *>(F.pa.ps)[k].d = F.pa.pd[k].d;
}

__global__ __launch_bounds__(kBlock) void k_tables_clear_seg(const FrontJob *__restrict__ jobs,
                                                            int J)
{
    const FrontJob &F = jobs[job_of(jobs, J, blockIdx.x, &FrontJob::bt0)];
    const int64_t i = ((int64_t)blockIdx.x - F.bt0) * kBlock + threadIdx.x;
    if (i < F.hcap) F.a.hash[i].key = kEmptyKey;
    if (i < F.nd2) reinterpret_cast<uint32_t *>(F.a.dense)[i] = 0u;
    if (i == 0) *F.counter = 0ull;
}

__global__ __launch_bounds__(kBlock) void k_cells_seg(const FrontJob *__restrict__ jobs, int J)
{
    const FrontJob &F = jobs[job_of(jobs, J, blockIdx.x, &FrontJob::b0)];
    const int64_t i = ((int64_t)blockIdx.x - F.b0) * kBlock + threadIdx.x;
    if (i < F.a.n) cells_one(F.a, i);
}

__global__ __launch_bounds__(kBlock) void k_csr_seg(const BackJob *__restrict__ jobs, int J)
{
    const BackJob &B = jobs[job_of(jobs, J, blockIdx.x, &BackJob::bc0)];
    const int64_t q = ((int64_t)blockIdx.x - B.bc0) * kBlock + threadIdx.x;
    if (q <= B.m) csr_one(B.srt, B.m, B.row_bits, B.n, B.rp, B.col, q);
}

void launch_keys_seg(const FrontJob *jobs, int J, int64_t nb, hipStream_t s)
{
    if (nb > 0) hipLaunchKernelGGL(k_keys_seg, dim3((unsigned)nb), dim3(kBlock), 0, s, jobs, J);
}

void launch_permute_seg(const FrontJob *jobs, int J, int64_t nb, hipStream_t s)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_permute_seg, dim3((unsigned)nb), dim3(kBlock), 0, s, jobs, J);
    hipLaunchKernelGGL(k_d0_copy_seg, dim3((unsigned)nb), dim3(kBlock), 0, s, jobs, J);
}

void launch_tables_seg(const FrontJob *jobs, int J, int64_t nbt, int64_t nb, hipStream_t s)
{
    if (nbt > 0)
        hipLaunchKernelGGL(k_tables_clear_seg, dim3((unsigned)nbt), dim3(kBlock), 0, s, jobs, J);
    if (nb > 0) hipLaunchKernelGGL(k_cells_seg, dim3((unsigned)nb), dim3(kBlock), 0, s, jobs, J);
}

void launch_csr_seg(const BackJob *jobs, int J, int64_t nbc, hipStream_t s)
{
    if (nbc > 0) hipLaunchKernelGGL(k_csr_seg, dim3((unsigned)nbc), dim3(kBlock), 0, s, jobs, J);
}

// ------------------------------------------------------- statistics
__global__ __launch_bounds__(kBlock) void k_max_degree(int64_t n, const int32_t *__restrict__ rp,
                                                      uint32_t *__restrict__ out)
{
    __shared__ uint32_t wm[kWavesPerBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t d = i < n ? (uint32_t)(rp[i + 1] - rp[i]) : 0u;
    for (int o = kWave / 2; o > 0; o >>= 1) d = max(d, (uint32_t)__shfl_xor(d, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) m = max(m, wm[k]);
        if (m) atomicMax(out, m);
    }
}

void launch_max_degree(int64_t n, const int32_t *rp, uint32_t *out, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_max_degree, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, rp, out);
}

}  // namespace rcp
