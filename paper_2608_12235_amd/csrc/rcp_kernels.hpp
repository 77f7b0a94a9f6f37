// Host-callable launchers of the HIP kernels (internal to the library).
#pragma once
#include "rcp_dev.hpp"

namespace rcp {

// ------------------------------------------------------------ k_sort.hip
// One array of a segmented sort (device descriptor): keys k[0] (values
// v[0], or nullptr) and the second buffers k[1], v[1]; n items in nt =
// ceil(n / 2048) tiles, t0 = tiles of the segments before it.
struct SortSeg {
    uint64_t *k[2];
    uint32_t *v[2];
    int64_t n, t0, nt;
};
constexpr int64_t kSortTile = 2048;
// Stable LSD radix sort of every segment sg[0..nseg) (device memory) on the
// low nbits of its keys, by one sequence of launches over all ntiles
// tiles; returns the buffer index (the same for all segments) that holds
// the result.  hist needs 256 * ntiles entries, totals 256 * nseg.
int radix_sort_segs(const SortSeg *sg, int nseg, int64_t ntiles, int nbits, bool vals,
                    uint32_t *hist, uint32_t *totals, hipStream_t s);
// Write nseg host descriptors to dst (device) in stream order.
void launch_put_segs(SortSeg *dst, const SortSeg *src, int nseg, hipStream_t s);

// -------------------------------------------------------- k_neighbor.hip
struct LevelGrid {
    double inv_w;    // cells per unit length (nc / L); cell = floor(x * inv_w)
    double dmax;     // largest D0 in the class
    int32_t nc;      // cells per axis
    int32_t count;   // particles in the class
    int64_t dbase;   // first entry of the level's dense cell table, -1: hashed
};

// One occupied cell: its key and the run [start, start + count) of sorted
// particles in it; 16 bytes so a probe is one load.
struct alignas(16) HashSlot {
    uint64_t key;
    int32_t start, count;
};

// Everything one segment's list build needs, passed by value.
struct BuildArgs {
    int64_t n;
    int32_t nlev, mb;       // classes; Morton bits below the class field
    int32_t tshift, tiles;  // key bit of the tile field; tiles per axis (power of 2)
    double L, hL, kb, opg, sk2;
    double hLa[3];          // per axis: hL, or +inf on an axis bounded by walls (no image)
    const P4 *pos;
    const uint8_t *lev;
    const uint64_t *skey;   // sorted keys (after the sort)
    struct HashSlot *hash;  // open-addressing table of occupied cells
    uint64_t hmask;
    int2 *dense;            // (start, count) per cell of the dense levels
    LevelGrid lv[kMaxLevels];
};

struct PermArgs {
    int64_t n;
    const uint32_t *perm;
    const P4 *ps;
    P4 *pd;
    float *xref[3];
    const double *ms[3]; double *md[3];
    const double *vs[3]; double *vd[3];
    const int32_t *os; int32_t *od;
    const uint8_t *ls; uint8_t *ld;
};

// One packing of a batch of list builds as the segmented build kernels see
// it (device table, one entry per packing; block ranges are prefixes over
// the batch).
struct FrontJob {
    BuildArgs a;            // geometry, permuted positions / levels, sorted keys, tables
    PermArgs pa;            // the permutation (pa.perm: sorted local indices)
    const P4 *pos0;         // positions before the permutation (keys)
    const uint8_t *lev0;
    uint64_t *keys;         // Morton keys out
    uint32_t *vals;         // local indices out
    unsigned long long *counter;   // search entry count (64-bit, so it cannot wrap),
                                   // zeroed with the tables
    uint64_t *list;         // search output: the list region and its capacity
    int64_t lcap;
    int32_t row_bits, pad;
    int64_t hcap, nd2;      // hash slots and dense words to clear
    int64_t b0;             // first block in the per-particle grids
    int64_t bt0;            // first block in the table-clear grid
};
struct BackJob {
    const uint64_t *srt;    // entries sorted by (row, col)
    int64_t m, n;
    int32_t row_bits, seg;
    int32_t *rp, *col;
    WorkItem *W;            // the packing's work-item slots
    int64_t nslots;
    int32_t row_cost, item_work;
    int32_t fill;           // 1: cut the rows into the slots here
    int32_t cur;
    double kb, disp_lim, kappa_lim;
    SegPtrs ptrs;
    int64_t bc0;            // first block in the entry grid (m + 1 threads a packing)
    int64_t bs0;            // first block in the slot grid
    int64_t br0;            // first block in the row grid
};
// Front steps for all packings of a batch (jobs in device memory): Morton
// keys (nb = blocks of the per-particle grid), permutation (then the D0 of
// the new order into the other position buffer), cell tables (nbt = blocks
// of the clear grid; clears the counters too).
void launch_keys_seg(const FrontJob *jobs, int J, int64_t nb, hipStream_t s);
void launch_permute_seg(const FrontJob *jobs, int J, int64_t nb, hipStream_t s);
void launch_tables_seg(const FrontJob *jobs, int J, int64_t nbt, int64_t nb, hipStream_t s);
// Back steps: rows and columns (nbc blocks), work items (nbs slot blocks,
// nbr row blocks), validity limits and pointer entries.
void launch_csr_seg(const BackJob *jobs, int J, int64_t nbc, hipStream_t s);
void launch_items_seg(const BackJob *jobs, int J, int64_t nbs, int64_t nbr, hipStream_t s);
void launch_after_seg(const BackJob *jobs, int J, SegState *S, SegPtrs *P, hipStream_t s);

// One pass over the particles: every listed pair (i, j) is appended twice
// to `list` as (row << row_bits) | col, rows and cols in sorted order, in an
// arbitrary order; *counter (zeroed by the caller) receives the number of
// entries, which may exceed cap (then only cap were stored).
void launch_search(const BuildArgs &a, uint64_t *list, unsigned long long *counter, int64_t cap,
                   int row_bits, int xcd_remap, hipStream_t s);
// The same, wave-cooperative (the same pairs, another append order), for
// jobs[0..J) (their list, lcap, row_bits and counter fields say where) over
// nb blocks of the per-particle grid starting at block b_base of the batch.
void launch_search_seg(const FrontJob *jobs, int J, int64_t nb, int max_nlev, int xcd_remap,
                       int64_t b_base, hipStream_t s);
// *out = longest row (max rp[i+1] - rp[i]); out must be zeroed first.
void launch_max_degree(int64_t n, const int32_t *rp, uint32_t *out, hipStream_t s);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);

// ---------------------------------------------------------- k_place.hip
// Random sequential addition in rounds (see k_place.hip).
struct alignas(16) PlaceSlot {
    uint64_t key;        // cell key, ~0 when empty
    int32_t head, pad;   // most recently pushed item of the cell (-1: none)
};
struct PlaceGrid {
    int64_t off;         // first slot of the class's table in the arena
    uint64_t mask;       // slots - 1 (a power of two)
    int64_t nc;          // cells per axis
    double inv_w;        // nc / L
    int32_t any, pad;    // the class has spheres
};
constexpr int kPlaceMaxClasses = 64;
struct PlaceArgs {
    int64_t n;
    double L, hL, kappa0;
    uint64_t seed;
    int64_t max_attempts;
    int32_t dim;             // 3, or 2: the z coordinate is 0
    int ncls;
    int32_t walls, round;    // hard walls (see inside_walls); bounded axes have no image
    int32_t pad;
    const int32_t *ord;      // rank -> sphere (largest first)
    const double *d0;        // by sphere
    double *x;               // (n, 3) by sphere: placed positions
    int32_t *att;            // by rank: next attempt
    uint8_t *placed;         // by rank
    int32_t *next;           // by sphere: next sphere of its cell
    PlaceSlot *tab;          // arena of the classes' cell tables
    double *prop;            // window x 3: the round's proposals
    uint8_t *valid;          // window
    int32_t *pnext;          // window: next proposal of its cell
    PlaceSlot *ptab;         // the round's proposal table
    uint64_t pmask;
    int64_t pcap;
    unsigned long long *first;   // lowest rank of the window still unplaced
    int32_t *fail;               // set when a sphere ran out of attempts
    PlaceGrid grid[kPlaceMaxClasses];
};

// Seating of the spheres that are not frozen in the voids of the frozen ones
// (a cascade stage; k_place.hip).  Frozen spheres sorted by cell of an nc^3
// grid: fxd[4 o .. 4 o + 3] = (x, y, z, diameter), cell q holds o in
// [start[q], start[q + 1]).  Sphere gidx[t] (user index, relative diameter
// gd[t]) gets the first proposal of the counter stream that overlaps no
// frozen sphere at the seating scale kappa0, written to x (user order, n x
// 3); *fail is set when one needs more than max_attempts.
struct SeatArgs {
    const double *fxd;
    const int32_t *start;
    const double *gd;
    const int32_t *gidx;
    double *x;
    int32_t *fail;
    int64_t nc;
    double inv_w, L, hL, kappa0;
    uint64_t seed;
    int64_t max_attempts;
    int32_t dim;             // 3, or 2: the z coordinate is 0
};
void launch_seat(const SeatArgs &a, int64_t ng, hipStream_t st);

// Frozen spheres of packing seg: the D0 field of every record in both
// position buffers gets the sign -1 where mask (user order) is set, +1
// elsewhere.
void launch_set_frozen(const SegPtrs *P, int seg, int64_t n, const uint8_t *mask, hipStream_t st);

// One round over ranks [lo, hi) of class c (clear the proposal table,
// propose and validate, resolve conflicts and commit).
void launch_place_round(const PlaceArgs &a, int c, int64_t lo, int64_t hi, hipStream_t st);

// -------------------------------------------------------- k_iterate.hip
// flags bit 0: XCD-aware block order; bit 1: the last block of each packing
// runs its tail (otherwise launch_tail must follow); bit 2: whole 32-byte
// position records written (else the three coordinates only).
// Work items of packing seg (nslots slots at W): rows are cut so that an
// item covers item_work units of row_cost * row + row pointer; rp == nullptr
// leaves every slot empty.
void launch_items(const int32_t *rp, int64_t n, int seg, int row_cost, int item_work,
                  WorkItem *W, int64_t nslots, hipStream_t st);
void launch_iterate(const SegPtrs *P, SegState *S, const WorkItem *W, double *partials,
                    int nitems, int flags, hipStream_t s);
// b0, nb: the work-item range of the only packing when nseg == 1 (its
// layout at launch or capture time), else ignored.
void launch_tail(SegState *S, const double *partials, int nseg, int64_t b0, int64_t nb,
                 hipStream_t s);
// nblocks and bfirst of every packing from lay (2 int64 per packing, device).
void launch_set_layout(SegState *S, int nseg, const int64_t *lay, hipStream_t s);
// Start a schedule on segment seg: copy the table, reset the position in it,
// set the first rung's parameters from the current kappa.
void launch_sched_start(SegState *S, int seg, const SchedDev &q, int reset_adam,
                        int64_t iter_limit, hipStream_t s);
void launch_set_flags(SegState *S, int seg, int32_t clear, int32_t set, hipStream_t s);

// Energy terms / gradient of one segment at positions given in user order
// (xu, n x 3 row-major, device) or at its current state (xu == nullptr).
struct EvalOut {
    double *part;     // per-block partials: E_ov, S_drd, max delta, n_overlap
    double *gu;       // dE/dx in user order (n x 3) or nullptr
};
void launch_eval(const SegPtrs *P, const SegState *S, int seg, int64_t n, const double *xu,
                 double kappa, const EvalOut &o, int nblocks, hipStream_t s);
// Final reduction of launch_eval partials into out[0..5]: E_ov, E_growth,
// gk_ov, gk_growth, max delta, n_overlap (mu and sum D0 given).
void launch_eval_finish(const double *part, int nblocks, double kappa, double mu,
                        const SegState *S, int seg, double *out, hipStream_t s);
// Max displacement^2 of xu (user order, n x 3) against the list's xref.
void launch_disp(const SegPtrs *P, const SegState *S, int seg, int64_t n, const double *xu,
                 double *part, int nblocks, hipStream_t s);
// Adam moments of segment seg to (dir 0) or from (dir 1) user-order arrays
// mu, vu (n x 3 row-major, device).
void launch_moments_io(const SegPtrs *P, int seg, int64_t n, double *mu, double *vu, int dir,
                       hipStream_t s);
// Gather user-order positions xu (n x 3) into the current SoA buffer.
void launch_set_positions(const SegPtrs *P, SegState *S, int seg, int64_t n, const double *xu,
                          int cur, hipStream_t s);
// Scatter the current positions into user order xu (n x 3, device).
void launch_get_positions(const SegPtrs *P, int seg, int64_t n, double *xu, int cur,
                          hipStream_t s);
// Shrink to contact: per-block minima of the pair contact scales in
// part[0..nblocks), their minimum in part[nblocks].
void launch_shrink(const SegPtrs *P, const SegState *S, int seg, int64_t n, double *part,
                   int nblocks, hipStream_t s);
// out[0] = max of part[0..nblocks)
void launch_max_finish(const double *part, int nblocks, double *out, hipStream_t s);

}  // namespace rcp
