// Host runtime of the library: contexts, buffers, the neighbour-list build
// pipeline, the iteration loop (HIP graphs of K iterations, one status read
// per graph), shrink to contact, and the C ABI of include/rcp.h.
#include "rcp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rcp_kernels.hpp"

namespace rcp {
double uniform01(uint64_t seed, uint64_t i, uint64_t attempt, int axis);
void place_uniform(int64_t n, double L, uint64_t seed, int dim, double *x);
int place_rsa(int64_t n, const double *d0, double L, double kappa0, uint64_t seed, int dim,
              int64_t max_attempts, double *x);
}  // namespace rcp

using namespace rcp;

// Events used only to time work on the context's stream: no system-scope
// fence when they are recorded (a fence writes back and invalidates the
// caches, which costs microseconds per event node and slows the launch that
// follows); their readers synchronise the stream first.
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

// ------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(RCP_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

#define CHK(call)                    \
    do {                             \
        int rc_ = (call);            \
        if (rc_ != RCP_OK) return rc_; \
    } while (0)

template <class T>
static int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(RCP_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    return RCP_OK;
}

template <class T>
static void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// grow a device buffer to at least `need` elements (contents discarded)
template <class T>
static int dgrow(T **p, int64_t *cap, int64_t need)
{
    if (need <= *cap && *p) return RCP_OK;
    int64_t c = std::max<int64_t>(need + need / 4, 1024);
    dfree(*p);
    CHK(dalloc(p, (size_t)c));
    *cap = c;
    return RCP_OK;
}

// ------------------------------------------------------------ context
struct Seg {
    int64_t n = 0;
    double L = 0, d0min = 0, d0max = 0, sumd0 = 0, sumd03 = 0, nvol = 0, kappa0 = 1;
    uint64_t seed = 0;
    int nlev = 1;
    std::vector<double> d0h;         // relative diameters (host copy, user order)
    std::vector<double> dmax_upto;   // max D0 over classes <= l
    std::vector<double> dmax_lev;    // max D0 in class l
    std::vector<int64_t> lev_count;
    // device arrays; M, V, ORIG, LEV are double-buffered for the Morton
    // permutation (live set `set`); positions with D0 ping-pong through Q
    P4 *Q[2] = {};
    double *M[2][3] = {}, *V[2][3] = {};
    int32_t *ORIG[2] = {};
    uint8_t *LEV[2] = {};
    float *XREF[3] = {};
    int32_t *rp = nullptr, *col = nullptr;
    int64_t col_cap = 0;
    int set = 0;
    int cur = 0;          // host copy of the live position buffer
    int64_t npairs = 0, nnz = 0, maxdeg = 0, list_est = 0;
    int blocks = 0;              // work-item slots of this packing
    int64_t first_item = 0;      // its first slot in the work table
    int64_t slot_entries = 0;    // list length the slots are sized for
    int64_t rebuilds = 0;
    int err = 0;                 // error that stopped this packing (census)
    bool built = false;
    bool parked = false;         // finished: no work-item slots until its next run
    // frozen spheres (a cascade stage): mask in user order, their D0 is an
    // absolute diameter; sum of D0^3 over the frozen and the other spheres
    bool mixed = false;
    std::vector<uint8_t> frozen;
    double sum3_frozen = 0, sum3_grow = 0;
    // hard walls (rcp_set_boundary): flat walls across the axes of `walls`,
    // a round container over the axes of `round`
    int32_t walls = 0, round = 0;
    // iteration count at the last list build and the length of the last
    // interval between builds (0: not yet known), for the graph length
    int64_t it_build = -1, interval = 0;
};

// A stream for the pair searches of a batch of list builds.
struct BuildLane {
    hipStream_t st = nullptr;
    bool own = false;
    hipEvent_t ev = nullptr;
    int64_t load = 0;                // particles assigned in the current batch
};

constexpr int kBuildLanes = 4;

struct rcp_ctx {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool any_mixed = false;         // some packing has frozen spheres
    bool any_walls = false;         // some packing has hard walls
    int dim = 3;                    // 3, or 2: disks in the plane z = 0
    rcp_params params{};
    rcp_tuning tuning{};
    std::vector<Seg> segs;
    SegPtrs *d_ptrs = nullptr;
    SegState *d_state = nullptr;
    SegState *h_state = nullptr;    // pinned mirror of d_state
    WorkItem *d_work = nullptr;
    int nitems = 0;
    int64_t items_cap = 0;
    double *d_partials = nullptr;
    uint32_t *totals = nullptr;      // small device counters
    // list builds: lane 0 runs on the context's stream, further lanes (for
    // builds of several packings at once) on streams of their own
    std::vector<BuildLane> lanes;
    hipEvent_t fork_ev = nullptr;
    // batch sort buffers: Morton keys and permutations of all packings being
    // built (key and value ping-pong), the second buffer of the entry sort,
    // histograms, digit totals, segment descriptors (device, pinned host)
    uint64_t *skA = nullptr, *skB = nullptr;
    uint32_t *svA = nullptr, *svB = nullptr;
    int64_t skA_cap = 0, skB_cap = 0, svA_cap = 0, svB_cap = 0;
    uint64_t *ltmp = nullptr;
    int64_t ltmp_cap = 0;
    uint32_t *shist = nullptr, *stot = nullptr;
    int64_t shist_cap = 0, stot_cap = 0;
    SortSeg *d_segs = nullptr;
    int64_t segs_cap = 0;
    std::vector<SortSeg> h_segs;
    uint64_t *larena = nullptr;      // list regions of the builds in flight
    int64_t larena_cap = 0;
    HashSlot *harena = nullptr;      // their cell hashes and dense cell tables
    int64_t harena_cap = 0;
    int2 *darena = nullptr;
    int64_t darena_cap = 0;
    FrontJob *d_fj = nullptr, *h_fj = nullptr;   // batch job tables (device, pinned host)
    BackJob *d_bj = nullptr, *h_bj = nullptr;
    int64_t fj_cap = 0, bj_cap = 0, hj_cap = 0;
    unsigned long long *bcount = nullptr;   // their entry counts (device, pinned host)
    int64_t bcount_cap = 0;
    unsigned long long *h_bcount = nullptr;
    int64_t h_bcount_cap = 0;
    double *part = nullptr;          // evaluation partials
    int64_t part_cap = 0;
    double *out = nullptr;           // small device results
    double *xtmp = nullptr;          // staging of user-order positions
    int64_t xtmp_cap = 0;
    double *h_out = nullptr;         // pinned small results
    // iteration graphs by length (see graph_len); graph_valid = false
    // drops them all before the next launch
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    bool graph_valid = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<hipEvent_t> kev;     // per-launch kernel timing events (3 per iteration)
    // rebuild timing: event pairs recorded around list builds, read (and
    // returned to the pool) at the next point where the stream is idle
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rb_pending, rb_pool;
    rcp_stats stats{};
    double *scratch = nullptr;       // this GPU's fixed scratch array (see below)
    int64_t *d_layout = nullptr;     // (blocks, first item) per packing: device,
    int64_t *h_layout = nullptr;     // and pinned host staging
};

static void ptrs_of(const Seg &s, SegPtrs &p)
{
    for (int b = 0; b < 2; ++b) p.p[b] = s.Q[b];
    for (int a = 0; a < 3; ++a) {
        p.m[a] = s.M[s.set][a];
        p.v[a] = s.V[s.set][a];
        p.xref[a] = s.XREF[a];
    }
    p.orig = s.ORIG[s.set];
    p.lev = s.LEV[s.set];
    p.rp = s.rp;
    p.col = s.col;
}

static int rebuild_events(rcp_ctx *c, std::pair<hipEvent_t, hipEvent_t> &ev)
{
    if (!c->rb_pool.empty()) {
        ev = c->rb_pool.back();
        c->rb_pool.pop_back();
        return RCP_OK;
    }
    HIPCHK(hipEventCreateWithFlags(&ev.first, kTimingEvent));
    HIPCHK(hipEventCreateWithFlags(&ev.second, kTimingEvent));
    return RCP_OK;
}

// Add the durations of completed list builds to the statistics.
static void flush_rebuild_times(rcp_ctx *c)
{
    for (auto &ev : c->rb_pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) c->stats.rebuild_ms += ms;
        c->rb_pool.push_back(ev);
    }
    c->rb_pending.clear();
}

static int pull_state(rcp_ctx *c)
{
    HIPCHK(hipMemcpyAsync(c->h_state, c->d_state, sizeof(SegState) * c->segs.size(),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    flush_rebuild_times(c);
    for (size_t k = 0; k < c->segs.size(); ++k) c->segs[k].cur = c->h_state[k].cur;
    return RCP_OK;
}

// write one host-owned field group of a segment's device record
template <class T>
static int put_field(rcp_ctx *c, int k, size_t offset, const T &v)
{
    HIPCHK(hipMemcpyAsync((char *)(c->d_state + k) + offset, &v, sizeof(T),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return RCP_OK;
}

// ------------------------------------------- fixed scratch (no allocation)
// Block partials and small results of rcp_energy_dev_static: a device array
// of this module, one copy per GPU, held until the process ends.  Its name
// is a host-side stand-in; the device address is looked up once per GPU.
constexpr int64_t kScratchBlocks = (int64_t)1 << 16;        // n <= 2^24 spheres
constexpr int64_t kScratchWords = 4 * kScratchBlocks + 64;  // 2 MiB + results
static __device__ __align__(256) double scratch[kScratchWords];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_addr;   // per device index

// Device address of the current GPU's scratch array (hipGetSymbolAddress on
// the first call for that device, with it current).
static int scratch_address(double **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_addr[dev] = (double *)p;
    }
    *out = g_scratch_addr[dev];
    return RCP_OK;
}

// Bound on |x - (double)(float)x| summed over the three axes for positions
// in [0, L), in units of L: sqrt(3) 2^-23 (twice the rounding bound).
constexpr double kXrefErr = 1.7320508075688772 * 0x1p-23;

// ------------------------------------------------------------ work table
// Work-item slots for packing k: enough for row_cost * n + slot_entries
// units of item_work each (see rcp_tuning), plus one.
static int64_t slots_for(const rcp_ctx *c, int64_t n, int64_t entries)
{
    const int64_t rc = c->tuning.row_cost, wk = c->tuning.item_work;
    return (rc * n + entries) / wk + 2;
}

// Cut the rows of a built packing into work items (device kernel on its
// row pointers); items of an unbuilt packing are left empty.
static void fill_items(rcp_ctx *c, int k, hipStream_t st)
{
    Seg &s = c->segs[k];
    WorkItem *w = c->d_work + s.first_item;
    launch_items(s.built ? s.rp : nullptr, s.n, k, c->tuning.row_cost, c->tuning.item_work, w,
                 s.blocks, st);
}

// Lay out the work-item slots of all packings (a graph captured before is
// invalid afterwards) and fill them.
static int build_work(rcp_ctx *c)
{
    int64_t total = 0;
    for (size_t k = 0; k < c->segs.size(); ++k) {
        Seg &s = c->segs[k];
        // a finished packing gets no slots (its blocks would only exit)
        const int64_t nb = s.parked ? 0 : slots_for(c, s.n, s.slot_entries);
        if (nb > (int64_t)INT32_MAX / 4 || total + nb > (int64_t)INT32_MAX / 4)
            return fail(RCP_ENOMEM, "work table too large");
        s.blocks = (int)nb;
        s.first_item = total;
        total += nb;
    }
    if (total > c->items_cap) {
        dfree(c->d_work);
        dfree(c->d_partials);
        c->d_work = nullptr;
        c->d_partials = nullptr;
        CHK(dalloc(&c->d_work, (size_t)total));
        CHK(dalloc(&c->d_partials, 4 * (size_t)total));
        c->items_cap = total;
    }
    c->nitems = (int)total;
    const int ns = (int)c->segs.size();
    for (int k = 0; k < ns; ++k) {
        c->h_layout[2 * k] = c->segs[k].blocks;
        c->h_layout[2 * k + 1] = c->segs[k].first_item;
    }
    HIPCHK(hipMemcpyAsync(c->d_layout, c->h_layout, sizeof(int64_t) * 2 * ns,
                          hipMemcpyHostToDevice, c->stream));
    launch_set_layout(c->d_state, ns, c->d_layout, c->stream);
    for (int k = 0; k < ns; ++k) fill_items(c, k, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->graph_valid = false;
    return RCP_OK;
}

// Packings that have finished for good (stop, cap, non-finite, abort) give
// up their work-item slots once they hold more than an eighth of the table:
// the iteration grid then covers only the packings still running.
static int park_finished(rcp_ctx *c)
{
    if (c->segs.size() < 2) return RCP_OK;
    int64_t freed = 0;
    bool any = false;
    for (size_t k = 0; k < c->segs.size(); ++k) {
        const int32_t f = c->h_state[k].flags;
        if (!c->segs[k].parked && (f & (F_STOP | F_CAP | F_NONFINITE | F_ABORT))) {
            any = true;
            freed += c->segs[k].blocks;
        }
    }
    if (!any || 8 * freed < (int64_t)c->nitems) return RCP_OK;
    for (size_t k = 0; k < c->segs.size(); ++k)
        if (c->h_state[k].flags & (F_STOP | F_CAP | F_NONFINITE | F_ABORT)) c->segs[k].parked = true;
    return build_work(c);
}

// ------------------------------------------------------------ list build
static int bits_for(int64_t v)   // bits needed to hold values 0..v
{
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

// A list build is split at its one host round trip, the entry count of the
// search.  All packings that need a build are built as one batch: their
// Morton keys are sorted by one segmented radix sort (one sequence of
// launches for the batch), then each packing's permutation, cell tables and
// search run on one of up to kBuildLanes streams (each with its own cell
// tables, so small packings' builds run side by side); the entry counts
// come back in one copy; one segmented sort orders every list by (row,
// col), and the rows, work items and validity limits follow per packing.
struct BuildJob {
    int k = 0;
    int lane = 0;
    double kappa = 0.0;
    BuildArgs a;
    int nbits = 0, row_bits = 0;
    int64_t ndense = 0, hcap = 0;
    int64_t lcap = 0, loff = 0;   // list region: entries and offset in the arena
    int64_t koff = 0;             // offset of the packing's keys in the batch key buffers
    int64_t hoff = 0, doff = 0;   // offsets of its hash and dense tables in their arenas
};

// Host arithmetic of a build of packing k at kb = kappa: grid levels, key
// layout, dense / hashed levels, list capacity (at least min_entries).
static int build_plan(rcp_ctx *c, int k, double kappa, int64_t min_entries, BuildJob &j)
{
    const Seg &s = c->segs[k];
    const int64_t n = s.n;
    const double g = c->params.skin_g, sk = c->params.skin_s;
    const double opg = 1.0 + g, sk2 = (2.0 * sk) * s.d0min;
    // with frozen spheres (absolute diameters |D0|, the others kappa D0) the
    // list is built at max(kappa, 1): every cutoff is then at least the
    // contact distance, and the build's growth allowance covers kappa up
    // to (1 + g) times that scale
    if (s.mixed && kappa < 1.0) kappa = 1.0;
    // largest cutoff must stay below half the box (minimum image)
    const double cmax = kappa * (opg * s.d0max + sk2);
    if (!(cmax < 0.5 * s.L))
        return fail(RCP_EBOX, "packing %d: listing cutoff %.17g is not below L/2 = %.17g", k,
                    cmax, 0.5 * s.L);
    j.k = k;
    j.kappa = kappa;
    BuildArgs &a = j.a;
    std::memset(&a, 0, sizeof a);
    a.n = n;
    a.nlev = s.nlev;
    a.L = s.L;
    a.hL = 0.5 * s.L;
    for (int ax = 0; ax < 3; ++ax)   // no image across an axis bounded by walls
        a.hLa[ax] = (((s.walls | s.round) >> ax) & 1) ? INFINITY : 0.5 * s.L;
    a.kb = kappa;
    a.opg = opg;
    a.sk2 = sk2;
    int maxbits = 1;
    for (int l = 0; l < s.nlev; ++l) {
        const double h = kappa * (opg * s.dmax_upto[l] + sk2) * (1.0 + 1e-12);
        int64_t nc = (int64_t)std::floor(s.L / h);
        nc = std::max<int64_t>(1, std::min<int64_t>(nc, (int64_t)1 << 19));
        a.lv[l].nc = (int32_t)nc;
        a.lv[l].inv_w = (double)nc / s.L;
        a.lv[l].dmax = s.dmax_lev[l];
        a.lv[l].count = (int32_t)s.lev_count[l];
        a.lv[l].dbase = -1;
        maxbits = std::max(maxbits, bits_for(nc - 1));
    }
    a.mb = 3 * maxbits;
    // spatial tiles ahead of the class field (see k_neighbor.hip): 4 x 4 x 4
    // when the key has room, else 2 x 2 x 2, else none
    const int lb = bits_for(s.nlev - 1);
    a.tshift = a.mb + lb;
    a.tiles = (a.tshift + 6 <= 63) ? 4 : ((a.tshift + 3 <= 63) ? 2 : 1);
    const int tbits = a.tiles == 4 ? 6 : (a.tiles == 2 ? 3 : 0);
    j.nbits = a.tshift + tbits;
    j.row_bits = std::max(1, bits_for(n - 1));
    // levels whose grid fits a budget of 8 cells a particle get a dense
    // (start, count) table, looked up without hashing; the rest are hashed
    j.ndense = 0;
    const int64_t dense_budget = 8 * n + 65536;
    int64_t nhashed = 0;
    for (int l = 0; l < s.nlev; ++l) {
        const int64_t nc = a.lv[l].nc, cells = nc * nc * nc;
        if (a.lv[l].count > 0 && j.ndense + cells <= dense_budget) {
            a.lv[l].dbase = j.ndense;
            j.ndense += cells;
        } else {
            nhashed += a.lv[l].count;
        }
    }
    // at most a quarter of the slots occupied: a lookup of an absent cell
    // (most lookups on the sparse levels) rarely meets another key and has to
    // follow a probe chain (each step a dependent load)
    j.hcap = 64;
    while (j.hcap < 4 * nhashed) j.hcap <<= 1;
    // the expected list length with room to spare
    j.lcap = std::max<int64_t>({s.list_est + s.list_est / 4, 8 * n, 1024, min_entries});
    return RCP_OK;
}

// Lanes 0..nl-1 exist (lane 0 is the context's stream).
static int ensure_lanes(rcp_ctx *c, int nl)
{
    if (!c->fork_ev) HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    while ((int)c->lanes.size() < nl) {
        BuildLane L;
        if (c->lanes.empty()) {
            L.st = c->stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
            L.own = true;
        }
        const hipError_t e = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming);
        c->lanes.push_back(L);
        HIPCHK(e);
    }
    return RCP_OK;
}

// Grow the lanes' cell tables, the batch key buffers, the list arena and
// the sort scratch for the planned builds (every stream involved is idle:
// buffers may be reallocated).
static int build_grow(rcp_ctx *c, std::vector<BuildJob> &jobs, int nl)
{
    (void)nl;
    int64_t ltot = 0, ntot = 0, tiles = 0, ltiles = 0, htot = 0, dtot = 0;
    for (auto &j : jobs) {
        j.loff = ltot;
        ltot += j.lcap;
        j.koff = ntot;
        ntot += j.a.n;
        j.hoff = htot;
        htot += j.hcap;
        j.doff = dtot;
        dtot += j.ndense;
        tiles += (j.a.n + kSortTile - 1) / kSortTile;
        ltiles += (j.lcap + kSortTile - 1) / kSortTile;
    }
    const int64_t J = (int64_t)jobs.size();
    CHK(dgrow(&c->harena, &c->harena_cap, htot));
    CHK(dgrow(&c->darena, &c->darena_cap, std::max<int64_t>(dtot, 1)));
    CHK(dgrow(&c->d_fj, &c->fj_cap, J));
    CHK(dgrow(&c->d_bj, &c->bj_cap, J));
    if (J > c->hj_cap) {
        if (c->h_fj) (void)hipHostFree(c->h_fj);
        if (c->h_bj) (void)hipHostFree(c->h_bj);
        c->h_fj = nullptr;
        c->h_bj = nullptr;
        c->hj_cap = 0;
        const int64_t cap = std::max<int64_t>(16, 2 * J);
        hipError_t e = hipHostMalloc((void **)&c->h_fj, sizeof(FrontJob) * cap, 0);
        if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_bj, sizeof(BackJob) * cap, 0);
        if (e != hipSuccess) return fail(RCP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        c->hj_cap = cap;
    }
    CHK(dgrow(&c->skA, &c->skA_cap, ntot));
    CHK(dgrow(&c->skB, &c->skB_cap, ntot));
    CHK(dgrow(&c->svA, &c->svA_cap, ntot));
    CHK(dgrow(&c->svB, &c->svB_cap, ntot));
    CHK(dgrow(&c->larena, &c->larena_cap, ltot));
    CHK(dgrow(&c->ltmp, &c->ltmp_cap, ltot));
    CHK(dgrow(&c->shist, &c->shist_cap, 256 * std::max(tiles, ltiles)));
    CHK(dgrow(&c->stot, &c->stot_cap, 256 * J));
    CHK(dgrow(&c->d_segs, &c->segs_cap, J));
    CHK(dgrow(&c->bcount, &c->bcount_cap, J));
    if ((int64_t)c->h_segs.size() < J) c->h_segs.resize(J);
    if (J > c->h_bcount_cap) {
        if (c->h_bcount) (void)hipHostFree(c->h_bcount);
        c->h_bcount = nullptr;
        c->h_bcount_cap = 0;
        const int64_t cap = std::max<int64_t>(64, 2 * J);
        const hipError_t e =
            hipHostMalloc((void **)&c->h_bcount, sizeof(unsigned long long) * cap, 0);
        if (e != hipSuccess) return fail(RCP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
        c->h_bcount_cap = cap;
    }
    return RCP_OK;
}

// Sort the segments h_segs[0..J) (host descriptors: t0 and nt are filled
// in here; they are passed to the device as kernel arguments) on the
// context's stream; *par receives the buffer index holding the results.
static int sort_segments(rcp_ctx *c, int J, int nbits, bool vals, int *par)
{
    int64_t t = 0;
    for (int q = 0; q < J; ++q) {
        c->h_segs[q].t0 = t;
        c->h_segs[q].nt = (c->h_segs[q].n + kSortTile - 1) / kSortTile;
        t += c->h_segs[q].nt;
    }
    launch_put_segs(c->d_segs, c->h_segs.data(), J, c->stream);
    *par = radix_sort_segs(c->d_segs, J, t, nbits, vals, c->shist, c->stot, c->stream);
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

// Lanes 1..nl-1 wait for the context's stream.
static int fork_lanes(rcp_ctx *c, int nl)
{
    if (nl <= 1) return RCP_OK;
    HIPCHK(hipEventRecord(c->fork_ev, c->stream));
    for (int l = 1; l < nl; ++l) HIPCHK(hipStreamWaitEvent(c->lanes[l].st, c->fork_ev, 0));
    return RCP_OK;
}

// Make the context's stream wait for lanes 1..nl-1.
static int join_lanes(rcp_ctx *c, int nl)
{
    for (int l = 1; l < nl; ++l) {
        HIPCHK(hipEventRecord(c->lanes[l].ev, c->lanes[l].st));
        HIPCHK(hipStreamWaitEvent(c->stream, c->lanes[l].ev, 0));
    }
    return RCP_OK;
}

// Front half of a batch of builds: Morton keys at the current positions
// and one segmented sort, the permutation of every per-particle array and
// the cell tables, each as one launch over all packings (job table
// jobs -> c->h_fj, copied to the device), then the pair searches, one per
// packing on its lane, appending every pair in both directions to each
// packing's list region (entry count of jobs[q] in bcount[q]).  Leaves the
// lanes forked.
static int build_fronts(rcp_ctx *c, std::vector<BuildJob> &jobs, int nl)
{
    const int J = (int)jobs.size();
    int nbits = 1;
    for (auto &j : jobs) nbits = std::max(nbits, j.nbits);
    const int spar = ((nbits + 7) / 8) & 1;   // buffer of the sorted keys (n >= 1 always)
    int64_t nb = 0, nbt = 0;
    for (int q = 0; q < J; ++q) {
        BuildJob &j = jobs[q];
        Seg &s = c->segs[j.k];
        FrontJob &F = c->h_fj[q];
        const int cur = s.cur, ncur = cur ^ 1, set = s.set, nset = set ^ 1;
        j.a.pos = s.Q[ncur];
        j.a.lev = s.LEV[nset];
        j.a.skey = (spar ? c->skB : c->skA) + j.koff;
        j.a.hash = c->harena + j.hoff;
        j.a.hmask = (uint64_t)j.hcap - 1;
        j.a.dense = c->darena + j.doff;
        F.a = j.a;
        PermArgs &pa = F.pa;
        pa.n = s.n;
        pa.perm = (spar ? c->svB : c->svA) + j.koff;
        pa.ps = s.Q[cur];
        pa.pd = s.Q[ncur];
        for (int ax = 0; ax < 3; ++ax) {
            pa.xref[ax] = s.XREF[ax];
            pa.ms[ax] = s.M[set][ax];
            pa.md[ax] = s.M[nset][ax];
            pa.vs[ax] = s.V[set][ax];
            pa.vd[ax] = s.V[nset][ax];
        }
        pa.os = s.ORIG[set];
        pa.od = s.ORIG[nset];
        pa.ls = s.LEV[set];
        pa.ld = s.LEV[nset];
        F.pos0 = s.Q[cur];
        F.lev0 = s.LEV[set];
        F.keys = c->skA + j.koff;
        F.vals = c->svA + j.koff;
        F.counter = c->bcount + q;
        F.list = c->larena + j.loff;
        F.lcap = j.lcap;
        F.row_bits = j.row_bits;
        F.pad = 0;
        F.hcap = j.hcap;
        F.nd2 = 2 * j.ndense;
        F.b0 = nb;
        nb += (s.n + kBlock - 1) / kBlock;
        F.bt0 = nbt;
        nbt += (std::max(F.hcap, F.nd2) + kBlock - 1) / kBlock;
        SortSeg &g = c->h_segs[q];
        g.k[0] = c->skA + j.koff;
        g.k[1] = c->skB + j.koff;
        g.v[0] = c->svA + j.koff;
        g.v[1] = c->svB + j.koff;
        g.n = s.n;
        s.set = nset;
        s.cur = ncur;
    }
    HIPCHK(hipMemcpyAsync(c->d_fj, c->h_fj, sizeof(FrontJob) * J, hipMemcpyHostToDevice,
                          c->stream));
    launch_keys_seg(c->d_fj, J, nb, c->stream);
    int par = 0;
    CHK(sort_segments(c, J, nbits, true, &par));
    if (par != spar) return fail(RCP_EDEVICE, "internal: key sort parity");
    launch_permute_seg(c->d_fj, J, nb, c->stream);
    launch_tables_seg(c->d_fj, J, nbt, nb, c->stream);
    // one search launch per packing, spread over the lanes: each packing's
    // grid is split by level and plane when it is small, which a single
    // launch over a large batch would not be
    CHK(fork_lanes(c, nl));
    const bool coop = (c->tuning.variant >> 6) & 1;
    for (int q = 0; q < J; ++q) {
        const BuildJob &j = jobs[q];
        hipStream_t st = c->lanes[j.lane].st;
        if (coop)
            launch_search_seg(c->d_fj + q, 1, (j.a.n + kBlock - 1) / kBlock, j.a.nlev,
                              c->tuning.xcd_remap, c->h_fj[q].b0, st);
        else
            launch_search(j.a, c->larena + j.loff, c->bcount + q, j.lcap, j.row_bits,
                          c->tuning.xcd_remap, st);
    }
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

// Back half for the jobs listed in qs, ms[q] entries in each list region:
// one segmented sort by (row, col) (full rows, partners ascending), then
// row pointers and columns, work items (*relayout when a packing's slots
// are too few: the caller lays out the work table again) and the validity
// limits and pointer entries, each as one launch over the batch (job table
// -> c->h_bj, copied to the device).
static int build_backs(rcp_ctx *c, std::vector<BuildJob> &jobs, const std::vector<int> &qs,
                       const std::vector<int64_t> &ms, bool *relayout)
{
    const int J = (int)qs.size();
    if (J == 0) return RCP_OK;
    int nbits = 1;
    int64_t ltiles = 0;
    for (int r = 0; r < J; ++r) {
        nbits = std::max(nbits, 2 * jobs[qs[r]].row_bits);
        ltiles += (ms[qs[r]] + kSortTile - 1) / kSortTile;
    }
    const int spar = ltiles > 0 ? ((nbits + 7) / 8) & 1 : 0;
    const double sk = c->params.skin_s, opg = 1.0 + c->params.skin_g;
    int64_t nbc = 0, nbs = 0, nbr = 0;
    for (int r = 0; r < J; ++r) {
        const BuildJob &j = jobs[qs[r]];
        const int64_t m = ms[qs[r]];
        Seg &s = c->segs[j.k];
        BackJob &B = c->h_bj[r];
        SortSeg &g = c->h_segs[r];
        g.k[0] = c->larena + j.loff;
        g.k[1] = c->ltmp + j.loff;
        g.v[0] = g.v[1] = nullptr;
        g.n = m;
        B.srt = (spar ? c->ltmp : c->larena) + j.loff;
        B.m = m;
        B.n = s.n;
        B.row_bits = j.row_bits;
        B.seg = j.k;
        B.rp = s.rp;
        B.col = s.col;
        B.W = c->d_work + s.first_item;
        B.nslots = s.blocks;
        B.row_cost = c->tuning.row_cost;
        B.item_work = c->tuning.item_work;
        s.list_est = m;
        s.built = true;
        // the work table holds this list's items; it is laid out again when
        // it is too small, or more than twice too large (idle items still
        // cost a launch slot and a partial for the tail to read)
        B.fill = (slots_for(c, s.n, m) <= s.blocks && slots_for(c, s.n, 2 * m) >= s.blocks) ? 1 : 0;
        if (!B.fill) {
            s.slot_entries = m + m / 4;
            *relayout = true;
        }
        B.cur = s.cur;
        B.kb = j.kappa;
        // the list-reference positions are kept in float: a coordinate in
        // [0, L) is off by at most L 2^-24, so the displacement allowance
        // shrinks by sqrt(3) L 2^-23 (never below zero: then every
        // iteration asks for a build, which is slow but sound)
        B.disp_lim = std::max(0.0, sk * j.kappa * s.d0min * (1.0 - 1e-9) - kXrefErr * s.L);
        B.kappa_lim = opg * j.kappa * (1.0 - 1e-12);
        ptrs_of(s, B.ptrs);
        B.bc0 = nbc;
        nbc += (m + 1 + kBlock - 1) / kBlock;
        B.bs0 = nbs;
        nbs += (s.blocks + kBlock - 1) / kBlock;
        B.br0 = nbr;
        nbr += (s.n + kBlock - 1) / kBlock;
        s.npairs = m / 2;
        s.nnz = m;
        s.rebuilds += 1;
        c->stats.rebuilds += 1;
    }
    HIPCHK(hipMemcpyAsync(c->d_bj, c->h_bj, sizeof(BackJob) * J, hipMemcpyHostToDevice,
                          c->stream));
    int par = 0;
    CHK(sort_segments(c, J, nbits, false, &par));
    if (par != spar) return fail(RCP_EDEVICE, "internal: entry sort parity");
    launch_csr_seg(c->d_bj, J, nbc, c->stream);
    launch_items_seg(c->d_bj, J, nbs, nbr, c->stream);
    launch_after_seg(c->d_bj, J, c->d_state, c->d_ptrs, c->stream);
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

// A list of m entries (each pair twice) is addressed with 32-bit row
// pointers and partner indices: longer lists are refused.
static int check_list_size(int k, int64_t m)
{
    if (m > (int64_t)INT32_MAX)
        return fail(RCP_ENOMEM,
                    "packing %d: neighbour list of %lld entries exceeds 2^31 - 1 (reduce the "
                    "listing skin)",
                    k, (long long)m);
    return RCP_OK;
}

// Build the lists of packings ks[i] at kb = kappas[i], sharing one host
// round trip.  rcs[i] receives each packing's status (RCP_EBOX leaves that
// packing untouched); the return value is the first error that is not a
// per-packing RCP_EBOX.
static int rebuild_batch(rcp_ctx *c, const std::vector<int> &ks, const std::vector<double> &kappas,
                         std::vector<int> &rcs)
{
    rcs.assign(ks.size(), RCP_OK);
    std::vector<BuildJob> jobs;
    for (size_t i = 0; i < ks.size(); ++i) {
        BuildJob j;
        const int rc = build_plan(c, ks[i], kappas[i], 0, j);
        if (rc == RCP_EBOX) {
            rcs[i] = rc;
            continue;
        }
        CHK(rc);
        jobs.push_back(j);
    }
    if (jobs.empty()) return RCP_OK;
    // lanes: largest packings first, each to the least loaded lane
    const int nl = (int)std::min<size_t>(kBuildLanes, jobs.size());
    CHK(ensure_lanes(c, nl));
    std::vector<int> order(jobs.size());
    for (size_t q = 0; q < jobs.size(); ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return jobs[x].a.n > jobs[y].a.n; });
    for (int l = 0; l < nl; ++l) c->lanes[l].load = 0;
    for (int q : order) {
        int best = 0;
        for (int l = 1; l < nl; ++l)
            if (c->lanes[l].load < c->lanes[best].load) best = l;
        jobs[q].lane = best;
        c->lanes[best].load += jobs[q].a.n;
    }
    CHK(build_grow(c, jobs, nl));
    std::pair<hipEvent_t, hipEvent_t> ev;
    CHK(rebuild_events(c, ev));
    HIPCHK(hipEventRecord(ev.first, c->stream));
    CHK(build_fronts(c, jobs, nl));
    CHK(join_lanes(c, nl));
    HIPCHK(hipMemcpyAsync(c->h_bcount, c->bcount, sizeof(unsigned long long) * jobs.size(),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipGetLastError());
    // columns sized before any back half is queued
    std::vector<int64_t> ms(jobs.size());
    std::vector<int> ok, redo;
    for (size_t q = 0; q < jobs.size(); ++q) {
        ms[q] = (int64_t)c->h_bcount[q];
        // row pointers, partner indices and work-item offsets are 32-bit
        CHK(check_list_size(jobs[q].k, ms[q]));
        if (ms[q] > jobs[q].lcap) {
            redo.push_back((int)q);
            continue;
        }
        ok.push_back((int)q);
        Seg &s = c->segs[jobs[q].k];
        if (ms[q] > s.col_cap) {
            dfree(s.col);
            s.col_cap = std::max<int64_t>(ms[q] + ms[q] / 4, 1024);
            CHK(dalloc(&s.col, (size_t)s.col_cap));
        }
    }
    bool relayout = false;
    CHK(build_backs(c, jobs, ok, ms, &relayout));
    // a list that outgrew its region is built again on its own, sized for
    // the count just seen (its particles are already in list order, so the
    // second sort keeps that order and the list is the same)
    for (int q : redo) {
        std::vector<BuildJob> one(1);
        CHK(build_plan(c, jobs[q].k, jobs[q].kappa, ms[q], one[0]));
        one[0].lane = 0;
        HIPCHK(hipStreamSynchronize(c->stream));
        CHK(build_grow(c, one, 1));
        CHK(build_fronts(c, one, 1));
        HIPCHK(hipMemcpyAsync(c->h_bcount, c->bcount, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        std::vector<int64_t> m1(1, (int64_t)c->h_bcount[0]);
        CHK(check_list_size(jobs[q].k, m1[0]));
        if (m1[0] > one[0].lcap) return fail(RCP_ENOMEM, "pair list overflow after regrowth");
        Seg &s = c->segs[jobs[q].k];
        if (m1[0] > s.col_cap) {
            dfree(s.col);
            s.col_cap = std::max<int64_t>(m1[0] + m1[0] / 4, 1024);
            CHK(dalloc(&s.col, (size_t)s.col_cap));
        }
        CHK(build_backs(c, one, std::vector<int>{0}, m1, &relayout));
    }
    HIPCHK(hipEventRecord(ev.second, c->stream));
    c->rb_pending.push_back(ev);
    if (relayout) CHK(build_work(c));
    return RCP_OK;
}

// Build the list of segment k at its current positions with kb = kappa.
static int rebuild(rcp_ctx *c, int k, double kappa)
{
    std::vector<int> rcs;
    CHK(rebuild_batch(c, {k}, {kappa}, rcs));
    return rcs[0];
}

// ------------------------------------------------------------ iteration loop
static int ensure_kernel_events(rcp_ctx *c, int K);

// Record event e on the context's stream.  While the stream is being
// captured, a plain hipEventRecord leaves no node in the graph, so the event
// node is added to the capture graph explicitly after the current capture
// dependencies, and becomes the new dependency.
static int record_event(rcp_ctx *c, hipEvent_t e)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t cg = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    HIPCHK(hipStreamGetCaptureInfo_v2(c->stream, &cs, &id, &cg, &deps, &nd));
    if (cs != hipStreamCaptureStatusActive) {
        HIPCHK(hipEventRecord(e, c->stream));
        return RCP_OK;
    }
    hipGraphNode_t node;
    HIPCHK(hipGraphAddEventRecordNode(&node, cg, deps, nd, e));
    HIPCHK(hipStreamUpdateCaptureDependencies(c->stream, &node, 1,
                                              hipStreamSetCaptureDependencies));
    return RCP_OK;
}

// Launches that carry timing events: the middle one of every batch of
// graph_iters (time_kernels = 1; away from the host synchronisation that
// precedes a batch) or all of them (time_kernels = 2).
static bool slot_timed(const rcp_ctx *c, int64_t slot)
{
    const int64_t mid = std::max(1, c->tuning.graph_iters) / 2;
    return slot >= 0 && (c->tuning.time_kernels == 2 || (c->tuning.time_kernels == 1 && slot == mid));
}

// Launch flags of the gradient + Adam kernel from the tuning (see
// launch_iterate; the fused tail is added by the callers that use it).
static int iterate_flags(const rcp_ctx *c)
{
    return (c->tuning.xcd_remap ? 1 : 0) | ((c->tuning.variant & 128) ? 4 : 0) |
           (c->any_mixed ? 16 : 0) | (c->any_walls ? 32 : 0) | (c->dim == 2 ? 64 : 0) |
           ((c->tuning.variant & 63) << 8);
}

// The tail runs inside the gradient kernel only when asked for and when no
// packing has frozen spheres or walls and the packings are 3-D (the other
// kernels have no fused tail).
static bool tail_fused(const rcp_ctx *c)
{
    return c->tuning.fused_tail && !c->any_mixed && !c->any_walls && c->dim == 3;
}

// One iteration: gradient + Adam kernel and tail kernel, bracketed by the
// slot's three events when the slot is timed.
static int launch_one_iteration(rcp_ctx *c, int slot)
{
    const int flags = iterate_flags(c) | (tail_fused(c) ? 2 : 0);
    const bool timed = slot_timed(c, slot) && 3 * slot + 2 < (int)c->kev.size();
    if (timed) CHK(record_event(c, c->kev[3 * slot]));
    if (c->nitems > 0)
        launch_iterate(c->d_ptrs, c->d_state, c->d_work, c->d_partials, c->nitems, flags,
                       c->stream);
    if (timed) CHK(record_event(c, c->kev[3 * slot + 1]));
    if (!tail_fused(c))
        launch_tail(c->d_state, c->d_partials, (int)c->segs.size(), c->segs[0].first_item,
                    c->segs[0].blocks, c->stream);
    if (timed) CHK(record_event(c, c->kev[3 * slot + 2]));
    return RCP_OK;
}

// Events for timing K launches (created once, reused by every graph).
static int ensure_kernel_events(rcp_ctx *c, int K)
{
    while ((int)c->kev.size() < 3 * K) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, kTimingEvent));
        c->kev.push_back(e);
    }
    return RCP_OK;
}

// Accumulate the durations of the timed launches among the first `worked`.
static void add_kernel_times(rcp_ctx *c, int64_t worked, int64_t nnz)
{
    for (int64_t b = 0; b < worked && 3 * b + 2 < (int64_t)c->kev.size(); ++b) {
        if (!slot_timed(c, b)) continue;
        float a = 0, t = 0;
        (void)hipEventElapsedTime(&a, c->kev[3 * b], c->kev[3 * b + 1]);
        (void)hipEventElapsedTime(&t, c->kev[3 * b + 1], c->kev[3 * b + 2]);
        c->stats.kernel_ms += a;
        c->stats.tail_kernel_ms += t;
        c->stats.kernel_launches += 1;
        c->stats.kernel_nnz += nnz;
    }
}

static bool seg_done(int32_t f);

// The graph of K iterations, captured on first use (every graph is dropped
// when the launch layout or the tuning changes).
static int graph_for(rcp_ctx *c, int K, hipGraphExec_t *out)
{
    if (!c->graph_valid) {
        for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
        c->graphs.clear();
        c->graph_valid = true;
    }
    for (auto &g : c->graphs)
        if (g.first == K) {
            *out = g.second;
            return RCP_OK;
        }
    if (c->tuning.time_kernels) CHK(ensure_kernel_events(c, std::max(1, c->tuning.graph_iters)));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    int rc = RCP_OK;
    for (int it = 0; it < K && rc == RCP_OK; ++it) rc = launch_one_iteration(c, it);
    const hipError_t ee = hipStreamEndCapture(c->stream, &g);
    if (rc != RCP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ee != hipSuccess) return fail(RCP_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    hipGraphExec_t x = nullptr;
    hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(RCP_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    c->graphs.push_back({K, x});
    *out = x;
    return RCP_OK;
}

// Graph lengths a context keeps: the tuning's K, and the powers of two from
// kMinGraph below it.
constexpr int kMinGraph = 8;

// Iterations of the next graph launch.  A packing whose list needs a
// rebuild idles for the rest of the graph (the host rebuilds between
// launches), so the launch is cut to about the iterations the busiest
// packing still has before its next build: its last interval between
// builds less the iterations since, or before a second build the
// displacement allowance left at the displacement rate so far (and no more
// than the iterations left before any limit); then the largest kept length
// not above that, at least kMinGraph.  Results do not depend on it, only
// how many launches idle.
static int graph_len(const rcp_ctx *c, int K)
{
    if (K <= kMinGraph) return K;
    int64_t want = 0;
    for (size_t k = 0; k < c->segs.size(); ++k) {
        const SegState &h = c->h_state[k];
        if (seg_done(h.flags)) continue;
        const Seg &s = c->segs[k];
        const int64_t since = s.it_build >= 0 ? h.iters - s.it_build : 0;
        int64_t r = K;
        if (s.interval > 0 && s.it_build >= 0) {
            r = s.interval - since;
        } else if (since > 0 && h.max_disp2 > 0.0 && h.disp_lim > 0.0) {
            const double d = std::sqrt(h.max_disp2);
            const double est = d < h.disp_lim ? (double)since * (h.disp_lim / d - 1.0) : 0.0;
            r = est < (double)K ? (int64_t)est : K;
        }
        if (h.iter_limit > 0) r = std::min<int64_t>(r, h.iter_limit - h.iters);
        want = std::max(want, r);
    }
    if (want >= K) return K;
    int G = kMinGraph;
    while (2 * G <= want && 2 * G < K) G *= 2;
    return G;
}

static bool seg_done(int32_t f)
{
    return (f & (F_STOP | F_CAP | F_NONFINITE | F_HOLD | F_ABORT)) != 0;
}

// Iterate every packing until each is done (stop, cap, non-finite, limit).
static int run_loop(rcp_ctx *c)
{
    const int K = std::max(1, c->tuning.graph_iters);
    CHK(pull_state(c));
    for (;;) {
        bool any = false;
        std::vector<int> ks;
        std::vector<double> kap;
        for (size_t k = 0; k < c->segs.size(); ++k) {
            const int32_t f = c->h_state[k].flags;
            if (seg_done(f)) continue;
            if (f & (F_REBUILD | F_STALE)) {
                ks.push_back((int)k);
                kap.push_back(c->h_state[k].kappa);
            }
            any = true;
        }
        if (!any) break;
        if (!ks.empty()) {
            std::vector<int> rcs;
            CHK(rebuild_batch(c, ks, kap, rcs));
            for (size_t i = 0; i < ks.size(); ++i) {
                if (rcs[i] == RCP_OK) {
                    Seg &sg = c->segs[ks[i]];
                    const int64_t it = c->h_state[ks[i]].iters;
                    if (sg.it_build >= 0 && it > sg.it_build) sg.interval = it - sg.it_build;
                    sg.it_build = it;
                    continue;
                }
                if (c->segs.size() == 1) return rcs[i];
                // one packing outgrew its box: stop it, let the others run
                const int k = ks[i];
                c->segs[k].err = rcs[i];
                launch_set_flags(c->d_state, k, 0, F_ABORT, c->stream);
                c->h_state[k].flags |= F_ABORT;
            }
            any = false;
            for (size_t k = 0; k < c->segs.size(); ++k)
                if (!seg_done(c->h_state[k].flags)) any = true;
            if (!any) break;
        }
        int64_t before = 0;
        for (size_t k = 0; k < c->segs.size(); ++k) before += c->h_state[k].iters;
        if (c->tuning.time_kernels) CHK(ensure_kernel_events(c, K));
        const int G = graph_len(c, K);
        HIPCHK(hipEventRecord(c->e0, c->stream));
        if (K > 1) {
            hipGraphExec_t gx = nullptr;
            CHK(graph_for(c, G, &gx));
            HIPCHK(hipGraphLaunch(gx, c->stream));
            c->stats.graph_launches += 1;
        } else {
            CHK(launch_one_iteration(c, 0));
        }
        HIPCHK(hipEventRecord(c->e1, c->stream));
        std::vector<int64_t> prev(c->segs.size());
        for (size_t k = 0; k < c->segs.size(); ++k) prev[k] = c->h_state[k].iters;
        CHK(pull_state(c));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, c->e0, c->e1));
        c->stats.iterate_ms += ms;
        CHK(park_finished(c));
        int64_t worked = 0, nnz = 0;
        for (size_t k = 0; k < c->segs.size(); ++k) {
            const int64_t d = c->h_state[k].iters - prev[k];
            c->stats.iterations += d;
            c->stats.particle_updates += d * c->segs[k].n;
            worked = std::max(worked, d);
            if (d > 0) nnz += c->segs[k].nnz;
        }
        // a packing runs consecutive launches until it goes idle, so the
        // first `worked` launches of this batch did work
        if (c->tuning.time_kernels) add_kernel_times(c, std::min<int64_t>(worked, K > 1 ? G : 1), nnz);
        (void)before;
    }
    return RCP_OK;
}

static int to_sched(const rcp_schedule *q, SchedDev &d)
{
    if (!q || q->size != sizeof(rcp_schedule)) return fail(RCP_EINVAL, "schedule: bad size field");
    if (q->n_rungs < 1 || q->n_rungs > RCP_MAX_RUNGS)
        return fail(RCP_EINVAL, "schedule: n_rungs %d out of [1, %d]", q->n_rungs, RCP_MAX_RUNGS);
    std::memset(&d, 0, sizeof d);
    d.n_rungs = q->n_rungs;
    d.absolute = q->absolute;
    d.tol = q->tol;
    for (int r = 0; r < q->n_rungs; ++r) {
        if (q->budget[r] < 1) return fail(RCP_EINVAL, "schedule: budget[%d] < 1", r);
        if (!std::isfinite(q->mu[r]) || !(q->eta_x[r] >= 0) || !(q->eta_k[r] >= 0) ||
            !(q->decay[r] > 0))
            return fail(RCP_EINVAL, "schedule: rung %d has a bad value", r);
        d.mu[r] = q->mu[r];
        d.eta_x[r] = q->eta_x[r];
        d.eta_k[r] = q->eta_k[r];
        d.decay[r] = q->decay[r];
        d.budget[r] = q->budget[r];
    }
    return RCP_OK;
}

static int reset_moments(rcp_ctx *c, int k)
{
    Seg &s = c->segs[k];
    for (int a = 0; a < 3; ++a) {
        launch_fill_f64(s.M[s.set][a], s.n, 0.0, c->stream);
        launch_fill_f64(s.V[s.set][a], s.n, 0.0, c->stream);
    }
    return RCP_OK;
}

// Volume (area in two dimensions) of packing k's domain: L per plain or
// flat-walled axis, the disk or ball of diameter L over the round axes.
static double domain_volume(const rcp_ctx *c, const Seg &s)
{
    int nr = 0;
    double v = 1.0;
    for (int a = 0; a < c->dim; ++a) {
        if ((s.round >> a) & 1) ++nr;
        else v = v * s.L;
    }
    if (nr == 2) v = v * ((M_PI / 4.0) * (s.L * s.L));
    if (nr == 3) v = v * ((M_PI / 6.0) * (s.L * s.L * s.L));
    return v;
}

static int shrink_seg(rcp_ctx *c, int k, double *kp_out, double *phi_out)
{
    CHK(pull_state(c));
    if (c->segs[k].mixed) {
        // a cascade stage: no shrink (the release that follows starts from
        // this state); phi from the frozen diameters and kappa D0 of the rest
        const Seg &s = c->segs[k];
        const double kp = c->h_state[k].kappa;
        *kp_out = kp;
        *phi_out = c->dim == 2 ? (M_PI / 4.0) * (s.sum3_frozen + kp * kp * s.sum3_grow) /
                                     (s.L * s.L)
                               : (M_PI / 6.0) * (s.sum3_frozen + kp * kp * kp * s.sum3_grow) /
                                     (s.L * s.L * s.L);
        return RCP_OK;
    }
    if (c->h_state[k].flags & (F_REBUILD | F_STALE)) CHK(rebuild(c, k, c->h_state[k].kappa));
    Seg &s = c->segs[k];
    const int nb = (int)std::max<int64_t>(1, (s.n + kBlock - 1) / kBlock);
    CHK(dgrow(&c->part, &c->part_cap, 4 * (int64_t)nb + 8));
    HIPCHK(hipEventRecord(c->e0, c->stream));
    launch_shrink(c->d_ptrs, c->d_state, k, s.n, c->part, nb, c->stream);
    HIPCHK(hipEventRecord(c->e1, c->stream));
    double kmin = 0;
    HIPCHK(hipMemcpyAsync(&kmin, c->part + nb, sizeof kmin, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->e0, c->e1));
    c->stats.shrink_ms += ms;
    const double kappa = c->h_state[k].kappa;
    const double kp = std::min(kappa, kmin);
    *kp_out = kp;
    // the volume fraction; the area fraction in two dimensions (over the
    // container's volume: L^d for a box, periodic or walled)
    *phi_out = c->dim == 2 ? (M_PI / 4.0) * (kp * kp) * s.sumd03 / domain_volume(c, s)
                           : (M_PI / 6.0) * (kp * kp * kp) * s.sumd03 / domain_volume(c, s);
    return RCP_OK;
}

// State in three coordinates per sphere (the boundary calls convert from and
// to (n, dim)).
static int set_state3(rcp_ctx *c, int k, const double *x, double kappa, int is_device);
static int get_state3(rcp_ctx *c, int k, double *x, double *kappa, double *diam);

// ------------------------------------------------------------ placement
// Random sequential addition in rounds on the device (k_place.hip) for
// packing k; the positions then replace the packing's state as
// rcp_set_state does (at its current kappa).
static int place_device(rcp_ctx *c, int k, uint64_t seed, int64_t window, int64_t max_attempts,
                        int64_t *rounds)
{
    CHK(pull_state(c));
    Seg &s = c->segs[k];
    const int64_t n = s.n;
    const std::vector<double> &d0 = s.d0h;
    const double kappa = c->h_state[k].kappa;   // placement at the current scale
    // ranks: largest first, ties by index; classes floor(log2(D0 / D0_min))
    std::vector<int32_t> ord(n);
    for (int64_t i = 0; i < n; ++i) ord[i] = (int32_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return d0[a] > d0[b]; });
    std::vector<int> cls(n);
    int ncls = 1;
    for (int64_t r = 0; r < n; ++r) {
        int e;
        std::frexp(d0[ord[r]] / s.d0min, &e);
        cls[r] = std::max(0, e - 1);
        ncls = std::max(ncls, cls[r] + 1);
    }
    if (ncls > kPlaceMaxClasses) return fail(RCP_EINVAL, "size ratio too large for placement");
    std::vector<int64_t> count(ncls, 0);
    std::vector<double> dmax(ncls, 0.0);
    for (int64_t r = 0; r < n; ++r) {
        count[cls[r]]++;
        dmax[cls[r]] = std::max(dmax[cls[r]], d0[ord[r]]);
    }
    PlaceArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = n;
    a.L = s.L;
    a.hL = 0.5 * s.L;
    a.kappa0 = kappa;
    a.seed = seed;
    a.max_attempts = max_attempts;
    a.dim = c->dim;
    a.ncls = ncls;
    a.walls = s.walls;
    a.round = s.round;
    int64_t tcap = 0;
    for (int q = 0; q < ncls; ++q) {
        PlaceGrid &g = a.grid[q];
        const double h = kappa * dmax[q] * (1.0 + 1e-12);
        int64_t nc = h > 0 ? (int64_t)std::floor(s.L / h) : 1;
        nc = std::max<int64_t>(1, std::min<int64_t>(nc, (int64_t)1 << 20));
        g.nc = nc;
        g.inv_w = (double)nc / s.L;
        g.any = count[q] > 0;
        uint64_t cap = 16;
        while (cap < (uint64_t)(2 * count[q] + 2)) cap <<= 1;
        g.off = tcap;
        g.mask = cap - 1;
        tcap += (int64_t)cap;
    }
    const int64_t W = std::max<int64_t>(1, std::min<int64_t>(window, n));
    uint64_t pc = 16;
    while (pc < (uint64_t)(2 * W)) pc <<= 1;
    a.pcap = (int64_t)pc;
    a.pmask = pc - 1;
    // device buffers for the placement only
    int32_t *d_ord = nullptr, *d_att = nullptr, *d_next = nullptr, *d_pnext = nullptr,
            *d_fail = nullptr;
    double *d_d0 = nullptr, *d_x = nullptr, *d_prop = nullptr;
    uint8_t *d_placed = nullptr, *d_valid = nullptr;
    PlaceSlot *d_tab = nullptr, *d_ptab = nullptr;
    unsigned long long *d_first = nullptr;
    auto release = [&]() {
        dfree(d_ord); dfree(d_att); dfree(d_next); dfree(d_pnext); dfree(d_fail);
        dfree(d_d0); dfree(d_x); dfree(d_prop); dfree(d_placed); dfree(d_valid);
        dfree(d_tab); dfree(d_ptab); dfree(d_first);
    };
    int rc = RCP_OK;
    do {
        if ((rc = dalloc(&d_ord, n)) || (rc = dalloc(&d_att, n)) || (rc = dalloc(&d_next, n)) ||
            (rc = dalloc(&d_pnext, W)) || (rc = dalloc(&d_fail, 1)) || (rc = dalloc(&d_d0, n)) ||
            (rc = dalloc(&d_x, 3 * n)) || (rc = dalloc(&d_prop, 3 * W)) ||
            (rc = dalloc(&d_placed, n)) || (rc = dalloc(&d_valid, W)) ||
            (rc = dalloc(&d_tab, tcap)) || (rc = dalloc(&d_ptab, a.pcap)) ||
            (rc = dalloc(&d_first, 1)))
            break;
        hipError_t e = hipMemcpyAsync(d_ord, ord.data(), sizeof(int32_t) * n,
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_d0, d0.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                               c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(d_att, 0, sizeof(int32_t) * n, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(d_placed, 0, n, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(d_fail, 0, sizeof(int32_t), c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(d_tab, 0xff, sizeof(PlaceSlot) * tcap, c->stream);
        if (e != hipSuccess) {
            rc = fail(RCP_EDEVICE, "placement set-up: %s", hipGetErrorString(e));
            break;
        }
        a.ord = d_ord;
        a.d0 = d_d0;
        a.x = d_x;
        a.att = d_att;
        a.placed = d_placed;
        a.next = d_next;
        a.tab = d_tab;
        a.prop = d_prop;
        a.valid = d_valid;
        a.pnext = d_pnext;
        a.ptab = d_ptab;
        a.first = d_first;
        a.fail = d_fail;
        int64_t nround = 0;
        int64_t cb = 0;
        while (cb < n && rc == RCP_OK) {
            int64_t ce = cb;
            while (ce < n && cls[ce] == cls[cb]) ++ce;
            int64_t lo = cb;
            while (lo < ce) {
                const int64_t hi = std::min(lo + W, ce);
                unsigned long long h_hi = (unsigned long long)hi;
                if ((e = hipMemcpyAsync(d_first, &h_hi, sizeof h_hi, hipMemcpyHostToDevice,
                                        c->stream)) != hipSuccess)
                    break;
                launch_place_round(a, cls[cb], lo, hi, c->stream);
                unsigned long long first = 0;
                int32_t failed = 0;
                if ((e = hipGetLastError()) != hipSuccess ||
                    (e = hipMemcpyAsync(&first, d_first, sizeof first, hipMemcpyDeviceToHost,
                                        c->stream)) != hipSuccess ||
                    (e = hipMemcpyAsync(&failed, d_fail, sizeof failed, hipMemcpyDeviceToHost,
                                        c->stream)) != hipSuccess ||
                    (e = hipStreamSynchronize(c->stream)) != hipSuccess)
                    break;
                ++nround;
                if (failed) {
                    rc = fail(RCP_EPLACE, "packing %d: a sphere exceeded %lld placement attempts",
                              k, (long long)max_attempts);
                    break;
                }
                lo = (int64_t)first;
            }
            if (e != hipSuccess && rc == RCP_OK)
                rc = fail(RCP_EDEVICE, "placement: %s", hipGetErrorString(e));
            cb = ce;
        }
        if (rc != RCP_OK) break;
        if (rounds) *rounds = nround;
        rc = set_state3(c, k, d_x, kappa, 1);
    } while (0);
    const hipError_t se = hipStreamSynchronize(c->stream);
    release();
    if (rc == RCP_OK && se != hipSuccess)
        return fail(RCP_EDEVICE, "placement: %s", hipGetErrorString(se));
    return rc;
}

// ------------------------------------------------------------ creation
static int validate_seg(int64_t n, const double *d0, double L, double kappa0)
{
    if (n <= 0) return fail(RCP_EINVAL, "n must be positive");
    // positions are gathered with 32-bit byte offsets (32 bytes a sphere)
    if (n >= (int64_t)1 << 27) return fail(RCP_EINVAL, "n too large (limit 2^27 - 1)");
    if (!d0) return fail(RCP_EINVAL, "null diameter list");
    if (!(L > 0) || !std::isfinite(L)) return fail(RCP_EINVAL, "box edge must be positive");
    if (!(kappa0 > 0) || !std::isfinite(kappa0)) return fail(RCP_EINVAL, "kappa0 must be positive");
    for (int64_t i = 0; i < n; ++i)
        if (!(d0[i] > 0) || !std::isfinite(d0[i]))
            return fail(RCP_EINVAL, "diameter %lld is not a positive finite number", (long long)i);
    return RCP_OK;
}

static int seg_setup(rcp_ctx *c, int k, int64_t n, const double *d0, double L, double kappa0,
                     uint64_t seed, int init_mode)
{
    Seg &s = c->segs[k];
    s.n = n;
    s.L = L;
    s.kappa0 = kappa0;
    s.seed = seed;
    s.d0h.assign(d0, d0 + n);
    s.d0min = d0[0];
    s.d0max = d0[0];
    double sum = 0, cs = 0, sum3 = 0, cs3 = 0, sum6 = 0, cs6 = 0;   // Neumaier sums
    auto nadd = [](double &acc, double &comp, double v) {
        double t = acc + v;
        if (std::fabs(acc) >= std::fabs(v)) comp += (acc - t) + v;
        else comp += (v - t) + acc;
        acc = t;
    };
    for (int64_t i = 0; i < n; ++i) {
        s.d0min = std::min(s.d0min, d0[i]);
        s.d0max = std::max(s.d0max, d0[i]);
        nadd(sum, cs, d0[i]);
        // D0^d: the volume (area in two dimensions) of a sphere up to a constant
        const double c3 = c->dim == 2 ? d0[i] * d0[i] : d0[i] * d0[i] * d0[i];
        nadd(sum3, cs3, c3);
        nadd(sum6, cs6, c3 * c3);
    }
    s.sumd0 = sum + cs;
    s.sumd03 = sum3 + cs3;
    s.nvol = (s.sumd03 * s.sumd03) / (sum6 + cs6);
    const double opg = 1.0 + c->params.skin_g, sk2 = (2.0 * c->params.skin_s) * s.d0min;
    if (!(kappa0 * (opg * s.d0max + sk2) < 0.5 * L))
        return fail(RCP_EBOX, "packing %d: listing cutoff at kappa0 is not below L/2", k);
    // size classes: class floor(log2(D0 / D0_min) / p); consecutive classes
    // share a level (one grid) while the level's cell width, kappa ((1 + g)
    // max D0 + 2 s D0_min), stays within twice that of its first class, so a
    // skin that dominates the small classes' cutoffs does not leave several
    // nearly identical, sparsely filled grids to be searched
    const int p = std::max(1, c->params.level_ratio_pow2);
    std::vector<int> cls(n);
    int ncls = 1;
    for (int64_t i = 0; i < n; ++i) {
        int e;
        std::frexp(d0[i] / s.d0min, &e);
        cls[i] = std::max(0, e - 1) / p;
        if (cls[i] >= 4 * kMaxLevels) return fail(RCP_EINVAL, "size ratio too large");
        ncls = std::max(ncls, cls[i] + 1);
    }
    std::vector<double> cmax(ncls, 0.0);
    for (int64_t i = 0; i < n; ++i) cmax[cls[i]] = std::max(cmax[cls[i]], d0[i]);
    for (int q = 1; q < ncls; ++q) cmax[q] = std::max(cmax[q], cmax[q - 1]);
    const double opg0 = 1.0 + c->params.skin_g, sk0 = (2.0 * c->params.skin_s) * s.d0min;
    std::vector<uint8_t> level_of(ncls);
    int nlev = 0;
    double h0 = 0.0;
    for (int q = 0; q < ncls; ++q) {
        const double h = opg0 * cmax[q] + sk0;
        if (q == 0 || h > 2.0 * h0) {
            if (nlev >= kMaxLevels) return fail(RCP_EINVAL, "more than %d size levels", kMaxLevels);
            ++nlev;
            h0 = h;
        }
        level_of[q] = (uint8_t)(nlev - 1);
    }
    std::vector<uint8_t> lev(n);
    for (int64_t i = 0; i < n; ++i) lev[i] = level_of[cls[i]];
    s.nlev = nlev;
    s.dmax_upto.assign(nlev, 0.0);
    s.lev_count.assign(nlev, 0);
    for (int64_t i = 0; i < n; ++i) {
        s.dmax_upto[lev[i]] = std::max(s.dmax_upto[lev[i]], d0[i]);
        s.lev_count[lev[i]]++;
    }
    s.dmax_lev = s.dmax_upto;
    for (int l = 1; l < nlev; ++l) s.dmax_upto[l] = std::max(s.dmax_upto[l], s.dmax_upto[l - 1]);
    // placement
    std::vector<double> x(3 * n, 0.0);
    if (init_mode == RCP_INIT_RSA) {
        if (place_rsa(n, d0, L, kappa0, seed, c->dim, (int64_t)1 << 22, x.data()) != 0)
            return fail(RCP_EPLACE, "packing %d: random sequential addition failed", k);
    } else if (init_mode == RCP_INIT_UNIFORM) {
        place_uniform(n, L, seed, c->dim, x.data());
    } else if (init_mode != RCP_INIT_NONE && init_mode != RCP_INIT_RSA_DEVICE) {
        return fail(RCP_EINVAL, "unknown init_mode %d", init_mode);
    }
    // device arrays
    for (int b = 0; b < 2; ++b) {
        for (int a = 0; a < 3; ++a) {
            CHK(dalloc(&s.M[b][a], n));
            CHK(dalloc(&s.V[b][a], n));
        }
        CHK(dalloc(&s.Q[b], n));
        CHK(dalloc(&s.ORIG[b], n));
        CHK(dalloc(&s.LEV[b], n));
    }
    for (int a = 0; a < 3; ++a) CHK(dalloc(&s.XREF[a], n));
    CHK(dalloc(&s.rp, n + 1));
    s.col_cap = std::max<int64_t>(8 * n, 1024);
    CHK(dalloc(&s.col, s.col_cap));
    s.slot_entries = s.col_cap;
    std::vector<float> soa(n);
    for (int a = 0; a < 3; ++a) {
        for (int64_t i = 0; i < n; ++i) soa[i] = (float)x[3 * i + a];
        HIPCHK(hipMemcpy(s.XREF[a], soa.data(), sizeof(float) * n, hipMemcpyHostToDevice));
        HIPCHK(hipMemset(s.M[0][a], 0, sizeof(double) * n));
        HIPCHK(hipMemset(s.V[0][a], 0, sizeof(double) * n));
    }
    {
        std::vector<P4> q(n);
        for (int64_t i = 0; i < n; ++i) q[i] = P4{x[3 * i], x[3 * i + 1], x[3 * i + 2], d0[i]};
        HIPCHK(hipMemcpy(s.Q[0], q.data(), sizeof(P4) * n, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(s.Q[1], q.data(), sizeof(P4) * n, hipMemcpyHostToDevice));
    }
    std::vector<int32_t> orig(n);
    for (int64_t i = 0; i < n; ++i) orig[i] = (int32_t)i;
    HIPCHK(hipMemcpy(s.ORIG[0], orig.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s.LEV[0], lev.data(), n, hipMemcpyHostToDevice));
    std::vector<int32_t> rp0(n + 1, 0);
    HIPCHK(hipMemcpy(s.rp, rp0.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
    s.set = 0;
    s.cur = 0;
    // state record
    SegState st;
    std::memset(&st, 0, sizeof st);
    st.n = n;
    st.L = L;
    st.hL = 0.5 * L;
    st.d0min = s.d0min;
    st.sumd0 = s.sumd0;
    st.nvol = s.nvol;
    st.d0max_k = s.d0max * (1.0 + 1e-9);
    st.beta1 = c->params.beta1;
    st.beta2 = c->params.beta2;
    st.eps_x = c->params.eps_x > 0 ? c->params.eps_x : 1e-12 / (kappa0 * s.d0max);
    st.eps_k = c->params.eps_k;
    st.kappa = kappa0;
    st.b1t = 1.0;
    st.b2t = 1.0;
    st.iL = 1.0 / L;
    seg_bias_terms(st);
    st.flags = F_STALE | F_HOLD;
    st.cur = 0;
    HIPCHK(hipMemcpy(c->d_state + k, &st, sizeof st, hipMemcpyHostToDevice));
    SegPtrs pp;
    ptrs_of(s, pp);
    HIPCHK(hipMemcpy(c->d_ptrs + k, &pp, sizeof pp, hipMemcpyHostToDevice));
    return RCP_OK;
}

static void destroy_ctx(rcp_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    for (auto &s : c->segs) {
        for (int b = 0; b < 2; ++b) {
            for (int a = 0; a < 3; ++a) {
                dfree(s.M[b][a]);
                dfree(s.V[b][a]);
            }
            dfree(s.Q[b]);
            dfree(s.ORIG[b]);
            dfree(s.LEV[b]);
        }
        for (int a = 0; a < 3; ++a) dfree(s.XREF[a]);
        dfree(s.rp);
        dfree(s.col);
    }
    dfree(c->d_ptrs);
    dfree(c->d_state);
    dfree(c->d_work);
    dfree(c->d_partials);
    for (auto &L : c->lanes) {
        if (L.own && L.st) (void)hipStreamSynchronize(L.st);
        if (L.ev) (void)hipEventDestroy(L.ev);
        if (L.own && L.st) (void)hipStreamDestroy(L.st);
    }
    c->lanes.clear();
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    dfree(c->totals);
    dfree(c->skA);
    dfree(c->skB);
    dfree(c->svA);
    dfree(c->svB);
    dfree(c->ltmp);
    dfree(c->shist);
    dfree(c->stot);
    dfree(c->d_segs);
    dfree(c->larena);
    dfree(c->harena);
    dfree(c->darena);
    dfree(c->d_fj);
    dfree(c->d_bj);
    if (c->h_fj) (void)hipHostFree(c->h_fj);
    if (c->h_bj) (void)hipHostFree(c->h_bj);
    dfree(c->bcount);
    if (c->h_bcount) (void)hipHostFree(c->h_bcount);
    dfree(c->part);
    dfree(c->out);
    dfree(c->xtmp);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->h_layout) (void)hipHostFree(c->h_layout);
    dfree(c->d_layout);
    for (auto &e : c->kev) (void)hipEventDestroy(e);
    c->kev.clear();
    for (auto *v : {&c->rb_pending, &c->rb_pool})
        for (auto &ev : *v) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    if (c->e0) (void)hipEventDestroy(c->e0);
    if (c->e1) (void)hipEventDestroy(c->e1);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// ------------------------------------------------------------ C ABI
extern "C" {

int rcp_version(void) { return RCP_VERSION; }

const char *rcp_last_error(void) { return g_err.c_str(); }

void rcp_params_default(rcp_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->size = sizeof(rcp_params);
    p->beta1 = 0.9;
    p->beta2 = 0.999;
    p->eps_x = 0.0;
    p->eps_k = 1e-12;
    p->skin_s = 0.5;
    p->skin_g = 0.02;
    p->level_ratio_pow2 = 1;
}

void rcp_tuning_default(rcp_tuning *t)
{
    if (!t) return;
    std::memset(t, 0, sizeof *t);
    t->size = sizeof(rcp_tuning);
    t->graph_iters = 32;
    t->xcd_remap = 1;
    t->fused_tail = 0;
    // cooperative pair search; whole 32-byte records written (measured at
    // least as fast as writing the three coordinates alone)
    t->variant = 64 | 128;
    // work items of about 185 rows on the C3 state: measured best with the
    // partner phase at issue priority 2 (8 / 2048 before it)
    t->row_cost = 6;
    t->item_work = 1536;
    t->time_kernels = 0;
}

// Default rung table; see include/rcp.h for the reading it encodes.
int rcp_schedule_default(int64_t n, int dim, double S, int Y, int X, int64_t n_min,
                         rcp_schedule *out)
{
    if (!out || n <= 0 || dim < 1) return fail(RCP_EINVAL, "bad arguments to rcp_schedule_default");
    std::memset(out, 0, sizeof *out);
    out->size = sizeof(rcp_schedule);
    const double nt_d = std::ceil(4000.0 * Y + X * std::sqrt((double)n * dim) - 2000.0);
    const int64_t nt = std::max<int64_t>((int64_t)nt_d, n_min);
    const double Sr = std::max(S, 1.0);
    const double fx = std::max(1.0, std::sqrt(Sr / 10.0));
    const double fk = std::min(1.0, std::sqrt(160.0 / Sr)) * std::min(1.0, std::pow(1e4 / Sr, 0.25));
    const double fb = 1.0 + std::max(0.0, std::log10(Sr / 10.0)) +
                      1.7 * std::max(0.0, std::log10(Sr / 1e4));
    struct R { double mu, ex, ek, hl, bf; };
    const R rungs[] = {
        {1e-2, 1e-2, 1e-3, 0.0, 1.0},      {1e-3, 5e-3, 5e-4, 0.0, 0.25},
        {1e-4, 2.5e-3, 2.5e-4, 0.0, 0.25}, {1e-3, 2.5e-3, 2.5e-4, 0.0, 0.125},
        {1e-4, 2.5e-3, 2.5e-4, 0.0, 0.125}, {1e-3, 2.5e-3, 2.5e-4, 0.0, 0.125},
        {1e-4, 2.5e-3, 2.5e-4, 0.0, 0.125}, {1e-5, 1.25e-3, 1.25e-4, 1.0 / 16, 2.0},
    };
    out->n_rungs = (int32_t)(sizeof rungs / sizeof rungs[0]);
    out->absolute = 0;
    out->tol = 5e-4;
    for (int r = 0; r < out->n_rungs; ++r) {
        out->mu[r] = rungs[r].mu;
        out->eta_x[r] = rungs[r].ex * fx;
        out->eta_k[r] = rungs[r].ek * fk;
        const double bf = rungs[r].bf * (r == 0 ? fb : 1.0);
        out->budget[r] = std::max<int64_t>(1, (int64_t)std::ceil(bf * (double)nt));
        out->decay[r] = rungs[r].hl <= 0 ? 1.0
                                         : std::pow(2.0, -1.0 / (rungs[r].hl * (double)out->budget[r]));
    }
    return RCP_OK;
}

int rcp_census_init(int dim, int n_prob, const int64_t *n, const double *const *d0,
                    const double *box, const double *kappa0, const uint64_t *seeds,
                    int init_mode, const rcp_params *params, void *stream, rcp_ctx **out)
{
    if (!out) return fail(RCP_EINVAL, "null output pointer");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(RCP_EINVAL, "dim must be 2 or 3 (got %d)", dim);
    if (n_prob < 1 || !n || !d0 || !box || !kappa0 || !seeds)
        return fail(RCP_EINVAL, "bad census arguments");
    if (params && params->size != sizeof(rcp_params)) return fail(RCP_EINVAL, "rcp_params: bad size");
    rcp_params P;
    if (params) P = *params;
    else rcp_params_default(&P);
    if (!(P.beta1 >= 0 && P.beta1 < 1) || !(P.beta2 >= 0 && P.beta2 < 1) || !(P.skin_s >= 0) ||
        !(P.skin_g >= 0) || !(P.eps_k > 0) || !std::isfinite(P.eps_k) ||
        !std::isfinite(P.eps_x) || !std::isfinite(P.skin_s) || !std::isfinite(P.skin_g))
        return fail(RCP_EINVAL, "bad rcp_params values");
    for (int k = 0; k < n_prob; ++k) CHK(validate_seg(n[k], d0[k], box[k], kappa0[k]));
    if (init_mode < RCP_INIT_NONE || init_mode > RCP_INIT_RSA_DEVICE)
        return fail(RCP_EINVAL, "unknown init_mode %d", init_mode);
    rcp_ctx *c = new rcp_ctx();
    c->params = P;
    rcp_tuning_default(&c->tuning);
    c->dim = dim;
    c->segs.resize(n_prob);
    int rc = RCP_OK;
    do {
        hipError_t e;
        if (stream) {
            c->stream = (hipStream_t)stream;
        } else {
            e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
            if (e != hipSuccess) { rc = fail(RCP_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)); break; }
            c->own_stream = true;
        }
        if ((e = hipEventCreateWithFlags(&c->e0, kTimingEvent)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&c->e1, kTimingEvent)) != hipSuccess) {
            rc = fail(RCP_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
            break;
        }
        if ((rc = scratch_address(&c->scratch)) != RCP_OK) break;
        if ((rc = dalloc(&c->d_ptrs, n_prob)) != RCP_OK) break;
        if ((rc = dalloc(&c->d_state, n_prob)) != RCP_OK) break;
        if ((rc = dalloc(&c->totals, 16)) != RCP_OK) break;
        if ((rc = dalloc(&c->out, 16)) != RCP_OK) break;
        if ((e = hipHostMalloc((void **)&c->h_state, sizeof(SegState) * n_prob, 0)) != hipSuccess) {
            rc = fail(RCP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
            break;
        }
        if ((e = hipHostMalloc((void **)&c->h_out, sizeof(double) * 16, 0)) != hipSuccess) {
            rc = fail(RCP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
            break;
        }
        if ((e = hipHostMalloc((void **)&c->h_layout, sizeof(int64_t) * 2 * n_prob, 0)) !=
            hipSuccess) {
            rc = fail(RCP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
            break;
        }
        if ((rc = dalloc(&c->d_layout, 2 * (size_t)n_prob)) != RCP_OK) break;
        for (int k = 0; k < n_prob && rc == RCP_OK; ++k)
            rc = seg_setup(c, k, n[k], d0[k], box[k], kappa0[k], seeds[k], init_mode);
        if (rc != RCP_OK) break;
        rc = build_work(c);
        for (int k = 0; k < n_prob && rc == RCP_OK && init_mode == RCP_INIT_RSA_DEVICE; ++k)
            rc = place_device(c, k, seeds[k], RCP_PLACE_WINDOW, (int64_t)1 << 22, nullptr);
    } while (0);
    if (rc != RCP_OK) {
        std::string msg = g_err;
        destroy_ctx(c);
        g_err = msg;
        return rc;
    }
    *out = c;
    return RCP_OK;
}

int rcp_pack_init(int dim, const double *box, int64_t n, const double *d0, double kappa0,
                  uint64_t seed, int init_mode, const rcp_params *params, void *stream,
                  rcp_ctx **out)
{
    if (dim != 2 && dim != 3) return fail(RCP_EINVAL, "dim must be 2 or 3 (got %d)", dim);
    if (!box) return fail(RCP_EINVAL, "null box");
    for (int a = 1; a < dim; ++a)
        if (box[a] != box[0]) return fail(RCP_EINVAL, "only cubic boxes are implemented");
    const double *dl[1] = {d0};
    const double L = box[0];
    return rcp_census_init(dim, 1, &n, dl, &L, &kappa0, &seed, init_mode, params, stream, out);
}

int rcp_set_skin(rcp_ctx *c, double skin_s, double skin_g)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    if (!(skin_s >= 0) || !(skin_g >= 0) || !std::isfinite(skin_s) || !std::isfinite(skin_g))
        return fail(RCP_EINVAL, "bad skin");
    CHK(pull_state(c));
    for (size_t k = 0; k < c->segs.size(); ++k) {
        const Seg &s = c->segs[k];
        const double kap = s.mixed ? std::max(1.0, c->h_state[k].kappa) : c->h_state[k].kappa;
        if (!(kap * ((1.0 + skin_g) * s.d0max + (2.0 * skin_s) * s.d0min) < 0.5 * s.L))
            return fail(RCP_EBOX, "packing %d: listing cutoff with this skin is not below L/2",
                        (int)k);
    }
    c->params.skin_s = skin_s;
    c->params.skin_g = skin_g;
    for (size_t k = 0; k < c->segs.size(); ++k)
        if (c->segs[k].built) launch_set_flags(c->d_state, (int)k, 0, F_REBUILD, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return pull_state(c);
}

int rcp_set_tuning(rcp_ctx *c, const rcp_tuning *t)
{
    if (!c || !t || t->size != sizeof(rcp_tuning)) return fail(RCP_EINVAL, "bad tuning");
    const int64_t max_rows = (t->variant & 32) ? 2 * kBlock : kBlock;
    if (t->graph_iters < 1 || t->graph_iters > 4096 || t->variant < 0 || t->variant > 255 ||
        t->row_cost < 1 || t->row_cost > 65536 || t->item_work < 1 ||
        (int64_t)t->item_work > max_rows * t->row_cost)
        return fail(RCP_EINVAL, "bad tuning values");
    if (t->time_kernels < 0 || t->time_kernels > 2) return fail(RCP_EINVAL, "bad tuning values");
    const bool relayout = t->row_cost != c->tuning.row_cost || t->item_work != c->tuning.item_work;
    c->tuning = *t;
    c->graph_valid = false;
    if (relayout && !c->segs.empty()) CHK(build_work(c));
    return RCP_OK;
}

static int check_k(rcp_ctx *c, int k)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    if (k < 0 || k >= (int)c->segs.size()) return fail(RCP_EINVAL, "packing index %d out of range", k);
    return RCP_OK;
}

// Positions at the boundary are (n, dim) row-major; inside, every packing
// keeps three coordinates (z = 0 in two dimensions).
static void expand_dim(const rcp_ctx *c, int64_t n, const double *xu, std::vector<double> &x3)
{
    x3.assign(3 * n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < c->dim; ++a) x3[3 * i + a] = xu[c->dim * i + a];
}

static void reduce_dim(const rcp_ctx *c, int64_t n, const double *x3, double *xu)
{
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < c->dim; ++a) xu[c->dim * i + a] = x3[3 * i + a];
}

int rcp_set_state(rcp_ctx *c, int k, const double *x, double kappa, int is_device)
{
    CHK(check_k(c, k));
    if (c->dim == 3 || !x) return set_state3(c, k, x, kappa, is_device);
    if (is_device) return fail(RCP_EINVAL, "device positions need dim = 3");
    std::vector<double> x3;
    expand_dim(c, c->segs[k].n, x, x3);
    return set_state3(c, k, x3.data(), kappa, 0);
}

static int set_state3(rcp_ctx *c, int k, const double *x, double kappa, int is_device)
{
    CHK(check_k(c, k));
    Seg &s = c->segs[k];
    if (!x || !(kappa > 0) || !std::isfinite(kappa)) return fail(RCP_EINVAL, "bad state");
    CHK(dgrow(&c->xtmp, &c->xtmp_cap, 3 * s.n));
    CHK(pull_state(c));
    if (is_device) {
        HIPCHK(hipMemcpyAsync(c->xtmp, x, sizeof(double) * 3 * s.n, hipMemcpyDeviceToDevice,
                              c->stream));
    } else {
        std::vector<double> w(x, x + 3 * s.n);
        const int32_t bounded = s.walls | s.round;
        for (size_t q = 0; q < w.size(); ++q) {
            double &v = w[q];
            if (!std::isfinite(v) || v < -s.L || v >= 2 * s.L)
                return fail(RCP_EINVAL, "position outside [-L, 2L)");
            if ((bounded >> (q % 3)) & 1) continue;   // no wrap across walls
            if (v < 0) v += s.L;
            if (v >= s.L) v -= s.L;
        }
        HIPCHK(hipMemcpyAsync(c->xtmp, w.data(), sizeof(double) * 3 * s.n,
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    launch_set_positions(c->d_ptrs, c->d_state, k, s.n, c->xtmp, s.cur, c->stream);
    CHK(reset_moments(c, k));
    SegState st = c->h_state[k];
    st.kappa = kappa;
    st.t = 0;
    st.b1t = 1.0;
    st.b2t = 1.0;
    seg_bias_terms(st);
    st.mk = 0;
    st.vk = 0;
    st.it_rung = 0;
    st.rung = 0;
    st.iters = 0;
    st.flags = F_STALE | F_HOLD;
    HIPCHK(hipMemcpyAsync(c->d_state + k, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    s.built = false;
    return RCP_OK;
}

int rcp_set_frozen(rcp_ctx *c, int k, const uint8_t *mask)
{
    CHK(check_k(c, k));
    Seg &s = c->segs[k];
    CHK(pull_state(c));
    const int64_t n = s.n;
    std::vector<uint8_t> fz(n, 0);
    if (mask)
        for (int64_t i = 0; i < n; ++i) fz[i] = mask[i] ? 1 : 0;
    // schedule scales over the spheres that are not frozen (they alone
    // inflate and move), compensated sums as at set-up
    double sum = 0, cs = 0, sum3 = 0, cs3 = 0, sum6 = 0, cs6 = 0, dmin = INFINITY, f3 = 0;
    int64_t ng = 0;
    auto nadd = [](double &a, double &comp, double v) {
        const double t = a + v;
        comp += std::fabs(a) >= std::fabs(v) ? (a - t) + v : (v - t) + a;
        a = t;
    };
    for (int64_t i = 0; i < n; ++i) {
        const double d = s.d0h[i];
        const double dd = c->dim == 2 ? d * d : d * d * d;   // D0^dim
        if (fz[i]) {
            f3 += dd;
            continue;
        }
        ++ng;
        dmin = std::min(dmin, d);
        nadd(sum, cs, d);
        nadd(sum3, cs3, dd);
        nadd(sum6, cs6, dd * dd);
    }
    if (ng == 0) return fail(RCP_EINVAL, "packing %d: every sphere frozen", k);
    if (ng < n && (s.walls | s.round))
        return fail(RCP_EINVAL, "packing %d: frozen spheres are not combined with walls", k);
    CHK(dgrow(&c->xtmp, &c->xtmp_cap, (n + 7) / 8));
    HIPCHK(hipMemcpyAsync(c->xtmp, fz.data(), (size_t)n, hipMemcpyHostToDevice, c->stream));
    launch_set_frozen(c->d_ptrs, k, n, reinterpret_cast<const uint8_t *>(c->xtmp), c->stream);
    SegState st = c->h_state[k];
    st.mixed = ng < n ? 1 : 0;
    st.sumd0 = sum + cs;
    st.nvol = ((sum3 + cs3) * (sum3 + cs3)) / (sum6 + cs6);
    st.d0min = dmin;
    HIPCHK(hipMemcpyAsync(c->d_state + k, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->h_state[k] = st;
    s.mixed = ng < n;
    s.frozen = s.mixed ? fz : std::vector<uint8_t>();
    s.sum3_frozen = f3;
    s.sum3_grow = sum3 + cs3;
    c->any_mixed = false;
    for (const Seg &q : c->segs) c->any_mixed = c->any_mixed || q.mixed;
    c->graph_valid = false;
    return RCP_OK;
}

int rcp_set_boundary(rcp_ctx *c, int k, uint32_t walls, uint32_t round)
{
    CHK(check_k(c, k));
    Seg &s = c->segs[k];
    const uint32_t axes = c->dim == 2 ? 3u : 7u;
    const int nround = (int)((round >> 0) & 1) + (int)((round >> 1) & 1) + (int)((round >> 2) & 1);
    if ((walls & ~axes) || (round & ~axes) || (walls & round) || nround == 1)
        return fail(RCP_EINVAL, "packing %d: bad boundary (walls 0x%x, round 0x%x, dim %d)", k,
                    walls, round, c->dim);
    if (s.mixed && (walls | round))
        return fail(RCP_EINVAL, "packing %d: frozen spheres are not combined with walls", k);
    CHK(pull_state(c));
    SegState st = c->h_state[k];
    st.walls = (int32_t)walls;
    st.round = (int32_t)round;
    st.flags |= F_STALE;   // the list depends on which axes have images
    HIPCHK(hipMemcpyAsync(c->d_state + k, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->h_state[k] = st;
    s.walls = (int32_t)walls;
    s.round = (int32_t)round;
    s.built = false;
    c->any_walls = false;
    for (const Seg &q : c->segs) c->any_walls = c->any_walls || (q.walls | q.round) != 0;
    c->graph_valid = false;
    return RCP_OK;
}

int rcp_seat_device(rcp_ctx *c, int k, double kappa0, uint64_t seed, int64_t max_attempts)
{
    CHK(check_k(c, k));
    Seg &s = c->segs[k];
    if (!(kappa0 > 0) || !std::isfinite(kappa0) || max_attempts < 1)
        return fail(RCP_EINVAL, "bad seating arguments");
    const int64_t n = s.n;
    std::vector<double> x(3 * n);
    double kap = 0;
    CHK(get_state3(c, k, x.data(), &kap, nullptr));
    // the frozen spheres, binned on a grid whose cells are at least as wide
    // as the largest seating distance (27 cells hold every frozen sphere a
    // proposal can overlap)
    double fdmax = 0, gdmax = 0;
    std::vector<int32_t> fidx, gidx;
    for (int64_t i = 0; i < n; ++i) {
        if (s.mixed && s.frozen[i]) {
            fidx.push_back((int32_t)i);
            fdmax = std::max(fdmax, s.d0h[i]);
        } else {
            gidx.push_back((int32_t)i);
            gdmax = std::max(gdmax, s.d0h[i]);
        }
    }
    const double wmin = 0.5 * (fdmax + kappa0 * gdmax) * (1.0 + 1e-12);
    int64_t nc = wmin > 0 ? (int64_t)std::floor(s.L / wmin) : 1;
    nc = std::max<int64_t>(1, std::min<int64_t>(nc, 64));
    const int64_t ncell = nc * nc * nc;
    SeatArgs a;
    std::memset(&a, 0, sizeof a);
    a.nc = nc;
    a.inv_w = (double)nc / s.L;
    a.L = s.L;
    a.hL = 0.5 * s.L;
    a.kappa0 = kappa0;
    a.seed = seed;
    a.max_attempts = max_attempts;
    a.dim = c->dim;
    const int64_t nf = (int64_t)fidx.size(), ng = (int64_t)gidx.size();
    std::vector<double> fxd(4 * std::max<int64_t>(nf, 1));
    std::vector<int32_t> start(ncell + 1, 0);
    std::vector<int64_t> cell(nf);
    auto cell_of = [&](double v) {
        int64_t q = (int64_t)(v * a.inv_w);
        return q < 0 ? 0 : (q >= nc ? nc - 1 : q);
    };
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t j = fidx[f];
        cell[f] = (cell_of(x[3 * j]) * nc + cell_of(x[3 * j + 1])) * nc + cell_of(x[3 * j + 2]);
        start[cell[f] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) start[q + 1] += start[q];
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t j = fidx[f], o = fill[cell[f]]++;
        fxd[4 * o] = x[3 * j];
        fxd[4 * o + 1] = x[3 * j + 1];
        fxd[4 * o + 2] = x[3 * j + 2];
        fxd[4 * o + 3] = s.d0h[j];
    }
    std::vector<double> gd(std::max<int64_t>(ng, 1));
    for (int64_t t = 0; t < ng; ++t) gd[t] = s.d0h[gidx[t]];
    double *d_f = nullptr, *d_g = nullptr, *d_x = nullptr;
    int32_t *d_start = nullptr, *d_gi = nullptr, *d_fail = nullptr;
    int rc = RCP_OK;
    do {
        if ((rc = dalloc(&d_f, fxd.size())) != RCP_OK) break;
        if ((rc = dalloc(&d_g, gd.size())) != RCP_OK) break;
        if ((rc = dalloc(&d_x, (size_t)(3 * n))) != RCP_OK) break;
        if ((rc = dalloc(&d_start, start.size())) != RCP_OK) break;
        if ((rc = dalloc(&d_gi, (size_t)std::max<int64_t>(ng, 1))) != RCP_OK) break;
        if ((rc = dalloc(&d_fail, 1)) != RCP_OK) break;
        hipError_t e = hipMemcpy(d_f, fxd.data(), sizeof(double) * fxd.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_g, gd.data(), sizeof(double) * gd.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_x, x.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_start, start.data(), sizeof(int32_t) * start.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && ng > 0) e = hipMemcpy(d_gi, gidx.data(), sizeof(int32_t) * ng, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(d_fail, 0, sizeof(int32_t));
        if (e != hipSuccess) { rc = fail(RCP_EDEVICE, "seating upload: %s", hipGetErrorString(e)); break; }
        a.fxd = d_f;
        a.gd = d_g;
        a.start = d_start;
        a.gidx = d_gi;
        a.x = d_x;
        a.fail = d_fail;
        launch_seat(a, ng, c->stream);
        int32_t failed = 0;
        e = hipMemcpyAsync(&failed, d_fail, sizeof failed, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(x.data(), d_x, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) { rc = fail(RCP_EDEVICE, "seating: %s", hipGetErrorString(e)); break; }
        if (failed) { rc = fail(RCP_EPLACE, "seating: a sphere exceeded %lld attempts", (long long)max_attempts); break; }
    } while (false);
    dfree(d_f); dfree(d_g); dfree(d_x); dfree(d_start); dfree(d_gi); dfree(d_fail);
    if (rc != RCP_OK) return rc;
    return set_state3(c, k, x.data(), kappa0, 0);
}

int rcp_get_state(rcp_ctx *c, int k, double *x, double *kappa, double *diam)
{
    CHK(check_k(c, k));
    if (c->dim == 3 || !x) return get_state3(c, k, x, kappa, diam);
    std::vector<double> x3(3 * c->segs[k].n);
    CHK(get_state3(c, k, x3.data(), kappa, diam));
    reduce_dim(c, c->segs[k].n, x3.data(), x);
    return RCP_OK;
}

static int get_state3(rcp_ctx *c, int k, double *x, double *kappa, double *diam)
{
    CHK(check_k(c, k));
    CHK(pull_state(c));
    Seg &s = c->segs[k];
    const int64_t n = s.n;
    if (!diam) {
        // positions scattered into user order on the device, one copy out
        if (x && n > 0) {
            CHK(dgrow(&c->xtmp, &c->xtmp_cap, 3 * n));
            launch_get_positions(c->d_ptrs, k, n, c->xtmp, s.cur, c->stream);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(x, c->xtmp, sizeof(double) * 3 * n, hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        if (kappa) *kappa = c->h_state[k].kappa;
        return RCP_OK;
    }
    std::vector<P4> q(n);
    std::vector<int32_t> orig(n);
    HIPCHK(hipMemcpy(orig.data(), s.ORIG[s.set], sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(q.data(), s.Q[s.cur], sizeof(P4) * n, hipMemcpyDeviceToHost));
    const double kap = c->h_state[k].kappa;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t u = orig[i];
        if (x) {
            x[3 * u] = q[i].x;
            x[3 * u + 1] = q[i].y;
            x[3 * u + 2] = q[i].z;
        }
        if (diam) diam[u] = q[i].d > 0.0 ? kap * q[i].d : -q[i].d;
    }
    if (kappa) *kappa = kap;
    return RCP_OK;
}

int rcp_get_optimizer(rcp_ctx *c, int k, double *m, double *v, rcp_optimizer *o)
{
    CHK(check_k(c, k));
    if (!o || o->size != sizeof(rcp_optimizer)) return fail(RCP_EINVAL, "rcp_optimizer: bad size");
    CHK(pull_state(c));
    const SegState &st = c->h_state[k];
    o->rung = st.rung;
    o->t = st.t;
    o->it_rung = st.it_rung;
    o->iterations = st.iters;
    o->m_kappa = st.mk;
    o->v_kappa = st.vk;
    o->mu = st.mu;
    o->eta_x = st.eta_x;
    o->eta_k = st.eta_k;
    if (m || v) {
        const Seg &s = c->segs[k];
        CHK(dgrow(&c->xtmp, &c->xtmp_cap, 6 * s.n));
        launch_moments_io(c->d_ptrs, k, s.n, c->xtmp, c->xtmp + 3 * s.n, 0, c->stream);
        HIPCHK(hipGetLastError());
        std::vector<double> h(6 * s.n);
        HIPCHK(hipMemcpyAsync(h.data(), c->xtmp, sizeof(double) * 6 * s.n, hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (m) reduce_dim(c, s.n, h.data(), m);
        if (v) reduce_dim(c, s.n, h.data() + 3 * s.n, v);
    }
    return RCP_OK;
}

int rcp_set_optimizer(rcp_ctx *c, int k, const double *m, const double *v,
                      const rcp_optimizer *o)
{
    CHK(check_k(c, k));
    if (!o || o->size != sizeof(rcp_optimizer)) return fail(RCP_EINVAL, "rcp_optimizer: bad size");
    CHK(pull_state(c));
    const int nr = c->h_state[k].sched.n_rungs;
    if (o->t < 0 || o->it_rung < 0 || o->iterations < 0 || o->rung < 0 ||
        (nr > 0 ? o->rung >= nr : o->rung != 0))
        return fail(RCP_EINVAL, "rcp_optimizer: step counter or schedule position out of range");
    if (!std::isfinite(o->m_kappa) || !(o->v_kappa >= 0) || !std::isfinite(o->v_kappa) ||
        !std::isfinite(o->mu) || !(o->eta_x >= 0) || !std::isfinite(o->eta_x) ||
        !(o->eta_k >= 0) || !std::isfinite(o->eta_k))
        return fail(RCP_EINVAL, "rcp_optimizer: bad value");
    const Seg &s = c->segs[k];
    const int64_t n3 = 3 * s.n, nd = (int64_t)c->dim * s.n;
    for (int64_t q = 0; m && q < nd; ++q)
        if (!std::isfinite(m[q])) return fail(RCP_EINVAL, "first moment %lld is not finite", (long long)q);
    for (int64_t q = 0; v && q < nd; ++q)
        if (!(v[q] >= 0) || !std::isfinite(v[q]))
            return fail(RCP_EINVAL, "second moment %lld is negative or not finite", (long long)q);
    std::vector<double> m3, v3;   // (n, 3) copies; the z moments stay 0 in two dimensions
    if (m) {
        expand_dim(c, s.n, m, m3);
        m = m3.data();
    }
    if (v) {
        expand_dim(c, s.n, v, v3);
        v = v3.data();
    }
    SegState st = c->h_state[k];
    st.t = o->t;
    // beta powers as repeated products, as the iteration forms them
    st.b1t = 1.0;
    st.b2t = 1.0;
    for (int64_t q = 0; q < o->t; ++q) {
        st.b1t *= st.beta1;
        st.b2t *= st.beta2;
    }
    seg_bias_terms(st);
    st.mk = o->m_kappa;
    st.vk = o->v_kappa;
    st.rung = o->rung;
    st.it_rung = o->it_rung;
    st.iters = o->iterations;
    st.mu = o->mu;
    st.eta_x = o->eta_x;
    st.eta_k = o->eta_k;
    if (m || v) {
        CHK(dgrow(&c->xtmp, &c->xtmp_cap, 6 * s.n));
        if (!m || !v) {   // keep the array not given
            launch_moments_io(c->d_ptrs, k, s.n, c->xtmp, c->xtmp + n3, 0, c->stream);
            HIPCHK(hipGetLastError());
        }
        if (m)
            HIPCHK(hipMemcpyAsync(c->xtmp, m, sizeof(double) * n3, hipMemcpyHostToDevice, c->stream));
        if (v)
            HIPCHK(hipMemcpyAsync(c->xtmp + n3, v, sizeof(double) * n3, hipMemcpyHostToDevice,
                                  c->stream));
        launch_moments_io(c->d_ptrs, k, s.n, c->xtmp, c->xtmp + n3, 1, c->stream);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(c->d_state + k, &st, sizeof st, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->h_state[k] = st;
    return RCP_OK;
}

int rcp_place_device(rcp_ctx *c, int k, uint64_t seed, int64_t window, int64_t *rounds)
{
    CHK(check_k(c, k));
    if (window < 1) return fail(RCP_EINVAL, "window must be at least 1");
    return place_device(c, k, seed, window, (int64_t)1 << 22, rounds);
}

int rcp_neighbor_build(rcp_ctx *c, int k, int64_t *n_pairs)
{
    CHK(check_k(c, k));
    CHK(pull_state(c));
    CHK(rebuild(c, k, c->h_state[k].kappa));
    if (n_pairs) *n_pairs = c->segs[k].npairs;
    return RCP_OK;
}

int rcp_get_pairs(rcp_ctx *c, int k, int32_t *pi, int32_t *pj, int64_t cap, int64_t *count)
{
    CHK(check_k(c, k));
    Seg &s = c->segs[k];
    if (!s.built) return fail(RCP_ESTATE, "no neighbour list built");
    HIPCHK(hipStreamSynchronize(c->stream));
    const int64_t n = s.n;
    std::vector<int32_t> rp(n + 1), orig(n), col(s.nnz);
    HIPCHK(hipMemcpy(rp.data(), s.rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(orig.data(), s.ORIG[s.set], sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (s.nnz) HIPCHK(hipMemcpy(col.data(), s.col, sizeof(int32_t) * s.nnz, hipMemcpyDeviceToHost));
    std::vector<std::pair<int32_t, int32_t>> pr;
    pr.reserve(s.npairs);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t a = orig[i], b = orig[col[q]];
            if (a < b) pr.emplace_back(a, b);
        }
    std::sort(pr.begin(), pr.end());
    const int64_t m = (int64_t)pr.size();
    for (int64_t q = 0; q < m && q < cap; ++q) {
        pi[q] = pr[q].first;
        pj[q] = pr[q].second;
    }
    if (count) *count = m;
    return RCP_OK;
}

static int eval_current(rcp_ctx *c, int k, const double *xu, double kappa, double mu,
                        double *gu_dev, hipStream_t st)
{
    Seg &s = c->segs[k];
    const int nb = (int)std::max<int64_t>(1, (s.n + kBlock - 1) / kBlock);
    CHK(dgrow(&c->part, &c->part_cap, 4 * (int64_t)nb + 8));
    EvalOut o;
    o.part = c->part;
    o.gu = gu_dev;
    launch_eval(c->d_ptrs, c->d_state, k, s.n, xu, kappa, o, nb, st);
    launch_eval_finish(c->part, nb, kappa, mu, c->d_state, k, c->out, st);
    return RCP_OK;
}

int rcp_energy_grad(rcp_ctx *c, int k, double mu, rcp_energy *e, double *grad_x)
{
    CHK(check_k(c, k));
    if (!e) return fail(RCP_EINVAL, "null output");
    CHK(pull_state(c));
    if (c->h_state[k].flags & (F_REBUILD | F_STALE)) {
        CHK(rebuild(c, k, c->h_state[k].kappa));
        CHK(pull_state(c));
    }
    Seg &s = c->segs[k];
    double *gdev = nullptr;
    if (grad_x) {
        CHK(dgrow(&c->xtmp, &c->xtmp_cap, 3 * s.n));
        gdev = c->xtmp;
    }
    CHK(eval_current(c, k, nullptr, c->h_state[k].kappa, mu, gdev, c->stream));
    double o[6];
    HIPCHK(hipMemcpyAsync(o, c->out, sizeof o, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> g3(grad_x && c->dim != 3 ? 3 * s.n : 0);
    if (grad_x)
        HIPCHK(hipMemcpyAsync(c->dim == 3 ? grad_x : g3.data(), gdev, sizeof(double) * 3 * s.n,
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (grad_x && c->dim != 3) reduce_dim(c, s.n, g3.data(), grad_x);
    e->E_overlap = o[0];
    e->E_growth = o[1];
    e->dE_dkappa_overlap = o[2];
    e->dE_dkappa_growth = o[3];
    e->max_overlap = o[4];
    e->n_overlap = (int64_t)std::llround(o[5]);
    return RCP_OK;
}

// Load a schedule on every packing and set its first rung; with
// reset_adam the optimiser starts afresh (moments and step counter zero).
static int start_schedule(rcp_ctx *c, const rcp_schedule *sched, int per_packing,
                          int64_t max_iters, bool reset_adam = true)
{
    CHK(pull_state(c));
    std::vector<SchedDev> qs(c->segs.size());
    for (size_t k = 0; k < c->segs.size(); ++k) CHK(to_sched(per_packing ? sched + k : sched, qs[k]));
    // every packing runs again: packings parked by an earlier run get slots
    bool parked = false;
    for (auto &s : c->segs) {
        parked = parked || s.parked;
        s.parked = false;
    }
    if (parked) CHK(build_work(c));
    for (size_t k = 0; k < c->segs.size(); ++k) {
        if (reset_adam) CHK(reset_moments(c, (int)k));
        c->segs[k].err = 0;
        launch_sched_start(c->d_state, (int)k, qs[k], reset_adam ? 1 : 0, max_iters, c->stream);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return RCP_OK;
}

int rcp_adam_step(rcp_ctx *c, double mu, double eta_x, double eta_k, int64_t n_steps)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    if (n_steps < 1 || !std::isfinite(mu) || !(eta_x >= 0) || !(eta_k >= 0))
        return fail(RCP_EINVAL, "bad adam_step arguments");
    rcp_schedule q;
    std::memset(&q, 0, sizeof q);
    q.size = sizeof q;
    q.n_rungs = 1;
    q.absolute = 1;
    q.tol = -1.0;
    q.mu[0] = mu;
    q.eta_x[0] = eta_x;
    q.eta_k[0] = eta_k;
    q.decay[0] = 1.0;
    q.budget[0] = n_steps;
    // the optimiser state carries over from the previous call
    CHK(start_schedule(c, &q, 0, 0, false));
    CHK(run_loop(c));
    CHK(pull_state(c));
    for (size_t k = 0; k < c->segs.size(); ++k)
        if (c->h_state[k].flags & F_NONFINITE)
            return fail(RCP_ENONFINITE, "packing %zu: non-finite energy or gradient", k);
    return RCP_OK;
}

// Result of packing k from its current state (shrink included).
static int seg_result(rcp_ctx *c, int k, rcp_result &r)
{
    CHK(pull_state(c));
    const SegState st = c->h_state[k];
    std::memset(&r, 0, sizeof r);
    r.kappa_before_shrink = st.kappa;
    r.max_overlap = st.max_delta;
    r.energy = st.E_ov;
    r.iterations = st.iters;
    r.rung = st.rung;
    if (c->segs[k].err) {
        r.status = c->segs[k].err;
        r.rebuilds = c->segs[k].rebuilds;
        return RCP_OK;
    }
    if (st.flags & F_NONFINITE) {
        r.status = RCP_ENONFINITE;
        r.rebuilds = c->segs[k].rebuilds;
        return RCP_OK;
    }
    if (st.flags & F_STOP) r.status = 0;
    else if (st.flags & F_CAP) r.status = RCP_ENOTCONV;
    else r.status = 1;
    if (!(st.flags & F_STOP)) {
        // the state is the one after the last update: evaluate it
        rcp_energy e;
        CHK(rcp_energy_grad(c, k, st.mu, &e, nullptr));
        r.max_overlap = e.max_overlap;
        r.energy = e.E_overlap;
    }
    CHK(shrink_seg(c, k, &r.kappa, &r.phi));
    r.rebuilds = c->segs[k].rebuilds;
    return RCP_OK;
}

__global__ void k_extend(SegState *S, int nseg, int64_t n_more)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nseg) return;
    S[k].iter_limit = n_more > 0 ? S[k].iters + n_more : 0;
    S[k].flags &= ~F_HOLD;
}

int rcp_run_start(rcp_ctx *c, const rcp_schedule *sched, int per_packing)
{
    if (!c || !sched) return fail(RCP_EINVAL, "null argument");
    CHK(start_schedule(c, sched, per_packing, 0));
    // hold every packing until rcp_run_continue
    for (size_t k = 0; k < c->segs.size(); ++k)
        launch_set_flags(c->d_state, (int)k, 0, F_HOLD, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    return RCP_OK;
}

int rcp_run_continue(rcp_ctx *c, int64_t n_iters, int32_t *active)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    if (n_iters < 0) return fail(RCP_EINVAL, "n_iters < 0");
    const int ns = (int)c->segs.size();
    hipLaunchKernelGGL(k_extend, dim3((ns + 63) / 64), dim3(64), 0, c->stream, c->d_state, ns,
                       n_iters);
    // run_loop returns right after reading every record back (nothing is
    // launched after its last read), so the host mirror is current here
    CHK(run_loop(c));
    int32_t a = 0;
    for (int k = 0; k < ns; ++k)
        if (!(c->h_state[k].flags & (F_STOP | F_CAP | F_NONFINITE))) ++a;
    if (active) *active = a;
    return RCP_OK;
}

int rcp_run_prepare(rcp_ctx *c)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    const int K = std::max(1, c->tuning.graph_iters);
    if (K <= 1) return RCP_OK;
    // every length the run loop may launch (see graph_len): K, and the
    // powers of two from kMinGraph below it
    std::vector<int> lens = {K};
    if (K > kMinGraph) {
        int G = kMinGraph;
        while (2 * G < K) G *= 2;
        for (; G >= kMinGraph; G /= 2) lens.push_back(G);
    }
    for (int G : lens) {
        hipGraphExec_t gx = nullptr;
        CHK(graph_for(c, G, &gx));
        HIPCHK(hipGraphUpload(gx, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return RCP_OK;
}

int rcp_run_result(rcp_ctx *c, int k, rcp_result *r)
{
    CHK(check_k(c, k));
    if (!r) return fail(RCP_EINVAL, "null result");
    return seg_result(c, k, *r);
}

int rcp_inflate_run(rcp_ctx *c, const rcp_schedule *sched, int per_packing, int64_t max_iters,
                    rcp_result *results)
{
    if (!c || !sched || !results) return fail(RCP_EINVAL, "null argument");
    if (max_iters < 0) return fail(RCP_EINVAL, "max_iters < 0");
    CHK(start_schedule(c, sched, per_packing, max_iters));
    CHK(run_loop(c));
    int rc = RCP_OK;
    for (size_t k = 0; k < c->segs.size(); ++k) {
        CHK(seg_result(c, (int)k, results[k]));
        const int st = results[k].status;
        if (st == RCP_EBOX) rc = RCP_EBOX;
        else if (st == RCP_ENONFINITE && rc != RCP_EBOX) rc = RCP_ENONFINITE;
        else if (st == RCP_ENOTCONV && rc == RCP_OK) rc = RCP_ENOTCONV;
    }
    if (rc == RCP_ENOTCONV) fail(RCP_ENOTCONV, "iteration cap reached before the stop test held");
    if (rc == RCP_ENONFINITE) fail(RCP_ENONFINITE, "non-finite energy or gradient");
    if (rc == RCP_EBOX)
        fail(RCP_EBOX, "a packing's listing cutoff reached L/2 (its result status is RCP_EBOX)");
    return rc;
}

int rcp_census_run(rcp_ctx *c, const rcp_schedule *sched, int per_packing, int64_t max_iters,
                   rcp_result *results)
{
    return rcp_inflate_run(c, sched, per_packing, max_iters, results);
}

int rcp_shrink(rcp_ctx *c, int k, double *kappa_shrunk, double *phi)
{
    CHK(check_k(c, k));
    double kp, ph;
    CHK(shrink_seg(c, k, &kp, &ph));
    if (kappa_shrunk) *kappa_shrunk = kp;
    if (phi) *phi = ph;
    return RCP_OK;
}

// Make the list valid for user-order device positions x_dev at kappa.
static int ensure_valid_at(rcp_ctx *c, const double *x_dev, double kappa, hipStream_t st)
{
    if (st != c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    CHK(pull_state(c));
    Seg &s = c->segs[0];
    SegState &h = c->h_state[0];
    bool ok = s.built && !(h.flags & (F_REBUILD | F_STALE));
    if (ok) {
        const int nb = (int)std::max<int64_t>(1, (s.n + kBlock - 1) / kBlock);
        CHK(dgrow(&c->part, &c->part_cap, 4 * (int64_t)nb + 8));
        launch_disp(c->d_ptrs, c->d_state, 0, s.n, x_dev, c->part, nb, st);
        launch_max_finish(c->part, nb, c->out + 8, st);
        double d2 = 0;
        HIPCHK(hipMemcpyAsync(&d2, c->out + 8, sizeof d2, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        // the test the iteration tail applies (see k_iterate.hip)
        const double excess = std::max(0.0, kappa - h.kappa_lim);
        ok = 2.0 * std::sqrt(d2) + excess * h.d0max_k <= 2.0 * h.disp_lim;
    }
    if (!ok) {
        HIPCHK(hipStreamSynchronize(st));
        CHK(rcp_set_state(c, 0, x_dev, kappa, 1));
        CHK(rebuild(c, 0, kappa));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return RCP_OK;
}

__global__ void k_energy_out(const double *o, double *E)
{
    E[0] = o[0] + o[1];
    E[1] = o[4];
}

__global__ void k_gk_out(const double *o, double *gk) { gk[0] = o[2] + o[3]; }

int rcp_energy_dev(rcp_ctx *c, const double *x_dev, double kappa, double mu, double *E_dev,
                   void *stream)
{
    if (!c || !x_dev || !E_dev) return fail(RCP_EINVAL, "null argument");
    if (c->dim != 3) return fail(RCP_EINVAL, "device position arrays need dim = 3");
    hipStream_t st = (hipStream_t)stream;   // NULL: the null stream
    CHK(ensure_valid_at(c, x_dev, kappa, st));
    CHK(eval_current(c, 0, x_dev, kappa, mu, nullptr, st));
    hipLaunchKernelGGL(k_energy_out, dim3(1), dim3(1), 0, st, c->out, E_dev);
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

int rcp_adjoint_dev(rcp_ctx *c, const double *x_dev, double kappa, double mu, double *gx_dev,
                    double *gk_dev, void *stream)
{
    if (!c || !x_dev || !gx_dev || !gk_dev) return fail(RCP_EINVAL, "null argument");
    if (c->dim != 3) return fail(RCP_EINVAL, "device position arrays need dim = 3");
    hipStream_t st = (hipStream_t)stream;   // NULL: the null stream
    CHK(ensure_valid_at(c, x_dev, kappa, st));
    CHK(eval_current(c, 0, x_dev, kappa, mu, gx_dev, st));
    hipLaunchKernelGGL(k_gk_out, dim3(1), dim3(1), 0, st, c->out, gk_dev);
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

int rcp_energy_dev_static(rcp_ctx *c, const double *x_dev, double kappa, double mu,
                          double *E_dev, void *stream)
{
    if (!c || !x_dev || !E_dev) return fail(RCP_EINVAL, "null argument");
    if (c->dim != 3) return fail(RCP_EINVAL, "device position arrays need dim = 3");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(mu))
        return fail(RCP_EINVAL, "bad kappa or mu");
    const Seg &s = c->segs[0];
    const int64_t nb = std::max<int64_t>(1, (s.n + kBlock - 1) / kBlock);
    if (nb > kScratchBlocks)
        return fail(RCP_EINVAL,
                    "rcp_energy_dev_static: n = %lld exceeds the fixed scratch (at most %lld "
                    "spheres)",
                    (long long)s.n, (long long)(kScratchBlocks * kBlock));
    if (!c->scratch) return fail(RCP_ESTATE, "no scratch address for this context");
    hipStream_t st = (hipStream_t)stream;   // NULL: the null stream
    if (st != c->stream) HIPCHK(hipStreamSynchronize(c->stream));
    // the context's record, read without touching any growable host list
    HIPCHK(hipMemcpyAsync(c->h_state, c->d_state, sizeof(SegState) * c->segs.size(),
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const SegState &h = c->h_state[0];
    if (!s.built || (h.flags & (F_REBUILD | F_STALE)))
        return fail(RCP_ESTATE, "rcp_energy_dev_static: packing 0 has no valid neighbour list");
    double *part = c->scratch, *res = c->scratch + 4 * kScratchBlocks;
    // the validity test of the iteration tail at (x_dev, kappa)
    launch_disp(c->d_ptrs, c->d_state, 0, s.n, x_dev, part, (int)nb, st);
    launch_max_finish(part, (int)nb, res, st);
    HIPCHK(hipMemcpyAsync(c->h_out, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double d2 = c->h_out[0];
    const double excess = std::max(0.0, kappa - h.kappa_lim);
    if (!(2.0 * std::sqrt(d2) + excess * h.d0max_k <= 2.0 * h.disp_lim))
        return fail(RCP_ESTATE,
                    "rcp_energy_dev_static: the neighbour list is not valid at these positions "
                    "and kappa (rebuild it with rcp_neighbor_build or rcp_energy_dev)");
    EvalOut o;
    o.part = part;
    o.gu = nullptr;
    launch_eval(c->d_ptrs, c->d_state, 0, s.n, x_dev, kappa, o, (int)nb, st);
    launch_eval_finish(part, (int)nb, kappa, mu, c->d_state, 0, res + 8, st);
    hipLaunchKernelGGL(k_energy_out, dim3(1), dim3(1), 0, st, res + 8, E_dev);
    HIPCHK(hipGetLastError());
    return RCP_OK;
}

int rcp_time_iterations(rcp_ctx *c, int64_t n_iters, double *iterate_us, double *tail_us,
                        int64_t *done)
{
    if (!c || n_iters < 1) return fail(RCP_EINVAL, "bad arguments");
    const int ns = (int)c->segs.size();
    hipLaunchKernelGGL(k_extend, dim3((ns + 63) / 64), dim3(64), 0, c->stream, c->d_state, ns,
                       n_iters);
    constexpr int kBatch = 32;
    std::vector<hipEvent_t> ev(3 * kBatch);
    for (auto &e : ev) HIPCHK(hipEventCreateWithFlags(&e, kTimingEvent));
    double it_ms = 0, tl_ms = 0;
    int64_t n_done = 0;
    int rc = RCP_OK;
    const int flags = iterate_flags(c);
    for (;;) {
        if ((rc = pull_state(c)) != RCP_OK) break;
        bool any = false;
        std::vector<int> ks;
        std::vector<double> kap;
        for (int k = 0; k < ns; ++k) {
            const int32_t f = c->h_state[k].flags;
            if (seg_done(f)) continue;
            if (f & (F_REBUILD | F_STALE)) {
                ks.push_back(k);
                kap.push_back(c->h_state[k].kappa);
            }
            any = true;
        }
        if (!any) break;
        if (!ks.empty()) {
            std::vector<int> rcs;
            if ((rc = rebuild_batch(c, ks, kap, rcs)) != RCP_OK) break;
            for (int r : rcs)
                if (r != RCP_OK) rc = r;
            if (rc != RCP_OK) break;
        }
        if ((rc = pull_state(c)) != RCP_OK) break;
        int64_t before = 0;
        for (int k = 0; k < ns; ++k) before += c->h_state[k].iters;
        for (int b = 0; b < kBatch && c->nitems > 0; ++b) {
            (void)hipEventRecord(ev[3 * b], c->stream);
            launch_iterate(c->d_ptrs, c->d_state, c->d_work, c->d_partials, c->nitems, flags,
                           c->stream);
            (void)hipEventRecord(ev[3 * b + 1], c->stream);
            launch_tail(c->d_state, c->d_partials, ns, c->segs[0].first_item, c->segs[0].blocks,
                        c->stream);
            (void)hipEventRecord(ev[3 * b + 2], c->stream);
        }
        if ((rc = pull_state(c)) != RCP_OK) break;
        int64_t after = 0;
        for (int k = 0; k < ns; ++k) after += c->h_state[k].iters;
        // a packing runs consecutive launches until it goes idle, so the
        // first (after - before) launches of a one-packing context did work
        const int64_t worked = std::min<int64_t>(after - before, kBatch);
        for (int64_t b = 0; b < worked; ++b) {
            float a = 0, t = 0;
            (void)hipEventElapsedTime(&a, ev[3 * b], ev[3 * b + 1]);
            (void)hipEventElapsedTime(&t, ev[3 * b + 1], ev[3 * b + 2]);
            it_ms += a;
            tl_ms += t;
        }
        n_done += worked;
        c->stats.iterations += after - before;
        if (after == before) break;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (rc != RCP_OK) return rc;
    if (iterate_us) *iterate_us = n_done ? 1e3 * it_ms / (double)n_done : 0.0;
    if (tail_us) *tail_us = n_done ? 1e3 * tl_ms / (double)n_done : 0.0;
    if (done) *done = n_done;
    return RCP_OK;
}

int rcp_get_stats(rcp_ctx *c, rcp_stats *s)
{
    if (!c || !s) return fail(RCP_EINVAL, "null argument");
    CHK(pull_state(c));   // completes and counts pending list-build timings
    *s = c->stats;
    s->nnz = 0;
    s->max_degree = 0;
    s->levels = 0;
    for (auto &g : c->segs) {
        s->nnz += g.nnz;
        s->levels = std::max<int64_t>(s->levels, g.nlev);
        if (!g.built || g.n <= 0) continue;
        // longest row of the current list, computed on request
        launch_fill_u32(c->totals + 1, 1, 0u, c->stream);
        launch_max_degree(g.n, g.rp, c->totals + 1, c->stream);
        uint32_t md = 0;
        HIPCHK(hipMemcpyAsync(&md, c->totals + 1, sizeof md, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        s->max_degree = std::max<int64_t>(s->max_degree, md);
    }
    return RCP_OK;
}

int rcp_reset_stats(rcp_ctx *c)
{
    if (!c) return fail(RCP_EINVAL, "null context");
    std::memset(&c->stats, 0, sizeof c->stats);
    return RCP_OK;
}

int rcp_num_packings(rcp_ctx *c) { return c ? (int)c->segs.size() : 0; }

int64_t rcp_num_particles(rcp_ctx *c, int k)
{
    if (!c || k < 0 || k >= (int)c->segs.size()) return -1;
    return c->segs[k].n;
}

void rcp_destroy(rcp_ctx *c) { destroy_ctx(c); }

}  // extern "C"
