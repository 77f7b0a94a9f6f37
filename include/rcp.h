/*
 * rcp.h -- C ABI of the MI355X library for the Adam-based inflation protocol
 * (random close packings of polydisperse spheres in a periodic cube, or
 * disks in a periodic square, optionally bounded by hard walls).
 *
 * The library keeps every per-particle array in device memory (FP64 SoA,
 * Morton order inside; user order at this boundary) and runs every step of
 * an inflation iteration in its own HIP kernels for gfx950.
 *
 * Problem statement (Sec. 1 and App. A of the paper): a list of N positive
 * relative diameters D0_i, the spatial dimension and the domain (a periodic
 * cube or square of edge L; rcp_set_boundary adds flat or round hard walls,
 * Sec. 2).  Diameters are D_i = kappa D0_i with one global
 * scale kappa.  The optimised energy is Eq. (energy):
 *     E(x, kappa) = 1/2 sum_{i<j} (1 - r_ij/d_ij)^2 Theta(1 - r_ij/d_ij)
 *                   - mu sum_i D_i,       d_ij = (D_i + D_j)/2,
 * minimised jointly over positions and kappa with Adam, mu annealed through
 * rungs whose length follows Eq. (trigger); the run stops in the final rung
 * once the largest fractional overlap 1 - r/d is below a tolerance (5e-4 in
 * App. A), after which kappa is reduced uniformly until no pair overlaps
 * (Sec. 2, App. A).
 *
 * Conventions for every call:
 *   - return value 0 on success, a negative RCP_E* code on failure; the
 *     message of the last failure on the calling thread is rcp_last_error();
 *   - positions (and gradients and Adam moments) at this boundary are
 *     row-major (n, dim) doubles in user order (dim = 3, or 2 for disks:
 *     Fig. 1 of the paper is 2-D); inside, a disk packing is a packing in the
 *     plane z = 0, whose z gradients vanish so its z coordinates never move;
 *   - host arrays are borrowed for the duration of the call and copied;
 *   - device arrays given to *_dev calls are borrowed until the work queued
 *     on the given stream has completed;
 *   - a context is bound to one HIP stream and is not thread safe; distinct
 *     contexts are independent;
 *   - arguments are validated before any device work is queued.
 */
#ifndef RCP_H
#define RCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RCP_VERSION 1
#define RCP_MAX_RUNGS 16

/* error codes */
#define RCP_OK 0
#define RCP_EINVAL -1      /* bad argument: n <= 0, D0 <= 0 or not finite, dim not 2 or 3,
                              non-cubic box, kappa <= 0, bad schedule              */
#define RCP_EBOX -2        /* largest listing cutoff >= L/2 (a sphere would meet its
                              own periodic image, Sec. 2)                          */
#define RCP_ENOMEM -3      /* device or host allocation failed                    */
#define RCP_EDEVICE -4     /* HIP runtime error (message has the HIP error string) */
#define RCP_ENOTCONV -5    /* iteration cap of the final rung reached; the result
                              struct is still filled                                */
#define RCP_ENONFINITE -6  /* NaN or Inf in the energy or a gradient               */
#define RCP_EPLACE -7      /* random sequential addition exceeded its attempts      */
#define RCP_ESTATE -8      /* call not valid in the context's current state        */

/* initial placement modes for rcp_pack_init */
#define RCP_INIT_NONE 0     /* positions come later from rcp_set_state            */
#define RCP_INIT_RSA 1      /* random sequential addition without overlap, largest
                               sphere first (App. A: dilute, non-overlapping start) */
#define RCP_INIT_UNIFORM 2  /* i.i.d. uniform positions, overlaps allowed         */
#define RCP_INIT_RSA_DEVICE 3  /* random sequential addition on the GPU, in rounds
                                  of RCP_PLACE_WINDOW proposals (rcp_place_device) */
#define RCP_PLACE_WINDOW 65536

typedef struct rcp_ctx rcp_ctx;

/* Optimiser and neighbour-list parameters.  size must be sizeof(rcp_params).
 *   beta1, beta2, eps_x, eps_k: Adam (Kingma and Ba) for positions and for
 *     kappa (App. A), 0 <= beta < 1; eps_x <= 0 selects
 *     1e-12 / (kappa0 * max D0), an explicit eps_x and eps_k must be
 *     positive and finite.
 *   skin_s, skin_g: a pair is listed at scale kb when
 *       r^2 < c^2,  c = kb ((1 + g)(D0_i + D0_j)/2 + 2 s D0_min),
 *     and the list stays valid while
 *       2 max|x - x_build| + max(0, kappa - (1 + g) kb) max D0 <= 2 s kb D0_min
 *     (App. A rebuilds on accumulated displacement; the skin form is ours:
 *     kappa may grow by the factor 1 + g for free, and beyond that at the
 *     expense of the displacement allowance).
 *   level_ratio_pow2: size classes are floor(log2(D0/D0_min) / p), p >= 1;
 *     consecutive classes share one cell grid while its cell width stays
 *     within twice that of the first of them.
 */
typedef struct {
    uint32_t size;
    double beta1, beta2, eps_x, eps_k;
    double skin_s, skin_g;
    int32_t level_ratio_pow2;
} rcp_params;

/* Launch tuning (performance only; results do not depend on it except
 * through summation order, which is fixed for a given tuning).  size must
 * be sizeof(rcp_tuning).
 *   graph_iters: iterations captured per HIP graph launch (1 = no graph);
 *   xcd_remap: 1 = map consecutive work items to the same XCD;
 *   fused_tail: 1 = the last block of a packing to finish an iteration
 *     reduces the partial sums and updates kappa and the schedule (one
 *     kernel per iteration), 0 = a separate one-block kernel does it;
 *   variant: gradient + Adam kernel variant, bit 0 = four partner gathers in
 *     flight per thread instead of two, bit 1 = the Adam operands are loaded
 *     before the partner loop (more latency hidden, more registers), bit 2 =
 *     a work item's partner indices are staged in LDS in one coalesced pass
 *     before the partner loop, bit 3 = persistent blocks that each take a
 *     sequence of work items and prefetch the next item's descriptor and row
 *     pointers (bits 1, 2 and fused_tail do not apply with bit 3), bit 4 =
 *     compiled for seven waves per SIMD (fewer registers, some spilling),
 *     bit 5 = work items of up to 512 rows, two per thread in the Adam phase
 *     (bits 1-4 and fused_tail do not apply with it); bit 6 selects the
 *     wave-cooperative pair search of the list build (the 64 lanes of a
 *     wave test the flattened candidates of all their cells together; the
 *     same pairs are listed); bit 7 = each update writes the whole 32-byte
 *     position record (x, y, z, D0) instead of the three coordinates;
 *   time_kernels: 0 = no timing; 1 = HIP events around the gradient + Adam
 *     and tail launches of the middle iteration (graph_iters / 2) of every
 *     batch of graph_iters (a uniform sample of one launch in graph_iters;
 *     event nodes cost a few microseconds each); 2 = around every launch
 *     (rcp_stats.kernel_ms and friends);
 *   row_cost, item_work: the rows of a packing (in list order) are cut into
 *     work items of item_work units, a row costing row_cost units plus one
 *     per listed partner, so each 256-thread block gets about the same
 *     gather work whether its rows are small spheres or large ones; 1 <=
 *     row_cost <= 65536 and 1 <= item_work <= R * row_cost, R = 512 with
 *     variant bit 5 and 256 otherwise (an item then never holds more than R
 *     rows). */
typedef struct {
    uint32_t size;
    int32_t graph_iters;
    int32_t xcd_remap;
    int32_t fused_tail;
    int32_t variant;
    int32_t row_cost;
    int32_t item_work;
    int32_t time_kernels;
} rcp_tuning;

/* Annealing schedule: a table of rungs run in order (App. A).  Rung r lasts
 * budget[r] iterations; the last rung is the final relaxation, where the
 * stop test max delta < tol is applied before each update, and budget of the
 * last rung is its iteration cap.  decay[r] multiplies mu and both step
 * sizes after every iteration of rung r.  When absolute == 0, at the start of rung r:
 *     mu    = (mu[r] * N_v) / (kappa * sum D0),  N_v = (sum D0^3)^2 / sum D0^6
 *     eta_x = eta_x[r] * (kappa * D0_min)
 *     eta_k = eta_k[r] * kappa
 * with kappa its value at that moment (N_v is formed with compensated
 * sums in index order); when absolute != 0 the three numbers
 * are used as given.  size must be sizeof(rcp_schedule). */
typedef struct {
    uint32_t size;
    int32_t n_rungs;
    int32_t absolute;
    double tol;
    double mu[RCP_MAX_RUNGS];
    double eta_x[RCP_MAX_RUNGS];
    double eta_k[RCP_MAX_RUNGS];
    double decay[RCP_MAX_RUNGS];
    int64_t budget[RCP_MAX_RUNGS];
} rcp_schedule;

/* Energy terms at the current state (rcp_energy_grad). */
typedef struct {
    double E_overlap;      /* 1/2 sum delta^2 over overlapping pairs          */
    double E_growth;       /* -mu kappa sum D0                                 */
    double dE_dkappa_overlap;  /* sum delta r / (kappa d)                      */
    double dE_dkappa_growth;   /* -mu sum D0                                   */
    double max_overlap;    /* max fractional overlap 1 - r/d (0 if none)       */
    int64_t n_overlap;     /* number of overlapping pairs                      */
} rcp_energy;

/* Outcome of an inflation run (per packing). */
typedef struct {
    double phi;                 /* volume fraction after shrink to contact     */
    double kappa;               /* kappa' after shrink                          */
    double kappa_before_shrink;
    double max_overlap;         /* at the returned (pre-shrink) state           */
    double energy;              /* overlap energy at the returned state         */
    int64_t iterations;         /* Adam updates taken                           */
    int64_t rebuilds;           /* neighbour-list builds                        */
    int32_t status;             /* 0 converged, RCP_ENOTCONV, RCP_ENONFINITE,
                                   1 = stopped by max_iters                     */
    int32_t rung;               /* rung index at return                          */
} rcp_result;

/* Timing and counters accumulated by a context (HIP events on its stream). */
typedef struct {
    int64_t iterations;         /* iterations executed (all packings, summed)  */
    int64_t particle_updates;   /* sum over iterations of the packing's N      */
    int64_t rebuilds;
    int64_t graph_launches;
    int64_t nnz;                /* listed partners (both directions) now        */
    int64_t max_degree;         /* longest row of the current lists             */
    double iterate_ms;          /* time in iteration launches                   */
    double rebuild_ms;          /* time in neighbour-list builds                */
    double shrink_ms;
    /* with rcp_tuning.time_kernels > 0: HIP events on the context's stream
     * around the sampled launches of the gradient + Adam kernel and of the
     * tail kernel, counted for launches in which some packing iterated */
    double kernel_ms;           /* summed gradient + Adam kernel durations       */
    double tail_kernel_ms;      /* summed tail kernel durations                  */
    int64_t kernel_launches;    /* launches timed                                */
    int64_t kernel_nnz;         /* sum over timed launches of the listed
                                   partners (all packings) at that launch        */
    int64_t levels;             /* cell-grid levels of the size classes (largest
                                   over the packings)                            */
} rcp_stats;

int rcp_version(void);
const char *rcp_last_error(void);
void rcp_params_default(rcp_params *p);
/* Defaults: graph_iters 32, xcd_remap 1, fused_tail 0, variant 192 (the
 * cooperative pair search, the two-gather gradient + Adam kernel writing
 * whole records), row_cost 6, item_work 1536, time_kernels 0. */
void rcp_tuning_default(rcp_tuning *t);

/* Default rung table for a packing of n spheres in dimension dim with size
 * ratio S = max D0 / min D0, with the principal budget of Eq. (trigger),
 * n_trig = ceil(4000 Y + X sqrt(n dim) - 2000), floored at n_min.  The rung
 * values are our reading (App. A does not list them): densify at mu~ = 1e-2
 * for n_trig updates, rungs at 1e-3 and 1e-4 (n_trig/4 each), two cycles
 * 1e-3 <-> 1e-4 (n_trig/8 each), final relaxation from 1e-5 with mu and
 * both step sizes halving every 1/16 of its cap (cap 2 n_trig), so mu is
 * annealed towards 0; stop tolerance 5e-4.  For broad
 * distributions the position steps are multiplied by max(1, sqrt(S/10)),
 * the kappa steps by min(1, sqrt(160/S)) min(1, (1e4/S)^(1/4)) and the
 * densification budget by 1 + max(0, log10(S/10)) + 1.7 max(0, log10(S/1e4)),
 * so that small spheres can move out of the way of growing large ones.  In relative schedules mu~ is turned into
 * mu = mu~ N_v / (kappa sum D0) at each rung start, N_v = (sum D0^3)^2 /
 * sum D0^6 (the volume participation number: N for equal spheres, about the
 * number of volume-carrying spheres for a broad distribution), so the
 * equilibrium summed overlap is mu~ N_v.  Returns RCP_EINVAL for n <= 0 or
 * dim < 1. */
int rcp_schedule_default(int64_t n, int dim, double S, int Y, int X, int64_t n_min,
                         rcp_schedule *out);

/* Create a context for n_prob independent packings (1 for a plain solve;
 * several for a batched census).  Packing k has n[k] spheres (1 <= n[k] <
 * 2^27) with relative
 * diameters d0[k][0..n[k]) (host), cube edge box[k], starting scale
 * kappa0[k] and placement seed seeds[k] (SplitMix64 counter stream, see
 * rcp_pack_init).  dim is 3, or 2 (Sec. 2: the dimension is an input; in
 * two dimensions placement does not draw the z axis, the schedule's
 * participation number is (sum D0^2)^2 / sum D0^4 and phi is the area
 * fraction; the iteration then runs a kernel instantiated for two
 * coordinates, which leaves the z moments and reference unread, whatever
 * the tuning variant, and the tail is not fused).  stream is a hipStream_t
 * (NULL: the library creates one).
 * Returns RCP_EBOX if a packing's largest cutoff is not below L/2. */
int rcp_census_init(int dim, int n_prob, const int64_t *n,
                    const double *const *d0, const double *box,
                    const double *kappa0, const uint64_t *seeds, int init_mode,
                    const rcp_params *params, void *stream, rcp_ctx **out);

/* One packing: the n_prob = 1 case of rcp_census_init.  box points at dim
 * edge lengths that must be equal.  Placement draws uniform numbers u =
 * (SplitMix64(seed, ((i << 24) | attempt) * 4 + axis) >> 11) * 2^-53 and
 * position u * L per axis (Steele, Lea and Flood 2014). */
int rcp_pack_init(int dim, const double *box, int64_t n, const double *d0,
                  double kappa0, uint64_t seed, int init_mode,
                  const rcp_params *params, void *stream, rcp_ctx **out);

/* Random sequential addition of packing k on the GPU, at its current kappa
 * (App. A: the run starts from a dilute configuration placed without
 * overlap with the help of a cell list; the procedure is our reading).
 * Spheres are ranked largest first (ties: lower index first) and placed
 * class by class, largest class first (class floor(log2(D0 / D0_min))).  A
 * round takes the ranks [lo, min(lo + window, end of the class)), lo the
 * lowest rank of the class not yet placed; each unplaced sphere i of the
 * round proposes attempt a_i of the SplitMix64 stream of rcp_pack_init,
 * (u(seed, i, a_i, axis) L); a proposal is valid when it overlaps no placed
 * sphere (r^2 < (kappa (D0_i + D0_j)/2)^2, minimum image, no contraction),
 * and a valid proposal is placed unless a valid proposal of a lower rank in
 * the same round overlaps it; the others move on to their next attempt.
 * With window = 1 this is the host placement of RCP_INIT_RSA attempt for
 * attempt.  The positions replace the packing's state as rcp_set_state
 * does.  rounds (may be NULL) receives the number of rounds.  RCP_EINVAL for
 * window < 1 or more than 64 size classes, RCP_EPLACE when a sphere needs
 * more than 2^22 attempts (a fraction above what random sequential addition
 * can reach, about 0.38 for equal spheres and 0.55 for equal disks, takes
 * that many rounds before it fails: minutes). */
int rcp_place_device(rcp_ctx *ctx, int k, uint64_t seed, int64_t window, int64_t *rounds);

/* Frozen spheres, for the stages of the sequential multimodal cascade
 * (Sec. 4: a finer class is seated in the voids of the coarser ones and
 * inflated with the coarser classes held fixed).  mask: n bytes in user
 * order (host, copied); mask[i] != 0 freezes sphere i: its D0 (as given at
 * creation) is then an absolute diameter that does not scale with kappa,
 * and it takes no Adam step; the others keep D = kappa D0.  The energy of
 * Eq. (energy) becomes E = 1/2 sum delta^2 - mu kappa sum over the spheres
 * not frozen of D0, with d_ij = (sigma_i + sigma_j) / 2 (sigma = D0 frozen,
 * kappa D0 otherwise), and dE/dkappa = sum delta (r / d^2) dd_ij/dkappa -
 * mu sum D0 over the spheres not frozen; the relative schedule's scales
 * (sum D0, N_v, D0_min) are taken over the spheres not frozen.  Lists are
 * built at max(kappa, 1).  No shrink is done for such a packing: its
 * result reports kappa and phi as they are (the release that follows, a
 * new context with every sphere free, ends with the shrink).  mask = NULL
 * (or all zero) frees every sphere.  While any packing of the context has
 * frozen spheres, the iteration uses the two-gather kernel whatever the
 * tuning variant, and the tail is not fused.  RCP_EINVAL when every sphere
 * would be frozen, or when the packing has walls (rcp_set_boundary). */
int rcp_set_frozen(rcp_ctx *ctx, int k, const uint8_t *mask);

/* Hard walls of packing k (Sec. 2: every coordinate direction may be
 * periodic or bounded by a flat or curved hard wall; rectilinear, circular,
 * cylindrical and spherical domains).  Bit a of `walls` puts flat walls at
 * x_a = 0 and x_a = L across axis a; `round` names the axes (two or three)
 * of a round container, the disk or ball of diameter L centred at L/2 on
 * them (a circle in two dimensions; in three, a cylinder along the
 * remaining axis, or a sphere); the remaining axes stay periodic.  A
 * bounded axis has no image and positions on it are not wrapped.  The
 * paper gives no wall energy; ours: a sphere of diameter sigma whose centre
 * is at distance h from a wall overlaps it when 2h < sigma, with
 * delta = 1 - 2h / sigma (the pair term of Eq. (energy) with the sphere's
 * mirror image) and energy delta^2 / 2, counted in E_overlap,
 * dE_dkappa_overlap (delta (2h / sigma) / kappa), max_overlap (so in the
 * stop test) and n_overlap.  2h is 2 x_a and 2 (L - x_a) for flat walls and
 * L - 2 rho for the round one, rho the distance from the container's axis
 * or centre.  Device placement (rcp_place_device) then accepts only
 * proposals that touch no wall at the placement scale (flat:
 * fl(kappa D0) <= 2 x_a and <= 2 (L - x_a); round: t = L - fl(kappa D0) >= 0
 * and t^2 >= 4 rho^2, no contraction), the shrink keeps every sphere clear
 * of the walls by the same tests, and phi divides by the container's
 * volume (L per plain axis, (pi/4) L^2 or (pi/6) L^3 over the round axes).
 * Host placement at creation (RCP_INIT_RSA) knows no walls: create with
 * RCP_INIT_NONE, set the boundary, then place with rcp_place_device or set
 * positions with rcp_set_state.  The list is rebuilt before the next
 * evaluation.  While any packing has walls, the iteration uses the
 * two-gather kernel whatever the tuning variant, and the tail is not
 * fused.  walls = round = 0 is the periodic box.  RCP_EINVAL for an axis
 * beyond dim, an axis in both masks, a round container of one axis, or a
 * packing with frozen spheres (walls and frozen spheres are not
 * combined). */
int rcp_set_boundary(rcp_ctx *ctx, int k, uint32_t walls, uint32_t round);

/* Seating of a new class in the voids of the frozen spheres (Sec. 4): every
 * sphere of packing k that is not frozen gets, independently, its first
 * proposal of the placement counter stream (the one of rcp_place_device,
 * attempt a = 0, 1, ...) that overlaps no frozen sphere at the seating scale
 * kappa0: r^2 < ((D_frozen + kappa0 D0_i) / 2)^2 rejects.  Spheres that are not
 * frozen may overlap one another (the inflation that follows separates
 * them).  Frozen positions are kept; then the state is set as by
 * rcp_set_state(positions, kappa0).  RCP_EINVAL for kappa0 <= 0 or
 * max_attempts < 1, RCP_EPLACE when a sphere needs more than max_attempts. */
int rcp_seat_device(rcp_ctx *ctx, int k, double kappa0, uint64_t seed, int64_t max_attempts);

/* Replace the launch tuning (see rcp_tuning); RCP_EINVAL for values out of
 * range.  A captured graph is re-captured at the next iteration.  Tuning
 * changes launch shapes only; the method (App. A) is unchanged. */
int rcp_set_tuning(rcp_ctx *ctx, const rcp_tuning *t);

/* Replace the listing skin (skin_s, skin_g of rcp_params) of every packing
 * of the context, e.g. by an autotuner between iterations of a run; every
 * built list is rebuilt before the next iteration.  The trajectory does not
 * depend on the skin beyond summation order.  RCP_EINVAL for a negative or
 * non-finite value, RCP_EBOX if a packing's largest cutoff at its current
 * kappa would not be below L/2 (nothing is changed then). */
int rcp_set_skin(rcp_ctx *ctx, double skin_s, double skin_g);

/* Replace positions (row-major (n, dim), user order) and kappa of packing k
 * (the state of the optimised energy, Eq. (energy) of App. A); x is a host
 * pointer (is_device == 0, every value in [-L, 2L), wrapped into [0, L)) or
 * a device pointer (is_device != 0, values already in [0, L); dim = 3
 * only).  Resets the
 * Adam moments and step counter (as after placement) and the schedule
 * position, and marks the neighbour list stale.  RCP_EINVAL for a bad
 * kappa or a host position outside [-L, 2L). */
int rcp_set_state(rcp_ctx *ctx, int k, const double *x, double kappa,
                  int is_device);

/* Copy positions (n, dim, user order), kappa and optionally the working
 * diameters kappa D0 (n) of packing k to host memory (App. A: the outputs
 * of a run are the positions and the scaled diameters).  x, kappa and diam
 * may each be NULL. */
int rcp_get_state(rcp_ctx *ctx, int k, double *x, double *kappa, double *diam);

/* Optimiser state of one packing beyond its positions and kappa: App. A
 * applies Adam (Kingma and Ba, bias corrected) to every coordinate and to
 * kappa with one step counter, and anneals mu through the rungs of a
 * schedule.  size must be sizeof(rcp_optimizer). */
typedef struct {
    uint32_t size;
    int32_t rung;          /* rung of the loaded schedule in force            */
    int64_t t;             /* Adam step counter (0 = no step taken)           */
    int64_t it_rung;       /* iterations taken in the current rung            */
    int64_t iterations;    /* iterations of the current run                   */
    double m_kappa, v_kappa;   /* first and second moments of kappa           */
    double mu, eta_x, eta_k;   /* growth pressure and step sizes in force     */
} rcp_optimizer;

/* Copy the optimiser state of packing k: the first and second moments of
 * every coordinate (m, v: (n, dim) row-major, user order, host; either may be
 * NULL) and the scalars in *opt.  Together with rcp_get_state this is a
 * complete checkpoint of a run in progress. */
int rcp_get_optimizer(rcp_ctx *ctx, int k, double *m, double *v, rcp_optimizer *opt);

/* Restore the optimiser state of packing k from a checkpoint (host arrays
 * as rcp_get_optimizer writes them; m or v NULL leaves that array as it
 * is).  To resume a run: rcp_set_state (positions, kappa), rcp_run_start
 * (loads the schedule and resets the optimiser), rcp_set_optimizer, then
 * rcp_run_continue.  The resumed trajectory equals the uninterrupted one up
 * to the summation order of the gradient (the neighbour list is rebuilt at
 * the resume point).  RCP_EINVAL for t < 0, a rung outside the loaded
 * schedule, v < 0 or non-finite values. */
int rcp_set_optimizer(rcp_ctx *ctx, int k, const double *m, const double *v,
                      const rcp_optimizer *opt);

/* Build the neighbour list of packing k at its current (x, kappa), with
 * kb = kappa (App. A keeps a neighbour structure that is rebuilt when the
 * accumulated displacement demands it; the listing rule is that of
 * rcp_params).  n_pairs (may be NULL) receives the number of listed pairs
 * (each counted once).  RCP_EBOX if the largest listing cutoff is not below
 * L/2; RCP_ENOMEM if the list would exceed 2^31 - 1 entries (both
 * directions counted). */
int rcp_neighbor_build(rcp_ctx *ctx, int k, int64_t *n_pairs);

/* Canonical pair set of the current list of packing k: every pair (i, j)
 * whose separation r (minimum image, Sec. 2) satisfies r^2 < c^2 with the
 * listing cutoff c of rcp_params, as i < j in user indices, lexicographic.
 * Writes min(count, cap) pairs to the host arrays i, j (NULL allowed with
 * cap = 0) and sets *count.  RCP_ESTATE if no list has been built. */
int rcp_get_pairs(rcp_ctx *ctx, int k, int32_t *i, int32_t *j, int64_t cap,
                  int64_t *count);

/* Energy terms and gradient of Eq. (energy) at packing k's current state
 * with the given mu; rebuilds the list first if it is not valid.  grad_x
 * (n, dim, user order, host) may be NULL. */
int rcp_energy_grad(rcp_ctx *ctx, int k, double mu, rcp_energy *e,
                    double *grad_x);

/* n_steps Adam updates (App. A: Adam on every coordinate and on kappa,
 * Kingma and Ba with bias correction) of every packing with fixed mu,
 * eta_x, eta_k (absolute numbers), the neighbour list rebuilt whenever its
 * validity test fails; no stop test.  The moments and the step counter
 * carry over from the previous call (adam_step(a) then adam_step(b) is
 * adam_step(a + b)); they start at zero after placement, rcp_set_state and
 * rcp_run_start.  RCP_EINVAL for n_steps < 1, a non-finite mu or a negative
 * step size; RCP_ENONFINITE if a gradient became NaN or Inf. */
int rcp_adam_step(rcp_ctx *ctx, double mu, double eta_x, double eta_k,
                  int64_t n_steps);

/* Inflation run of App. A: Adam on positions and kappa under the annealing
 * schedule (rungs of Eq. (trigger) length), stop test in the final rung,
 * then shrink to contact (Sec. 2).  Starts from the current positions and
 * kappa with fresh optimiser moments.
 * Run the schedule (sched[k] for packing k, or sched[0] for all when
 * per_packing == 0) until every packing has stopped, hit its cap, or
 * max_iters iterations were taken (0: no limit); then shrink each packing
 * to contact.  results has n_prob entries.  Returns 0, or RCP_ENOTCONV /
 * RCP_ENONFINITE / RCP_EBOX if any packing ended that way (its result's
 * status says which).  In a context with several packings, a packing whose
 * listing cutoff reaches L/2 is stopped with status RCP_EBOX and the others
 * run on; with one packing the call fails at that point. */
int rcp_inflate_run(rcp_ctx *ctx, const rcp_schedule *sched, int per_packing,
                    int64_t max_iters, rcp_result *results);

/* The run of rcp_inflate_run in steps: rcp_run_start loads the schedule(s)
 * and resets the optimiser state of every packing without iterating;
 * rcp_run_continue then advances every active packing by up to n_iters
 * iterations (0: until each has stopped or reached its cap) and reports
 * in *active how many packings can still continue.  No shrink is done;
 * rcp_run_result fills a result for packing k from its current state
 * (shrink included) without changing that state. */
int rcp_run_start(rcp_ctx *ctx, const rcp_schedule *sched, int per_packing);
int rcp_run_continue(rcp_ctx *ctx, int64_t n_iters, int32_t *active);

/* Capture the HIP graph of graph_iters iterations (App. A's iteration, as
 * rcp_run_continue launches it) ahead of the next rcp_run_continue, which
 * then does not pay for the capture.  The graph stays valid until the
 * tuning or the work-item layout changes (a list build that changes the
 * number of work items); the graph is uploaded to the device, nothing is
 * launched.  No-op for graph_iters 1. */
int rcp_run_prepare(rcp_ctx *ctx);
int rcp_run_result(rcp_ctx *ctx, int k, rcp_result *result);

/* Census entry point (Sec. 3 generates its census of packings one run at a
 * time; here the runs of a batch share every launch): rcp_inflate_run over
 * every packing of a context made by rcp_census_init, one launch per
 * iteration for the whole batch.  Every packing's result is the one a
 * context of its own would give. */
int rcp_census_run(rcp_ctx *ctx, const rcp_schedule *sched, int per_packing,
                   int64_t max_iters, rcp_result *results);

/* Shrink to contact of packing k at its current state (Sec. 2, App. A):
 * kappa' is the largest double <= kappa such that every listed pair has
 * fl(fl(kappa' d0)^2) <= r^2 with d0 = (D0_i + D0_j)/2 and, with walls
 * (rcp_set_boundary), every sphere clears them by the placement tests at
 * scale kappa'; phi is the volume (area) fraction at kappa' over the
 * container's volume. */
int rcp_shrink(rcp_ctx *ctx, int k, double *kappa_shrunk, double *phi);

/* Raw device entry points for torch.autograd.Function (packing 0; App. A,
 * Eq. (energy) and its gradient; dim = 3 only).  x_dev: (n, 3) row-major positions in user
 * order on the device, borrowed until the work on `stream` completes.
 * stream is the caller's hipStream_t and NULL means the null stream (not
 * the context's own): reads of x_dev and writes of the outputs are ordered
 * on it.  The list is rebuilt at (x_dev, kappa) if it is not valid there
 * (this synchronises the stream): packing 0 then takes x_dev and kappa as
 * its state, exactly as rcp_set_state would (its optimiser state is reset),
 * so a context used for evaluation should not also carry a run.
 * rcp_energy_dev writes E = E_overlap + E_growth to E_dev[0] and max overlap
 * to E_dev[1].  rcp_adjoint_dev writes dE/dx (n, 3, user order) to gx_dev
 * and dE/dkappa to gk_dev[0]. */
int rcp_energy_dev(rcp_ctx *ctx, const double *x_dev, double kappa, double mu,
                   double *E_dev, void *stream);
int rcp_adjoint_dev(rcp_ctx *ctx, const double *x_dev, double kappa, double mu,
                    double *gx_dev, double *gk_dev, void *stream);

/* For callers that cannot allocate device memory (code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
 * energy of rcp_energy_dev (E = E_overlap + E_growth to E_dev[0], max overlap
 * to E_dev[1]; same arguments, same kernels and summation order, so the same
 * bits) with no allocation and no list rebuild.  Its block partials live in
 * a fixed device array of the library, one per GPU, sized for at most 2^24
 * spheres (2 MiB plus 512 bytes), held until the process ends.  Packing 0's
 * neighbour list must already be valid at (x_dev, kappa) (rcp_neighbor_build
 * or an rcp_energy_dev call at nearby positions builds one); RCP_ESTATE
 * otherwise, RCP_EINVAL for more than 2^24 spheres, a null pointer or a bad
 * kappa or mu.  The array keeps the last call's contents and is shared by
 * every call on that GPU, whatever the context: calls that overlap on one
 * GPU (several threads or streams) race, and the caller must serialise them.
 * The call synchronises the context's stream and `stream` (the validity test
 * reads one number back). */
int rcp_energy_dev_static(rcp_ctx *ctx, const double *x_dev, double kappa, double mu,
                          double *E_dev, void *stream);

/* Kernel timing of the running schedule: like rcp_run_continue(ctx,
 * n_iters) but each iteration is launched on its own, with HIP events
 * recorded on the context's stream around the gradient + Adam kernel and
 * around the tail kernel.  Writes the mean durations (microseconds) over
 * the iterations that did work, and how many those were (*done).  Rebuilds
 * that fall in the window run as usual and are not timed here. */
int rcp_time_iterations(rcp_ctx *ctx, int64_t n_iters, double *iterate_us, double *tail_us,
                        int64_t *done);

/* Counters and timings accumulated by the context (see rcp_stats; the
 * particle-update rate of App. A's iterations is particle_updates divided
 * by the iteration time); rcp_reset_stats zeroes them. */
int rcp_get_stats(rcp_ctx *ctx, rcp_stats *s);
int rcp_reset_stats(rcp_ctx *ctx);
/* Number of packings of a context, and spheres in packing k (-1 for a bad
 * context or index). */
int rcp_num_packings(rcp_ctx *ctx);
int64_t rcp_num_particles(rcp_ctx *ctx, int k);
/* Release every device and host buffer of the context (waits for its
 * stream).  NULL is ignored. */
void rcp_destroy(rcp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* RCP_H */
