/*
 * FP64 CPU oracle for the Adam-based inflation protocol.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding
 * may include, link or call this file; it is built and called by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark.  It
 * shares no code with the HIP path.
 *
 * What is computed, and where the paper defines it:
 *   - soft finite-range overlap energy E = (eps/2) sum_{i<j} (1 - r/d)^2
 *     Theta(1 - r/d) - mu sum_i D_i with d = (D_i + D_j)/2 and D_i = kappa D0_i
 *     (App. A, Eq. (energy)); eps = 1 (Adam is invariant to its scale);
 *   - the gradient of E w.r.t. the positions and kappa (derived from
 *     Eq. (energy); the paper does not print it);
 *   - Adam (Kingma and Ba, bias corrected) on every coordinate and on kappa
 *     (App. A);
 *   - the annealing schedule, read as a table of rungs (App. A and
 *     Eq. (trigger)); the rung values themselves are unstated in the paper;
 *   - the stop rule: in the final rung, max fractional overlap below the
 *     tolerance (5e-4 in App. A);
 *   - shrink to contact: the largest kappa' <= kappa with no overlapping pair
 *     (Sec. 2, App. A);
 *   - random sequential addition at low volume fraction (App. A mentions a
 *     cell-list placement without overlap; the algorithm is our reading);
 *   - candidate pairs: brute force O(N^2), per-row brute force for subsets,
 *     and a plain size-class cell list (App. A uses a k-d tree; any method
 *     that returns the same pair set is equivalent);
 *   - frozen spheres for the stages of the sequential multimodal cascade
 *     (Sec. 4): a frozen sphere keeps its position and an absolute
 *     diameter while the other spheres inflate (see orc_set_frozen), and
 *     the seating of a new class in the voids of the frozen ones;
 *   - the spatial dimension d (the paper's input, Sec. 2; Fig. 1 is
 *     2-D): d = 2 packs disks in the plane z = 0 (see orc_set_dim);
 *   - hard walls (Sec. 2: each axis periodic or bounded by a flat or curved
 *     hard wall): flat walls per axis and a round container over two or
 *     three axes (see orc_set_boundary).
 *
 * Floating point: compiled with -ffp-contract=off; every quantity is double.
 * Sums of many terms (energy, kappa gradient) use Neumaier compensation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_RUNGS 16

/* ------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014), addressed as a counter stream */
/* ------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_u01(uint64_t seed, uint64_t i, uint64_t attempt, int axis)
{
    uint64_t k = ((i << 24) | attempt) * 4u + (uint64_t)axis;
    return (double)(orc_splitmix64(seed, k) >> 11) * 0x1p-53;
}

/* The spatial dimension, 3 or 2 (see orc_set_dim). */
static int g_dim = 3;

/* Boundary (see orc_set_boundary): bit a of g_walls = flat walls across
 * axis a, bit a of g_round = axis a is one of the round container's. */
static unsigned g_walls = 0, g_round = 0;

static inline int periodic(int a) { return !(((g_walls | g_round) >> a) & 1u); }

/* Coordinate ax of attempt a of sphere i: u(seed, i, a, ax) L in [0, L);
 * 0 for ax = 2 in two dimensions (not drawn). */
static inline double coord_draw(uint64_t seed, int64_t i, int64_t a, int ax, double L)
{
    if (ax == 2 && g_dim == 2) return 0.0;
    double v = orc_u01(seed, (uint64_t)i, (uint64_t)a, ax) * L;
    if (v >= L) v -= L;
    return v;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Minimum image and the canonical pair predicate                      */
/* ------------------------------------------------------------------ */
/* Positions live in [0, L).  The separation is shifted by one box length
 * when it exceeds half a box (the largest sphere may not meet its own image,
 * Sec. 2).  Exactly at +-L/2 no shift is applied. */
static inline double mimg(double d, double L, double hL)
{
    if (d > hL) return d - L;
    if (d < -hL) return d + L;
    return d;
}

/* Along an axis bounded by walls there is no image: the plain difference. */
static inline double mimg_ax(double d, int a, double L, double hL)
{
    return periodic(a) ? mimg(d, L, hL) : d;
}

static inline double sep2(const double *x, int64_t i, int64_t j, double L,
                          double hL, double *dx, double *dy, double *dz)
{
    *dx = mimg_ax(x[3 * j] - x[3 * i], 0, L, hL);
    *dy = mimg_ax(x[3 * j + 1] - x[3 * i + 1], 1, L, hL);
    *dz = mimg_ax(x[3 * j + 2] - x[3 * i + 2], 2, L, hL);
    return (*dx * *dx + *dy * *dy) + *dz * *dz;
}

/* Neighbour-list cutoff of a pair listed at scale kb:
 *   c = kb * ((1 + g) * (0.5 * (D0_i + D0_j)) + 2 s D0_min).
 * The pair is listed iff r^2 < c^2.  opg = 1 + g and sk2 = (2 s) D0_min are
 * computed once by the caller. */
static inline double cutoff(double di, double dj, double kb, double opg,
                            double sk2)
{
    return kb * (opg * (0.5 * (di + dj)) + sk2);
}

/* ------------------------------------------------------------------ */
/* Pair sets                                                          */
/* ------------------------------------------------------------------ */
typedef struct { int32_t i, j; } pair_t;

static int cmp_pair(const void *a, const void *b)
{
    const pair_t *p = a, *q = b;
    if (p->i != q->i) return p->i < q->i ? -1 : 1;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    return 0;
}

/* All pairs i<j with r^2 < c^2, by testing every pair.  Output is already
 * lexicographic.  Returns the number of pairs (may exceed cap; then only
 * cap are written). */
int64_t orc_pairs_brute(int64_t n, const double *x, const double *d0, double L,
                        double kb, double s, double g, double d0min,
                        int32_t *pi, int32_t *pj, int64_t cap)
{
    const double hL = 0.5 * L, opg = 1.0 + g, sk2 = (2.0 * s) * d0min;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double dx, dy, dz;
            double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
            double c = cutoff(d0[i], d0[j], kb, opg, sk2);
            if (r2 < c * c) {
                if (cnt < cap) { pi[cnt] = (int32_t)i; pj[cnt] = (int32_t)j; }
                ++cnt;
            }
        }
    return cnt;
}

/* For each requested row i, every j != i with r^2 < c^2, ascending j, by
 * testing all N candidates.  Pass nbr == NULL to get the counts only.
 * offs[k] is where row k's list starts in nbr (caller computes it from the
 * counts of a first call). */
void orc_rows_pairs(int64_t n, const double *x, const double *d0, double L,
                    double kb, double s, double g, double d0min,
                    const int64_t *rows, int64_t nrows, int64_t *counts,
                    const int64_t *offs, int32_t *nbr)
{
    const double hL = 0.5 * L, opg = 1.0 + g, sk2 = (2.0 * s) * d0min;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k], c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
            double cc = cutoff(d0[i], d0[j], kb, opg, sk2);
            if (r2 < cc * cc) {
                if (nbr) nbr[offs[k] + c] = (int32_t)j;
                ++c;
            }
        }
        counts[k] = c;
    }
}

/* Size-class cell list.  Class of particle i: floor(log2(D0_i / D0_min)).
 * Class l gets a cubic grid whose cells are at least as wide as the largest
 * cutoff between a class-l particle and any particle of class <= l, so a
 * particle of class <= l finds every listed partner of class l in the 27
 * cells around it.  Each particle searches its own class (partners with a
 * larger index only) and every larger class. */
typedef struct { int64_t key; int32_t idx; } kv_t;

static int cmp_kv(const void *a, const void *b)
{
    const kv_t *p = a, *q = b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

typedef struct {
    int nlev;
    int *lev;          /* class of each particle */
    int64_t *nc;       /* cells per axis per class */
    double *w;         /* cell width per class */
    int64_t *start;    /* start of class l in kv */
    int64_t *count;
    kv_t *kv;          /* particles sorted by (class, cell) */
} cells_t;

static int64_t cell_of(double xv, double w, int64_t nc)
{
    int64_t c = (int64_t)(xv / w);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

static void cells_build(cells_t *C, int64_t n, const double *x, const double *d0,
                        double L, double kb, double opg, double sk2, double d0min)
{
    C->lev = malloc(sizeof(int) * (size_t)n);
    int nlev = 1;
    for (int64_t i = 0; i < n; ++i) {
        int l = (int)floor(log2(d0[i] / d0min));
        if (l < 0) l = 0;
        C->lev[i] = l;
        if (l + 1 > nlev) nlev = l + 1;
    }
    C->nlev = nlev;
    double *dmax = calloc((size_t)nlev, sizeof(double));
    C->count = calloc((size_t)nlev, sizeof(int64_t));
    C->start = calloc((size_t)nlev + 1, sizeof(int64_t));
    C->nc = calloc((size_t)nlev, sizeof(int64_t));
    C->w = calloc((size_t)nlev, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        if (d0[i] > dmax[C->lev[i]]) dmax[C->lev[i]] = d0[i];
        C->count[C->lev[i]]++;
    }
    double run = 0.0;
    for (int l = 0; l < nlev; ++l) {
        if (dmax[l] > run) run = dmax[l];
        double h = kb * (opg * run + sk2) * (1.0 + 1e-12);
        int64_t nc = (int64_t)floor(L / h);
        if (nc < 1) nc = 1;
        if (nc > (1 << 20)) nc = 1 << 20;
        C->nc[l] = nc;
        C->w[l] = L / (double)nc;
        C->start[l + 1] = C->start[l] + C->count[l];
    }
    C->kv = malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = calloc((size_t)nlev, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int l = C->lev[i];
        int64_t nc = C->nc[l];
        double w = C->w[l];
        int64_t cx = cell_of(x[3 * i], w, nc), cy = cell_of(x[3 * i + 1], w, nc),
                cz = cell_of(x[3 * i + 2], w, nc);
        kv_t e = {(cx * nc + cy) * nc + cz, (int32_t)i};
        C->kv[C->start[l] + fill[l]++] = e;
    }
    for (int l = 0; l < nlev; ++l)
        qsort(C->kv + C->start[l], (size_t)C->count[l], sizeof(kv_t), cmp_kv);
    free(fill);
    free(dmax);
}

static void cells_free(cells_t *C)
{
    free(C->lev); free(C->nc); free(C->w); free(C->start); free(C->count);
    free(C->kv);
}

static int64_t lower_key(const kv_t *a, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid].key < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Half pairs found from particle i: partners of the same class with a larger
 * index, and partners of every larger class.  Writes up to cap partners
 * into out (if non-NULL) and returns how many there are. */
static int64_t cells_search(const cells_t *C, int64_t i, const double *x,
                            const double *d0, double L, double kb, double opg,
                            double sk2, int32_t *out)
{
    const double hL = 0.5 * L;
    int64_t cnt = 0;
    for (int l = C->lev[i]; l < C->nlev; ++l) {
        if (C->count[l] == 0) continue;
        int64_t nc = C->nc[l];
        double w = C->w[l];
        int64_t c[3];
        for (int a = 0; a < 3; ++a) c[a] = cell_of(x[3 * i + a], w, nc);
        int64_t lo = nc >= 3 ? -1 : 0, hi = nc >= 3 ? 1 : nc - 1;
        const kv_t *kv = C->kv + C->start[l];
        for (int64_t ox = lo; ox <= hi; ++ox)
            for (int64_t oy = lo; oy <= hi; ++oy)
                for (int64_t oz = lo; oz <= hi; ++oz) {
                    int64_t ax, ay, az;
                    if (nc >= 3) {
                        ax = (c[0] + ox + nc) % nc;
                        ay = (c[1] + oy + nc) % nc;
                        az = (c[2] + oz + nc) % nc;
                    } else {
                        ax = ox; ay = oy; az = oz;
                    }
                    int64_t key = (ax * nc + ay) * nc + az;
                    for (int64_t p = lower_key(kv, C->count[l], key);
                         p < C->count[l] && kv[p].key == key; ++p) {
                        int64_t j = kv[p].idx;
                        if (l == C->lev[i] && j <= i) continue;
                        double dx, dy, dz;
                        double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
                        double cc = cutoff(d0[i], d0[j], kb, opg, sk2);
                        if (r2 < cc * cc) {
                            if (out) out[cnt] = (int32_t)j;
                            ++cnt;
                        }
                    }
                }
    }
    return cnt;
}

/* Half pair list in search order (deterministic, independent of threads). */
static int64_t cells_half_pairs(int64_t n, const double *x, const double *d0,
                                double L, double kb, double s, double g,
                                double d0min, int32_t **pi_out, int32_t **pj_out)
{
    const double opg = 1.0 + g, sk2 = (2.0 * s) * d0min;
    cells_t C;
    cells_build(&C, n, x, d0, L, kb, opg, sk2, d0min);
    int64_t *cnt = malloc(sizeof(int64_t) * (size_t)(n + 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        cnt[i] = cells_search(&C, i, x, d0, L, kb, opg, sk2, NULL);
    int64_t tot = 0;
    for (int64_t i = 0; i < n; ++i) { int64_t c = cnt[i]; cnt[i] = tot; tot += c; }
    cnt[n] = tot;
    int32_t *pi = malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    int32_t *pj = malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = cells_search(&C, i, x, d0, L, kb, opg, sk2, pj + cnt[i]);
        for (int64_t q = 0; q < k; ++q) pi[cnt[i] + q] = (int32_t)i;
    }
    free(cnt);
    cells_free(&C);
    *pi_out = pi;
    *pj_out = pj;
    return tot;
}

/* Canonical pair set from the cell list: (min, max) per pair, sorted. */
int64_t orc_pairs_cells(int64_t n, const double *x, const double *d0, double L,
                        double kb, double s, double g, double d0min,
                        int32_t *pi, int32_t *pj, int64_t cap)
{
    int32_t *a, *b;
    int64_t tot = cells_half_pairs(n, x, d0, L, kb, s, g, d0min, &a, &b);
    pair_t *p = malloc(sizeof(pair_t) * (size_t)(tot > 0 ? tot : 1));
    for (int64_t k = 0; k < tot; ++k) {
        p[k].i = a[k] < b[k] ? a[k] : b[k];
        p[k].j = a[k] < b[k] ? b[k] : a[k];
    }
    qsort(p, (size_t)tot, sizeof(pair_t), cmp_pair);
    for (int64_t k = 0; k < tot && k < cap; ++k) { pi[k] = p[k].i; pj[k] = p[k].j; }
    free(p); free(a); free(b);
    return tot;
}

/* ------------------------------------------------------------------ */
/* Spatial dimension (Sec. 2: the dimension is an input; Fig. 1, 2-D)  */
/* ------------------------------------------------------------------ */
/* d = 3 (default) or 2.  With d = 2 every position has z = 0: placement
 * proposes only x and y (axis 2 of the counter stream is not drawn), the
 * energy, its gradient (whose z components then vanish) and Adam are the
 * 3-D ones restricted to the plane, the volume participation number of
 * the schedule is (sum D^2)^2 / sum D^4 and the packing fraction is the
 * area fraction (pi / 4) sum D^2 / L^2. */
void orc_set_dim(int d) { g_dim = (d == 2) ? 2 : 3; }

/* ------------------------------------------------------------------ */
/* Hard walls (Sec. 2: every axis periodic or bounded by a flat or     */
/* curved hard wall; Fig. capabilities)                                */
/* ------------------------------------------------------------------ */
/* The paper names the boundaries but prints no wall energy.  Our reading:
 *   - flat walls across axis a (bit a of walls): planes x_a = 0 and
 *     x_a = L;
 *   - a round container over the axes of `round` (two or three of them):
 *     the ball of diameter L centred at L/2 on those axes (a circle in
 *     2-D, a cylinder along the remaining axis or a sphere in 3-D);
 *   - other axes stay periodic; a bounded axis has no image;
 *   - a sphere of diameter sigma whose centre is at distance h from a wall
 *     overlaps it when 2h < sigma, with delta = 1 - 2h / sigma (the overlap
 *     depth over the radius, as 1 - r/d is the depth over the contact
 *     distance of a pair; equivalently the pair term with the sphere's
 *     mirror image, r = 2h and d = sigma) and energy delta^2 / 2, added to
 *     the pair energy of Eq. (energy) and to the max overlap of the stop
 *     rule;
 *   - 2h is 2 x_a and 2 (L - x_a) for the flat walls and L - 2 rho for the
 *     round one, rho the distance from the axis (or centre) over the round
 *     axes, summed in axis order;
 *   - gradient: d delta / d x_a = -2 / sigma and +2 / sigma for the lower and
 *     upper flat walls, 2 (x_a - L/2) / (sigma rho) for the round wall;
 *     dE/dkappa gains delta (2h / sigma) / kappa (sigma = kappa D0);
 *   - the packing fraction is the sphere volume over the domain's volume
 *     (the round axes contribute the disk or ball of diameter L);
 *   - placement accepts only proposals that touch no wall at the placement
 *     scale, and shrink to contact keeps every sphere clear of the walls.
 * Frozen spheres are not combined with walls. */
void orc_set_boundary(unsigned walls, unsigned round)
{
    g_walls = walls & 7u;
    g_round = round & 7u;
}

/* rho^2 of position p over the round axes, in axis order. */
static inline double round_rho2(const double *p, double L)
{
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a)
        if ((g_round >> a) & 1u) {
            const double u = p[a] - 0.5 * L;
            r2 = r2 + u * u;
        }
    return r2;
}

/* Wall terms of a sphere of diameter sig at p: e += delta^2 / 2, s +=
 * delta (2h / sig), m = max(m, delta), *cnt += contacts; g3 += dE/dx and
 * gs3 += |dE/dx| (each may be NULL). */
static void wall_terms(const double *p, double sig, double L, double *g3, double *gs3,
                       double *e, double *s, double *m, int64_t *cnt)
{
    for (int a = 0; a < 3; ++a) {
        if (!((g_walls >> a) & 1u)) continue;
        for (int side = 0; side < 2; ++side) {
            const double gap = side == 0 ? 2.0 * p[a] : 2.0 * (L - p[a]);
            if (!(gap < sig)) continue;
            const double delta = 1.0 - gap / sig;
            *e += 0.5 * delta * delta;
            *s += delta * (gap / sig);
            if (delta > *m) *m = delta;
            ++*cnt;
            const double c = (side == 0 ? -2.0 : 2.0) * delta / sig;
            if (g3) g3[a] += c;
            if (gs3) gs3[a] += fabs(c);
        }
    }
    if (g_round) {
        const double rho = sqrt(round_rho2(p, L));
        const double gap = L - 2.0 * rho;
        if (gap < sig) {
            const double delta = 1.0 - gap / sig;
            *e += 0.5 * delta * delta;
            *s += delta * (gap / sig);
            if (delta > *m) *m = delta;
            ++*cnt;
            if (rho > 0.0)
                for (int a = 0; a < 3; ++a)
                    if ((g_round >> a) & 1u) {
                        const double c = 2.0 * delta * (p[a] - 0.5 * L) / (sig * rho);
                        if (g3) g3[a] += c;
                        if (gs3) gs3[a] += fabs(c);
                    }
        }
    }
}

/* Does a sphere of diameter fl(k D0) at p clear the round wall?  In squares,
 * so that the answer is fixed by the rounding of + and * alone:
 * t = L - k D0 >= 0 and t^2 >= 4 rho^2 (the same as L - 2 rho >= k D0). */
static inline int round_clear(double k, double d0, double L, double q4)
{
    const double t = L - k * d0;
    return t >= 0.0 && t * t >= q4;
}

/* Largest double k with fl(k D0) <= gap (a flat wall), or with
 * round_clear (the round wall); 0 when even k = 0 does not clear. */
static double flat_kmax(double gap, double d0)
{
    if (!(gap > 0.0)) return 0.0;
    double k = gap / d0;
    while (k > 0.0 && k * d0 > gap) k = nextafter(k, 0.0);
    for (;;) {
        const double up = nextafter(k, INFINITY);
        if (up * d0 <= gap) k = up; else break;
    }
    return k;
}

static double round_kmax(double q4, double d0, double L)
{
    if (!round_clear(0.0, d0, L, q4)) return 0.0;
    double k = (L - sqrt(q4)) / d0;
    if (k < 0.0) k = 0.0;
    while (k > 0.0 && !round_clear(k, d0, L, q4)) k = nextafter(k, 0.0);
    for (;;) {
        const double up = nextafter(k, INFINITY);
        if (round_clear(up, d0, L, q4)) k = up; else break;
    }
    return k;
}

/* Largest scale at which sphere i (relative diameter d0) at p clears every
 * wall (INFINITY with no walls). */
static double wall_kmax(const double *p, double d0, double L)
{
    double k = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (!((g_walls >> a) & 1u)) continue;
        const double lo = flat_kmax(2.0 * p[a], d0), hi = flat_kmax(2.0 * (L - p[a]), d0);
        if (lo < k) k = lo;
        if (hi < k) k = hi;
    }
    if (g_round) {
        const double r = round_kmax(4.0 * round_rho2(p, L), d0, L);
        if (r < k) k = r;
    }
    return k;
}

/* Placement test: a sphere of diameter sig at p touches no wall (touching
 * allowed), with the predicates of the shrink. */
static int inside_walls(const double *p, double sig, double L)
{
    for (int a = 0; a < 3; ++a) {
        if (!((g_walls >> a) & 1u)) continue;
        if (!(sig <= 2.0 * p[a]) || !(sig <= 2.0 * (L - p[a]))) return 0;
    }
    if (g_round) {
        const double t = L - sig;
        if (!(t >= 0.0 && t * t >= 4.0 * round_rho2(p, L))) return 0;
    }
    return 1;
}

/* Volume (area in 2-D) of the domain: L per plain axis, the disk or ball of
 * diameter L over the round axes. */
static double domain_volume(double L)
{
    int k = 0;
    double v = 1.0;
    for (int a = 0; a < g_dim; ++a) {
        if ((g_round >> a) & 1u) ++k;
        else v = v * L;
    }
    if (k == 2) v = v * ((M_PI / 4.0) * (L * L));
    if (k == 3) v = v * ((M_PI / 6.0) * (L * L * L));
    return v;
}

/* ------------------------------------------------------------------ */
/* Frozen spheres (Sec. 4, the sequential multimodal cascade)          */
/* ------------------------------------------------------------------ */
/* A cascade stage seats a finer class in the voids of the coarser ones
 * and inflates it with the coarser classes held fixed.  Our reading of
 * "held fixed": a frozen sphere keeps its position and its diameter,
 * given as an absolute value in D0 (it does not scale with kappa); the
 * other spheres have D = kappa D0 as in Eq. (energy).  With
 *   sigma_i = D0_i (frozen) or kappa D0_i,   d_ij = (sigma_i + sigma_j) / 2,
 *   E = 1/2 sum delta^2 - mu kappa sum_{i not frozen} D0_i,
 * the position gradient keeps its form and
 *   dE/dkappa = sum_pairs delta (r / d^2) w_ij - mu sum_{not frozen} D0_i,
 *   w_ij = dd_ij / dkappa = (g_i D0_i + g_j D0_j) / 2,
 * g = 0 for a frozen sphere and 1 otherwise.  Frozen spheres take no Adam
 * step.  With no mask set (the default) nothing is frozen and every
 * function below is the plain protocol. */
static const unsigned char *g_frozen = NULL;

void orc_set_frozen(const unsigned char *mask) { g_frozen = mask; }

static inline int frozen(int64_t i) { return g_frozen != NULL && g_frozen[i] != 0; }

static inline double sigma(const double *d0, int64_t i, double kappa)
{
    return frozen(i) ? d0[i] : kappa * d0[i];
}

static inline double wgrow(const double *d0, int64_t i) { return frozen(i) ? 0.0 : d0[i]; }

/* ------------------------------------------------------------------ */
/* Energy and gradient                                                 */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } nsum_t;   /* Neumaier running sum */

static inline void nadd(nsum_t *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum_t *a) { return a->s + a->c; }

/* Energy terms over a list of half pairs (i, j); pairs with r >= d add
 * nothing; with walls, then every sphere's wall terms in index order.
 * out = [E_overlap, E_growth, dE/dkappa overlap part, dE/dkappa growth
 * part, max fractional overlap, number overlapping (pairs and wall
 * contacts)].
 * gx (n x 3, may be NULL): dE/dx.  gscale (n x 3, may be NULL): per
 * component sum of |pair contributions|, the scale used by the parity
 * tolerance.  Pairs are processed in the order given. */
void orc_energy_grad(int64_t n, const double *x, const double *d0, double L,
                     double kappa, double mu, int64_t np, const int32_t *pi,
                     const int32_t *pj, double *out, double *gx, double *gscale)
{
    const double hL = 0.5 * L;
    nsum_t E = {0, 0}, S = {0, 0}, D = {0, 0};
    double maxd = 0.0;
    int64_t nov = 0;
    if (gx) memset(gx, 0, sizeof(double) * 3 * (size_t)n);
    if (gscale) memset(gscale, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t p = 0; p < np; ++p) {
        int64_t i = pi[p], j = pj[p];
        double dx, dy, dz;
        double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
        double r = sqrt(r2);
        double d = g_frozen ? 0.5 * (sigma(d0, i, kappa) + sigma(d0, j, kappa))
                            : kappa * (0.5 * (d0[i] + d0[j]));
        if (!(r < d)) continue;
        double delta = 1.0 - r / d;
        nadd(&E, 0.5 * delta * delta);
        if (g_frozen)   /* the pair's dE/dkappa: delta (r / d^2) w_ij */
            nadd(&S, delta * (r / d) * ((0.5 * (wgrow(d0, i) + wgrow(d0, j))) / d));
        else
            nadd(&S, delta * r / d);
        if (delta > maxd) maxd = delta;
        ++nov;
        if (r > 0.0) {
            double f = delta / (d * r);   /* dE/dx_i = f (x_j - x_i)_mi */
            double c[3] = {f * dx, f * dy, f * dz};
            for (int a = 0; a < 3; ++a) {
                if (gx) { gx[3 * i + a] += c[a]; gx[3 * j + a] -= c[a]; }
                if (gscale) {
                    gscale[3 * i + a] += fabs(c[a]);
                    gscale[3 * j + a] += fabs(c[a]);
                }
            }
        }
    }
    if (g_walls | g_round)
        for (int64_t i = 0; i < n; ++i) {
            double e = 0.0, sw = 0.0;
            wall_terms(x + 3 * i, kappa * d0[i], L, gx ? gx + 3 * i : NULL,
                       gscale ? gscale + 3 * i : NULL, &e, &sw, &maxd, &nov);
            nadd(&E, e);
            nadd(&S, sw);
        }
    for (int64_t i = 0; i < n; ++i) nadd(&D, wgrow(d0, i));
    out[0] = nval(&E);
    out[1] = -mu * kappa * nval(&D);
    out[2] = g_frozen ? nval(&S) : nval(&S) / kappa;
    out[3] = -mu * nval(&D);
    out[4] = maxd;
    out[5] = (double)nov;
}

/* Per-row quantities for a subset of rows, by testing all N partners with
 * the true overlap condition r < d (no list).  For row k (particle i):
 * g[3k..3k+2] = dE/dx_i, gscale likewise, rowstat[3k] = sum_j delta^2/2
 * (each pair's energy counted in full for this row), rowstat[3k+1] =
 * sum_j delta r / d, rowstat[3k+2] = max_j delta; the row's wall terms
 * (with walls) are included in all of them. */
void orc_rows_grad(int64_t n, const double *x, const double *d0, double L,
                   double kappa, const int64_t *rows, int64_t nrows, double *g,
                   double *gscale, double *rowstat)
{
    const double hL = 0.5 * L;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        double gg[3] = {0, 0, 0}, sc[3] = {0, 0, 0}, e = 0, s = 0, m = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy, dz;
            double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
            double d = kappa * (0.5 * (d0[i] + d0[j]));
            if (!(r2 < d * d)) continue;
            double r = sqrt(r2);
            if (!(r < d)) continue;
            double delta = 1.0 - r / d;
            e += 0.5 * delta * delta;
            s += delta * r / d;
            if (delta > m) m = delta;
            if (r > 0.0) {
                double f = delta / (d * r);
                double c[3] = {f * dx, f * dy, f * dz};
                for (int a = 0; a < 3; ++a) { gg[a] += c[a]; sc[a] += fabs(c[a]); }
            }
        }
        if (g_walls | g_round) {
            int64_t cnt = 0;
            wall_terms(x + 3 * i, kappa * d0[i], L, gg, sc, &e, &s, &m, &cnt);
        }
        for (int a = 0; a < 3; ++a) {
            g[3 * k + a] = gg[a];
            if (gscale) gscale[3 * k + a] = sc[a];
        }
        if (rowstat) { rowstat[3 * k] = e; rowstat[3 * k + 1] = s; rowstat[3 * k + 2] = m; }
    }
}

/* ------------------------------------------------------------------ */
/* Shrink to contact (Sec. 2; App. A)                                  */
/* ------------------------------------------------------------------ */
/* Largest double k with fl(fl(k dd) * fl(k dd)) <= r2, where dd is the pair's
 * relative mean diameter.  That map is monotone in k, so the admissible
 * k form a down-set and this maximum is unique. */
static double pair_kmax(double r2, double dd)
{
    double k = sqrt(r2) / dd;
    while (k > 0.0 && (k * dd) * (k * dd) > r2) k = nextafter(k, 0.0);
    for (;;) {
        double up = nextafter(k, INFINITY);
        if ((up * dd) * (up * dd) <= r2) k = up; else break;
    }
    return k;
}

/* kappa' = min(kappa, min over the pairs of pair_kmax, and with walls the
 * min over the spheres of wall_kmax).  Touching (r = d, 2h = sigma) counts
 * as no overlap. */
double orc_shrink(int64_t n, const double *x, const double *d0, double L,
                  double kappa, int64_t np, const int32_t *pi, const int32_t *pj)
{
    const double hL = 0.5 * L;
    double kp = kappa;
    for (int64_t p = 0; p < np; ++p) {
        double dx, dy, dz;
        double r2 = sep2(x, pi[p], pj[p], L, hL, &dx, &dy, &dz);
        double dd = 0.5 * (d0[pi[p]] + d0[pj[p]]);
        double k = pair_kmax(r2, dd);
        if (k < kp) kp = k;
    }
    if (g_walls | g_round)
        for (int64_t i = 0; i < n; ++i) {
            const double k = wall_kmax(x + 3 * i, d0[i], L);
            if (k < kp) kp = k;
        }
    return kp;
}

double orc_phi(int64_t n, const double *d0, double L, double kappa)
{
    nsum_t s = {0, 0};
    if (g_dim == 2) {
        for (int64_t i = 0; i < n; ++i) nadd(&s, d0[i] * d0[i]);
        return (M_PI / 4.0) * (kappa * kappa) * nval(&s) / domain_volume(L);
    }
    for (int64_t i = 0; i < n; ++i) nadd(&s, d0[i] * d0[i] * d0[i]);
    return (M_PI / 6.0) * (kappa * kappa * kappa) * nval(&s) / domain_volume(L);
}

/* Volume fraction with the frozen mask: sum over i of sigma_i^3. */
double orc_phi_frozen(int64_t n, const double *d0, double L, double kappa)
{
    nsum_t s = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double si = sigma(d0, i, kappa);
        nadd(&s, g_dim == 2 ? si * si : si * si * si);
    }
    return g_dim == 2 ? (M_PI / 4.0) * nval(&s) / domain_volume(L)
                      : (M_PI / 6.0) * nval(&s) / domain_volume(L);
}

/* Seating of a new class (Sec. 4: the finer class is seated in the voids
 * left by the coarser ones).  Every sphere i that is not frozen is placed
 * on its own: attempt a proposes p = (u(seed,i,a,0) L, u(seed,i,a,1) L,
 * u(seed,i,a,2) L) and is accepted when no frozen sphere j overlaps it at
 * the seating scale, r^2 < dd^2 with dd = (D0_j + kappa0 D0_i) / 2 and the
 * separation x_j - p (minimum image).  Spheres that are not frozen may
 * overlap one another (the inflation that follows separates them).
 * x holds the frozen positions on input.  Returns 0, or -1 when a sphere
 * needs more than max_attempts.  Brute force over the frozen spheres. */
int orc_seat(int64_t n, const double *d0, double L, double kappa0, uint64_t seed,
             int64_t max_attempts, double *x)
{
    const double hL = 0.5 * L;
    int64_t nf = 0;
    for (int64_t j = 0; j < n; ++j) nf += frozen(j);
    int64_t *fz = malloc(sizeof(int64_t) * (size_t)(nf > 0 ? nf : 1));
    nf = 0;
    for (int64_t j = 0; j < n; ++j)
        if (frozen(j)) fz[nf++] = j;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(min : rc)
    for (int64_t i = 0; i < n; ++i) {
        if (frozen(i)) continue;
        int64_t a;
        for (a = 0; a < max_attempts; ++a) {
            double p[3];
            for (int ax = 0; ax < 3; ++ax) p[ax] = coord_draw(seed, i, a, ax, L);
            int ok = 1;
            for (int64_t q = 0; q < nf && ok; ++q) {
                const int64_t j = fz[q];
                double dx = mimg_ax(x[3 * j] - p[0], 0, L, hL);
                double dy = mimg_ax(x[3 * j + 1] - p[1], 1, L, hL);
                double dz = mimg_ax(x[3 * j + 2] - p[2], 2, L, hL);
                double r2 = (dx * dx + dy * dy) + dz * dz;
                double dd = 0.5 * (d0[j] + kappa0 * d0[i]);
                if (r2 < dd * dd) ok = 0;
            }
            if (ok) {
                for (int ax = 0; ax < 3; ++ax) x[3 * i + ax] = p[ax];
                break;
            }
        }
        if (a == max_attempts) rc = -1;
    }
    free(fz);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Random sequential addition (App. A: dilute start without overlap)   */
/* ------------------------------------------------------------------ */
/* Largest sphere first (ties: lower index first).  Attempt a of sphere i
 * proposes (u(seed,i,a,0) L, u(seed,i,a,1) L, u(seed,i,a,2) L) and is
 * rejected when r^2 < (kappa0 * 0.5 * (D0_i + D0_j))^2 for a placed j, or
 * (with walls) when the sphere at scale kappa0 would overlap a wall.
 * Returns 0, or -1 when a sphere needs more than max_attempts. */
typedef struct { double d; int64_t i; } ord_t;

static int cmp_ord(const void *a, const void *b)
{
    const ord_t *p = a, *q = b;
    if (p->d != q->d) return p->d > q->d ? -1 : 1;
    return p->i < q->i ? -1 : (p->i > q->i);
}

int orc_rsa(int64_t n, const double *d0, double L, double kappa0, uint64_t seed,
            int64_t max_attempts, double *x)
{
    const double hL = 0.5 * L;
    ord_t *ord = malloc(sizeof(ord_t) * (size_t)n);
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        ord[i].d = d0[i]; ord[i].i = i;
        if (d0[i] > dmax) dmax = d0[i];
    }
    qsort(ord, (size_t)n, sizeof(ord_t), cmp_ord);
    /* one uniform grid, cells at least kappa0 * dmax wide */
    int64_t nc = (int64_t)floor(L / (kappa0 * dmax * (1.0 + 1e-12)));
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    double w = L / (double)nc;
    int64_t ncell = nc * nc * nc;
    int64_t *head = malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    int rc = 0;
    for (int64_t k = 0; k < n && rc == 0; ++k) {
        int64_t i = ord[k].i;
        int64_t a;
        for (a = 0; a < max_attempts; ++a) {
            double p[3];
            for (int ax = 0; ax < 3; ++ax) {
                p[ax] = coord_draw(seed, i, a, ax, L);
                x[3 * i + ax] = p[ax];
            }
            if (!inside_walls(p, kappa0 * d0[i], L)) continue;
            int64_t c[3];
            for (int ax = 0; ax < 3; ++ax) c[ax] = cell_of(p[ax], w, nc);
            int ok = 1;
            int64_t lo = nc >= 3 ? -1 : 0, hi = nc >= 3 ? 1 : nc - 1;
            for (int64_t ox = lo; ox <= hi && ok; ++ox)
                for (int64_t oy = lo; oy <= hi && ok; ++oy)
                    for (int64_t oz = lo; oz <= hi && ok; ++oz) {
                        int64_t ax_, ay_, az_;
                        if (nc >= 3) {
                            ax_ = (c[0] + ox + nc) % nc;
                            ay_ = (c[1] + oy + nc) % nc;
                            az_ = (c[2] + oz + nc) % nc;
                        } else { ax_ = ox; ay_ = oy; az_ = oz; }
                        for (int64_t j = head[(ax_ * nc + ay_) * nc + az_]; j >= 0;
                             j = next[j]) {
                            double dx, dy, dz;
                            double r2 = sep2(x, i, j, L, hL, &dx, &dy, &dz);
                            double dd = kappa0 * (0.5 * (d0[i] + d0[j]));
                            if (r2 < dd * dd) { ok = 0; break; }
                        }
                    }
            if (ok) break;
        }
        if (a == max_attempts) { rc = -1; break; }
        int64_t cell = (cell_of(x[3 * i], w, nc) * nc + cell_of(x[3 * i + 1], w, nc)) * nc +
                       cell_of(x[3 * i + 2], w, nc);
        next[i] = head[cell];
        head[cell] = i;
    }
    free(head); free(next); free(ord);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Random sequential addition in rounds (App. A: dilute start without  */
/* overlap, placed with the help of a cell list)                       */
/* ------------------------------------------------------------------ */
/* The sequential procedure above tries one sphere at a time.  This one
 * tries up to W spheres at a time, the same proposals in the same order of
 * attempts, so that a parallel machine can place them in rounds:
 *   - spheres are ranked largest first (ties: lower index first) and binned
 *     in size classes floor(log2(D0 / D0_min)); classes are placed from the
 *     largest down, so a sphere only meets spheres of its own class or
 *     larger ones;
 *   - a round takes the window of ranks [lo, min(lo + W, end of the class)),
 *     lo the lowest rank of the class not yet placed; every unplaced sphere
 *     i of the window proposes the position of its next attempt a_i,
 *     (u(seed, i, a_i, 0) L, u(seed, i, a_i, 1) L, u(seed, i, a_i, 2) L);
 *   - a proposal is valid when it overlaps no placed sphere (r^2 < dd^2,
 *     dd = kappa0 (D0_i + D0_j) / 2, separation x_j - p_i, minimum image)
 *     and, with walls, no wall at scale kappa0;
 *   - a valid proposal is accepted unless a valid proposal of a lower rank
 *     in the same round overlaps it (separation p_j - p_i);
 *   - accepted spheres are placed; every other sphere of the window that
 *     proposed moves on to its next attempt (more than max_attempts: -1).
 * No two accepted proposals overlap (of two overlapping valid proposals the
 * higher rank is rejected), and with W = 1 a round holds a single proposal,
 * so the procedure is the sequential one, attempt for attempt.  Returns 0
 * (rounds in *rounds) or -1.  Brute force over the placed spheres of the
 * current class and larger: for test sizes only. */
int orc_rsa_rounds(int64_t n, const double *d0, double L, double kappa0, uint64_t seed,
                   int64_t window, int64_t max_attempts, double *x, int64_t *rounds)
{
    const double hL = 0.5 * L;
    ord_t *ord = malloc(sizeof(ord_t) * (size_t)n);
    double d0min = d0[0];
    for (int64_t i = 0; i < n; ++i) {
        ord[i].d = d0[i]; ord[i].i = i;
        if (d0[i] < d0min) d0min = d0[i];
    }
    qsort(ord, (size_t)n, sizeof(ord_t), cmp_ord);
    int *cls = malloc(sizeof(int) * (size_t)n);      /* by rank */
    for (int64_t k = 0; k < n; ++k) {
        int e;
        frexp(ord[k].d / d0min, &e);                    /* ratio in [2^(e-1), 2^e) */
        cls[k] = e - 1 > 0 ? e - 1 : 0;
    }
    int64_t *att = calloc((size_t)n, sizeof(int64_t));
    unsigned char *placed = calloc((size_t)n, 1);
    int64_t *placed_list = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t nplaced = 0;
    double *prop = malloc(sizeof(double) * 3 * (size_t)(window > 0 ? window : 1));
    unsigned char *valid = malloc((size_t)(window > 0 ? window : 1));
    unsigned char *acc = malloc((size_t)(window > 0 ? window : 1));
    int64_t nround = 0;
    int rc = 0;
    int64_t cb = 0;
    while (cb < n && rc == 0) {
        int64_t ce = cb;
        while (ce < n && cls[ce] == cls[cb]) ++ce;       /* class ranks [cb, ce) */
        int64_t lo = cb;
        while (lo < ce && rc == 0) {
            int64_t hi = lo + window < ce ? lo + window : ce;
            ++nround;
            /* proposals and their validity against the placed spheres */
            for (int64_t k = lo; k < hi; ++k) {
                int64_t s = k - lo, i = ord[k].i;
                valid[s] = 0;
                if (placed[k]) continue;
                double *p = prop + 3 * s;
                for (int ax = 0; ax < 3; ++ax) p[ax] = coord_draw(seed, i, att[k], ax, L);
                int ok = inside_walls(p, kappa0 * d0[i], L);
                for (int64_t q = 0; q < nplaced && ok; ++q) {
                    int64_t j = placed_list[q];
                    double dx = mimg_ax(x[3 * j] - p[0], 0, L, hL);
                    double dy = mimg_ax(x[3 * j + 1] - p[1], 1, L, hL);
                    double dz = mimg_ax(x[3 * j + 2] - p[2], 2, L, hL);
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    double dd = kappa0 * (0.5 * (d0[i] + d0[j]));
                    if (r2 < dd * dd) ok = 0;
                }
                valid[s] = (unsigned char)ok;
            }
            /* conflicts among the valid proposals: the lower rank wins */
            for (int64_t k = lo; k < hi; ++k) {
                int64_t s = k - lo, i = ord[k].i;
                acc[s] = 0;
                if (placed[k] || !valid[s]) continue;
                int ok = 1;
                for (int64_t k2 = lo; k2 < k && ok; ++k2) {
                    int64_t s2 = k2 - lo, j = ord[k2].i;
                    if (placed[k2] || !valid[s2]) continue;
                    const double *pi_ = prop + 3 * s, *pj_ = prop + 3 * s2;
                    double dx = mimg_ax(pj_[0] - pi_[0], 0, L, hL);
                    double dy = mimg_ax(pj_[1] - pi_[1], 1, L, hL);
                    double dz = mimg_ax(pj_[2] - pi_[2], 2, L, hL);
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    double dd = kappa0 * (0.5 * (d0[i] + d0[j]));
                    if (r2 < dd * dd) ok = 0;
                }
                acc[s] = (unsigned char)ok;
            }
            /* placements and next attempts take effect at the end of the round */
            for (int64_t k = lo; k < hi; ++k) {
                int64_t s = k - lo, i = ord[k].i;
                if (placed[k]) continue;
                if (acc[s]) {
                    for (int ax = 0; ax < 3; ++ax) x[3 * i + ax] = prop[3 * s + ax];
                    placed[k] = 1;
                    placed_list[nplaced++] = i;
                } else if (++att[k] >= max_attempts) {
                    rc = -1;
                }
            }
            while (lo < ce && placed[lo]) ++lo;
        }
        cb = ce;
    }
    if (rounds) *rounds = nround;
    free(ord); free(cls); free(att); free(placed); free(placed_list); free(prop); free(valid);
    free(acc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Schedule, Adam and the whole inflation run (App. A)                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t n_rungs;
    int32_t absolute;   /* 1: mu, eta_x, eta_k below are used as given */
    double tol;         /* stop tolerance on the max fractional overlap */
    double mu[ORC_MAX_RUNGS];
    double eta_x[ORC_MAX_RUNGS];
    double eta_k[ORC_MAX_RUNGS];
    double decay[ORC_MAX_RUNGS];    /* per-iteration factor on mu, eta_x, eta_k */
    int64_t budget[ORC_MAX_RUNGS];
} orc_sched;

typedef struct {
    double beta1, beta2, eps_x, eps_k, skin_s, skin_g;
} orc_params;

typedef struct {
    double phi, kappa_shrunk, kappa, max_overlap, energy;
    int64_t iterations, rebuilds;
    int32_t status;      /* 0 converged, 1 iteration cap reached */
    int32_t rung;
} orc_result;

/* Full neighbour rows (both directions) from a half-pair list; each row
 * keeps the order in which its partners appear in the half list. */
static void full_rows(int64_t n, int64_t np, const int32_t *pi, const int32_t *pj,
                      int64_t **rp_out, int32_t **col_out)
{
    int64_t *rp = calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t p = 0; p < np; ++p) { rp[pi[p] + 1]++; rp[pj[p] + 1]++; }
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(fill, rp, sizeof(int64_t) * (size_t)n);
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(2 * np > 0 ? 2 * np : 1));
    for (int64_t p = 0; p < np; ++p) {
        col[fill[pi[p]]++] = pj[p];
        col[fill[pj[p]]++] = pi[p];
    }
    free(fill);
    *rp_out = rp;
    *col_out = col;
}

/* Debug mode of the run: before every gradient evaluation, test by brute
 * force (n <= 4096) that every overlapping pair (r < d at the current kappa)
 * is in the current list, and count the pairs that are not.  The
 * displacement allowance of the rebuild test can be scaled (1 = the rule
 * as stated; a larger factor plants a mistake the check must catch). */
static int g_list_check = 0;
static int64_t g_list_misses = 0;
static double g_trigger_scale = 1.0;

void orc_set_list_check(int on, double trigger_scale)
{
    g_list_check = on;
    g_list_misses = 0;
    g_trigger_scale = trigger_scale > 0 ? trigger_scale : 1.0;
}

int64_t orc_list_misses(void) { return g_list_misses; }

typedef struct {
    int64_t n;
    double L, hL, d0min, sumd0;
    const double *d0;
    double *x, *m, *v, *xref, *g;
    int64_t np;
    int32_t *pi, *pj;        /* half pairs of the current list */
    int64_t *rp;
    int32_t *col;
    double kb;               /* kappa at the last list build */
    int64_t rebuilds;
    double *gsmax;           /* optional: per component, the largest sum of
                                |pair contributions| over the evaluations */
} run_t;

/* With frozen spheres (absolute D0) the list is built at scale
 * max(kappa, 1): every cutoff is then at least the contact distance. */
static void run_rebuild(run_t *R, double kappa, const orc_params *P)
{
    if (g_frozen && kappa < 1.0) kappa = 1.0;
    free(R->pi); free(R->pj); free(R->rp); free(R->col);
    if (R->n <= 2048) {
        int64_t cap = 1024, np;
        for (;;) {
            R->pi = malloc(sizeof(int32_t) * (size_t)cap);
            R->pj = malloc(sizeof(int32_t) * (size_t)cap);
            np = orc_pairs_brute(R->n, R->x, R->d0, R->L, kappa, P->skin_s,
                                 P->skin_g, R->d0min, R->pi, R->pj, cap);
            if (np <= cap) break;
            free(R->pi); free(R->pj);
            cap = np;
        }
        R->np = np;
    } else {
        R->np = cells_half_pairs(R->n, R->x, R->d0, R->L, kappa, P->skin_s,
                                 P->skin_g, R->d0min, &R->pi, &R->pj);
    }
    full_rows(R->n, R->np, R->pi, R->pj, &R->rp, &R->col);
    memcpy(R->xref, R->x, sizeof(double) * 3 * (size_t)R->n);
    R->kb = kappa;
    R->rebuilds++;
}

/* Debug check (see orc_set_list_check): every pair with r < d at kappa
 * must be one of the listed pairs. */
static void list_check(const run_t *R, double kappa)
{
    const int64_t n = R->n;
    unsigned char *in = calloc((size_t)(n * n), 1);
    for (int64_t p = 0; p < R->np; ++p) {
        in[(int64_t)R->pi[p] * n + R->pj[p]] = 1;
        in[(int64_t)R->pj[p] * n + R->pi[p]] = 1;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            double dx, dy, dz;
            double r2 = sep2(R->x, i, j, R->L, R->hL, &dx, &dy, &dz);
            double d = 0.5 * (sigma(R->d0, i, kappa) + sigma(R->d0, j, kappa));
            if (r2 < d * d && !in[i * n + j]) ++g_list_misses;
        }
    free(in);
}

/* Gradient over full rows (parallel over rows, each row summed in list
 * order), plus E_ov, sum delta r/d and max delta accumulated per row and
 * then over rows in index order. */
static void run_grad(run_t *R, double kappa, double *Eov, double *Sdrd,
                     double *maxd)
{
    const int64_t n = R->n;
    double *re = malloc(sizeof(double) * 3 * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double gg[3] = {0, 0, 0}, ga[3] = {0, 0, 0}, e = 0, s = 0, m = 0;
        for (int64_t q = R->rp[i]; q < R->rp[i + 1]; ++q) {
            int64_t j = R->col[q];
            double dx, dy, dz;
            double r2 = sep2(R->x, i, j, R->L, R->hL, &dx, &dy, &dz);
            double r = sqrt(r2);
            double d = g_frozen ? 0.5 * (sigma(R->d0, i, kappa) + sigma(R->d0, j, kappa))
                                : kappa * (0.5 * (R->d0[i] + R->d0[j]));
            if (!(r < d)) continue;
            double delta = 1.0 - r / d;
            e += 0.25 * delta * delta;    /* each pair appears in two rows */
            if (g_frozen)   /* half the pair's dE/dkappa (see orc_set_frozen) */
                s += 0.5 * (delta * (r / d) *
                            ((0.5 * (wgrow(R->d0, i) + wgrow(R->d0, j))) / d));
            else
                s += 0.5 * (delta * r / d);
            if (delta > m) m = delta;
            if (r > 0.0) {
                double f = delta / (d * r);
                gg[0] += f * dx; gg[1] += f * dy; gg[2] += f * dz;
                ga[0] += fabs(f * dx); ga[1] += fabs(f * dy); ga[2] += fabs(f * dz);
            }
        }
        if (g_walls | g_round) {   /* the row's wall terms, in full */
            int64_t cnt = 0;
            wall_terms(R->x + 3 * i, kappa * R->d0[i], R->L, gg, ga, &e, &s, &m, &cnt);
        }
        R->g[3 * i] = gg[0]; R->g[3 * i + 1] = gg[1]; R->g[3 * i + 2] = gg[2];
        if (R->gsmax)
            for (int a = 0; a < 3; ++a)
                if (ga[a] > R->gsmax[3 * i + a]) R->gsmax[3 * i + a] = ga[a];
        re[3 * i] = e; re[3 * i + 1] = s; re[3 * i + 2] = m;
    }
    nsum_t E = {0, 0}, S = {0, 0};
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        nadd(&E, re[3 * i]);
        nadd(&S, re[3 * i + 1]);
        if (re[3 * i + 2] > mx) mx = re[3 * i + 2];
    }
    free(re);
    *Eov = nval(&E);
    *Sdrd = nval(&S);
    *maxd = mx;
}

/* Rung parameters at the start of rung r, from kappa at that moment.
 * Relative schedules scale mu so that the equilibrium summed overlap is
 * mu~ N_v (from dE/dkappa = 0), where N_v = (sum D0^3)^2 / sum D0^6 is the
 * volume participation number (N for equal spheres; for a broad
 * distribution about the number of spheres that carry the solid volume and
 * hence the contact network), and the step sizes by the current length and
 * kappa scales; absolute schedules take the numbers as they are. */
static void rung_start(const orc_sched *S, int r, double kappa, double nvol,
                       double sumd0, double d0min, double *mu, double *ex,
                       double *ek)
{
    if (S->absolute) {
        *mu = S->mu[r]; *ex = S->eta_x[r]; *ek = S->eta_k[r];
    } else {
        *mu = (S->mu[r] * nvol) / (kappa * sumd0);
        *ex = S->eta_x[r] * (kappa * d0min);
        *ek = S->eta_k[r] * kappa;
    }
}

/* One Adam update of parameter th with gradient g (Kingma and Ba 2015,
 * Algorithm 1 with bias correction; b1t = beta1^t, b2t = beta2^t). */
static inline double adam(double th, double g, double *m, double *v, double b1,
                          double b2, double b1t, double b2t, double eta,
                          double eps)
{
    *m = b1 * *m + (1.0 - b1) * g;
    *v = b2 * *v + (1.0 - b2) * (g * g);
    double mh = *m / (1.0 - b1t);
    double vh = *v / (1.0 - b2t);
    return th - eta * mh / (sqrt(vh) + eps);
}

/* The inflation run.  One iteration:
 *   1. rebuild the list if the displacement / growth criterion failed;
 *   2. evaluate the energy terms and gradients at (x_t, kappa_t);
 *   3. in the final rung, stop if max delta < tol (state x_t is returned);
 *   4. t += 1, Adam on every coordinate and on kappa, wrap positions;
 *   5. decay mu and the step sizes, advance the rung counter; at the end of a
 *      rung start the next one (its mu and etas from the new kappa); at the
 *      end of the final rung stop with status 1;
 *   6. test the list validity for the next iteration.
 * x (n x 3), kappa, m, v (n x 3), mk_vk[2] are in/out so a run can be split
 * into calls; ctl holds the schedule position:
 *   ctl[0] = t, ctl[1] = rung, ctl[2] = iterations done in the rung,
 *   ctl[3] = 1 when the rung's parameters still have to be set.
 * etas[0..2] = mu, eta_x, eta_k in force (in/out).
 * max_iters bounds the number of iterations of this call (status 2 when hit).
 * trace (may be NULL): per iteration (max delta, kappa, E_ov) up to trace_cap.
 * gsmax (n x 3, may be NULL): raised to the largest per-component sum of
 * |pair contributions| of any gradient evaluated (a scale for tolerances). */
int orc_run(int64_t n, double *x, const double *d0, double L, double *kappa,
            double *m, double *v, double *mk_vk, int64_t *ctl, double *etas,
            const orc_params *P, const orc_sched *S, int64_t max_iters,
            orc_result *res, double *trace, int64_t trace_cap, double *gsmax)
{
    run_t R;
    memset(&R, 0, sizeof R);
    R.gsmax = gsmax;
    R.n = n; R.L = L; R.hL = 0.5 * L; R.d0 = d0; R.x = x; R.m = m; R.v = v;
    R.xref = malloc(sizeof(double) * 3 * (size_t)n);
    R.g = malloc(sizeof(double) * 3 * (size_t)n);
    /* schedule scales (sum D0, N_v, D0_min) over the spheres that are not
     * frozen: they alone inflate and move */
    R.d0min = INFINITY;
    nsum_t sd = {0, 0}, s3 = {0, 0}, s6 = {0, 0};
    for (int64_t i = 0; i < n; ++i) {
        if (frozen(i)) continue;
        if (d0[i] < R.d0min) R.d0min = d0[i];
        nadd(&sd, d0[i]);
        /* volume (area in 2-D) participation number */
        const double c3 = g_dim == 2 ? d0[i] * d0[i] : d0[i] * d0[i] * d0[i];
        nadd(&s3, c3);
        nadd(&s6, c3 * c3);
    }
    R.sumd0 = nval(&sd);
    const double nvol = (nval(&s3) * nval(&s3)) / nval(&s6);
    const double b1 = P->beta1, b2 = P->beta2;
    int64_t t = ctl[0];
    int r = (int)ctl[1];
    int64_t itr = ctl[2];
    double mu = etas[0], ex = etas[1], ek = etas[2];
    if (ctl[3]) {
        rung_start(S, r, *kappa, nvol, R.sumd0, R.d0min, &mu, &ex, &ek);
        ctl[3] = 0;
    }
    /* beta powers as repeated products (the same rounding on every side) */
    double b1t = 1.0, b2t = 1.0;
    for (int64_t k = 0; k < t; ++k) { b1t *= b1; b2t *= b2; }
    double mk = mk_vk[0], vk = mk_vk[1];
    int status = 2;
    int need_build = 1;
    double Eov = 0, Sdrd = 0, maxd = 0;
    int64_t it;
    for (it = 0; it < max_iters; ++it) {
        if (need_build) run_rebuild(&R, *kappa, P);
        if (g_list_check && n <= 4096) list_check(&R, *kappa);
        run_grad(&R, *kappa, &Eov, &Sdrd, &maxd);
        if (trace && it < trace_cap) {
            trace[3 * it] = maxd; trace[3 * it + 1] = *kappa; trace[3 * it + 2] = Eov;
        }
        if (r == S->n_rungs - 1 && maxd < S->tol) { status = 0; break; }
        double gk = g_frozen ? Sdrd - mu * R.sumd0 : Sdrd / *kappa - mu * R.sumd0;
        t += 1;
        b1t *= b1; b2t *= b2;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 3 * n; ++q) {
            if (frozen(q / 3)) continue;   /* held fixed: no step */
            double th = adam(x[q], R.g[q], &m[q], &v[q], b1, b2, b1t, b2t, ex,
                             P->eps_x);
            if (periodic((int)(q % 3))) {   /* no wrap across walls */
                if (th < 0.0) th += L;
                if (th >= L) th -= L;
            }
            x[q] = th;
        }
        *kappa = adam(*kappa, gk, &mk, &vk, b1, b2, b1t, b2t, ek, P->eps_k);
        mu *= S->decay[r];
        ex *= S->decay[r];
        ek *= S->decay[r];
        itr += 1;
        if (itr >= S->budget[r]) {
            if (r == S->n_rungs - 1) { status = 1; ++it; break; }
            r += 1;
            itr = 0;
            rung_start(S, r, *kappa, nvol, R.sumd0, R.d0min, &mu, &ex, &ek);
        }
        /* list validity for the next iteration */
        double lim = g_trigger_scale * (P->skin_s * R.kb * R.d0min);
        double md2 = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double dx = mimg_ax(x[3 * i] - R.xref[3 * i], 0, L, R.hL);
            double dy = mimg_ax(x[3 * i + 1] - R.xref[3 * i + 1], 1, L, R.hL);
            double dz = mimg_ax(x[3 * i + 2] - R.xref[3 * i + 2], 2, L, R.hL);
            double d2 = (dx * dx + dy * dy) + dz * dz;
            if (d2 > md2) md2 = d2;
        }
        need_build = (md2 > lim * lim) || (*kappa > (1.0 + P->skin_g) * R.kb);
    }
    ctl[0] = t; ctl[1] = r; ctl[2] = itr;
    etas[0] = mu; etas[1] = ex; etas[2] = ek;
    mk_vk[0] = mk; mk_vk[1] = vk;
    if (res) {
        res->iterations = it;
        res->rebuilds = R.rebuilds;
        res->status = status;
        res->rung = r;
        res->kappa = *kappa;
        res->energy = Eov;
        if (status != 0) {
            /* state after the last step: evaluate it for the report */
            run_rebuild(&R, *kappa, P);
            run_grad(&R, *kappa, &Eov, &Sdrd, &maxd);
            res->rebuilds = R.rebuilds;
            res->energy = Eov;
        }
        res->max_overlap = maxd;
        if (g_frozen) {
            /* a cascade stage: no shrink (the release that follows resolves
             * the remaining overlaps below the tolerance) */
            res->kappa_shrunk = *kappa;
            res->phi = orc_phi_frozen(n, d0, L, *kappa);
        } else {
            double kp = orc_shrink(n, x, d0, L, *kappa, R.np, R.pi, R.pj);
            res->kappa_shrunk = kp;
            res->phi = orc_phi(n, d0, L, kp);
        }
    }
    free(R.xref); free(R.g); free(R.pi); free(R.pj); free(R.rp); free(R.col);
    return status;
}

/* Timing helper for the CPU baseline: `iters` evaluations of gradient +
 * Adam on a fixed list (no schedule logic, no rebuilds), in place.  The
 * list is built with every thread; the timed loop runs on `threads`
 * threads (0: every thread). */
double orc_time_iterations(int64_t n, double *x, const double *d0, double L,
                           double kappa, double mu, double eta_x, double s,
                           double g, int64_t iters, int64_t *np_out, int threads)
{
    run_t R;
    memset(&R, 0, sizeof R);
    R.n = n; R.L = L; R.hL = 0.5 * L; R.d0 = d0; R.x = x;
    R.xref = malloc(sizeof(double) * 3 * (size_t)n);
    R.g = malloc(sizeof(double) * 3 * (size_t)n);
    double *m = calloc(3 * (size_t)n, sizeof(double));
    double *v = calloc(3 * (size_t)n, sizeof(double));
    R.d0min = d0[0];
    for (int64_t i = 0; i < n; ++i) if (d0[i] < R.d0min) R.d0min = d0[i];
    orc_params P = {0.9, 0.999, 1e-15, 1e-12, s, g};
    run_rebuild(&R, kappa, &P);
    if (np_out) *np_out = R.np;
    double b1t = 1.0, b2t = 1.0, Eov, Sdrd, maxd;
    double t0;
#ifdef _OPENMP
    const int all = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
    t0 = omp_get_wtime();
#else
    (void)threads;
    t0 = 0;
#endif
    for (int64_t it = 0; it < iters; ++it) {
        run_grad(&R, kappa, &Eov, &Sdrd, &maxd);
        b1t *= 0.9; b2t *= 0.999;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 3 * n; ++q) {
            double th = adam(x[q], R.g[q], &m[q], &v[q], 0.9, 0.999, b1t, b2t,
                             eta_x, P.eps_x);
            if (th < 0.0) th += L;
            if (th >= L) th -= L;
            x[q] = th;
        }
        (void)mu;
    }
    double t1;
#ifdef _OPENMP
    t1 = omp_get_wtime();
    omp_set_num_threads(all);
#else
    t1 = 0;
#endif
    free(R.xref); free(R.g); free(R.pi); free(R.pj); free(R.rp); free(R.col);
    free(m); free(v);
    return t1 - t0;
}
