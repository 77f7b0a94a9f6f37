// Initial placement on the host (App. A: particles start dilute and
// non-overlapping, placed with a cell-list procedure; the paper gives no
// algorithm, random sequential addition is our reading).
//
// Uniform numbers come from the SplitMix64 output function (Steele, Lea and
// Flood, OOPSLA 2014) evaluated at counter (i << 24 | attempt) * 4 + axis.
// Compiled without floating-point contraction so that the accept / reject
// decisions are reproducible: a proposal for sphere i is rejected when
//     r2 < dd * dd,  r2 = (dx dx + dy dy) + dz dz,  dx = mi(x_j - x_i),
//     dd = kappa0 * (0.5 * (D0_i + D0_j))
// for some placed sphere j.  In two dimensions (dim = 2) every sphere lies
// in the plane z = 0: axis 2 of the counter stream is not drawn.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace rcp {

// Open-addressing map from a cell key to the most recently placed sphere in
// that cell (the rest of the cell's spheres follow through `next`).
struct CellHeads {
    std::vector<uint64_t> key;
    std::vector<int64_t> head;
    uint64_t mask = 0;
    static constexpr uint64_t kEmpty = ~0ull;
    void init(int64_t expected)
    {
        uint64_t cap = 16;
        while (cap < (uint64_t)(2 * expected + 2)) cap <<= 1;
        key.assign(cap, kEmpty);
        head.assign(cap, -1);
        mask = cap - 1;
    }
    static uint64_t mix(uint64_t k)
    {
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        return k;
    }
    int64_t find(uint64_t k) const
    {
        for (uint64_t s = mix(k) & mask;; s = (s + 1) & mask) {
            if (key[s] == k) return head[s];
            if (key[s] == kEmpty) return -1;
        }
    }
    // returns the previous head of the cell (or -1) and makes i the head
    int64_t push(uint64_t k, int64_t i)
    {
        for (uint64_t s = mix(k) & mask;; s = (s + 1) & mask) {
            if (key[s] == k) {
                const int64_t prev = head[s];
                head[s] = i;
                return prev;
            }
            if (key[s] == kEmpty) {
                key[s] = k;
                head[s] = i;
                return -1;
            }
        }
    }
};

static inline uint64_t sm64_mix(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t i, uint64_t attempt, int axis)
{
    const uint64_t k = ((i << 24) | attempt) * 4u + (uint64_t)axis;
    return (double)(sm64_mix(seed, k) >> 11) * 0x1p-53;
}

static inline double mimage(double d, double L, double hL)
{
    return d > hL ? d - L : (d < -hL ? d + L : d);
}

void place_uniform(int64_t n, double L, uint64_t seed, int dim, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double p = a < dim ? uniform01(seed, (uint64_t)i, 0, a) * L : 0.0;
            if (p >= L) p -= L;
            x[3 * i + a] = p;
        }
}

// Largest sphere first (ties: smaller index first).  Placed spheres are
// binned by size class (floor(log2(D0 / D0_min))) on one grid per class
// with cells no narrower than kappa0 times the class's largest diameter;
// since every placed sphere is at least as large as the candidate, a
// candidate only has to look at its own and larger classes.
int place_rsa(int64_t n, const double *d0, double L, double kappa0, uint64_t seed, int dim,
              int64_t max_attempts, double *x)
{
    const double hL = 0.5 * L;
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return d0[a] > d0[b]; });
    double d0min = d0[0];
    for (int64_t i = 0; i < n; ++i) d0min = std::min(d0min, d0[i]);
    std::vector<int> cls(n);
    int ncls = 1;
    for (int64_t i = 0; i < n; ++i) {
        int e;
        std::frexp(d0[i] / d0min, &e);   // ratio in [2^(e-1), 2^e)
        cls[i] = std::max(0, e - 1);
        ncls = std::max(ncls, cls[i] + 1);
    }
    std::vector<double> dmax(ncls, 0.0);
    for (int64_t i = 0; i < n; ++i) dmax[cls[i]] = std::max(dmax[cls[i]], d0[i]);
    for (int c = 1; c < ncls; ++c) dmax[c] = std::max(dmax[c], dmax[c - 1]);
    std::vector<int64_t> nc(ncls);
    std::vector<double> w(ncls);
    for (int c = 0; c < ncls; ++c) {
        double h = kappa0 * dmax[c] * (1.0 + 1e-12);
        int64_t k = h > 0 ? (int64_t)std::floor(L / h) : 1;
        k = std::max<int64_t>(1, std::min<int64_t>(k, 1 << 20));
        nc[c] = k;
        w[c] = L / (double)k;
    }
    std::vector<CellHeads> head(ncls);
    {
        std::vector<int64_t> per(ncls, 0);
        for (int64_t i = 0; i < n; ++i) per[cls[i]]++;
        for (int c = 0; c < ncls; ++c) head[c].init(per[c]);
    }
    std::vector<int64_t> next(n, -1);
    std::vector<int64_t> placed_in(ncls, 0);
    auto cell = [&](double v, int c) {
        int64_t k = (int64_t)(v / w[c]);
        return std::min<int64_t>(std::max<int64_t>(k, 0), nc[c] - 1);
    };
    auto key = [&](int64_t cx, int64_t cy, int64_t cz, int c) {
        return ((uint64_t)cx * (uint64_t)nc[c] + (uint64_t)cy) * (uint64_t)nc[c] + (uint64_t)cz;
    };
    for (int64_t k = 0; k < n; ++k) {
        const int64_t i = order[k];
        int64_t a;
        for (a = 0; a < max_attempts; ++a) {
            double p[3];
            for (int ax = 0; ax < 3; ++ax) {
                p[ax] = ax < dim ? uniform01(seed, (uint64_t)i, (uint64_t)a, ax) * L : 0.0;
                if (p[ax] >= L) p[ax] -= L;
            }
            bool ok = true;
            for (int c = cls[i]; c < ncls && ok; ++c) {
                if (placed_in[c] == 0) continue;
                const int64_t m = nc[c];
                const int64_t cx = cell(p[0], c), cy = cell(p[1], c), cz = cell(p[2], c);
                const int64_t lo = m >= 3 ? -1 : 0, hi = m >= 3 ? 1 : m - 1;
                for (int64_t ox = lo; ox <= hi && ok; ++ox)
                    for (int64_t oy = lo; oy <= hi && ok; ++oy)
                        for (int64_t oz = lo; oz <= hi && ok; ++oz) {
                            auto wrap = [m](int64_t v) { return v < 0 ? v + m : (v >= m ? v - m : v); };
                            const int64_t ax = m >= 3 ? wrap(cx + ox) : ox;
                            const int64_t ay = m >= 3 ? wrap(cy + oy) : oy;
                            const int64_t az = m >= 3 ? wrap(cz + oz) : oz;
                            for (int64_t j = head[c].find(key(ax, ay, az, c)); j >= 0; j = next[j]) {
                                const double dx = mimage(x[3 * j] - p[0], L, hL);
                                const double dy = mimage(x[3 * j + 1] - p[1], L, hL);
                                const double dz = mimage(x[3 * j + 2] - p[2], L, hL);
                                const double r2 = (dx * dx + dy * dy) + dz * dz;
                                const double dd = kappa0 * (0.5 * (d0[i] + d0[j]));
                                if (r2 < dd * dd) {
                                    ok = false;
                                    break;
                                }
                            }
                        }
            }
            if (ok) {
                for (int ax = 0; ax < 3; ++ax) x[3 * i + ax] = p[ax];
                break;
            }
        }
        if (a == max_attempts) return -1;
        const int c = cls[i];
        const uint64_t kk = key(cell(x[3 * i], c), cell(x[3 * i + 1], c), cell(x[3 * i + 2], c), c);
        next[i] = head[c].push(kk, i);
        placed_in[c]++;
    }
    return 0;
}

}  // namespace rcp
