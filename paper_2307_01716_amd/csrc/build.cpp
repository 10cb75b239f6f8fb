// Host construction of APRIL A- and F-lists (Sec. 6).
//
// Per polygon:
//  1. Boundary cells (Sec. 6.1, edge traversal): every edge is walked row by
//     row; in each row of cells it spans, the x-extent of the edge inside the
//     row gives the run of cells whose closed square it meets, and the
//     extent inside the open row gives the cells whose interior it crosses.
//     A cell met by an edge is "touched"; a touched cell whose interior no
//     edge crosses only has boundary on its border.
//  2. Point-in-polygon by row tables (scanline idea, Sec. 6.1): for every row
//     of cells, the x-positions where edges cross the row's centre line,
//     sorted.  A cell centre is inside iff an odd number of them lie left of
//     it.
//  3. One-step intervalization (Sec. 6.2, Alg. 3): walk the touched cells in
//     Hilbert order.  Runs of consecutive ids extend the current A-interval.
//     Each gap between touched ids is a run of untouched, hence same-class,
//     cells (consecutive Hilbert cells share an edge and no boundary passes
//     between them): one point-in-polygon test of its first cell labels the
//     whole gap.  Inside -> the gap is an F-interval and the A-interval runs
//     on; outside -> the A-interval ends at the gap.  A touched cell joins
//     the F-list too when no edge crosses its interior and its centre is
//     inside (the polygon only touches it along its border).
//  Cells before the first and after the last touched id are outside: the
//  curve starts and ends in the outer ring, which no polygon reaches.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>

#include "internal.hpp"

namespace april {
namespace {

typedef __int128 i128;

inline int64_t floor_div(i128 a, i128 b) {  // b > 0
    i128 q = a / b;
    if ((a % b) != 0 && a < 0) q--;
    return int64_t(q);
}
inline int64_t ceil_div(i128 a, i128 b) { return -floor_div(-a, b); }

struct Poly {
    std::vector<int64_t> x, y;   // lattice units relative to the grid origin
};

struct Result {
    std::vector<uint32_t> a, f;  // flattened (start, end) pairs
    int rc = APRIL_OK;
    std::string msg;
};

class Builder {
public:
    Builder(const LatticeGrid &g) : g_(g) {}
    void set_grid(const LatticeGrid &g) { g_ = g; }

    int run(const Poly &p, Result &out);
    // the sorted, distinct ids of the cells the open chain p meets (its
    // segments only; no closing edge)
    void chain_cells(const Poly &p, std::vector<uint64_t> &ids);
    // the same lists, with the steps split over `threads` threads (for one
    // large polygon)
    int run_parallel(const Poly &p, Result &out, int threads);

private:
    void edge_cells(int64_t ax, int64_t ay, int64_t bx, int64_t by, std::vector<uint64_t> &out) const;
    void row_tables(const Poly &p, int threads = 1);
    void intervalize(const uint8_t *cls, size_t m, Result &out) const;
    void edge_crossings(int64_t ax, int64_t ay, int64_t bx, int64_t by);
    bool centre_inside(uint32_t i, uint32_t j) const;
    void push_f(uint64_t s, uint64_t e, std::vector<uint32_t> &f) const;

    LatticeGrid g_;
    std::vector<uint64_t> touched_;          // (hilbert id << 1) | interior crossed
    int64_t jmin_ = 0, jmax_ = 0;
    std::vector<uint32_t> row_off_;          // CSR of crossings per row
    std::vector<int64_t> row_x_;             // floor of crossing x, doubled units
    std::vector<uint32_t> row_fill_;
    std::vector<uint8_t> cls_;               // class bits per touched cell
};

// Cells met by the edge a-b, with the interior-crossed flag.
void Builder::edge_cells(int64_t ax, int64_t ay, int64_t bx, int64_t by, std::vector<uint64_t> &out) const {
    const int64_t w = g_.w;
    if (ay > by) { std::swap(ax, bx); std::swap(ay, by); }
    const bool horiz = (ay == by);
    const i128 D = horiz ? 1 : i128(by - ay);
    const int64_t j0 = ceil_div(ay, w) - 1, j1 = floor_div(by, w);
    for (int64_t j = j0; j <= j1; j++) {
        const int64_t ylo = std::max<int64_t>(ay, j * w), yhi = std::min<int64_t>(by, (j + 1) * w);
        // x-extent of the edge within the closed row, as N/D
        i128 n0, n1;
        if (horiz) {
            n0 = std::min(ax, bx);
            n1 = std::max(ax, bx);
        } else {
            const i128 u = i128(ax) * D + i128(ylo - ay) * (bx - ax);
            const i128 v = i128(ax) * D + i128(yhi - ay) * (bx - ax);
            n0 = std::min(u, v);
            n1 = std::max(u, v);
        }
        const i128 Dw = D * w;
        const int64_t i0 = ceil_div(n0, Dw) - 1, i1 = floor_div(n1, Dw);
        // the edge runs through the open row iff it has a piece strictly inside it
        const bool open_row = horiz ? (j * w < ay && ay < (j + 1) * w) : (ylo < yhi);
        int64_t o0 = 1, o1 = 0;
        if (open_row) { o0 = floor_div(n0, Dw); o1 = ceil_div(n1, Dw) - 1; }
        for (int64_t i = i0; i <= i1; i++) {
            const uint64_t d = hilbert_xy2d(g_.order, uint32_t(i), uint32_t(j));
            out.push_back((d << 1) | uint64_t(i >= o0 && i <= o1));
        }
    }
}

// Crossings of the edge a-b with the centre lines of cell rows (half-open
// rule: the edge crosses y = c iff exactly one endpoint is above c).
void Builder::edge_crossings(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
    if (ay == by) return;
    if (ay > by) { std::swap(ax, bx); std::swap(ay, by); }
    const int64_t w = g_.w;
    // rows whose doubled centre c = (2j+1) w satisfies 2ay <= c < 2by
    const int64_t j0 = std::max<int64_t>(jmin_, ceil_div(2 * i128(ay) - w, 2 * i128(w)));
    const int64_t j1 = std::min<int64_t>(jmax_, ceil_div(2 * i128(by) - w, 2 * i128(w)) - 1);
    const i128 D = by - ay;
    for (int64_t j = j0; j <= j1; j++) {
        const i128 c = i128(2 * j + 1) * w;
        // doubled x of the crossing = 2ax + (c - 2ay)(bx - ax)/(by - ay)
        const i128 N = 2 * i128(ax) * D + (c - 2 * i128(ay)) * (bx - ax);
        const size_t r = size_t(j - jmin_);
        row_x_[row_off_[r] + row_fill_[r]++] = floor_div(N, D);
    }
}

// Is the centre of cell (i, j) inside?  Only asked for cells whose interior
// no edge crosses, so the centre never lies on the boundary and the crossing
// count to its left has the parity of the count to its right.
bool Builder::centre_inside(uint32_t i, uint32_t j) const {
    const int64_t jj = int64_t(j);
    if (jj < jmin_ || jj > jmax_) return false;
    const size_t r = size_t(jj - jmin_);
    const int64_t X = (2 * int64_t(i) + 1) * g_.w;
    const int64_t *b = row_x_.data() + row_off_[r], *e = row_x_.data() + row_off_[r + 1];
    // floor(x) < X  <=>  x < X for integer X
    return (std::lower_bound(b, e, X) - b) & 1;
}

void Builder::push_f(uint64_t s, uint64_t e, std::vector<uint32_t> &f) const {
    if (!f.empty() && f.back() == s) f.back() = uint32_t(e);   // contiguous: extend
    else { f.push_back(uint32_t(s)); f.push_back(uint32_t(e)); }
}

// Centre-line crossing tables of every row the polygon spans.
void Builder::row_tables(const Poly &p, int threads) {
    const size_t nv = p.x.size();
    int64_t ymin = p.y[0], ymax = p.y[0];
    for (size_t k = 0; k < nv; k++) { ymin = std::min(ymin, p.y[k]); ymax = std::max(ymax, p.y[k]); }
    jmin_ = floor_div(ymin, g_.w) - 1;
    jmax_ = floor_div(ymax, g_.w) + 1;
    const size_t rows = size_t(jmax_ - jmin_ + 1);
    row_off_.assign(rows + 1, 0);
    row_fill_.assign(rows, 0);
    // count, then fill
    for (size_t k = 0; k < nv; k++) {
        const size_t k2 = (k + 1 == nv) ? 0 : k + 1;
        int64_t ay = p.y[k], by = p.y[k2];
        if (ay == by) continue;
        if (ay > by) std::swap(ay, by);
        const int64_t w = g_.w;
        const int64_t j0 = std::max<int64_t>(jmin_, ceil_div(2 * i128(ay) - w, 2 * i128(w)));
        const int64_t j1 = std::min<int64_t>(jmax_, ceil_div(2 * i128(by) - w, 2 * i128(w)) - 1);
        for (int64_t j = j0; j <= j1; j++) row_off_[size_t(j - jmin_) + 1]++;
    }
    for (size_t r = 0; r < rows; r++) row_off_[r + 1] += row_off_[r];
    row_x_.resize(row_off_[rows]);
    for (size_t k = 0; k < nv; k++) {
        const size_t k2 = (k + 1 == nv) ? 0 : k + 1;
        edge_crossings(p.x[k], p.y[k], p.x[k2], p.y[k2]);
    }
    parallel(threads, [&](int t) {
        for (size_t r = rows * size_t(t) / size_t(threads); r < rows * size_t(t + 1) / size_t(threads); r++)
            std::sort(row_x_.begin() + row_off_[r], row_x_.begin() + row_off_[r + 1]);
    });
}

// Classes of the sorted, merged touched cells (cls[t] bit 0: touched cell t is
// Full, i.e. border-only contact with its centre inside; bit 1: the gap after
// it is inside), turned into the A- and F-lists by one walk in Hilbert order.
void Builder::intervalize(const uint8_t *cls, size_t m, Result &out) const {
    auto &A = out.a;
    auto &F = out.f;
    A.clear();
    F.clear();
    uint64_t a_start = touched_[0] >> 1;
    for (size_t t = 0; t < m; t++) {
        const uint64_t d = touched_[t] >> 1;
        if (cls[t] & 1) push_f(d, d + 1, F);
        if (t + 1 == m) break;
        const uint64_t nxt = touched_[t + 1] >> 1;
        if (nxt == d + 1) continue;
        // gap [d+1, nxt): one class throughout
        if (cls[t] & 2) {
            push_f(d + 1, nxt, F);
        } else {
            A.push_back(uint32_t(a_start));
            A.push_back(uint32_t(d + 1));
            a_start = nxt;
        }
    }
    A.push_back(uint32_t(a_start));
    A.push_back(uint32_t((touched_[m - 1] >> 1) + 1));
}

// class bits of touched cell t (see intervalize)
#define APRIL_CELL_CLASS(t, m)                                                              \
    ([&](size_t t_) -> uint8_t {                                                            \
        uint8_t c = 0;                                                                      \
        uint32_t ci, cj;                                                                    \
        const uint64_t d = touched_[t_] >> 1;                                               \
        if (!(touched_[t_] & 1)) {                                                          \
            hilbert_d2xy(g_.order, d, &ci, &cj);                                            \
            if (centre_inside(ci, cj)) c |= 1;                                              \
        }                                                                                   \
        if (t_ + 1 < (m) && (touched_[t_ + 1] >> 1) != d + 1) {                             \
            hilbert_d2xy(g_.order, d + 1, &ci, &cj);                                        \
            if (centre_inside(ci, cj)) c |= 2;                                              \
        }                                                                                   \
        return c;                                                                           \
    })(t)

void Builder::chain_cells(const Poly &p, std::vector<uint64_t> &ids) {
    touched_.clear();
    for (size_t k = 0; k + 1 < p.x.size(); k++) edge_cells(p.x[k], p.y[k], p.x[k + 1], p.y[k + 1], touched_);
    ids.clear();
    for (uint64_t t : touched_) ids.push_back(t >> 1);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
}

int Builder::run(const Poly &p, Result &out) {
    const size_t nv = p.x.size();
    touched_.clear();
    // 1. boundary cells
    for (size_t k = 0; k < nv; k++) {
        const size_t k2 = (k + 1 == nv) ? 0 : k + 1;
        edge_cells(p.x[k], p.y[k], p.x[k2], p.y[k2], touched_);
    }
    std::sort(touched_.begin(), touched_.end());
    // merge duplicates: keep one entry per cell, interior flag ORed
    size_t m = 0;
    for (size_t t = 0; t < touched_.size(); t++) {
        if (m && (touched_[m - 1] >> 1) == (touched_[t] >> 1)) touched_[m - 1] |= touched_[t] & 1;
        else touched_[m++] = touched_[t];
    }
    touched_.resize(m);
    // 2. centre-line crossings per row
    row_tables(p);
    // 3. one-step intervalization
    cls_.resize(m);
    for (size_t t = 0; t < m; t++) cls_[t] = APRIL_CELL_CLASS(t, m);
    intervalize(cls_.data(), m, out);
    return APRIL_OK;
}

int Builder::run_parallel(const Poly &p, Result &out, int T) {
    const size_t nv = p.x.size();
    // 1. boundary cells, edges split over the threads
    std::vector<std::vector<uint64_t>> part(T);
    parallel(T, [&](int t) {
        const size_t k0 = nv * size_t(t) / size_t(T), k1 = nv * size_t(t + 1) / size_t(T);
        for (size_t k = k0; k < k1; k++) {
            const size_t k2 = (k + 1 == nv) ? 0 : k + 1;
            edge_cells(p.x[k], p.y[k], p.x[k2], p.y[k2], part[t]);
        }
    });
    // 2. sample sort by cell id: T - 1 splitters from evenly spaced samples
    //    of every part; each part is cut into the T id ranges, and range b
    //    (bucket b) is gathered, sorted and merged by thread b
    std::vector<uint64_t> sample;
    for (int t = 0; t < T; t++)
        for (size_t q = 1; q <= 32 && !part[t].empty(); q++) sample.push_back(part[t][part[t].size() * q / 33] >> 1);
    std::sort(sample.begin(), sample.end());
    std::vector<uint64_t> spl(T, 0);   // bucket b holds ids in [spl[b], spl[b + 1])
    for (int b = 1; b < T; b++) spl[b] = sample.empty() ? 0 : sample[sample.size() * size_t(b) / size_t(T)];
    auto bucket_of = [&](uint64_t key) {
        return int(std::upper_bound(spl.begin() + 1, spl.end(), key >> 1) - spl.begin()) - 1;
    };
    std::vector<std::vector<size_t>> cnt(T, std::vector<size_t>(T + 1, 0));   // [part][bucket]
    parallel(T, [&](int t) {
        for (uint64_t v : part[t]) cnt[t][bucket_of(v) + 1]++;
        for (int b = 0; b < T; b++) cnt[t][b + 1] += cnt[t][b];
        // counting sort of the part by bucket (stable, in place via a copy)
        std::vector<uint64_t> tmp(part[t].size());
        std::vector<size_t> pos(cnt[t].begin(), cnt[t].end() - 1);
        for (uint64_t v : part[t]) tmp[pos[bucket_of(v)]++] = v;
        part[t].swap(tmp);
    });
    std::vector<std::vector<uint64_t>> bucket(T);
    parallel(T, [&](int b) {
        auto &v = bucket[b];
        size_t n = 0;
        for (int t = 0; t < T; t++) n += cnt[t][b + 1] - cnt[t][b];
        v.reserve(n);
        for (int t = 0; t < T; t++) v.insert(v.end(), part[t].begin() + cnt[t][b], part[t].begin() + cnt[t][b + 1]);
        std::sort(v.begin(), v.end());
        size_t m = 0;
        for (size_t t = 0; t < v.size(); t++) {
            if (m && (v[m - 1] >> 1) == (v[t] >> 1)) v[m - 1] |= v[t] & 1;
            else v[m++] = v[t];
        }
        v.resize(m);
    });
    part.clear();
    std::vector<size_t> boff(T + 1, 0);
    for (int b = 0; b < T; b++) boff[b + 1] = boff[b] + bucket[b].size();
    const size_t m = boff[T];
    touched_.resize(m);
    parallel(T, [&](int b) {
        std::copy(bucket[b].begin(), bucket[b].end(), touched_.begin() + boff[b]);
        std::vector<uint64_t>().swap(bucket[b]);
    });
    // 3. row tables, every cell's classes, then the walk, each split over
    //    the threads; the walk's segments are stitched at their ends
    row_tables(p, T);
    cls_.resize(m);
    std::vector<Result> seg(T);
    std::vector<uint64_t> first_start(T), last_start(T);   // first A interval's start slot; carried a_start
    std::vector<char> emitted(T, 0);
    parallel(T, [&](int t) {
        const size_t t0 = m * size_t(t) / size_t(T), t1 = m * size_t(t + 1) / size_t(T);
        for (size_t i = t0; i < t1; i++) cls_[i] = APRIL_CELL_CLASS(i, m);
        // walk [t0, t1): A intervals whose start is not yet known use the
        // carried start of the segments before (filled in below)
        auto &A = seg[t].a;
        auto &F = seg[t].f;
        uint64_t a_start = t0 < t1 ? touched_[t0] >> 1 : 0;
        bool open = true;   // the current A interval started before this segment
        for (size_t i = t0; i < t1; i++) {
            const uint64_t d = touched_[i] >> 1;
            if (cls_[i] & 1) push_f(d, d + 1, F);
            if (i + 1 == m) break;
            const uint64_t nxt = touched_[i + 1] >> 1;
            if (nxt == d + 1) continue;
            if (cls_[i] & 2) {
                push_f(d + 1, nxt, F);
            } else {
                if (open) { emitted[t] = 1; first_start[t] = 0; }
                A.push_back(open ? 0u : uint32_t(a_start));
                A.push_back(uint32_t(d + 1));
                a_start = nxt;
                open = false;
            }
        }
        last_start[t] = open ? ~uint64_t(0) : a_start;
    });
    auto &A = out.a;
    auto &F = out.f;
    A.clear();
    F.clear();
    uint64_t carry = touched_[0] >> 1;
    for (int t = 0; t < T; t++) {
        auto &a = seg[t].a;
        if (emitted[t]) a[0] = uint32_t(carry);   // the interval open at the segment's start
        A.insert(A.end(), a.begin(), a.end());
        if (last_start[t] != ~uint64_t(0)) carry = last_start[t];
        for (size_t k = 0; k < seg[t].f.size(); k += 2) push_f(seg[t].f[k], seg[t].f[k + 1], F);
    }
    A.push_back(uint32_t(carry));
    A.push_back(uint32_t((touched_[m - 1] >> 1) + 1));
    return APRIL_OK;
}

#undef APRIL_CELL_CLASS

}  // namespace
}  // namespace april

using namespace april;

namespace {

// Build every polygon k on grid lg[gid(k)]; one collection out.
template <class GridOf>
int build_collection(const std::vector<LatticeGrid> &lg, GridOf gid, const april_grid_t &desc,
                     uint64_t key, const double *xy, const uint64_t *vtx_off, uint64_t n, uint32_t flags,
                     april_lists_t **out, int max_threads) {
    for (uint64_t k = 0; k < n; k++)
        if (vtx_off[k + 1] < vtx_off[k] + 3) return fail(APRIL_E_INVALID, "polygon with < 3 vertices");
    const bool strict = flags & APRIL_STRICT;
    std::vector<Result> res(n);
    std::atomic<uint64_t> next{0};
    std::atomic<int> err{0};
    const int T = int(std::min<uint64_t>(std::max(1, max_threads), n));
    // with fewer polygons than threads, a large polygon is built by several
    // threads (about this many boundary cells or more: APRIL_PAR_BUILD_CELLS)
    const int inner = std::max(1, max_threads / std::max(1, T));
    const char *pe = getenv("APRIL_PAR_BUILD_CELLS");
    const double par_cells = pe ? atof(pe) : 65536.0;
    parallel(T, [&](int) {
        Builder b(lg[0]);
        Poly p;
        for (;;) {
            const uint64_t k = next.fetch_add(1);
            if (k >= n || err.load()) break;
            const LatticeGrid &g = lg[gid(k)];
            b.set_grid(g);
            const uint64_t v0 = vtx_off[k], v1 = vtx_off[k + 1];
            p.x.clear();
            p.y.clear();
            int rc = APRIL_OK;
            for (uint64_t v = v0; v < v1 && rc == APRIL_OK; v++) {
                int64_t c[2];
                for (int a = 0; a < 2; a++) {
                    const double q = (xy[2 * v + a] - (a ? g.y0 : g.x0)) * 1073741824.0;
                    const double r = std::nearbyint(q);
                    if (!(std::fabs(r) < 4.0e15)) { rc = APRIL_E_GRID; break; }
                    if (strict && r != q) { rc = APRIL_E_INVALID; break; }
                    c[a] = int64_t(r);
                }
                if (rc) break;
                // the outer ring of cells must stay untouched
                if (c[0] <= g.w || c[1] <= g.w || c[0] >= (g.cells - 1) * g.w || c[1] >= (g.cells - 1) * g.w) {
                    rc = APRIL_E_GRID;
                    break;
                }
                // drop repeated vertices (zero-length edges)
                if (!p.x.empty() && p.x.back() == c[0] && p.y.back() == c[1]) continue;
                p.x.push_back(c[0]);
                p.y.push_back(c[1]);
            }
            while (rc == APRIL_OK && p.x.size() > 1 && p.x.front() == p.x.back() && p.y.front() == p.y.back()) {
                p.x.pop_back();
                p.y.pop_back();
            }
            if (rc == APRIL_OK && p.x.size() < 3) rc = APRIL_E_INVALID;
            if (rc == APRIL_OK) {
                double cells = 0;   // boundary cells, estimated from the edges' extents
                if (inner > 1)
                    for (size_t v = 0; v < p.x.size(); v++) {
                        const size_t v2 = v + 1 == p.x.size() ? 0 : v + 1;
                        cells += double(std::llabs(p.x[v2] - p.x[v]) + std::llabs(p.y[v2] - p.y[v])) / double(g.w) + 2;
                    }
                rc = (inner > 1 && cells >= par_cells) ? b.run_parallel(p, res[k], inner) : b.run(p, res[k]);
            }
            if (rc) {
                res[k].rc = rc;
                int z = 0;
                err.compare_exchange_strong(z, int(k + 1 > 0x7fffffff ? 0x7fffffff : k + 1));
            }
        }
    });
    if (err.load()) {
        const uint64_t k = uint64_t(err.load()) - 1;
        const int rc = res[k].rc;
        return fail(rc, rc == APRIL_E_GRID ? "polygon " + std::to_string(k) + " reaches the outer cell ring or leaves the grid"
                        : rc == APRIL_E_INVALID ? "polygon " + std::to_string(k) + " has a non-lattice coordinate or < 3 distinct vertices"
                                                : "polygon " + std::to_string(k) + " failed");
    }
    auto *L = new (std::nothrow) april_lists;
    if (!L) return fail(APRIL_E_NOMEM, "out of host memory");
    try {
        L->grid = desc;
        L->partition_key = key;
        L->n = n;
        L->off_a.resize(n + 1);
        L->off_f.resize(n + 1);
        uint64_t na = 0, nf = 0;
        for (uint64_t k = 0; k < n; k++) {
            L->off_a[k] = na;
            L->off_f[k] = nf;
            na += res[k].a.size() / 2;
            nf += res[k].f.size() / 2;
        }
        L->off_a[n] = na;
        L->off_f[n] = nf;
        L->n_a = na;
        L->n_f = nf;
        L->start_a.resize(na);
        L->end_a.resize(na);
        L->start_f.resize(nf);
        L->end_f.resize(nf);
        std::atomic<uint64_t> nk{0};
        parallel(T, [&](int) {
            for (;;) {
                const uint64_t k = nk.fetch_add(1);
                if (k >= n) break;
                uint64_t o = L->off_a[k];
                for (size_t t = 0; t < res[k].a.size(); t += 2, o++) {
                    L->start_a[o] = res[k].a[t];
                    L->end_a[o] = res[k].a[t + 1];
                }
                o = L->off_f[k];
                for (size_t t = 0; t < res[k].f.size(); t += 2, o++) {
                    L->start_f[o] = res[k].f[t];
                    L->end_f[o] = res[k].f[t + 1];
                }
                std::vector<uint32_t>().swap(res[k].a);
                std::vector<uint32_t>().swap(res[k].f);
            }
        });
    } catch (...) {
        delete L;
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    *out = L;
    return APRIL_OK;
}

}  // namespace

extern "C" int april_build_lists(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off,
                                 uint64_t n, uint32_t flags, april_lists_t **out) {
    clear_error();
    if (!grid || !xy || !vtx_off || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no polygons");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    std::vector<LatticeGrid> lg(1);
    if (int rc = lattice_grid(grid, &lg[0])) return rc;
    return build_collection(lg, [](uint64_t) { return 0u; }, *grid, 0, xy, vtx_off, n, flags, out, host_threads());
}

namespace april {
int build_lists_threads(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off, uint64_t n,
                        uint32_t flags, int max_threads, april_lists_t **out) {
    clear_error();
    if (!grid || !xy || !vtx_off || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no polygons");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    std::vector<LatticeGrid> lg(1);
    if (int rc = lattice_grid(grid, &lg[0])) return rc;
    return build_collection(lg, [](uint64_t) { return 0u; }, *grid, 0, xy, vtx_off, n, flags, out, max_threads);
}
}  // namespace april

extern "C" int april_build_lists_partitioned(const april_grid_t *grids, uint32_t n_grids,
                                             const uint32_t *grid_of, const double *xy,
                                             const uint64_t *vtx_off, uint64_t n, uint32_t flags,
                                             april_lists_t **out) {
    clear_error();
    if (!grids || !grid_of || !xy || !vtx_off || !out || n_grids == 0)
        return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no polygons");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    std::vector<LatticeGrid> lg(n_grids);
    uint64_t key = 1469598103934665603ull;   // FNV-1a over the grid descriptors
    for (uint32_t t = 0; t < n_grids; t++) {
        if (int rc = lattice_grid(&grids[t], &lg[t])) return rc;
        const unsigned char *b = reinterpret_cast<const unsigned char *>(&grids[t]);
        for (size_t u = 0; u < sizeof(april_grid_t); u++) key = (key ^ b[u]) * 1099511628211ull;
    }
    for (uint64_t k = 0; k < n; k++)
        if (grid_of[k] >= n_grids) return fail(APRIL_E_INVALID, "grid index out of range");
    april_grid_t desc = grids[0];
    desc.flags = APRIL_GRID_PARTITIONED;
    return build_collection(lg, [&](uint64_t k) { return grid_of[k]; }, desc, key, xy, vtx_off, n, flags,
                            out, host_threads());
}

extern "C" int april_build_cells(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off, uint64_t n,
                                 uint32_t flags, april_cells_t **out) {
    clear_error();
    if (!grid || !xy || !vtx_off || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no linestrings");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    LatticeGrid g;
    if (int rc = lattice_grid(grid, &g)) return rc;
    for (uint64_t k = 0; k < n; k++)
        if (vtx_off[k + 1] < vtx_off[k] + 2) return fail(APRIL_E_INVALID, "linestring with < 2 vertices");
    const bool strict = flags & APRIL_STRICT;
    std::vector<std::vector<uint32_t>> per(n);
    std::atomic<uint64_t> next{0};
    std::atomic<int> err{0};
    std::atomic<uint64_t> bad{~0ull};
    const int T = int(std::min<uint64_t>(uint64_t(host_threads()), n));
    parallel(T, [&](int) {
        Builder b(g);
        Poly p;
        std::vector<uint64_t> ids;
        for (;;) {
            const uint64_t k = next.fetch_add(1);
            if (k >= n || err.load()) break;
            p.x.clear();
            p.y.clear();
            int rc = APRIL_OK;
            for (uint64_t v = vtx_off[k]; v < vtx_off[k + 1] && rc == APRIL_OK; v++) {
                int64_t c[2];
                for (int a = 0; a < 2 && rc == APRIL_OK; a++) {
                    const double q = (xy[2 * v + a] - (a ? g.y0 : g.x0)) * 1073741824.0;
                    const double r = std::nearbyint(q);
                    if (!(std::fabs(r) < 4.0e15)) rc = APRIL_E_GRID;
                    else if (strict && r != q) rc = APRIL_E_INVALID;
                    else c[a] = int64_t(r);
                }
                if (rc == APRIL_OK &&
                    (c[0] <= g.w || c[1] <= g.w || c[0] >= (g.cells - 1) * g.w || c[1] >= (g.cells - 1) * g.w))
                    rc = APRIL_E_GRID;
                if (rc == APRIL_OK) {
                    p.x.push_back(c[0]);
                    p.y.push_back(c[1]);
                }
            }
            if (rc != APRIL_OK) {
                int z = 0;
                err.compare_exchange_strong(z, rc);
                bad.store(k);
                break;
            }
            b.chain_cells(p, ids);
            per[k].assign(ids.begin(), ids.end());
        }
    });
    if (int rc = err.load())
        return fail(rc, "linestring " + std::to_string(bad.load()) +
                            (rc == APRIL_E_GRID ? " reaches the outer cell ring or leaves the grid"
                                                : " has a non-lattice coordinate"));
    auto *C = new (std::nothrow) april_cells;
    if (!C) return fail(APRIL_E_NOMEM, "out of host memory");
    try {
        C->grid = *grid;
        C->n = n;
        C->off.resize(n + 1);
        C->off[0] = 0;
        for (uint64_t k = 0; k < n; k++) C->off[k + 1] = C->off[k] + per[k].size();
        C->n_ids = C->off[n];
        C->ids.resize(C->n_ids);
        for (uint64_t k = 0; k < n; k++) std::copy(per[k].begin(), per[k].end(), C->ids.begin() + C->off[k]);
    } catch (...) {
        delete C;
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    *out = C;
    return APRIL_OK;
}
