// GPU construction of APRIL A- and F-lists (Sec. 6), for a whole collection
// at once.  The lists are identical to the host builder's (build.cpp): the
// same exact edge traversal, the same centre-line crossing rule, the same
// one-step intervalization -- reorganized as data-parallel passes:
//
//  1. one thread per vertex: lattice coordinates relative to the grid origin
//     and the checks (lattice, grid ring);
//  2. one thread per edge: how many (cell, row) entries it produces -- the
//     cells whose closed square it meets, row by row (Sec. 6.1 traversal),
//     and the centre lines of cell rows it crosses; exclusive scans give
//     every edge its output range;
//  3. one thread per edge writes its entries: key (polygon, Hilbert id,
//     interior-crossed flag) for cells, key (polygon, row) and crossing x
//     for centre lines;
//  4. radix sorts: for each polygon the touched cells are then in Hilbert
//     order, and each row's crossings contiguous and in x order;
//  5. one thread per entry keeps the last entry of every (polygon, cell) run
//     (its flag is the OR of the run's), and a scan compacts them;
//  6. one thread per touched cell takes the class bits of Alg. 3 (centre of
//     a border-only cell inside; first cell of the gap after it inside) from
//     the parity of the crossings left of the centre in its row (two binary
//     searches);
//  7. one thread per touched cell decides which A- and F-interval ends it
//     owns -- a run of A or F cells starts or stops only at a touched cell or
//     at a gap next to it -- and scans give each end its slot.
//
// Two host synchronizations read the sizes that the output buffers need.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <new>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t fdiv(int64_t a, int64_t b) {   // floor(a / b), b > 0
    const int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}
__device__ __forceinline__ int64_t fdiv(__int128 a, __int128 b) {
    const __int128 q = a / b;
    return int64_t((a % b != 0 && a < 0) ? q - 1 : q);
}
template <typename T>
__device__ __forceinline__ int64_t cdiv(T a, T b) { return -fdiv(T(-a), b); }

// Hilbert curve, the library's variant: quadrants lower-left, upper-left,
// upper-right, lower-right; the first sub-curve transposed, the last one
// reflected in the anti-diagonal.  A state is one of the four symmetries
// (0 identity, 1 transpose, 2 anti-transpose, 3 half turn); they compose by
// XOR.
__device__ __forceinline__ void sym(uint32_t s, uint32_t bx, uint32_t by, uint32_t &ox, uint32_t &oy) {
    const uint32_t swap = (s ^ (s >> 1)) & 1u, flip = (s >> 1) & 1u;
    ox = (swap ? by : bx) ^ flip;
    oy = (swap ? bx : by) ^ flip;
}
__device__ __forceinline__ uint32_t child(uint32_t digit) { return digit == 0 ? 1u : digit == 3 ? 2u : 0u; }

__device__ uint32_t hilbert_d(int order, uint32_t x, uint32_t y) {
    uint32_t state = 0, d = 0;
    for (int lvl = order - 1; lvl >= 0; lvl--) {
        uint32_t qx, qy;
        sym(state, (x >> lvl) & 1u, (y >> lvl) & 1u, qx, qy);
        const uint32_t digit = (qx * 3u) ^ qy;   // (0,0)->0 (0,1)->1 (1,1)->2 (1,0)->3
        d = (d << 2) | digit;
        state ^= child(digit);
    }
    return d;
}

__device__ void hilbert_xy(int order, uint32_t d, uint32_t &x, uint32_t &y) {
    uint32_t state = 0, X = 0, Y = 0;
    for (int lvl = order - 1; lvl >= 0; lvl--) {
        const uint32_t digit = (d >> (2 * lvl)) & 3u;
        uint32_t bx, by;
        sym(state, digit >> 1, (digit ^ (digit >> 1)) & 1u, bx, by);   // quadrant of the digit
        X = (X << 1) | bx;
        Y = (Y << 1) | by;
        state ^= child(digit);
    }
    x = X;
    y = Y;
}

struct Geo {
    double x0, y0;     // grid origin
    int64_t w;         // cell side, lattice units
    int64_t cells;     // 2^order
    int order;
    uint32_t strict;
};

// error word: (polygon << 32) | (vertex in polygon << 8) | code; the
// smallest wins, so the report names the first failing polygon and, in it,
// the first failing check in vertex order (as the host builder does)
enum : uint64_t { kErrGrid = 1, kErrLattice = 2, kErrDistinct = 3 };
constexpr uint64_t kErrNoVertex = 0xffffff;

__global__ void k_vertices(const double *xy, const uint64_t *voff, uint64_t n, uint64_t nv, Geo g, int64_t *X,
                           int64_t *Y, uint32_t *poly, uint8_t *bad, unsigned long long *err) {
    const uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    // polygon of vertex v: the last k with voff[k] <= v
    uint64_t lo = 0, hi = n;   // voff[lo] <= v < voff[hi]
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (voff[mid] <= v) lo = mid;
        else hi = mid;
    }
    poly[v] = uint32_t(lo);
    uint64_t code = 0;
    int64_t c[2] = {0, 0};
    for (int a = 0; a < 2 && !code; a++) {
        const double q = (xy[2 * v + a] - (a ? g.y0 : g.x0)) * 1073741824.0;
        const double r = rint(q);
        if (!(fabs(r) < 4.0e15)) code = kErrGrid;
        else if (g.strict && r != q) code = kErrLattice;
        else c[a] = int64_t(r);
    }
    // the outer ring of cells must stay untouched
    if (!code && (c[0] <= g.w || c[1] <= g.w || c[0] >= (g.cells - 1) * g.w || c[1] >= (g.cells - 1) * g.w))
        code = kErrGrid;
    X[v] = c[0];
    Y[v] = c[1];
    if (code) {
        bad[lo] = 1;
        const uint64_t vl = min<uint64_t>(v - voff[lo], kErrNoVertex - 1);
        atomicMin(err, (unsigned long long)((lo << 32) | (vl << 8) | code));
    }
}

// Cells met by the edge a-b (closed squares), row by row; with EMIT, their
// keys.  T is the product type: int64 when the grid spans few enough lattice
// units, else 128-bit.
template <typename T, bool EMIT>
__device__ uint64_t edge_cells(int64_t ax, int64_t ay, int64_t bx, int64_t by, const Geo &g, uint64_t key_hi,
                               uint64_t *out) {
    const int64_t w = g.w;
    if (ay > by) {
        const int64_t tx = ax, ty = ay;
        ax = bx; ay = by; bx = tx; by = ty;
    }
    const bool horiz = ay == by;
    const T D = horiz ? T(1) : T(by - ay);
    const int64_t j0 = cdiv<int64_t>(ay, w) - 1, j1 = fdiv(by, w);
    uint64_t cnt = 0;
    for (int64_t j = j0; j <= j1; j++) {
        const int64_t ylo = max(ay, j * w), yhi = min(by, (j + 1) * w);
        T n0, n1;
        if (horiz) {
            n0 = T(min(ax, bx));
            n1 = T(max(ax, bx));
        } else {
            const T u = T(ax) * D + T(ylo - ay) * T(bx - ax);
            const T v = T(ax) * D + T(yhi - ay) * T(bx - ax);
            n0 = u < v ? u : v;
            n1 = u < v ? v : u;
        }
        const T Dw = D * T(w);
        const int64_t i0 = cdiv<T>(n0, Dw) - 1, i1 = fdiv(n1, Dw);
        if (EMIT) {
            const bool open_row = horiz ? (j * w < ay && ay < (j + 1) * w) : (ylo < yhi);
            int64_t o0 = 1, o1 = 0;
            if (open_row) {
                o0 = fdiv(n0, Dw);
                o1 = cdiv<T>(n1, Dw) - 1;
            }
            for (int64_t i = i0; i <= i1; i++) {
                const uint64_t d = hilbert_d(g.order, uint32_t(i), uint32_t(j));
                out[cnt + uint64_t(i - i0)] = key_hi | (d << 1) | uint64_t(i >= o0 && i <= o1);
            }
        }
        cnt += uint64_t(i1 - i0 + 1);
    }
    return cnt;
}

// Crossings of the edge a-b with the centre lines of cell rows (half-open:
// y = c is crossed iff exactly one endpoint lies above c); with EMIT, the
// floor of each crossing's doubled x.
template <typename T, bool EMIT>
__device__ uint64_t edge_crossings(int64_t ax, int64_t ay, int64_t bx, int64_t by, const Geo &g, uint64_t key_hi,
                                   uint64_t *okey, int64_t *ox) {
    if (ay == by) return 0;
    if (ay > by) {
        const int64_t tx = ax, ty = ay;
        ax = bx; ay = by; bx = tx; by = ty;
    }
    const int64_t w = g.w;
    const int64_t j0 = cdiv<int64_t>(2 * ay - w, 2 * w), j1 = cdiv<int64_t>(2 * by - w, 2 * w) - 1;
    if (j1 < j0) return 0;
    if (EMIT) {
        const T D = T(by - ay);
        for (int64_t j = j0; j <= j1; j++) {
            const T c = T(2 * j + 1) * T(w);
            const T N = T(2) * T(ax) * D + (c - T(2) * T(ay)) * T(bx - ax);
            okey[j - j0] = key_hi | uint64_t(j);
            ox[j - j0] = fdiv(N, D);
        }
    }
    return uint64_t(j1 - j0 + 1);
}

struct EdgeArgs {
    const int64_t *X, *Y;
    const uint32_t *poly;
    const uint64_t *voff;
    const uint8_t *bad;
    uint64_t nv;
    Geo g;
    uint32_t wide;
};

__device__ __forceinline__ uint64_t next_vertex(const EdgeArgs &a, uint64_t v, uint32_t k) {
    return v + 1 == a.voff[k + 1] ? a.voff[k] : v + 1;
}

__global__ void k_edges_count(EdgeArgs a, uint64_t *ccount, uint64_t *xcount, uint32_t *ndistinct) {
    const uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const bool valid = v < a.nv;
    const uint32_t k = valid ? a.poly[v] : 0xffffffffu;
    bool distinct = false;
    uint64_t cc = 0, xc = 0;
    if (valid && !a.bad[k]) {
        const uint64_t v2 = next_vertex(a, v, k);
        const int64_t ax = a.X[v], ay = a.Y[v], bx = a.X[v2], by = a.Y[v2];
        distinct = ax != bx || ay != by;
        if (a.wide) {
            cc = edge_cells<__int128, false>(ax, ay, bx, by, a.g, 0, nullptr);
            xc = edge_crossings<__int128, false>(ax, ay, bx, by, a.g, 0, nullptr, nullptr);
        } else {
            cc = edge_cells<int64_t, false>(ax, ay, bx, by, a.g, 0, nullptr);
            xc = edge_crossings<int64_t, false>(ax, ay, bx, by, a.g, 0, nullptr, nullptr);
        }
    }
    if (valid) {
        ccount[v] = cc;
        xcount[v] = xc;
    }
    // distinct edges per polygon, one atomic per run of equal polygon ids in
    // the wave (ids are non-decreasing in v; a polygon of 10^5 vertices would
    // otherwise take 10^5 atomics on one word)
    const uint32_t kp = __shfl_up(k, 1);
    const bool head = lane == 0 || kp != k;
    const uint64_t heads = __ballot(head), flags = __ballot(distinct);
    if (head && k != 0xffffffffu) {
        const uint64_t above = lane == 63 ? 0 : heads & ~((2ull << lane) - 1);
        const uint32_t next = above ? uint32_t(__builtin_ctzll(above)) : 64u;
        const uint64_t upto = next == 64 ? ~0ull : (1ull << next) - 1;
        const uint32_t c = uint32_t(__popcll(flags & upto & ~((1ull << lane) - 1)));
        if (c) atomicAdd(&ndistinct[k], c);
    }
}

__global__ void k_check_distinct(const uint32_t *ndistinct, uint64_t n, unsigned long long *err) {
    const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n && ndistinct[k] < 3) atomicMin(err, (unsigned long long)((k << 32) | (kErrNoVertex << 8) | kErrDistinct));
}

// Each edge writes exactly the entries it counted (same loops), inside its
// scanned range [coff[v], coff[v] + ccount[v]); the range is checked against
// the totals first.
__global__ void k_edges_emit(EdgeArgs a, const uint64_t *coff, const uint64_t *ccount, const uint64_t *xoff,
                             const uint64_t *xcount, uint64_t ne, uint64_t nx, uint64_t *ckey, uint64_t *xkey,
                             int64_t *xval) {
    const uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= a.nv) return;
    const uint32_t k = a.poly[v];
    if (a.bad[k] || coff[v] + ccount[v] > ne || xoff[v] + xcount[v] > nx) return;
    const uint64_t v2 = next_vertex(a, v, k);
    const int64_t ax = a.X[v], ay = a.Y[v], bx = a.X[v2], by = a.Y[v2];
    const uint64_t chi = uint64_t(k) << 33, xhi = uint64_t(k) << 16;
    if (a.wide) {
        edge_cells<__int128, true>(ax, ay, bx, by, a.g, chi, ckey + coff[v]);
        edge_crossings<__int128, true>(ax, ay, bx, by, a.g, xhi, xkey + xoff[v], xval + xoff[v]);
    } else {
        edge_cells<int64_t, true>(ax, ay, bx, by, a.g, chi, ckey + coff[v]);
        edge_crossings<int64_t, true>(ax, ay, bx, by, a.g, xhi, xkey + xoff[v], xval + xoff[v]);
    }
}

// keep the last entry of every (polygon, cell) run: its flag is the run's OR
__global__ void k_keep(const uint64_t *key, uint64_t ne, uint64_t *keep) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    keep[i] = (i + 1 == ne || (key[i] >> 1) != (key[i + 1] >> 1)) ? 1 : 0;
}

__global__ void k_compact(const uint64_t *key, const uint64_t *keep, const uint64_t *pos, uint64_t ne,
                          uint64_t *cell, unsigned long long *m_out) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    if (keep[i]) cell[pos[i]] = key[i];
    if (i + 1 == ne) *m_out = pos[i] + keep[i];
}

// first touched cell of every polygon (each polygon has at least one)
__global__ void k_first(const uint64_t *cell, const unsigned long long *m_in, uint64_t n, uint64_t *first) {
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t m = *m_in;
    if (t == 0) first[n] = m;
    if (t >= m) return;
    const uint64_t k = cell[t] >> 33;
    if (t == 0 || (cell[t - 1] >> 33) != k) first[k] = t;
}

// Is the centre of cell (i, j) of polygon k inside?  Asked only for cells
// whose interior no edge crosses, so the centre is not on the boundary: the
// parity of the row's crossings left of it decides.
__device__ bool centre_inside(const uint64_t *xkey, const int64_t *xval, uint64_t nx, uint64_t k, uint32_t i,
                              uint32_t j, int64_t w) {
    const uint64_t target = (k << 16) | j;
    const int64_t Xc = (2 * int64_t(i) + 1) * w;
    // crossings are sorted by (polygon, row), x ascending within a row: the
    // count left of the centre is the distance between the row's first entry
    // and the first entry at or right of the centre
    uint64_t lo = 0, hi = nx;   // first index with key >= target
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (xkey[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    uint64_t a = lo, b = nx;    // first index with (key, x) >= (target, Xc)
    while (a < b) {
        const uint64_t mid = (a + b) / 2;
        if (xkey[mid] == target && xval[mid] < Xc) a = mid + 1;
        else b = mid;
    }
    return (a - lo) & 1u;
}

struct CellArgs {
    const uint64_t *cell, *first;
    const unsigned long long *m;
    const uint64_t *xkey;
    const int64_t *xval;
    uint64_t nx;
    Geo g;
};

// class bits of Alg. 3: bit 0 the touched cell is Full (no edge crosses its
// interior and its centre is inside), bit 1 the gap after it is inside
__global__ void k_classify(CellArgs a, uint64_t bound, uint8_t *cls) {
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= bound || t >= *a.m) return;
    const uint64_t key = a.cell[t], k = key >> 33;
    const uint32_t d = uint32_t(key >> 1);
    uint8_t c = 0;
    uint32_t ci, cj;
    if (!(key & 1)) {
        hilbert_xy(a.g.order, d, ci, cj);
        if (centre_inside(a.xkey, a.xval, a.nx, k, ci, cj, a.g.w)) c |= 1;
    }
    if (t + 1 < a.first[k + 1] && t + 1 < *a.m && uint32_t(a.cell[t + 1] >> 1) != d + 1) {
        hilbert_xy(a.g.order, d + 1, ci, cj);
        if (centre_inside(a.xkey, a.xval, a.nx, k, ci, cj, a.g.w)) c |= 2;
    }
    cls[t] = c;
}

// The interval ends a touched cell t owns (cells of its polygon in Hilbert
// order, u = t's rank, m its count).  A-intervals: a run of touched cells
// and inside gaps; it starts at the first cell or after an outside gap, and
// ends at the last cell or before an outside gap.  F-intervals: maximal runs
// of Full touched cells and inside gaps.
struct Ends {
    bool a_start, a_end;
    bool f_start, f_end;     // at most one of each per cell
    uint32_t f_start_at, f_end_at;
};

__device__ __forceinline__ Ends cell_ends(const CellArgs &a, const uint8_t *cls, uint64_t t) {
    const uint64_t key = a.cell[t], k = key >> 33;
    const uint32_t d = uint32_t(key >> 1);
    const uint64_t f0 = a.first[k], f1 = a.first[k + 1];
    const bool has_prev = t > f0, has_next = t + 1 < f1 && t + 1 < *a.m;
    const uint32_t dp = has_prev ? uint32_t(a.cell[t - 1] >> 1) : 0, dn = has_next ? uint32_t(a.cell[t + 1] >> 1) : 0;
    const uint8_t c = cls[t], cp = has_prev ? cls[t - 1] : 0, cn = has_next ? cls[t + 1] : 0;
    const bool gap_before = has_prev && dp + 1 != d, gap_after = has_next && dn != d + 1;
    Ends e;
    e.a_start = !has_prev || (gap_before && !(cp & 2));
    e.a_end = !has_next || (gap_after && !(c & 2));
    const bool full = c & 1;
    const bool prev_f = has_prev && (gap_before ? (cp & 2) : (cp & 1));
    const bool next_f = has_next && (gap_after ? (c & 2) : (cn & 1));
    const bool gap_in = gap_after && (c & 2);
    e.f_start = false;
    e.f_end = false;
    e.f_start_at = e.f_end_at = 0;
    if (full && !prev_f) { e.f_start = true; e.f_start_at = d; }
    if (gap_in && !full) { e.f_start = true; e.f_start_at = d + 1; }
    if (full && !next_f) { e.f_end = true; e.f_end_at = d + 1; }
    if (gap_in && !(cn & 1)) { e.f_end = true; e.f_end_at = dn; }
    return e;
}

__global__ void k_count_ends(CellArgs a, const uint8_t *cls, uint64_t bound, uint64_t *na, uint64_t *nf) {
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= bound) return;
    if (t >= *a.m) {
        na[t] = nf[t] = 0;
        return;
    }
    const Ends e = cell_ends(a, cls, t);
    na[t] = e.a_start;
    nf[t] = e.f_start;
}

__global__ void k_totals(const uint64_t *na, const uint64_t *ai, const uint64_t *nf, const uint64_t *fi,
                         uint64_t bound, unsigned long long *tot) {
    tot[0] = ai[bound - 1] + na[bound - 1];
    tot[1] = fi[bound - 1] + nf[bound - 1];
}

// Every slot is checked against the sizes the host allocated; a slot out of
// range (which consistent class bits never give) sets *bad_slot instead.
__global__ void k_scatter(CellArgs a, const uint8_t *cls, uint64_t bound, const uint64_t *na, const uint64_t *ai,
                          const uint64_t *nf, const uint64_t *fi, uint64_t n, const unsigned long long *tot,
                          uint64_t n_a, uint64_t n_f, uint64_t *off_a, uint64_t *off_f, uint32_t *sa, uint32_t *ea,
                          uint32_t *sf, uint32_t *ef, unsigned int *bad_slot) {
    const uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t == 0) {
        off_a[n] = tot[0];
        off_f[n] = tot[1];
    }
    if (t >= bound || t >= *a.m) return;
    const uint64_t key = a.cell[t], k = key >> 33;
    const uint32_t d = uint32_t(key >> 1);
    if (t == a.first[k]) {
        off_a[k] = ai[t];
        off_f[k] = fi[t];
    }
    const Ends e = cell_ends(a, cls, t);
    // slots as unsigned: "- 1" below zero wraps past every bound
    const uint64_t s_a = ai[t], e_a = ai[t] + na[t] - 1, s_f = fi[t], e_f = fi[t] + nf[t] - 1;
    if ((e.a_start && s_a >= n_a) || (e.a_end && e_a >= n_a) || (e.f_start && s_f >= n_f) ||
        (e.f_end && e_f >= n_f)) {
        atomicOr(bad_slot, 1u);
        return;
    }
    if (e.a_start) sa[s_a] = d;
    if (e.a_end) ea[e_a] = d + 1;
    if (e.f_start) sf[s_f] = e.f_start_at;
    if (e.f_end) ef[e_f] = e.f_end_at;
}

uint32_t blocks_for(uint64_t n) { return uint32_t(std::max<uint64_t>(1, (n + kThreads - 1) / kThreads)); }

// Stream-ordered scratch, freed when the call returns (in stream order).
struct Scratch {
    hipStream_t s;
    std::vector<void *> held;
    hipError_t err = hipSuccess;
    template <typename T>
    T *get(uint64_t count) {
        void *p = nullptr;
        if (err == hipSuccess) err = hipMallocAsync(&p, std::max<uint64_t>(count, 1) * sizeof(T), s);
        if (err != hipSuccess) return nullptr;
        held.push_back(p);
        return static_cast<T *>(p);
    }
    ~Scratch() {
        for (void *p : held) (void)hipFreeAsync(p, s);
    }
};

}  // namespace
}  // namespace april

using namespace april;

#define BG_TRY(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(APRIL_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" int april_build_lists_gpu(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off,
                                     uint64_t n, uint32_t flags, void *hip_stream, april_lists_t **out) {
    clear_error();
    if (!xy || !vtx_off || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no polygons");
    if (n >= (1ull << 31)) return fail(APRIL_E_INVALID, "more than 2^31 - 1 polygons");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    LatticeGrid lg;
    if (int rc = lattice_grid(grid, &lg)) return rc;
    for (uint64_t k = 0; k < n; k++)
        if (vtx_off[k + 1] < vtx_off[k] + 3) return fail(APRIL_E_INVALID, "polygon with < 3 vertices");
    const uint64_t nv = vtx_off[n] - vtx_off[0];
    DeviceState *st = nullptr;
    if (int rc = device_state(&st)) return rc;
    int dev = 0;
    BG_TRY(hipGetDevice(&dev));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);

    Geo g{lg.x0, lg.y0, lg.w, lg.cells, lg.order, (flags & APRIL_STRICT) ? 1u : 0u};
    // 64-bit products are exact while the grid spans at most 1.25 * 2^30
    // lattice units (|products| <= 4 E^2 < 2^63)
    const uint32_t wide = double(lg.w) * double(lg.cells) > 1.25 * 1073741824.0 ? 1u : 0u;

    Scratch sc{s};
    double *d_xy = sc.get<double>(2 * nv);
    uint64_t *d_voff = sc.get<uint64_t>(n + 1);
    int64_t *d_X = sc.get<int64_t>(nv), *d_Y = sc.get<int64_t>(nv);
    uint32_t *d_poly = sc.get<uint32_t>(nv), *d_ndist = sc.get<uint32_t>(n);
    uint8_t *d_bad = sc.get<uint8_t>(n);
    uint64_t *d_cc = sc.get<uint64_t>(nv), *d_xc = sc.get<uint64_t>(nv);
    uint64_t *d_coff = sc.get<uint64_t>(nv), *d_xoff = sc.get<uint64_t>(nv);
    unsigned long long *d_small = sc.get<unsigned long long>(8);   // err, m, totals
    if (sc.err != hipSuccess) return fail(APRIL_E_NOMEM, std::string("build scratch: ") + hipGetErrorString(sc.err));
    std::vector<uint64_t> voff_rel(n + 1);
    for (uint64_t k = 0; k <= n; k++) voff_rel[k] = vtx_off[k] - vtx_off[0];
    BG_TRY(hipMemcpyAsync(d_xy, xy + 2 * vtx_off[0], 16 * nv, hipMemcpyHostToDevice, s));
    BG_TRY(hipMemcpyAsync(d_voff, voff_rel.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));
    BG_TRY(hipMemsetAsync(d_ndist, 0, 4 * n, s));
    BG_TRY(hipMemsetAsync(d_bad, 0, n, s));
    BG_TRY(hipMemsetAsync(d_small, 0xff, 8, s));   // err = none

    // 1-2: vertices, then per-edge counts and their scans
    k_vertices<<<blocks_for(nv), kThreads, 0, s>>>(d_xy, d_voff, n, nv, g, d_X, d_Y, d_poly, d_bad, d_small);
    EdgeArgs ea{d_X, d_Y, d_poly, d_voff, d_bad, nv, g, wide};
    k_edges_count<<<blocks_for(nv), kThreads, 0, s>>>(ea, d_cc, d_xc, d_ndist);
    k_check_distinct<<<blocks_for(n), kThreads, 0, s>>>(d_ndist, n, d_small);
    BG_TRY(hipGetLastError());
    size_t tmp_bytes = 0, need = 0;
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need, d_cc, d_coff, nv, s));
    tmp_bytes = std::max(tmp_bytes, need);
    void *d_tmp = sc.get<char>(tmp_bytes);
    if (!d_tmp) return fail(APRIL_E_NOMEM, "build scratch");
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(d_tmp, tmp_bytes, d_cc, d_coff, nv, s));
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(d_tmp, tmp_bytes, d_xc, d_xoff, nv, s));
    uint64_t h[5] = {0, 0, 0, 0, 0};   // err, last coff, last cc, last xoff, last xc
    BG_TRY(hipMemcpyAsync(&h[0], d_small, 8, hipMemcpyDeviceToHost, s));
    BG_TRY(hipMemcpyAsync(&h[1], d_coff + nv - 1, 8, hipMemcpyDeviceToHost, s));
    BG_TRY(hipMemcpyAsync(&h[2], d_cc + nv - 1, 8, hipMemcpyDeviceToHost, s));
    BG_TRY(hipMemcpyAsync(&h[3], d_xoff + nv - 1, 8, hipMemcpyDeviceToHost, s));
    BG_TRY(hipMemcpyAsync(&h[4], d_xc + nv - 1, 8, hipMemcpyDeviceToHost, s));
    BG_TRY(hipStreamSynchronize(s));
    if (h[0] != ~0ull) {
        const uint64_t k = h[0] >> 32, code = h[0] & 0xff;
        return fail(code == kErrGrid ? APRIL_E_GRID : APRIL_E_INVALID,
                    "polygon " + std::to_string(k) +
                        (code == kErrGrid ? " reaches the outer cell ring or leaves the grid"
                                          : " has a non-lattice coordinate or < 3 distinct vertices"));
    }
    const uint64_t ne = h[1] + h[2], nx = h[3] + h[4];
    if (ne == 0) return fail(APRIL_E_INVALID, "no boundary cells");
    if (ne >= (1ull << 32) || nx >= (1ull << 32))
        return fail(APRIL_E_NOMEM, "more than 2^32 boundary-cell entries in one call: split the collection");

    // 3-4: emit, then sort both key sets
    uint64_t *d_ck = sc.get<uint64_t>(ne), *d_ck2 = sc.get<uint64_t>(ne);
    uint64_t *d_xk = sc.get<uint64_t>(nx), *d_xk2 = sc.get<uint64_t>(nx);
    int64_t *d_xv = sc.get<int64_t>(nx), *d_xv2 = sc.get<int64_t>(nx);
    if (sc.err != hipSuccess) return fail(APRIL_E_NOMEM, std::string("build scratch: ") + hipGetErrorString(sc.err));
    k_edges_emit<<<blocks_for(nv), kThreads, 0, s>>>(ea, d_coff, d_cc, d_xoff, d_xc, ne, nx, d_ck, d_xk, d_xv);
    BG_TRY(hipGetLastError());
    int kbits = 1;
    while (kbits < 31 && (1ull << kbits) < n) kbits++;
    need = 0;
    BG_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, need, d_ck, d_ck2, ne, 0, 33 + kbits, s));
    size_t need2 = 0;
    BG_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, need2, d_xk2, d_xk, reinterpret_cast<uint64_t *>(d_xv2),
                                              reinterpret_cast<uint64_t *>(d_xv), nx, 0, 16 + kbits, s));
    size_t need3 = 0;
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, need3, d_ck, d_ck2, ne, s));
    // doubled crossing x < 2 * cells * w
    int xbits = 1;
    while (xbits < 64 && double(uint64_t(1) << xbits) <= 2.0 * double(lg.cells) * double(lg.w)) xbits++;
    size_t need4 = 0;
    BG_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, need4, reinterpret_cast<uint64_t *>(d_xv),
                                              reinterpret_cast<uint64_t *>(d_xv2), d_xk, d_xk2, nx, 0, xbits, s));
    const size_t tmp2 = std::max({need, need2, need3, need4});
    void *d_tmp2 = sc.get<char>(tmp2);
    if (!d_tmp2) return fail(APRIL_E_NOMEM, "build scratch");
    if (ne) BG_TRY(hipcub::DeviceRadixSort::SortKeys(d_tmp2, need, d_ck, d_ck2, ne, 0, 33 + kbits, s));
    // crossings: by x first, then (stable) by (polygon, row), so that x is
    // ascending within a row; x >= 0 (relative coordinates are positive)
    if (nx) {
        uint64_t *xv = reinterpret_cast<uint64_t *>(d_xv), *xv2 = reinterpret_cast<uint64_t *>(d_xv2);
        BG_TRY(hipcub::DeviceRadixSort::SortPairs(d_tmp2, need4, xv, xv2, d_xk, d_xk2, nx, 0, xbits, s));
        BG_TRY(hipcub::DeviceRadixSort::SortPairs(d_tmp2, need2, d_xk2, d_xk, xv2, xv, nx, 0, 16 + kbits, s));
    }

    // 5: one entry per (polygon, cell); d_ck is free again and holds the flags
    uint64_t *keep = d_ck, *pos = sc.get<uint64_t>(ne), *cell = sc.get<uint64_t>(ne);
    uint64_t *first = sc.get<uint64_t>(n + 1);
    uint8_t *cls = sc.get<uint8_t>(ne);
    uint64_t *na = sc.get<uint64_t>(ne), *ai = sc.get<uint64_t>(ne), *nf = sc.get<uint64_t>(ne), *fi = sc.get<uint64_t>(ne);
    if (sc.err != hipSuccess) return fail(APRIL_E_NOMEM, std::string("build scratch: ") + hipGetErrorString(sc.err));
    unsigned long long *d_m = d_small + 1, *d_tot = d_small + 2;
    k_keep<<<blocks_for(ne), kThreads, 0, s>>>(d_ck2, ne, keep);
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(d_tmp2, need3, keep, pos, ne, s));
    k_compact<<<blocks_for(ne), kThreads, 0, s>>>(d_ck2, keep, pos, ne, cell, d_m);
    k_first<<<blocks_for(ne), kThreads, 0, s>>>(cell, d_m, n, first);
    // 6-7: classes, interval ends and their slots
    CellArgs ca{cell, first, d_m, d_xk, d_xv, nx, g};
    k_classify<<<blocks_for(ne), kThreads, 0, s>>>(ca, ne, cls);
    k_count_ends<<<blocks_for(ne), kThreads, 0, s>>>(ca, cls, ne, na, nf);
    BG_TRY(hipGetLastError());
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(d_tmp2, need3, na, ai, ne, s));
    BG_TRY(hipcub::DeviceScan::ExclusiveSum(d_tmp2, need3, nf, fi, ne, s));
    k_totals<<<1, 1, 0, s>>>(na, ai, nf, fi, ne, d_tot);
    BG_TRY(hipGetLastError());
    uint64_t tot[2] = {0, 0};
    BG_TRY(hipMemcpyAsync(tot, d_tot, 16, hipMemcpyDeviceToHost, s));
    BG_TRY(hipStreamSynchronize(s));
    const uint64_t n_a = tot[0], n_f = tot[1];

    // the lists, in the layout april_lists_to_device gives raw lists
    auto *L = new (std::nothrow) april_lists;
    if (!L) return fail(APRIL_E_NOMEM, "out of host memory");
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_off = up(8 * (n + 1)), b_a = up(4 * std::max<uint64_t>(n_a, 1)), b_f = up(4 * std::max<uint64_t>(n_f, 1));
    const size_t total = 2 * b_off + 2 * b_a + 2 * b_f;
    hipError_t e = hipMalloc(&L->d.block, total);
    if (e != hipSuccess) {
        delete L;
        return fail(APRIL_E_NOMEM, std::string("hipMalloc lists: ") + hipGetErrorString(e));
    }
    char *p = static_cast<char *>(L->d.block);
    L->d.off_a = reinterpret_cast<uint64_t *>(p); p += b_off;
    L->d.off_f = reinterpret_cast<uint64_t *>(p); p += b_off;
    L->d.start_a = reinterpret_cast<uint32_t *>(p); p += b_a;
    L->d.end_a = reinterpret_cast<uint32_t *>(p); p += b_a;
    L->d.start_f = reinterpret_cast<uint32_t *>(p); p += b_f;
    L->d.end_f = reinterpret_cast<uint32_t *>(p);
    L->d.bytes = total;
    unsigned int *d_bad_slot = reinterpret_cast<unsigned int *>(d_small + 4);
    e = hipMemsetAsync(d_bad_slot, 0, 4, s);
    if (e == hipSuccess) {
        k_scatter<<<blocks_for(ne), kThreads, 0, s>>>(ca, cls, ne, na, ai, nf, fi, n, d_tot, n_a, n_f, L->d.off_a,
                                                      L->d.off_f, L->d.start_a, L->d.end_a, L->d.start_f,
                                                      L->d.end_f, d_bad_slot);
        e = hipGetLastError();
    }
    unsigned int bad_slot = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad_slot, d_bad_slot, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the scratch is released after this call
    if (e != hipSuccess || bad_slot) {
        (void)hipFree(L->d.block);
        delete L;
        return e != hipSuccess ? fail(APRIL_E_HIP, std::string("build: ") + hipGetErrorString(e))
                               : fail(APRIL_E_CORRUPT, "build: inconsistent interval ends");
    }
    L->grid = *grid;
    L->partition_key = 0;
    L->n = n;
    L->n_a = n_a;
    L->n_f = n_f;
    L->device = dev;
    L->codec = APRIL_CODEC_RAW;
    *out = L;
    return APRIL_OK;
}
