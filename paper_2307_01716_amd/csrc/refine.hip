// Exact refinement of candidate pairs (the step after the intermediate
// filter, Sec. 2): do the two polygons share a point?
//
// Polygons are kept on the device as exact lattice coordinates (multiples
// of 2^-30 as int64), so every predicate is an integer sign: orientations
// are 128-bit cross products of 64-bit differences.  Two closed polygons
// share a point iff an edge of one meets an edge of the other, or, with no
// boundary contact at all, one lies inside the other -- then any vertex of
// the inner one is strictly inside the outer one.
//
// Work: pairs are taken 64 at a time from per-XCD ranges (as in the
// filter); a lane reads one pair's ids and verdict; pairs the filter already
// decided are answered from the verdict, the others are tested one after
// another by the whole wave.  Only edges whose box meets the intersection
// of the two MBRs can meet (a common boundary point lies in both MBRs), so
// the others are skipped.  The wave holds 64 edges of S in registers and
// walks R's edges (scalar loads); a ballot ends the pair at the first
// meeting.  The inside test counts, over the outer polygon's edges in
// parallel, the crossings of the horizontal ray from the vertex.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "device.hpp"
#include "internal.hpp"

struct april_polys {
    uint64_t n = 0, nv = 0;
    int device = -1;
    void *mem = nullptr;         // one allocation: off, box, x, y
    const uint64_t *off = nullptr;
    const int64_t *box = nullptr;   // per polygon: xmin, ymin, xmax, ymax
    const int64_t *x = nullptr, *y = nullptr;
};

namespace april {
namespace {

struct PolyView {
    const uint64_t *off;
    const int64_t *box, *x, *y;
    uint64_t n;
};

struct RefineArgs {
    PolyView R, S;
    const uint32_t *r, *s;
    const uint8_t *verdict;
    uint8_t *out;
    unsigned long long *counts;
    unsigned int *xhead;
    uint64_t n_pairs;
    uint32_t xcds;
};

__device__ __forceinline__ int sgn(__int128 v) { return (v > 0) - (v < 0); }

// sign of (b - a) x (c - a)
__device__ __forceinline__ int orient(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy) {
    return sgn(__int128(bx - ax) * (cy - ay) - __int128(by - ay) * (cx - ax));
}

__device__ __forceinline__ bool within(int64_t a, int64_t b, int64_t p) { return min(a, b) <= p && p <= max(a, b); }

// do the closed segments ab and cd share a point?
__device__ __forceinline__ bool segments_meet(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy,
                                              int64_t dx, int64_t dy) {
    const int o1 = orient(ax, ay, bx, by, cx, cy), o2 = orient(ax, ay, bx, by, dx, dy);
    const int o3 = orient(cx, cy, dx, dy, ax, ay), o4 = orient(cx, cy, dx, dy, bx, by);
    if (o1 * o2 < 0 && o3 * o4 < 0) return true;    // proper crossing
    // an endpoint on the other segment (covers touching and collinear overlap)
    return (o1 == 0 && within(ax, bx, cx) && within(ay, by, cy)) ||
           (o2 == 0 && within(ax, bx, dx) && within(ay, by, dy)) ||
           (o3 == 0 && within(cx, dx, ax) && within(cy, dy, ay)) ||
           (o4 == 0 && within(cx, dx, bx) && within(cy, dy, by));
}

// The same predicates on coordinates relative to a pair's origin, when every
// vertex of both polygons lies within 2^31 - 1 lattice units of it on each
// axis: differences fit in 32 bits, cross products in 64.
__device__ __forceinline__ int orient32(int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t cx, int32_t cy) {
    const int64_t v = int64_t(bx - ax) * int64_t(cy - ay) - int64_t(by - ay) * int64_t(cx - ax);
    return (v > 0) - (v < 0);
}

__device__ __forceinline__ bool within32(int32_t a, int32_t b, int32_t p) { return min(a, b) <= p && p <= max(a, b); }

__device__ __forceinline__ bool segments_meet32(int4 u, int4 w) {
    const int o1 = orient32(u.x, u.y, u.z, u.w, w.x, w.y), o2 = orient32(u.x, u.y, u.z, u.w, w.z, w.w);
    const int o3 = orient32(w.x, w.y, w.z, w.w, u.x, u.y), o4 = orient32(w.x, w.y, w.z, w.w, u.z, u.w);
    if (o1 * o2 < 0 && o3 * o4 < 0) return true;
    return (o1 == 0 && within32(u.x, u.z, w.x) && within32(u.y, u.w, w.y)) ||
           (o2 == 0 && within32(u.x, u.z, w.z) && within32(u.y, u.w, w.w)) ||
           (o3 == 0 && within32(w.x, w.z, u.x) && within32(w.y, w.w, u.y)) ||
           (o4 == 0 && within32(w.x, w.z, u.z) && within32(w.y, w.w, u.w));
}

__device__ __forceinline__ bool boxes_meet32(int4 u, int4 w) {
    return max(u.x, u.z) >= min(w.x, w.z) && min(u.x, u.z) <= max(w.x, w.z) && max(u.y, u.w) >= min(w.y, w.w) &&
           min(u.y, u.w) <= max(w.y, w.w);
}

__device__ __forceinline__ int64_t gl64(const int64_t *p, uint64_t i) {
    return ((const int64_t __attribute__((address_space(1))) *)p)[i];
}

// edges of one side staged in LDS per wave (x0, y0, x1, y1 relative to the
// pair's origin)
constexpr uint32_t kEdgeChunk = 128;

struct Pair {
    uint64_t a0, b0;       // first vertex of each polygon
    uint32_t na, nb;       // vertex (= edge) counts
    int64_t ox, oy;        // origin: lower-left corner of the union of the MBRs
    int32_t bx0, by0, bx1, by1;   // intersection of the MBRs, relative
};

// Append to `out` (from 0) the edges of polygon P (vertices [p0, p0 + n))
// whose boxes meet the pair's MBR intersection, starting at edge *pos and
// taking whole blocks of 64 edges while at most kEdgeChunk can result.
// Returns the count; *pos is the first edge not yet scanned.  Whole wave.
__device__ uint32_t gather_edges(const PolyView &P, uint64_t p0, uint32_t n, uint32_t &pos, const Pair &q,
                                 int4 *out, uint32_t lane) {
    uint32_t cnt = 0;
    wave_lds_sync();   // earlier readers of `out` are done
    while (pos < n && cnt + 64 <= kEdgeChunk) {
        const uint32_t e = pos + lane;
        const bool v = e < n;
        const uint32_t e1 = v ? e : 0, e2 = e1 + 1 == n ? 0 : e1 + 1;
        const int4 E = make_int4(int32_t(gl64(P.x, p0 + e1) - q.ox), int32_t(gl64(P.y, p0 + e1) - q.oy),
                                 int32_t(gl64(P.x, p0 + e2) - q.ox), int32_t(gl64(P.y, p0 + e2) - q.oy));
        const bool keep = v && max(E.x, E.z) >= q.bx0 && min(E.x, E.z) <= q.bx1 && max(E.y, E.w) >= q.by0 &&
                          min(E.y, E.w) <= q.by1;
        const uint64_t m = __ballot(keep);
        if (keep) out[cnt + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0))] = E;
        cnt += uint32_t(__popcll(m));
        pos += 64;
    }
    wave_lds_sync();
    return cnt;
}

// Does any of the na edges in ea meet any of the nb edges in eb?  The
// na * nb pairs are dealt out 64 at a time (lane t takes pair t, row-major).
__device__ bool edges_meet(const int4 *ea, uint32_t na, const int4 *eb, uint32_t nb, uint32_t lane) {
    if (na == 0 || nb == 0) return false;
    const uint32_t total = na * nb, q = 64 / nb, rem = 64 % nb;
    uint32_t i = lane / nb, j = lane % nb;
    for (uint32_t t0 = 0; t0 < total; t0 += 64) {
        bool h = false;
        if (t0 + lane < total) {
            const int4 u = ea[i], w = eb[j];
            h = boxes_meet32(u, w) && segments_meet32(u, w);
        }
        if (__any(h)) return true;
        i += q;
        j += rem;
        if (j >= nb) {
            j -= nb;
            i++;
        }
    }
    return false;
}

// Is the point (px, py) (relative) inside polygon P?  Asked only when the
// two boundaries do not meet, so the point is not on P's boundary.  Counts
// the edges crossing the horizontal line through the point to its right
// (an edge crosses when exactly one endpoint lies strictly above).
__device__ bool inside32(const PolyView &P, uint64_t p0, uint32_t n, const Pair &q, int32_t px, int32_t py,
                         uint32_t lane) {
    uint32_t crossings = 0;
    for (uint32_t e0 = 0; e0 < n; e0 += 64) {
        const uint32_t e = e0 + lane;
        bool c = false;
        if (e < n) {
            const uint32_t e2 = e + 1 == n ? 0 : e + 1;
            const int32_t ax = int32_t(gl64(P.x, p0 + e) - q.ox), ay = int32_t(gl64(P.y, p0 + e) - q.oy);
            const int32_t bx = int32_t(gl64(P.x, p0 + e2) - q.ox), by = int32_t(gl64(P.y, p0 + e2) - q.oy);
            if ((ay > py) != (by > py)) {
                const int o = orient32(ax, ay, bx, by, px, py);
                c = by > ay ? o > 0 : o < 0;   // the crossing lies right of the point
            }
        }
        crossings += uint32_t(__popcll(__ballot(c)));
    }
    return crossings & 1u;
}

// Wide pairs (some vertex 2^31 or more lattice units from the origin): the
// same test in 128-bit arithmetic, one edge of A (scalar) against 64 edges
// of B per step.
__device__ bool boundaries_meet_wide(const PolyView &A, uint64_t a0, uint32_t na, const PolyView &B, uint64_t b0,
                                     uint32_t nb, int64_t bx0, int64_t by0, int64_t bx1, int64_t by1,
                                     uint32_t lane) {
    for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
        const uint32_t q = q0 + lane;
        const bool qv = q < nb;
        const uint32_t qq = qv ? q : 0, q2 = qq + 1 == nb ? 0 : qq + 1;
        const int64_t cx = gl64(B.x, b0 + qq), cy = gl64(B.y, b0 + qq);
        const int64_t dx = gl64(B.x, b0 + q2), dy = gl64(B.y, b0 + q2);
        const bool qin = qv && max(cx, dx) >= bx0 && min(cx, dx) <= bx1 && max(cy, dy) >= by0 && min(cy, dy) <= by1;
        if (!__any(qin)) continue;
        int64_t ax = gl64(A.x, a0), ay = gl64(A.y, a0);
        for (uint32_t k = 0; k < na; k++) {
            const uint32_t k2 = k + 1 == na ? 0 : k + 1;
            const int64_t ex = gl64(A.x, a0 + k2), ey = gl64(A.y, a0 + k2);
            if (max(ax, ex) >= bx0 && min(ax, ex) <= bx1 && max(ay, ey) >= by0 && min(ay, ey) <= by1) {
                const bool h = qin && max(ax, ex) >= min(cx, dx) && min(ax, ex) <= max(cx, dx) &&
                               max(ay, ey) >= min(cy, dy) && min(ay, ey) <= max(cy, dy) &&
                               segments_meet(ax, ay, ex, ey, cx, cy, dx, dy);
                if (__any(h)) return true;
            }
            ax = ex;
            ay = ey;
        }
    }
    return false;
}

__device__ bool inside_wide(const PolyView &B, uint64_t b0, uint32_t nb, int64_t px, int64_t py, uint32_t lane) {
    uint32_t crossings = 0;
    for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
        const uint32_t q = q0 + lane;
        bool c = false;
        if (q < nb) {
            const uint32_t q2 = q + 1 == nb ? 0 : q + 1;
            const int64_t ax = gl64(B.x, b0 + q), ay = gl64(B.y, b0 + q);
            const int64_t bx = gl64(B.x, b0 + q2), by = gl64(B.y, b0 + q2);
            if ((ay > py) != (by > py)) {
                const int o = orient(ax, ay, bx, by, px, py);
                c = by > ay ? o > 0 : o < 0;
            }
        }
        crossings += uint32_t(__popcll(__ballot(c)));
    }
    return crossings & 1u;
}

__device__ __forceinline__ bool in_box(const int64_t *b, int64_t x, int64_t y) {
    return b[0] <= x && x <= b[2] && b[1] <= y && y <= b[3];
}

// marks a pair left for the wide pass
constexpr uint8_t kWidePending = 0xFE;

struct PairGeom {
    uint64_t r0, s0;
    uint32_t nr, ns;
    const int64_t *br, *bs;
};

__device__ __forceinline__ PairGeom pair_geom(const RefineArgs &a, uint32_t r, uint32_t s) {
    PairGeom g;
    g.r0 = a.R.off[r];
    g.s0 = a.S.off[s];
    g.nr = uint32_t(a.R.off[r + 1] - g.r0);
    g.ns = uint32_t(a.S.off[s + 1] - g.s0);
    g.br = a.R.box + 4 * uint64_t(r);
    g.bs = a.S.box + 4 * uint64_t(s);
    return g;
}

// 1 / 0, or kWidePending when some vertex lies 2^31 or more lattice units
// from the pair's origin (the 64-bit predicates would not be exact).
__device__ uint8_t refine_pair(const RefineArgs &a, uint32_t r, uint32_t s, int4 *ea, int4 *eb, uint32_t lane) {
    const PairGeom g = pair_geom(a, r, s);
    const int64_t *br = g.br, *bs = g.bs;
    const int64_t bx0 = max(br[0], bs[0]), by0 = max(br[1], bs[1]);
    const int64_t bx1 = min(br[2], bs[2]), by1 = min(br[3], bs[3]);
    if (bx0 > bx1 || by0 > by1) return 0;   // the MBRs do not meet
    const int64_t ux0 = min(br[0], bs[0]), uy0 = min(br[1], bs[1]);
    const int64_t ux1 = max(br[2], bs[2]), uy1 = max(br[3], bs[3]);
    // extents as unsigned differences (exact for any int64 inputs)
    if (uint64_t(ux1) - uint64_t(ux0) >= (1ull << 31) || uint64_t(uy1) - uint64_t(uy0) >= (1ull << 31))
        return kWidePending;
    Pair q;
    q.ox = ux0;
    q.oy = uy0;
    q.bx0 = int32_t(bx0 - ux0);
    q.by0 = int32_t(by0 - uy0);
    q.bx1 = int32_t(bx1 - ux0);
    q.by1 = int32_t(by1 - uy0);
    const uint64_t r0 = g.r0, s0 = g.s0;
    const uint32_t nr = g.nr, ns = g.ns;
    // chunks of R's edges against chunks of S's edges, both culled to the
    // MBR intersection; S's edges are gathered once when they fit one chunk
    uint32_t pr = 0, ps, cs = 0;
    bool s_once = false;
    while (pr < nr) {
        const uint32_t cr = gather_edges(a.R, r0, nr, pr, q, ea, lane);
        if (cr == 0) continue;
        if (s_once) {
            if (edges_meet(ea, cr, eb, cs, lane)) return 1;
            continue;
        }
        ps = 0;
        uint32_t gathers = 0;
        do {
            cs = gather_edges(a.S, s0, ns, ps, q, eb, lane);
            gathers++;
            if (edges_meet(ea, cr, eb, cs, lane)) return 1;
        } while (ps < ns);
        s_once = gathers == 1;   // eb holds all of S's culled edges: keep it
    }
    // no boundary contact: one polygon inside the other, or disjoint
    const int64_t rx0 = a.R.x[r0], ry0 = a.R.y[r0], sx0 = a.S.x[s0], sy0 = a.S.y[s0];
    if (in_box(bs, rx0, ry0) && inside32(a.S, s0, ns, q, int32_t(rx0 - q.ox), int32_t(ry0 - q.oy), lane))
        return 1;
    return in_box(br, sx0, sy0) && inside32(a.R, r0, nr, q, int32_t(sx0 - q.ox), int32_t(sy0 - q.oy), lane) ? 1 : 0;
}

__device__ uint8_t refine_pair_wide(const RefineArgs &a, uint32_t r, uint32_t s, uint32_t lane) {
    const PairGeom g = pair_geom(a, r, s);
    const int64_t *br = g.br, *bs = g.bs;
    const int64_t bx0 = max(br[0], bs[0]), by0 = max(br[1], bs[1]);
    const int64_t bx1 = min(br[2], bs[2]), by1 = min(br[3], bs[3]);
    if (boundaries_meet_wide(a.R, g.r0, g.nr, a.S, g.s0, g.ns, bx0, by0, bx1, by1, lane)) return 1;
    const int64_t rx0 = a.R.x[g.r0], ry0 = a.R.y[g.r0], sx0 = a.S.x[g.s0], sy0 = a.S.y[g.s0];
    if (in_box(bs, rx0, ry0) && inside_wide(a.S, g.s0, g.ns, rx0, ry0, lane)) return 1;
    return in_box(br, sx0, sy0) && inside_wide(a.R, g.r0, g.nr, sx0, sy0, lane) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_refine(RefineArgs a) {
    __shared__ int4 lds[kWavesPerBlock][2][kEdgeChunk];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int4 *ea = lds[wave][0], *eb = lds[wave][1];
    unsigned long long c_hit = 0, c_tested = 0;
    const uint32_t my_xcd = blockIdx.x % a.xcds;
    for (uint32_t k = 0; k < a.xcds; k++) {
        const uint32_t seg = (my_xcd + k) % a.xcds;
        const uint64_t lo = a.n_pairs * seg / a.xcds, hi = a.n_pairs * (seg + 1) / a.xcds;
        for (;;) {
            unsigned int got = 0;
            if (lane == 0) got = atomicAdd(&a.xhead[seg], 64u);
            const uint64_t g0 = lo + uniform(__shfl(got, 0));
            if (g0 >= hi) break;
            const uint64_t p = g0 + lane;
            uint32_t out = APRIL_BAD_PAIR, r = 0, s = 0;
            bool test = false;
            if (p < hi) {
                r = a.r[p];
                s = a.s[p];
                if (r < a.R.n && s < a.S.n) {
                    const uint8_t v = a.verdict ? a.verdict[p] : uint8_t(APRIL_INDECISIVE);
                    if (v == APRIL_TN) out = 0;
                    else if (v == APRIL_TH) out = 1;
                    else test = true;
                }
            }
            uint64_t todo = __ballot(test);
            while (todo) {
                const uint32_t k2 = uint32_t(__builtin_ctzll(todo));
                todo &= todo - 1;
                const uint32_t v = refine_pair(a, uniform(__builtin_amdgcn_readlane(r, k2)),
                                               uniform(__builtin_amdgcn_readlane(s, k2)), ea, eb, lane);
                out = lane == k2 ? v : out;
            }
            if (p < hi) {
                a.out[p] = uint8_t(out);
                c_hit += out == 1;
                c_tested += test;
            }
        }
    }
    if (a.counts) {
        for (int off = 32; off > 0; off >>= 1) {
            c_hit += __shfl_down(c_hit, off);
            c_tested += __shfl_down(c_tested, off);
        }
        if (lane == 0) {
            if (c_hit) atomicAdd(&a.counts[0], c_hit);
            if (c_tested) atomicAdd(&a.counts[1], c_tested);
        }
    }
}

// Second pass: the pairs k_refine left as kWidePending, in 128-bit
// arithmetic.  Every wave scans its share of the outputs 64 at a time.
__global__ __launch_bounds__(kBlock) void k_refine_wide(RefineArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    unsigned long long c_hit = 0;
    for (uint64_t g0 = wave * 64; g0 < a.n_pairs; g0 += waves * 64) {
        const uint64_t p = g0 + lane;
        const bool wide = p < a.n_pairs && a.out[p] == kWidePending;
        uint64_t todo = __ballot(wide);
        if (!todo) continue;
        const uint32_t r = wide ? a.r[p] : 0, s = wide ? a.s[p] : 0;
        uint32_t out = 0;
        while (todo) {
            const uint32_t k2 = uint32_t(__builtin_ctzll(todo));
            todo &= todo - 1;
            const uint32_t v = refine_pair_wide(a, uniform(__builtin_amdgcn_readlane(r, k2)),
                                                uniform(__builtin_amdgcn_readlane(s, k2)), lane);
            out = lane == k2 ? v : out;
        }
        if (wide) {
            a.out[p] = uint8_t(out);
            c_hit += out;
        }
    }
    if (a.counts) {
        for (int off = 32; off > 0; off >>= 1) c_hit += __shfl_down(c_hit, off);
        if (lane == 0 && c_hit) atomicAdd(&a.counts[0], c_hit);
    }
}

__global__ void k_zero_refine(unsigned int *xhead, unsigned long long *counts) {
    if (threadIdx.x < 64) xhead[threadIdx.x] = 0;
    if (counts && threadIdx.x < 2) counts[threadIdx.x] = 0;
}

PolyView view(const april_polys_t *P) { return PolyView{P->off, P->box, P->x, P->y, P->n}; }

}  // namespace
}  // namespace april

using namespace april;

extern "C" int april_polys_to_device(const double *xy, const uint64_t *vtx_off, uint64_t n, uint32_t flags,
                                     void *hip_stream, april_polys_t **out) {
    clear_error();
    if (!xy || !vtx_off || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (n == 0) return fail(APRIL_E_INVALID, "no polygons");
    if (flags & ~APRIL_STRICT) return fail(APRIL_E_INVALID, "unknown flags");
    const bool strict = flags & APRIL_STRICT;
    const uint64_t nv = vtx_off[n];
    for (uint64_t k = 0; k < n; k++)
        if (vtx_off[k + 1] < vtx_off[k] + 3 || vtx_off[k + 1] - vtx_off[k] > (1ull << 31))
            return fail(APRIL_E_INVALID, "polygon with < 3 or > 2^31 vertices");
    // host staging: off[n+1], box[4n], x[nv], y[nv] (one block, one copy)
    const uint64_t words = (n + 1) + 4 * n + 2 * nv;
    std::vector<int64_t> h;
    try {
        h.resize(words);
    } catch (...) {
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    uint64_t *off = reinterpret_cast<uint64_t *>(h.data());
    int64_t *box = h.data() + (n + 1), *x = box + 4 * n, *y = x + nv;
    std::atomic<int> err{0};
    const int T = int(std::min<uint64_t>(host_threads(), n));
    parallel(T, [&](int t) {
        for (uint64_t k = n * uint64_t(t) / uint64_t(T); k < n * uint64_t(t + 1) / uint64_t(T); k++) {
            off[k] = vtx_off[k] - vtx_off[0];
            int64_t b[4] = {INT64_MAX, INT64_MAX, INT64_MIN, INT64_MIN};
            for (uint64_t v = vtx_off[k]; v < vtx_off[k + 1]; v++) {
                int64_t c[2];
                for (int a = 0; a < 2; a++) {
                    const double q = xy[2 * v + a] * 1073741824.0;
                    const double rr = std::nearbyint(q);
                    if (!(std::fabs(rr) < 4.6e18)) { err.store(APRIL_E_INVALID); return; }
                    if (strict && rr != q) { err.store(APRIL_E_INVALID); return; }
                    c[a] = int64_t(rr);
                }
                const uint64_t i = v - vtx_off[0];
                x[i] = c[0];
                y[i] = c[1];
                b[0] = std::min(b[0], c[0]);
                b[1] = std::min(b[1], c[1]);
                b[2] = std::max(b[2], c[0]);
                b[3] = std::max(b[3], c[1]);
            }
            for (int a = 0; a < 4; a++) box[4 * k + a] = b[a];
        }
    });
    if (err.load()) return fail(APRIL_E_INVALID, "non-lattice coordinate (APRIL_STRICT) or coordinate out of range");
    off[n] = nv - vtx_off[0];
    auto *P = new (std::nothrow) april_polys;
    if (!P) return fail(APRIL_E_NOMEM, "out of host memory");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipMalloc(&P->mem, words * sizeof(int64_t)) != hipSuccess) {
        delete P;
        return fail(APRIL_E_NOMEM, "device allocation of the polygons failed");
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(P->mem, h.data(), words * sizeof(int64_t), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {   // the staging buffer dies here
        (void)hipFree(P->mem);
        delete P;
        return fail(APRIL_E_HIP, "copy of the polygons to the device failed");
    }
    int64_t *d = static_cast<int64_t *>(P->mem);
    P->n = n;
    P->nv = nv - vtx_off[0];
    P->device = dev;
    P->off = reinterpret_cast<const uint64_t *>(d);
    P->box = d + (n + 1);
    P->x = P->box + 4 * n;
    P->y = P->x + P->nv;
    *out = P;
    return APRIL_OK;
}

extern "C" void april_polys_free(april_polys_t *P) {
    if (!P) return;
    if (P->mem) (void)hipFree(P->mem);
    delete P;
}

extern "C" int april_refine_pairs(const april_polys_t *R, const april_polys_t *S, const uint32_t *d_r,
                                  const uint32_t *d_s, uint64_t n_pairs, const uint8_t *d_verdict, uint8_t *d_out,
                                  unsigned long long *d_counts, void *hip_stream) {
    clear_error();
    if (!R || !S) return fail(APRIL_E_INVALID, "NULL polygon collection");
    if (n_pairs && (!d_r || !d_s || !d_out)) return fail(APRIL_E_INVALID, "NULL pair or output array");
    if (n_pairs >= (1ull << 32)) return fail(APRIL_E_INVALID, "more than 2^32 - 1 pairs in one call");
    DeviceState *st = nullptr;
    if (int rc = device_state(&st)) return rc;
    int dev = 0;
    APRIL_HIP_TRY(hipGetDevice(&dev));
    if (R->device != dev || S->device != dev) return fail(APRIL_E_INVALID, "polygons live on another device");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    RefineArgs a;
    a.R = view(R);
    a.S = view(S);
    a.r = d_r;
    a.s = d_s;
    a.verdict = d_verdict;
    a.out = d_out;
    a.counts = d_counts;
    a.n_pairs = n_pairs;
    a.xcds = uint32_t(xcd_count(st->cus));
    // per-XCD range counters in a stream-ordered scratch of 256 bytes, so
    // calls on different streams never share them
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, 256, stream);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("refine scratch: ") + hipGetErrorString(e));
    a.xhead = static_cast<unsigned int *>(ws);
    k_zero_refine<<<1, 64, 0, stream>>>(a.xhead, d_counts);
    e = hipGetLastError();
    if (e == hipSuccess && n_pairs) {
        // 7 workgroups per CU: the residency its registers allow
        k_refine<<<dim3(uint32_t(st->cus) * 7), dim3(kBlock), 0, stream>>>(a);
        e = hipGetLastError();
        if (e == hipSuccess) {
            k_refine_wide<<<dim3(uint32_t(st->cus)), dim3(kBlock), 0, stream>>>(a);
            e = hipGetLastError();
        }
    }
    APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("refine launch: ") + hipGetErrorString(e));
    return APRIL_OK;
}
