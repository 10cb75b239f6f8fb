// Exact refinement of candidate pairs (the step after the intermediate
// filter, Sec. 2): do the two polygons share a point?
//
// Polygons are kept on the device as exact lattice coordinates (multiples
// of 2^-30 as int64), so every predicate is an integer sign.  Two closed
// polygons share a point iff an edge of one meets an edge of the other, or,
// with no boundary contact at all, one lies inside the other -- then any
// vertex of the inner one is strictly inside the outer one.
//
// Layout: one 64-byte record per polygon (first vertex index, vertex count,
// MBR, first vertex) and the vertices as interleaved (x, y) int64 pairs.
//
// Work: waves take G pairs at a time from per-XCD ranges (G = 64 for large
// calls, down to 4 when there are few pairs per wave); a lane reads one pair's
// ids, verdict and both polygon records.  Pairs the filter already decided
// are answered from the verdict; the others are tested one after another by
// the whole wave.  Only edges whose box meets the intersection B of the two
// MBRs can meet (a common point lies in both MBRs), so the others are
// dropped; the kept edges of each side are staged in LDS and tested
// all-pairs, 64 edge pairs per step, with coordinates relative to the lower
// left corner of the MBRs' union: when both polygons span less than 2^31
// lattice units, differences fit in 32 bits and cross products in 64.  The
// ray-crossing counts that decide containment are taken in the same pass
// over the edges.  Wider pairs are marked and left to a second kernel that
// works in 128-bit arithmetic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>

#include "device.hpp"
#include "internal.hpp"

struct april_polys {
    uint64_t n = 0, nv = 0;
    int device = -1;
    void *mem = nullptr;            // one allocation: records, then vertices
    const int64_t *rec = nullptr;   // per polygon: vtx0, nv, xmin, ymin, xmax, ymax, x0, y0
    const int64_t *xy = nullptr;    // vertices, (x, y) interleaved
};

namespace april {
namespace {

constexpr int kRecWords = 8;

struct PolyView {
    const int64_t *rec, *xy;
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
    uint32_t grab;   // pairs per grab, 4 .. 64
};

typedef int64_t i64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ i64x2 gl128(const int64_t *p, uint64_t i) {
    return ((const i64x2 __attribute__((address_space(1))) *)p)[i];
}

__device__ __forceinline__ int sgn(__int128 v) { return (v > 0) - (v < 0); }

// sign of (b - a) x (c - a), 128-bit
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

// The same predicates on coordinates relative to a pair's origin, every
// coordinate in [0, 2^31): differences fit in 32 bits, cross products in 64.
__device__ __forceinline__ int orient32(int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t cx, int32_t cy) {
    const int64_t v = int64_t(bx - ax) * int64_t(cy - ay) - int64_t(by - ay) * int64_t(cx - ax);
    return (v > 0) - (v < 0);
}

__device__ __forceinline__ bool within32(int32_t a, int32_t b, int32_t p) { return min(a, b) <= p && p <= max(a, b); }

// edges as (x0, y0, x1, y1)
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

// Does the edge u cross the horizontal line through (px, py) to the right of
// the point?  It crosses the line when exactly one endpoint lies strictly
// above; the crossing is right of the point when the point lies left of the
// upward-directed edge.  Never asked for a point on the edge.
__device__ __forceinline__ bool crosses_right32(int4 u, int32_t px, int32_t py) {
    if ((u.y > py) == (u.w > py)) return false;
    const int o = orient32(u.x, u.y, u.z, u.w, px, py);
    return u.w > u.y ? o > 0 : o < 0;
}

// A pair in relative coordinates (origin: lower-left corner of the MBRs'
// union); B = intersection of the MBRs.
struct Pair {
    uint64_t r0, s0;               // first vertex of each polygon
    uint32_t nr, ns;               // vertex (= edge) counts
    int64_t ox, oy;
    int32_t bx0, by0, bx1, by1;    // B
    int32_t rx, ry, sx, sy;        // first vertex of R and of S
    bool r_in_bs, s_in_br;         // R's first vertex in S's MBR, and S's in R's
};

enum : uint32_t { kDisjoint = 0, kNarrow = 1, kWide = 2 };

// workgroups of k_refine per CU: the residency its registers allow
constexpr int kRefineBlocksPerCU = 5;

// marks a pair left for the wide pass
constexpr uint8_t kWidePending = 0xFE;

__device__ __forceinline__ int4 rel_edge(const int64_t *xy, uint64_t p0, uint32_t e, uint32_t n, int64_t ox,
                                         int64_t oy) {
    const uint32_t e2 = e + 1 == n ? 0 : e + 1;
    const i64x2 a = gl128(xy, p0 + e), b = gl128(xy, p0 + e2);
    return make_int4(int32_t(a.x - ox), int32_t(a.y - oy), int32_t(b.x - ox), int32_t(b.y - oy));
}

__device__ __forceinline__ bool in_b(const Pair &q, int4 E) {
    return max(E.x, E.z) >= q.bx0 && min(E.x, E.z) <= q.bx1 && max(E.y, E.w) >= q.by0 && min(E.y, E.w) <= q.by1;
}

// write the lanes' edges flagged in `keep` to out[base ...] in lane order
__device__ __forceinline__ uint32_t append(int4 *out, uint32_t base, bool keep, int4 E) {
    const uint64_t m = __ballot(keep);
    if (keep) out[base + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0))] = E;
    return uint32_t(__popcll(m));
}

// edges of one side staged in LDS per wave
constexpr uint32_t kEdgeChunk = 128;

// Append to `out` (from 0) the edges of a polygon (vertices [p0, p0 + n))
// that meet B, starting at edge *pos and taking whole blocks of 64 edges
// while at most kEdgeChunk can result; *pos becomes the first edge not
// scanned.  *cross accumulates, over every scanned edge, the crossings of
// the ray from (px, py).  Returns the count.  Whole wave.
__device__ uint32_t gather_edges(const int64_t *xy, uint64_t p0, uint32_t n, uint32_t &pos, const Pair &q,
                                 int32_t px, int32_t py, uint32_t &cross, int4 *out, uint32_t lane) {
    uint32_t cnt = 0;
    wave_lds_sync();   // earlier readers of `out` are done
    while (pos < n && cnt + 64 <= kEdgeChunk) {
        const uint32_t e = pos + lane;
        const bool v = e < n;
        const int4 E = rel_edge(xy, p0, v ? e : 0, n, q.ox, q.oy);
        cross += uint32_t(__popcll(__ballot(v && crosses_right32(E, px, py))));
        cnt += append(out, cnt, v && in_b(q, E), E);
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

// the containment decision once no boundary contact was found: cross_s
// counts the ray from R's first vertex over S's edges, cross_r the ray from
// S's first vertex over R's edges
__device__ __forceinline__ uint8_t contained(const Pair &q, uint32_t cross_s, uint32_t cross_r) {
    return ((q.r_in_bs && (cross_s & 1u)) || (q.s_in_br && (cross_r & 1u))) ? 1 : 0;
}

// Both polygons with at most 64 edges: one load round for both.
__device__ uint8_t refine_small(const RefineArgs &a, const Pair &q, int4 *ea, int4 *eb, uint32_t lane) {
    const bool vr = lane < q.nr, vs = lane < q.ns;
    const int4 Er = rel_edge(a.R.xy, q.r0, vr ? lane : 0, q.nr, q.ox, q.oy);
    const int4 Es = rel_edge(a.S.xy, q.s0, vs ? lane : 0, q.ns, q.ox, q.oy);
    wave_lds_sync();
    const uint32_t cr = append(ea, 0, vr && in_b(q, Er), Er);
    const uint32_t cs = append(eb, 0, vs && in_b(q, Es), Es);
    const uint32_t cross_s = uint32_t(__popcll(__ballot(vs && crosses_right32(Es, q.rx, q.ry))));
    const uint32_t cross_r = uint32_t(__popcll(__ballot(vr && crosses_right32(Er, q.sx, q.sy))));
    wave_lds_sync();
    if (edges_meet(ea, cr, eb, cs, lane)) return 1;
    return contained(q, cross_s, cross_r);
}

__device__ uint8_t refine_chunked(const RefineArgs &a, const Pair &q, int4 *ea, int4 *eb, uint32_t lane) {
    // chunks of R's edges against chunks of S's edges; S is gathered once
    // when its kept edges fit one chunk
    uint32_t pr = 0, cs = 0, cross_r = 0, cross_s = 0;
    bool s_counted = false, s_once = false;
    while (pr < q.nr) {
        const uint32_t cr = gather_edges(a.R.xy, q.r0, q.nr, pr, q, q.sx, q.sy, cross_r, ea, lane);
        if (cr == 0) continue;
        if (s_once) {
            if (edges_meet(ea, cr, eb, cs, lane)) return 1;
            continue;
        }
        uint32_t ps = 0, gathers = 0, cross = 0;
        do {
            cs = gather_edges(a.S.xy, q.s0, q.ns, ps, q, q.rx, q.ry, cross, eb, lane);
            gathers++;
            if (edges_meet(ea, cr, eb, cs, lane)) return 1;
        } while (ps < q.ns);
        if (!s_counted) {
            cross_s = cross;
            s_counted = true;
        }
        s_once = gathers == 1;
    }
    if (!s_counted && q.r_in_bs) {   // no kept edge of R: one pass over S for the ray count
        for (uint32_t e0 = 0; e0 < q.ns; e0 += 64) {
            const uint32_t e = e0 + lane;
            const bool v = e < q.ns;
            const int4 E = rel_edge(a.S.xy, q.s0, v ? e : 0, q.ns, q.ox, q.oy);
            cross_s += uint32_t(__popcll(__ballot(v && crosses_right32(E, q.rx, q.ry))));
        }
    }
    return contained(q, cross_s, cross_r);
}

// --------------------------------------------------------- wide pairs

__device__ __forceinline__ bool in_box(const int64_t *rec, int64_t x, int64_t y) {
    return rec[2] <= x && x <= rec[4] && rec[3] <= y && y <= rec[5];
}

// one edge of A (uniform) against 64 edges of B per step, both culled to B
__device__ bool boundaries_meet_wide(const int64_t *axy, uint64_t a0, uint32_t na, const int64_t *bxy, uint64_t b0,
                                     uint32_t nb, int64_t bx0, int64_t by0, int64_t bx1, int64_t by1,
                                     uint32_t lane) {
    for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
        const uint32_t q = q0 + lane;
        const bool qv = q < nb;
        const uint32_t qq = qv ? q : 0, q2 = qq + 1 == nb ? 0 : qq + 1;
        const i64x2 c = gl128(bxy, b0 + qq), d = gl128(bxy, b0 + q2);
        const bool qin =
            qv && max(c.x, d.x) >= bx0 && min(c.x, d.x) <= bx1 && max(c.y, d.y) >= by0 && min(c.y, d.y) <= by1;
        if (!__any(qin)) continue;
        i64x2 u = gl128(axy, a0);
        for (uint32_t k = 0; k < na; k++) {
            const uint32_t k2 = k + 1 == na ? 0 : k + 1;
            const i64x2 w = gl128(axy, a0 + k2);
            if (max(u.x, w.x) >= bx0 && min(u.x, w.x) <= bx1 && max(u.y, w.y) >= by0 && min(u.y, w.y) <= by1) {
                const bool h = qin && max(u.x, w.x) >= min(c.x, d.x) && min(u.x, w.x) <= max(c.x, d.x) &&
                               max(u.y, w.y) >= min(c.y, d.y) && min(u.y, w.y) <= max(c.y, d.y) &&
                               segments_meet(u.x, u.y, w.x, w.y, c.x, c.y, d.x, d.y);
                if (__any(h)) return true;
            }
            u = w;
        }
    }
    return false;
}

__device__ bool inside_wide(const int64_t *xy, uint64_t p0, uint32_t n, int64_t px, int64_t py, uint32_t lane) {
    uint32_t crossings = 0;
    for (uint32_t q0 = 0; q0 < n; q0 += 64) {
        const uint32_t q = q0 + lane;
        bool c = false;
        if (q < n) {
            const uint32_t q2 = q + 1 == n ? 0 : q + 1;
            const i64x2 u = gl128(xy, p0 + q), w = gl128(xy, p0 + q2);
            if ((u.y > py) != (w.y > py)) {
                const int o = orient(u.x, u.y, w.x, w.y, px, py);
                c = w.y > u.y ? o > 0 : o < 0;
            }
        }
        crossings += uint32_t(__popcll(__ballot(c)));
    }
    return crossings & 1u;
}

__device__ uint8_t refine_pair_wide(const RefineArgs &a, uint32_t r, uint32_t s, uint32_t lane) {
    const int64_t *br = a.R.rec + kRecWords * uint64_t(r), *bs = a.S.rec + kRecWords * uint64_t(s);
    const uint64_t r0 = uint64_t(br[0]), s0 = uint64_t(bs[0]);
    const uint32_t nr = uint32_t(br[1]), ns = uint32_t(bs[1]);
    const int64_t bx0 = max(br[2], bs[2]), by0 = max(br[3], bs[3]);
    const int64_t bx1 = min(br[4], bs[4]), by1 = min(br[5], bs[5]);
    if (boundaries_meet_wide(a.R.xy, r0, nr, a.S.xy, s0, ns, bx0, by0, bx1, by1, lane)) return 1;
    if (in_box(bs, br[6], br[7]) && inside_wide(a.S.xy, s0, ns, br[6], br[7], lane)) return 1;
    return in_box(br, bs[6], bs[7]) && inside_wide(a.R.xy, r0, nr, bs[6], bs[7], lane) ? 1 : 0;
}

// ------------------------------------------------------------- kernels

__device__ __forceinline__ uint32_t rl32(uint32_t v, uint32_t k) { return uniform(__builtin_amdgcn_readlane(v, k)); }
__device__ __forceinline__ int32_t rli(int32_t v, uint32_t k) { return int32_t(rl32(uint32_t(v), k)); }
__device__ __forceinline__ uint64_t rl64(uint64_t v, uint32_t k) {
    return uint64_t(rl32(uint32_t(v), k)) | (uint64_t(rl32(uint32_t(v >> 32), k)) << 32);
}

__global__ __launch_bounds__(kBlock) void k_refine(RefineArgs a) {
    __shared__ int4 lds[kWavesPerBlock][2][kEdgeChunk];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int4 *ea = lds[wave][0], *eb = lds[wave][1];
    unsigned long long c_hit = 0, c_tested = 0;
    const uint32_t my_xcd = blockIdx.x % a.xcds, G = a.grab;
    for (uint32_t k = 0; k < a.xcds; k++) {
        const uint32_t seg = (my_xcd + k) % a.xcds;
        const uint64_t lo = a.n_pairs * seg / a.xcds, hi = a.n_pairs * (seg + 1) / a.xcds;
        if (k > 0 && range_drained(a.xhead, seg, lo, hi, lane)) continue;
        for (;;) {
            unsigned int got = 0;
            if (lane == 0) got = atomicAdd(&a.xhead[seg * kCtrStride], G);
            const uint64_t g0 = lo + uniform(__shfl(got, 0));
            if (g0 >= hi) break;
            const uint64_t p = g0 + lane;
            const bool mine = lane < G && p < hi;
            uint32_t out = APRIL_BAD_PAIR, kind = kDisjoint;
            bool test = false;
            // this lane's pair: ids, verdict, both records
            Pair m = {};
            if (mine) {
                const uint32_t r = a.r[p], s = a.s[p];
                if (r < a.R.n && s < a.S.n) {
                    const uint8_t v = a.verdict ? a.verdict[p] : uint8_t(APRIL_INDECISIVE);
                    if (v == APRIL_TN) out = 0;
                    else if (v == APRIL_TH) out = 1;
                    else test = true;
                }
                if (test) {
                    const int64_t *pr = a.R.rec + kRecWords * uint64_t(r), *ps = a.S.rec + kRecWords * uint64_t(s);
                    const i64x2 r01 = gl128(pr, 0), r23 = gl128(pr, 1), r45 = gl128(pr, 2), r67 = gl128(pr, 3);
                    const i64x2 s01 = gl128(ps, 0), s23 = gl128(ps, 1), s45 = gl128(ps, 2), s67 = gl128(ps, 3);
                    const int64_t bx0 = max(r23.x, s23.x), by0 = max(r23.y, s23.y);
                    const int64_t bx1 = min(r45.x, s45.x), by1 = min(r45.y, s45.y);
                    const int64_t ux0 = min(r23.x, s23.x), uy0 = min(r23.y, s23.y);
                    const int64_t ux1 = max(r45.x, s45.x), uy1 = max(r45.y, s45.y);
                    if (bx0 > bx1 || by0 > by1) {
                        kind = kDisjoint;   // the MBRs do not meet
                    } else if (uint64_t(ux1) - uint64_t(ux0) >= (1ull << 31) ||
                               uint64_t(uy1) - uint64_t(uy0) >= (1ull << 31)) {
                        kind = kWide;       // (unsigned differences: exact for any int64)
                    } else {
                        kind = kNarrow;
                        m.r0 = uint64_t(r01.x);
                        m.nr = uint32_t(r01.y);
                        m.s0 = uint64_t(s01.x);
                        m.ns = uint32_t(s01.y);
                        m.ox = ux0;
                        m.oy = uy0;
                        m.bx0 = int32_t(bx0 - ux0);
                        m.by0 = int32_t(by0 - uy0);
                        m.bx1 = int32_t(bx1 - ux0);
                        m.by1 = int32_t(by1 - uy0);
                        m.rx = int32_t(r67.x - ux0);
                        m.ry = int32_t(r67.y - uy0);
                        m.sx = int32_t(s67.x - ux0);
                        m.sy = int32_t(s67.y - uy0);
                        m.r_in_bs = s23.x <= r67.x && r67.x <= s45.x && s23.y <= r67.y && r67.y <= s45.y;
                        m.s_in_br = r23.x <= s67.x && s67.x <= r45.x && r23.y <= s67.y && s67.y <= r45.y;
                    }
                }
            }
            uint64_t todo = __ballot(test && kind == kNarrow);
            if (test && kind != kNarrow) out = kind == kWide ? kWidePending : 0;
            while (todo) {
                const uint32_t k2 = uint32_t(__builtin_ctzll(todo));
                todo &= todo - 1;
                Pair q;
                q.r0 = rl64(m.r0, k2);
                q.s0 = rl64(m.s0, k2);
                q.nr = rl32(m.nr, k2);
                q.ns = rl32(m.ns, k2);
                q.ox = int64_t(rl64(uint64_t(m.ox), k2));
                q.oy = int64_t(rl64(uint64_t(m.oy), k2));
                q.bx0 = rli(m.bx0, k2);
                q.by0 = rli(m.by0, k2);
                q.bx1 = rli(m.bx1, k2);
                q.by1 = rli(m.by1, k2);
                q.rx = rli(m.rx, k2);
                q.ry = rli(m.ry, k2);
                q.sx = rli(m.sx, k2);
                q.sy = rli(m.sy, k2);
                q.r_in_bs = rl32(m.r_in_bs, k2) != 0;
                q.s_in_br = rl32(m.s_in_br, k2) != 0;
                const uint32_t v = q.nr <= 64 && q.ns <= 64 ? refine_small(a, q, ea, eb, lane)
                                                           : refine_chunked(a, q, ea, eb, lane);
                out = lane == k2 ? v : out;
            }
            if (mine) {
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
        const unsigned long long v[2] = {c_hit, c_tested};
        if (lane == 0) add_totals(a.xhead, blockIdx.x * kWavesPerBlock + wave, v, 2);
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
            const uint32_t v = refine_pair_wide(a, rl32(r, k2), rl32(s, k2), lane);
            out = lane == k2 ? v : out;
        }
        if (wide) {
            a.out[p] = uint8_t(out);
            c_hit += out;
        }
    }
    if (a.counts) {
        for (int off = 32; off > 0; off >>= 1) c_hit += __shfl_down(c_hit, off);
        if (lane == 0) add_totals(a.xhead, uint32_t(wave), &c_hit, 1);
    }
}


PolyView view(const april_polys_t *P) { return PolyView{P->rec, P->xy, P->n}; }

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
    // host staging: records [8n], then vertices [2nv] (one block, one copy)
    const uint64_t words = uint64_t(kRecWords) * n + 2 * (nv - vtx_off[0]);
    std::vector<int64_t> h;
    try {
        h.resize(words);
    } catch (...) {
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    int64_t *rec = h.data(), *vxy = rec + uint64_t(kRecWords) * n;
    std::atomic<int> err{0};
    const int T = int(std::min<uint64_t>(host_threads(), n));
    parallel(T, [&](int t) {
        for (uint64_t k = n * uint64_t(t) / uint64_t(T); k < n * uint64_t(t + 1) / uint64_t(T); k++) {
            int64_t b[4] = {INT64_MAX, INT64_MAX, INT64_MIN, INT64_MIN};
            for (uint64_t v = vtx_off[k]; v < vtx_off[k + 1]; v++) {
                int64_t c[2];
                for (int d = 0; d < 2; d++) {
                    const double q = xy[2 * v + d] * 1073741824.0;
                    const double rr = std::nearbyint(q);
                    if (!(std::fabs(rr) < 4.6e18)) { err.store(APRIL_E_INVALID); return; }
                    if (strict && rr != q) { err.store(APRIL_E_INVALID); return; }
                    c[d] = int64_t(rr);
                }
                const uint64_t i = v - vtx_off[0];
                vxy[2 * i] = c[0];
                vxy[2 * i + 1] = c[1];
                b[0] = std::min(b[0], c[0]);
                b[1] = std::min(b[1], c[1]);
                b[2] = std::max(b[2], c[0]);
                b[3] = std::max(b[3], c[1]);
            }
            int64_t *o = rec + uint64_t(kRecWords) * k;
            const uint64_t first = vtx_off[k] - vtx_off[0];
            o[0] = int64_t(first);
            o[1] = int64_t(vtx_off[k + 1] - vtx_off[k]);
            for (int d = 0; d < 4; d++) o[2 + d] = b[d];
            o[6] = vxy[2 * first];
            o[7] = vxy[2 * first + 1];
        }
    });
    if (err.load()) return fail(APRIL_E_INVALID, "non-lattice coordinate (APRIL_STRICT) or coordinate out of range");
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
    P->rec = d;
    P->xy = d + uint64_t(kRecWords) * n;
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
    // 64 pairs per grab, fewer when that would leave waves idle (about two
    // grabs per wave), but at least 4: each grab costs an atomic
    const uint64_t blocks = uint64_t(st->cus) * kRefineBlocksPerCU, waves = blocks * kWavesPerBlock;
    a.grab = uint32_t(std::min<uint64_t>(64, std::max<uint64_t>(4, n_pairs / (waves * 2))));
    // per-XCD range counters in a stream-ordered scratch, so calls on
    // different streams never share them
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, kCtrBytes, stream);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("refine scratch: ") + hipGetErrorString(e));
    a.xhead = static_cast<unsigned int *>(ws);
    k_zero_ctrs<<<1, 64, 0, stream>>>(a.xhead);
    e = hipGetLastError();
    if (e == hipSuccess && n_pairs) {
        k_refine<<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(a);
        e = hipGetLastError();
        if (e == hipSuccess) {
            k_refine_wide<<<dim3(uint32_t(st->cus)), dim3(kBlock), 0, stream>>>(a);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && d_counts) {
        k_sum_totals<<<1, 64, 0, stream>>>(a.xhead, d_counts, 2);
        e = hipGetLastError();
    }
    APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("refine launch: ") + hipGetErrorString(e));
    return APRIL_OK;
}
