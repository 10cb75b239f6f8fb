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

__device__ __forceinline__ int64_t gl64(const int64_t *p, uint64_t i) {
    return ((const int64_t __attribute__((address_space(1))) *)p)[i];
}

// Any edge of polygon a (global indices [a0, a0 + na)) meeting an edge of
// polygon b ([b0, b0 + nb)) inside the box bx0..by1?  Whole wave.
__device__ bool boundaries_meet(const PolyView &A, uint64_t a0, uint32_t na, const PolyView &B, uint64_t b0,
                                uint32_t nb, int64_t bx0, int64_t by0, int64_t bx1, int64_t by1, uint32_t lane) {
    for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
        // this lane's edge of b, and whether it reaches into the box
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
            // edge a_k a_k2 (uniform) against the lane's edge
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

// Is point (px, py) inside polygon b?  Only asked when no boundary meets the
// other polygon's, so the point is not on b's boundary.  Whole wave.
__device__ bool inside(const PolyView &B, uint64_t b0, uint32_t nb, int64_t px, int64_t py, uint32_t lane) {
    uint32_t crossings = 0;
    for (uint32_t q0 = 0; q0 < nb; q0 += 64) {
        const uint32_t q = q0 + lane;
        bool c = false;
        if (q < nb) {
            const uint32_t q2 = q + 1 == nb ? 0 : q + 1;
            const int64_t ax = gl64(B.x, b0 + q), ay = gl64(B.y, b0 + q);
            const int64_t bx = gl64(B.x, b0 + q2), by = gl64(B.y, b0 + q2);
            if ((ay > py) != (by > py)) {
                // the edge crosses the line y = py; count it when the crossing
                // lies right of the point
                const int o = orient(ax, ay, bx, by, px, py);
                c = by > ay ? o > 0 : o < 0;
            }
        }
        crossings += uint32_t(__popcll(__ballot(c)));
    }
    return crossings & 1u;
}

__device__ uint8_t refine_pair(const RefineArgs &a, uint32_t r, uint32_t s, uint32_t lane) {
    const uint64_t r0 = a.R.off[r], s0 = a.S.off[s];
    const uint32_t nr = uint32_t(a.R.off[r + 1] - r0), ns = uint32_t(a.S.off[s + 1] - s0);
    const int64_t *br = a.R.box + 4 * uint64_t(r), *bs = a.S.box + 4 * uint64_t(s);
    const int64_t bx0 = max(br[0], bs[0]), by0 = max(br[1], bs[1]);
    const int64_t bx1 = min(br[2], bs[2]), by1 = min(br[3], bs[3]);
    if (bx0 > bx1 || by0 > by1) return 0;   // the MBRs do not meet
    // walk the polygon with fewer vertices as the scalar side
    const bool rs = nr <= ns;
    if (rs ? boundaries_meet(a.R, r0, nr, a.S, s0, ns, bx0, by0, bx1, by1, lane)
           : boundaries_meet(a.S, s0, ns, a.R, r0, nr, bx0, by0, bx1, by1, lane))
        return 1;
    if (inside(a.S, s0, ns, a.R.x[r0], a.R.y[r0], lane)) return 1;
    return inside(a.R, r0, nr, a.S.x[s0], a.S.y[s0], lane) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_refine(RefineArgs a) {
    const uint32_t lane = threadIdx.x & 63;
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
                                               uniform(__builtin_amdgcn_readlane(s, k2)), lane);
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
        k_refine<<<dim3(uint32_t(st->cus) * 4), dim3(kBlock), 0, stream>>>(a);
        e = hipGetLastError();
    }
    APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("refine launch: ") + hipGetErrorString(e));
    return APRIL_OK;
}
