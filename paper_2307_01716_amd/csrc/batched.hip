// Batched schedule of the APRIL filter: a length-binning pass, a persistent
// kernel for the workgroup bin, and a persistent kernel for everything else.
//
// Join kernel used here.  For sorted, disjoint interval lists X and Y,
// IntervalJoin of Alg. 2 returns true iff some X_i overlaps some Y_j.  That
// predicate can be decided from Y's side alone: for Y_j let i*(j) be the
// first i with X_i.end > Y_j.start; then
//     some X_i overlaps Y_j   <=>   i*(j) exists and X_{i*(j)}.start < Y_j.end.
// (<=: the pair is an overlap.  =>: an overlapping X_i has X_i.end >
// Y_j.start, so i*(j) <= i and X_{i*(j)}.start <= X_i.start < Y_j.end.)
// So one object's lists X are kept in LDS and every lane takes an element of
// the other object's list Y, read in coalesced chunks, and binary-searches X
// for i*(j); a ballot gives the join's result after each chunk (early exit).
// Elements of Y that end before X starts or start after X ends cannot
// overlap; long streamed lists are first cut to that window by a 64-ary
// search.
//
// The three joins of Alg. 2 (AA, AF = A(r) x F(s), FA = F(r) x A(s)) are
// symmetric in r and s, so the LDS side can be either object.  With X the
// resident object and Y the streamed one, one pass over Y.A gives AA and,
// since every F interval lies inside an A interval, FA as well: an X.F
// interval that overlaps Y_j lies in an X.A interval that overlaps Y_j, so
// X.F needs to be searched only for the Y.A elements that hit X.A.  A second
// pass over Y.F gives AF.  The verdict is Alg. 2's: no AA overlap -> true
// negative; else an overlap in either of the other two -> true hit; else
// indecisive.
//
// LDS layout and search.  A wave's resident lists are four arrays of TILE
// words (A.end, A.start, F.end, F.start).  Slots from the list's length up
// to TILE hold 0xFFFFFFFF, which is never at or below a
// start value (starts are below 2^32 - 1), so the search for i*(j) is a
// fixed sequence of compare-and-step rounds with no bounds tests, and the
// slot it lands on past the list's end holds a start that overlaps nothing.
//
// Lists longer than a tile.  X is cut into pieces by Hilbert key: piece k
// covers keys [k_k, k_{k+1}) and holds every X.A and X.F element that meets
// that range (at most TILE - 1 of each); the streamed Y elements are those
// that meet it.  An overlap at key p is found in the piece whose range holds
// p, because both elements meet that range; the F-inside-A argument above
// holds per piece for the same reason.
//
// Work distribution.  Pairs of two long objects (the workgroup bin, see
// "binning" below) are queued by a binning pass and joined first, each by
// the four waves of a workgroup.  Every other pair is handled by one wave of
// a second persistent kernel, in input order (pairs close in the input share
// lists, and the library's MBR join emits them grouped by R object).  Each
// XCD drains its own contiguous range of the input (so those lists meet in
// that XCD's L2), then helps the others.  A wave takes `grab` pairs at a time, one lane per
// pair's metadata, and fewer once the range is nearly drained so that waves
// finish together.  The object whose lists fit a tile is resident (R when
// both do, kept while consecutive pairs share it); when neither fits, the
// one with the shorter lists is resident piece by piece.  Pairs whose four
// lists are all very short run Alg. 2 sequentially, one lane per pair.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

// Join modes of the kernel: Alg. 2 on one grid; Alg. 2 across two orders
// (Sec. 5.3); within joins
// (Sec. 4.3.2); polygon-linestring joins (Sec. 4.3.3).
constexpr int kAlg2 = 0, kMixedOrders = 1, kWithinJoin = 2, kLinestrings = 3;

constexpr uint32_t kSideS = 0x80000000u;   // resident-object key: the object is from S
constexpr uint32_t kNone = 0xffffffffu;    // no resident object / no upper key bound

struct BatchArgs {
    FilterArgs f;
    unsigned int *xhead;         // pairs taken from XCD k's range: xhead[k * kCtrStride]
    uint32_t xcds;
    uint32_t thread_max;
    uint32_t search_min;
    uint32_t grab;               // pairs per grab (<= 64)
    uint32_t tail_grab;          // pairs per grab near a range's end
    uint64_t tail_pairs;         // "near the end": fewer pairs than this left
    uint32_t shift_r, shift_s;   // mixed orders: bits dropped from the finer side's A
    // workgroup bin (Alg. 2 only): pairs whose shorter object spans at least
    // wg_min intervals in a list (kNone: no workgroup bin)
    uint32_t wg_min;
    uint32_t qcap;               // queue entries per XCD range
    unsigned int *qfill;         // big pairs binned into XCD k's queue: qfill[k * kCtrStride]
    unsigned int *qhead;         // queue entries taken by workgroups: qhead[k * kCtrStride]
    uint32_t *queue;             // XCD k's queue: queue[k * qcap ...]
    unsigned long long *times;   // APRIL_WAVE_TIMES: call start; first, last end of the wave
                                 // kernel; first, last end of the workgroup kernel (or null)
};

// ---------------------------------------------------------------- binning
//
// Every pair falls in one bin, decided from its four list lengths alone (so
// the binning pass and the persistent kernel agree without a per-pair
// table).  With mr, ms the longer of each object's A and F lengths:
//   lane       both objects' lists have at most thread_max intervals:
//              one lane runs Alg. 2 sequentially;
//   workgroup  neither object fits a wave's tile and the shorter one spans
//              at least wg_min intervals (Alg. 2 mode only): the four waves
//              of a workgroup share one resident tile four times a wave's,
//              cut into pieces by Hilbert key, and split the other object's
//              stream between them;
//   wave       everything else: one wave, the object that fits resident (or
//              pieces of the shorter one).
// The binning pass appends the workgroup bin's pairs to one queue per XCD
// range (the range holding the pair) and marks their verdict bytes; a pair
// that finds its queue full is marked for the wave bin instead.
constexpr uint8_t kQueued = 0xFE;     // verdict byte of a pair in a workgroup queue
constexpr uint8_t kOverflow = 0xFD;   // verdict byte of a workgroup-bin pair left to the wave bin

__device__ __forceinline__ bool wg_bin(uint32_t mr, uint32_t ms, uint32_t tile, uint32_t wg_min) {
    return mr >= tile && ms >= tile && min(mr, ms) >= wg_min;
}

// XCD range of pair p: the k with n * k / xcds <= p < n * (k + 1) / xcds
__device__ __forceinline__ uint32_t range_of(uint64_t p, uint64_t n, uint32_t xcds) {
    uint32_t k = uint32_t((p * xcds) / n);
    if (k > 0 && p < n * k / xcds) k--;
    if (k + 1 < xcds && p >= n * (k + 1) / xcds) k++;
    return k;
}

// The binning pass: a thread per pair (grid-stride), one atomic per run of
// same-range queued lanes in a wave.
__global__ __launch_bounds__(256) void k_bin(BatchArgs b, uint32_t tile) {
    const FilterArgs &a = b.f;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); base < a.n_pairs;
         base += stride) {
        const uint64_t p = base + lane;
        bool big = false;
        if (p < a.n_pairs) {
            const uint32_t r = a.r[p], s = a.s[p];
            if ((r < a.n_r) & (s < a.n_s)) {
                const uint32_t mr = uint32_t(max(a.Ar.off[r + 1] - a.Ar.off[r], a.Fr.off[r + 1] - a.Fr.off[r]));
                const uint32_t ms = uint32_t(max(a.As.off[s + 1] - a.As.off[s], a.Fs.off[s + 1] - a.Fs.off[s]));
                big = wg_bin(mr, ms, tile, b.wg_min);
            }
        }
        const uint32_t k = p < a.n_pairs ? range_of(p, a.n_pairs, b.xcds) : 0u;
        uint64_t todo = __ballot(big);
        while (todo) {
            // lanes of the first pending lane's range
            const uint32_t k0 = uniform(__shfl(k, int(__builtin_ctzll(todo))));
            const uint64_t mine = __ballot(big && k == k0) & todo;
            todo &= ~mine;
            unsigned int got = 0;
            if (lane == uint32_t(__builtin_ctzll(mine)))
                got = atomicAdd(&b.qfill[k0 * kCtrStride], uint32_t(__popcll(mine)));
            got = __shfl(got, int(__builtin_ctzll(mine)));
            if ((mine >> lane) & 1) {
                const uint32_t slot = got + uint32_t(__popcll(mine & ((1ull << lane) - 1)));
                if (slot < b.qcap) {
                    b.queue[uint64_t(k0) * b.qcap + slot] = uint32_t(p);
                    a.verdict[p] = kQueued;
                } else {
                    a.verdict[p] = kOverflow;
                }
            }
        }
    }
}


// ------------------------------------------------------------ join pieces

// v[i] through the global address space (scalar base + 32-bit byte offset)
__device__ __forceinline__ uint32_t gload(const uint32_t *v, uint32_t i) {
    const char __attribute__((address_space(1))) *b = (const char __attribute__((address_space(1))) *)v;
    return *(const uint32_t __attribute__((address_space(1))) *)(b + (i << 2));
}

__device__ __forceinline__ uint64_t gload64(const uint64_t *v, uint64_t i) {
    return ((const uint64_t __attribute__((address_space(1))) *)v)[i];
}

__device__ __forceinline__ uint32_t gload32(const uint32_t *v, uint64_t i) {
    return ((const uint32_t __attribute__((address_space(1))) *)v)[i];
}

// first j in [0, m) with v[j] > key (m if none), v sorted: wave-cooperative
// 64-ary search, one global round trip per factor of 64
__device__ uint32_t wave_first_above(const uint32_t *__restrict__ v, uint32_t m, uint32_t key, uint32_t lane) {
    uint32_t lo = 0, hi = m;
    while (hi - lo > 64) {
        const uint64_t step = (uint64_t(hi - lo) + 63) >> 6;
        const uint64_t probe = lo + (lane + 1) * step - 1;
        const bool pred = probe >= hi ? true : (gload(v, uint32_t(probe)) > key);
        const uint64_t mask = __ballot(pred);
        if (!mask) { lo = hi; break; }
        const uint64_t f = __builtin_ctzll(mask);
        const uint64_t pf = lo + (f + 1) * step - 1;
        const uint32_t nlo = uint32_t(lo + f * step);
        hi = uniform(pf < hi ? uint32_t(pf) : hi);
        lo = uniform(nlo);
    }
    if (hi - lo == 0) return lo;
    const uint32_t j = lo + lane;
    const bool pred = j >= hi ? true : (gload(v, j) > key);
    const uint64_t mask = __ballot(pred);
    return mask ? lo + uint32_t(__builtin_ctzll(mask)) : hi;
}

// Resident lists of one wave: SoA in LDS, padded with sentinels to TILE
// entries.
struct Resident {
    uint32_t *as, *ae, *fs, *fe;
    uint32_t na, nf;
};

// Search of a resident end array E (sorted, padded with 0xFFFFFFFF to TILE
// entries): the address of the first entry above key, in log2(TILE) fixed
// rounds with no bounds tests and no per-round branch.  The matching start
// lies TILE entries further on (the arrays are laid out end, start).
template <int TILE>
__device__ __forceinline__ const uint32_t *lds_first_above(const uint32_t *E, uint32_t key) {
    const uint32_t *p = E;   // stepping the address keeps each round to one add
#pragma unroll
    for (uint32_t S = TILE / 2; S > 0; S >>= 1) p = p[S - 1] <= key ? p + S : p;
    return p;
}

// the same search in two arrays at once (independent LDS reads overlap)
template <int TILE>
__device__ __forceinline__ void lds_first_above2(const uint32_t *E1, const uint32_t *E2, uint32_t key,
                                                 const uint32_t *&p1, const uint32_t *&p2) {
    const uint32_t *p = E1, *q = E2;
#pragma unroll
    for (uint32_t S = TILE / 2; S > 0; S >>= 1) {
        const uint32_t u = p[S - 1], v = q[S - 1];
        p = u <= key ? p + S : p;
        q = v <= key ? q + S : q;
    }
    p1 = p;
    p2 = q;
}

// Copy X's A and F lists (na, nf < TILE intervals) into the resident arrays
// and pad all TILE slots.  The copy goes from global memory straight into
// LDS (no registers); every load is issued before the one wait, so the copy
// costs one memory round trip.
__device__ __forceinline__ void dma_dword(const uint32_t *src, uint32_t *lds_chunk) {
    // lane l's word lands at lds_chunk[l]
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_chunk, 4, 0, 0);
}

template <int TILE>
__device__ __forceinline__ void load_resident(const Resident &x, const uint32_t *__restrict__ as,
                                              const uint32_t *__restrict__ ae, uint32_t na,
                                              const uint32_t *__restrict__ fs, const uint32_t *__restrict__ fe,
                                              uint32_t nf, uint32_t lane) {
#pragma unroll 1
    for (int i = 0; i < TILE / 64; i++) {
        const uint32_t t = i * 64 + lane;
        if (t < na) {
            dma_dword(as + t, x.as + i * 64);
            dma_dword(ae + t, x.ae + i * 64);
        } else {
            x.as[t] = 0xffffffffu;
            x.ae[t] = 0xffffffffu;
        }
        if (t < nf) {
            dma_dword(fs + t, x.fs + i * 64);
            dma_dword(fe + t, x.fe + i * 64);
        } else {
            x.fs[t] = 0xffffffffu;
            x.fe[t] = 0xffffffffu;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // the copies have landed in LDS
}

// Stream Y[j..m) (sorted, disjoint) against the resident A-list until an
// element starts at or after `stop`; true iff some element overlaps it.  With
// FA, each element that overlaps the A-list is also tested against the
// resident F-list, and an overlap there sets *th and ends the scan.
//
// MAP says how a streamed element is read: kAsIs; or kShifted, the finer
// side's A-interval mapped to the resident (coarser) grid as [s >> sh,
// ((e - 1) >> sh) + 1), mapped elements staying sorted by start and by end
// (they may touch or overlap each other), which is all the scan needs.
constexpr int kAsIs = 0, kShifted = 1;

// After this many chunks a stream skips the chunks that cannot meet the
// resident list (512-interval instances; see stream_piece).
constexpr uint32_t kSkipChunks = 4;

// The chunks of Y from jj (64 * C elements) against the resident list:
// 0 = go on, 1 = the scan's answer is true, 2 = the chunk starts at or
// after the piece's end (and so do all later ones).
template <int TILE, int C, bool FA, int MAP>
__device__ __forceinline__ uint32_t stream_chunk(const Resident &x, const uint32_t *__restrict__ ys,
                                                 const uint32_t *__restrict__ ye, uint32_t jj, uint32_t m,
                                                 uint32_t stop, uint32_t lane, bool *th, uint32_t sh, bool &any) {
    uint32_t s[C], e[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        // lanes past the end load nothing and take an empty [0, 0)
        const uint32_t k = jj + c * 64 + lane;
        s[c] = k < m ? gload(ys, k) : 0u;
        e[c] = k < m ? gload(ye, k) : 0u;
        if (MAP == kShifted) {
            s[c] >>= sh;
            e[c] = k < m ? ((e[c] - 1) >> sh) + 1 : 0u;
        }
    }
    // this chunk and all later ones start at or after the piece's end
    if (uniform(s[0]) >= stop) return 2;
    bool hit = false, f = false;
#pragma unroll
    for (int c = 0; c < C; c++) {
        if (FA) {
            // the F search runs beside the A search; its answer counts
            // only where the element overlaps the A-list
            const uint32_t *pa, *pf;
            lds_first_above2<TILE>(x.ae, x.fe, s[c], pa, pf);
            const uint32_t sa = pa[TILE], sf = pf[TILE];
            const bool h = sa < e[c];
            hit |= h;
            f |= h & (sf < e[c]);
        } else {
            hit |= lds_first_above<TILE>(x.ae, s[c])[TILE] < e[c];
        }
    }
    if (__any(hit)) {
        if (!FA) return 1;
        any = true;
        if (__any(f)) {
            *th = true;
            return 1;
        }
    }
    return 0;
}

template <int TILE, int C, bool FA, int MAP>
__device__ __forceinline__ bool stream_piece(const Resident &x, const uint32_t *__restrict__ ys,
                                             const uint32_t *__restrict__ ye, uint32_t j, uint32_t m,
                                             uint32_t stop, uint32_t lane, bool *th, uint32_t sh) {
    bool any = false;
    if constexpr (TILE < 512 || MAP != kAsIs) {
        for (; j < m; j += 64 * C) {
            uint32_t s[C], e[C];
#pragma unroll
            for (int c = 0; c < C; c++) {
                // lanes past the end load nothing and take an empty [0, 0)
                const uint32_t k = j + c * 64 + lane;
                s[c] = k < m ? gload(ys, k) : 0u;
                e[c] = k < m ? gload(ye, k) : 0u;
                if (MAP == kShifted) {
                    s[c] >>= sh;
                    e[c] = k < m ? ((e[c] - 1) >> sh) + 1 : 0u;
                }
            }
            // this chunk and all later ones start at or after the piece's end
            if (uniform(s[0]) >= stop) break;
            bool hit = false, f = false;
#pragma unroll
            for (int c = 0; c < C; c++) {
                if (FA) {
                    // the F search runs beside the A search; its answer counts
                    // only where the element overlaps the A-list
                    const uint32_t *pa, *pf;
                    lds_first_above2<TILE>(x.ae, x.fe, s[c], pa, pf);
                    const uint32_t sa = pa[TILE], sf = pf[TILE];
                    const bool h = sa < e[c];
                    hit |= h;
                    f |= h & (sf < e[c]);
                } else {
                    hit |= lds_first_above<TILE>(x.ae, s[c])[TILE] < e[c];
                }
            }
            if (__any(hit)) {
                if (!FA) return true;
                any = true;
                if (__any(f)) {
                    *th = true;
                    return true;
                }
            }
        }
        return any;
    } else {
        constexpr uint32_t CH = 64 * C;
        for (uint32_t n = 0; j < m && n < kSkipChunks; j += CH, n++) {
            const uint32_t r = stream_chunk<TILE, C, FA, MAP>(x, ys, ye, j, m, stop, lane, th, sh, any);
            if (r == 1) return true;
            if (r == 2) return any;
        }
        // The rest of a long stream is taken 64 chunks at a time: lane l
        // tests chunk l, whose elements lie in [its first start, the next
        // chunk's first start) (Y is sorted and disjoint); only a resident
        // interval meeting that range can meet one of them (with FA, an F
        // overlap needs an A overlap: F lies inside A), so only the chunks
        // that pass are read.
        for (uint32_t q0 = j; q0 < m; q0 += 64 * CH) {
            const uint32_t cj = q0 + lane * CH;
            const bool in = cj < m;
            const uint32_t cs = in ? gload(ys, cj) : 0xffffffffu;
            const uint32_t cn = cj + CH < m ? gload(ys, cj + CH) : 0xffffffffu;
            const bool need = in && cs < stop && lds_first_above<TILE>(x.ae, cs)[TILE] < cn;
            uint64_t mask = __ballot(need);
            const bool past = __any(in && cs >= stop);   // from that chunk on, past the piece's end
            while (mask) {
                const uint32_t jj = q0 + uint32_t(__builtin_ctzll(mask)) * CH;
                mask &= mask - 1;
                if (stream_chunk<TILE, C, FA, MAP>(x, ys, ye, jj, m, stop, lane, th, sh, any) == 1) return true;
            }
            if (past) break;
        }
        return any;
    }
}

// Does every element of Y[j..m) that starts below `stop` lie inside one
// resident F interval?  The first F interval ending after the element's
// start is the only candidate (F is sorted and disjoint); a ballot of misses
// ends the scan.
template <int TILE, int C>
__device__ __forceinline__ bool stream_inside(const Resident &x, const uint32_t *__restrict__ ys,
                                              const uint32_t *__restrict__ ye, uint32_t j, uint32_t m,
                                              uint32_t stop, uint32_t lane) {
    for (; j < m; j += 64 * C) {
        uint32_t s[C], e[C];
#pragma unroll
        for (int c = 0; c < C; c++) {
            const uint32_t k = j + c * 64 + lane;
            s[c] = k < m ? gload(ys, k) : stop;   // lanes past the end take no part
            e[c] = k < m ? gload(ye, k) : 0u;
        }
        if (uniform(s[0]) >= stop) break;
        bool miss = false;
#pragma unroll
        for (int c = 0; c < C; c++) {
            if (s[c] < stop) {
                const uint32_t *p = lds_first_above<TILE>(x.fe, s[c]);
                miss |= !(p[TILE] <= s[c] && e[c] <= p[0]);
            }
        }
        if (__any(miss)) return false;
    }
    return true;
}

// One pair's lists as the wave sees them: X resident, Y streamed.
struct PairLists {
    const uint32_t *xas, *xae, *xfs, *xfe;
    const uint32_t *yas, *yae, *yfs, *yfe;
    uint32_t nxa, nxf, nya, nyf;
};

// Probe join, for a resident object X of few intervals spread over a wide
// key range (its Hilbert key range crosses a large part of the curve) and a
// long Y: streaming Y's elements in X's key window would read mostly
// elements that fall in X's gaps.  Instead every lane takes one of X's
// intervals from LDS and binary-searches Y in global memory with the same
// formulation as the streamed join, roles swapped: X_t overlaps some Y_j iff
// Y_{j*}.start < X_t.end, with j* the first j with Y_j.end > X_t.start.
// Alg. 2's joins in its order: X.A in Y.A (AA); then X.A in Y.F and X.F in
// Y.A (AF, FA).  Y.A is searched in its window [ja, jb) (elements ending
// above X's first start and starting below X's last end: every overlap lies
// there), Y.F whole.  Returns 0 = no AA overlap, 1 = a true hit, 2 = AA
// overlaps only.
__device__ __forceinline__ bool probe_any(const uint32_t *xs, const uint32_t *xe, uint32_t nx,
                                          const uint32_t *__restrict__ ys, const uint32_t *__restrict__ ye,
                                          uint32_t lo0, uint32_t hi0, uint32_t lane) {
    for (uint32_t t0 = 0; t0 < nx; t0 += 64) {
        const uint32_t t = t0 + lane;
        const uint32_t key = t < nx ? xs[t] : 0u, end = t < nx ? xe[t] : 0u;
        uint32_t lo = lo0, hi = t < nx ? hi0 : lo0;
        while (__any(lo < hi)) {
            const uint32_t m = (lo + hi) >> 1;
            if (lo < hi) {
                if (gload(ye, m) > key) hi = m;
                else lo = m + 1;
            }
        }
        if (__any(t < nx && lo < hi0 && gload(ys, lo) < end)) return true;
    }
    return false;
}

__device__ __forceinline__ uint32_t probe_join(const Resident &x, const PairLists &L, uint32_t ja, uint32_t jb,
                                               uint32_t lane) {
    if (!probe_any(x.as, x.ae, x.na, L.yas, L.yae, ja, jb, lane)) return 0;
    if (probe_any(x.as, x.ae, x.na, L.yfs, L.yfe, 0, L.nyf, lane)) return 1;
    return probe_any(x.fs, x.fe, x.nf, L.yas, L.yae, ja, jb, lane) ? 1u : 2u;
}

// A single resident piece takes the probe join when its window in Y.A holds
// more than this many elements per 64 resident intervals (a streamed chunk
// of 128 elements costs about one memory round trip, a probe round about
// eighteen dependent ones).
constexpr uint32_t kProbeWindowPerRound = 2048;

// Joins of one resident piece (key range [k0, k1)) with the streamed lists:
// 0 = no AA overlap, 1 = a true hit (FA or AF overlap), 2 = AA overlap only.
// Every value here is wave-uniform; uniform() says so to the compiler.
//
// kMixedOrders: Y is the finer side's A-list mapped to X's grid (shift sh),
// and only the coarse side's F decides a true hit (Sec. 5.3): no AF pass.
// kLinestrings: X is the polygon, Y the linestring's cells as runs of
// consecutive ids; the first pass decides (a cell inside F(p): a true hit).
// kWithinJoin: X is s, Y is A(r); bit 0 of the result is an AA overlap in
// this piece, bit 1 that every element of A(r) meeting [k0, k1) lies inside
// one F(s) interval; `want` says which of the two to find (a piece answers
// 0 for a test it skips).
template <int TILE, int C, int MODE>
__device__ __forceinline__ uint32_t join_piece(const Resident &res, const PairLists &L, uint32_t k0, uint32_t k1,
                                               uint32_t search_min, uint32_t lane, uint32_t sh, uint32_t want) {
    constexpr int MAP = MODE == kMixedOrders ? kShifted : kAsIs;
    // Y elements that can meet this piece: end above x_lo, start below x_hi
    const uint32_t x_lo = max(k0, uniform(res.as[0]));
    const uint32_t x_hi = min(k1, uniform(res.ae[res.na - 1]));
    const bool narrow = k0 > 0;
    bool th = false;
    // a mapped end ((e - 1) >> sh) + 1 is above x_lo iff e is above x_lo << sh
    const uint32_t ja =
        (narrow || L.nya > search_min) ? uniform(wave_first_above(L.yae, L.nya, MAP == kShifted ? x_lo << sh : x_lo, lane)) : 0;
    // (the 512-interval instance only: it has the registers to spare, and
    // long objects, which a wide window needs, make the library pick it)
    if (MODE == kAlg2 && TILE >= 512 && !narrow && k1 == kNone) {
        const uint32_t rounds = (max(res.na, res.nf) + 63) / 64;
        if (L.nya - ja > kProbeWindowPerRound * rounds) {
            const uint32_t jb = ja + uniform(wave_first_above(L.yas + ja, L.nya - ja, x_hi - 1, lane));
            if (jb - ja > kProbeWindowPerRound * rounds) return probe_join(res, L, ja, jb, lane);
        }
    }
    if (MODE == kWithinJoin) {
        const bool aa = (want & 1) && stream_piece<TILE, C, false, kAsIs>(res, L.yas, L.yae, ja, L.nya, x_hi, lane,
                                                                          &th, 0);
        if ((want & 1) && !aa && !narrow && k1 == kNone) return 0;   // one piece and no overlap
        bool in = false;
        if (want & 2) {
            // every element meeting [k0, k1), not only the resident window:
            // one outside X's intervals is not inside F(s)
            const uint32_t jc = (narrow || L.nya > search_min) ? uniform(wave_first_above(L.yae, L.nya, k0, lane)) : 0;
            in = stream_inside<TILE, C>(res, L.yas, L.yae, jc, L.nya, k1, lane);
        }
        return (aa ? 1u : 0u) | (in ? 2u : 0u);
    }
    if (!stream_piece<TILE, C, true, MAP>(res, L.yas, L.yae, ja, L.nya, x_hi, lane, &th, sh)) return 0;
    if (th) return 1;
    if (MODE == kMixedOrders || MODE == kLinestrings) return 2;
    const uint32_t jf = (narrow || L.nyf > search_min) ? uniform(wave_first_above(L.yfe, L.nyf, x_lo, lane)) : 0;
    return stream_piece<TILE, C, false, kAsIs>(res, L.yfs, L.yfe, jf, L.nyf, x_hi, lane, &th, 0) ? 1 : 2;
}

// Alg. 2's verdict for one pair, by the whole wave.  When both of X's lists
// are shorter than TILE they are one piece, kept resident for the next pair
// with the same `key`; otherwise X is loaded piece by piece.
template <int TILE, int C, int MODE>
__device__ uint32_t wave_pair(Resident &res, uint32_t &cached, uint32_t key, const PairLists &L,
                              uint32_t search_min, uint32_t lane, uint32_t sh, uint32_t &pcached, uint32_t *pw) {
    if (L.nxa == 0 || L.nya == 0) return APRIL_TN;
    if (L.nxa < TILE && L.nxf < TILE) {
        if (key != cached) {
            wave_lds_sync();
            load_resident<TILE>(res, L.xas, L.xae, L.nxa, L.xfs, L.xfe, L.nxf, lane);
            wave_lds_sync();
            res.na = L.nxa;
            res.nf = L.nxf;
            cached = key;
            pcached = kNone;
        }
        const uint32_t j = join_piece<TILE, C, MODE>(res, L, 0, kNone, search_min, lane, sh, 3);
        if (MODE == kWithinJoin) return !(j & 1) ? APRIL_TN : (j & 2) ? APRIL_TH : APRIL_INDECISIVE;
        return j == 0 ? APRIL_TN : j == 1 ? APRIL_TH : APRIL_INDECISIVE;
    }
    cached = kNone;
    bool aa = false, in = true;   // (within joins: every piece so far has A(r) inside F(s))
    uint32_t a0 = 0, f0 = 0, k0 = 0;
    // 512-interval Alg. 2 instance: the piece the previous pair left resident,
    // when it belongs to this object, is joined first (any order of pieces
    // finds an overlap, and consecutive pairs sharing an object tend to meet
    // it in the same place), then skipped in the walk below; its bounds are
    // in the wave's words pw (a0, a1, f0, f1, k0, k1)
    constexpr bool kHold = TILE >= 512 && MODE == kAlg2;
    uint32_t held_a0 = kNone;
    if constexpr (kHold) {
        if (pcached == key) {
            const uint32_t j = join_piece<TILE, C, MODE>(res, L, uniform(pw[4]), uniform(pw[5]), search_min, lane, sh, 3);
            if (j == 1) return APRIL_TH;
            aa |= j == 2;
            held_a0 = uniform(pw[0]);
        }
    }
    for (;;) {
        // at most TILE - 1 A elements from a0; the range ends where the next
        // one starts; then at most TILE - 1 F elements
        uint32_t a1 = L.nxa, f1 = L.nxf, k1 = kNone;
        if (L.nxa - a0 > TILE - 1) {
            a1 = a0 + TILE - 1;
            k1 = uniform(gload(L.xas, a1));
            f1 = f0 + uniform(wave_first_above(L.xfs + f0, L.nxf - f0, k1 - 1, lane));
        }
        if (f1 - f0 > TILE - 1) {
            f1 = f0 + TILE - 1;
            k1 = uniform(gload(L.xfs, f1));
            a1 = a0 + uniform(wave_first_above(L.xas + a0, a1 - a0, k1 - 1, lane));
        }
        if (kHold && a0 == held_a0) {
            // the held piece, joined above
        } else {
        wave_lds_sync();
        load_resident<TILE>(res, L.xas + a0, L.xae + a0, a1 - a0, L.xfs + f0, L.xfe + f0, f1 - f0, lane);
        wave_lds_sync();
        res.na = a1 - a0;
        res.nf = f1 - f0;
        if constexpr (kHold) {
            // this piece is resident now
            if (lane == 0) {
                pw[0] = a0;
                pw[1] = a1;
                pw[2] = f0;
                pw[3] = f1;
                pw[4] = k0;
                pw[5] = k1;
            }
            pcached = key;
        }
        if (MODE == kWithinJoin) {
            const uint32_t j =
                join_piece<TILE, C, MODE>(res, L, k0, k1, search_min, lane, sh, (aa ? 0u : 1u) | (in ? 2u : 0u));
            aa |= (j & 1) != 0;
            in = in && (j & 2);
            if (aa && !in) return APRIL_INDECISIVE;
        } else {
            const uint32_t j = join_piece<TILE, C, MODE>(res, L, k0, k1, search_min, lane, sh, 3);
            if (j == 1) return APRIL_TH;
            aa |= j == 2;
        }
        }
        if (k1 == kNone) break;
        // next piece: the first elements that end above k1
        k0 = k1;
        a0 = uniform(gload(L.xae, a1 - 1)) > k1 ? a1 - 1 : a1;
        f0 = (f1 > 0 && uniform(gload(L.xfe, f1 - 1)) > k1) ? f1 - 1 : f1;
    }
    if (MODE == kWithinJoin) return !aa ? APRIL_TN : in ? APRIL_TH : APRIL_INDECISIVE;
    return aa ? APRIL_INDECISIVE : APRIL_TN;
}

// --------------------------------------------------- workgroup schedule
//
// A pair of two long objects (the workgroup bin) is joined by the four
// waves of a workgroup together.  Their LDS holds one resident tile of
// TW = 4 * TILE intervals per list (A.end, A.start, F.end, F.start, padded
// with 0xFFFFFFFF as for a wave), so the shorter object X is cut into a
// quarter as many pieces, and the waves split the streamed object Y: wave w
// takes chunks w, w + 4, w + 8, ... of 64 * C elements.  An overlap raises
// a flag in LDS; a true hit ends every wave's stream at its next chunk.
//
// Pieces are visited in key order, so the streamed lists are merged rather
// than searched: piece k + 1 starts its stream where piece k's stopped.  A
// wave stops at its first chunk that starts at or after the piece's end
// (x_hi); with c* the smallest such chunk over the four waves, every chunk
// before c* was streamed and started below x_hi, so every element before
// chunk c* - 1 ends at or below x_hi, which is at most the next piece's
// first key: the next piece restarts at chunk c* - 1.  (An element streamed
// again, or one outside the piece's range, can only show a real overlap:
// the LDS search compares it with real intervals of X.)

struct WgShared {
    uint32_t grab;      // queue entry taken by the workgroup
    uint32_t bits;      // this pass: 1 = overlap with X.A, 2 = true hit
    uint32_t cstop;     // this pass: smallest stop chunk over the waves
    uint32_t pad;
};

constexpr uint32_t kHitAA = 1, kHitTH = 2;

// One chunk of a workgroup pass (see wg_stream), from Y[j]: true when the
// wave's pass ends there (the end of Y, a chunk starting at or after
// `stop`, or a true hit, its own or another wave's).
template <int TW, int C, bool FA>
__device__ __forceinline__ bool wg_chunk(const Resident &x, const uint32_t *__restrict__ ys,
                                         const uint32_t *__restrict__ ye, uint32_t j, uint32_t m, uint32_t stop,
                                         uint32_t lane, WgShared *sh) {
    if (j >= m) return true;
    if (uniform(__hip_atomic_load(&sh->bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) & kHitTH) return true;
    uint32_t s[C], e[C];
#pragma unroll
    for (int q = 0; q < C; q++) {
        const uint32_t k = j + q * 64 + lane;
        s[q] = k < m ? gload(ys, k) : 0u;
        e[q] = k < m ? gload(ye, k) : 0u;
    }
    if (uniform(s[0]) >= stop) return true;
    bool hit = false, f = false;
#pragma unroll
    for (int q = 0; q < C; q++) {
        if (FA) {
            const uint32_t *pa, *pf;
            lds_first_above2<TW>(x.ae, x.fe, s[q], pa, pf);
            const bool h = pa[TW] < e[q];
            hit |= h;
            f |= h & (pf[TW] < e[q]);
        } else {
            hit |= lds_first_above<TW>(x.ae, s[q])[TW] < e[q];
        }
    }
    const bool any_hit = __any(hit);
    const bool th = FA ? (any_hit && __any(f)) : any_hit;
    if (any_hit && lane == 0)
        __hip_atomic_fetch_or(&sh->bits, th ? (kHitAA | kHitTH) : kHitAA, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_WORKGROUP);
    return th;
}

// One pass of the workgroup over Y[j0, m) against the resident tile, up to
// the first chunk starting at or after `stop`.  FA: the pass over Y.A (an
// A-list overlap sets kHitAA; one that also meets X.F sets kHitTH); else
// the pass over Y.F (an overlap with X.A sets kHitTH).  Wave w takes chunks
// w, w + 4, ...: its first kSkipChunks one by one, then 64 of them at a
// time, lane l testing the wave's l-th next chunk (its elements lie between
// its first start and the next chunk's), and reading only the chunks a
// resident interval can meet.  The chunk at which the wave stops (its first
// chunk past Y's end or starting at or after `stop`, whether read or only
// tested) goes to cstop either way.
template <int TW, int C, bool FA>
__device__ __forceinline__ void wg_stream(const Resident &x, const uint32_t *__restrict__ ys,
                                          const uint32_t *__restrict__ ye, uint32_t j0, uint32_t m,
                                          uint32_t stop, uint32_t w, uint32_t lane, WgShared *sh) {
    constexpr uint32_t CH = 64 * C;
    uint32_t c = w;
    bool done = false;
    for (uint32_t n = 0; n < kSkipChunks && !done; n++) {
        done = wg_chunk<TW, C, FA>(x, ys, ye, j0 + c * CH, m, stop, lane, sh);
        if (!done) c += kWavesPerBlock;
    }
    while (!done) {
        if (uniform(__hip_atomic_load(&sh->bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) & kHitTH) break;
        const uint32_t cj = j0 + (c + lane * kWavesPerBlock) * CH;   // this lane's chunk
        const bool in = cj < m;
        const uint32_t cs = in ? gload(ys, cj) : 0xffffffffu;
        const uint32_t cn = cj + CH < m ? gload(ys, cj + CH) : 0xffffffffu;
        const bool need = in && cs < stop && lds_first_above<TW>(x.ae, cs)[TW] < cn;
        const uint64_t ends = __ballot(!in || cs >= stop);   // the wave's pass ends at the first of these
        uint64_t mask = __ballot(need);                      // all below it: starts increase with the chunk
        while (mask && !done) {
            const uint32_t l = uint32_t(__builtin_ctzll(mask));
            mask &= mask - 1;
            if (wg_chunk<TW, C, FA>(x, ys, ye, j0 + (c + l * kWavesPerBlock) * CH, m, stop, lane, sh)) {
                c += l * kWavesPerBlock;
                done = true;
            }
        }
        if (done) break;
        if (ends) {
            c += uint32_t(__builtin_ctzll(ends)) * kWavesPerBlock;
            break;
        }
        c += 64 * kWavesPerBlock;
    }
    if (lane == 0) __hip_atomic_fetch_min(&sh->cstop, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Copy X's piece (na, nf < TW intervals) into the workgroup's tile: wave w
// copies slots w * 64, (w + 4) * 64, ... and pads the rest.
template <int TW>
__device__ __forceinline__ void wg_load(const Resident &x, const uint32_t *__restrict__ as,
                                        const uint32_t *__restrict__ ae, uint32_t na,
                                        const uint32_t *__restrict__ fs, const uint32_t *__restrict__ fe,
                                        uint32_t nf, uint32_t w, uint32_t lane) {
#pragma unroll 1
    for (uint32_t i = w; i < TW / 64; i += kWavesPerBlock) {
        const uint32_t t = i * 64 + lane;
        if (t < na) {
            dma_dword(as + t, x.as + i * 64);
            dma_dword(ae + t, x.ae + i * 64);
        } else {
            x.as[t] = 0xffffffffu;
            x.ae[t] = 0xffffffffu;
        }
        if (t < nf) {
            dma_dword(fs + t, x.fs + i * 64);
            dma_dword(fe + t, x.fe + i * 64);
        } else {
            x.fs[t] = 0xffffffffu;
            x.fe[t] = 0xffffffffu;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Alg. 2's verdict for one workgroup-bin pair, by the whole workgroup.
// Every value that steers control flow is the same in all four waves (the
// same scalar loads, or LDS words read after a barrier), so every wave
// reaches every barrier.
template <int TW, int C>
__device__ uint32_t wg_pair(const Resident &res, const PairLists &L, uint32_t search_min, uint32_t w,
                            uint32_t lane, WgShared *sh) {
    bool aa = false;
    uint32_t a0 = 0, f0 = 0, k0 = 0;
    uint32_t ja = kNone, jf = kNone;   // stream restart points (kNone: search first)
    bool jf_tight = false;             // jf was set by the previous piece's F pass
    for (;;) {
        uint32_t a1 = L.nxa, f1 = L.nxf, k1 = kNone;
        if (L.nxa - a0 > TW - 1) {
            a1 = a0 + TW - 1;
            k1 = uniform(gload(L.xas, a1));
            f1 = f0 + uniform(wave_first_above(L.xfs + f0, L.nxf - f0, k1 - 1, lane));
        }
        if (f1 - f0 > TW - 1) {
            f1 = f0 + TW - 1;
            k1 = uniform(gload(L.xfs, f1));
            a1 = a0 + uniform(wave_first_above(L.xas + a0, a1 - a0, k1 - 1, lane));
        }
        __syncthreads();   // every wave is done with the previous piece's tile and flags
        if (w == 0 && lane == 0) {
            sh->bits = 0;
            sh->cstop = kNone;
        }
        wg_load<TW>(res, L.xas + a0, L.xae + a0, a1 - a0, L.xfs + f0, L.xfe + f0, f1 - f0, w, lane);
        __syncthreads();   // the tile and the cleared flags are in place
        const uint32_t na = a1 - a0;
        const uint32_t x_lo = max(k0, uniform(res.as[0]));
        const uint32_t x_hi = min(k1, uniform(res.ae[na - 1]));
        if (ja == kNone)
            ja = L.nya > search_min ? uniform(wave_first_above(L.yae, L.nya, x_lo, lane)) : 0u;
        wg_stream<TW, C, true>(res, L.yas, L.yae, ja, L.nya, x_hi, w, lane, sh);
        __syncthreads();
        uint32_t bits = uniform(sh->bits);
        uint32_t cs = uniform(sh->cstop);
        if (bits & kHitTH) return APRIL_TH;
        ja = ja + (cs > 0 ? (cs - 1) * (64 * C) : 0u);
        if (bits & kHitAA) {
            aa = true;
            // AF: Y.F against X.A over the same key range
            if (!jf_tight) {
                const uint32_t from = jf == kNone ? 0u : jf;
                jf = from + uniform(wave_first_above(L.yfe + from, L.nyf - from, x_lo, lane));
            }
            __syncthreads();   // every wave has read the flags of the A pass
            if (w == 0 && lane == 0) sh->cstop = kNone;
            __syncthreads();
            wg_stream<TW, C, false>(res, L.yfs, L.yfe, jf, L.nyf, x_hi, w, lane, sh);
            __syncthreads();
            bits = uniform(sh->bits);
            cs = uniform(sh->cstop);
            if (bits & kHitTH) return APRIL_TH;
            jf = jf + (cs > 0 ? (cs - 1) * (64 * C) : 0u);
            jf_tight = true;
        } else {
            jf_tight = false;
        }
        if (k1 == kNone) break;
        k0 = k1;
        a0 = uniform(gload(L.xae, a1 - 1)) > k1 ? a1 - 1 : a1;
        f0 = (f1 > 0 && uniform(gload(L.xfe, f1 - 1)) > k1) ? f1 - 1 : f1;
    }
    return aa ? APRIL_INDECISIVE : APRIL_TN;
}

// ------------------------------------------------------------- persistent

__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) { return (uint64_t(hi) << 32) | lo; }

__device__ __forceinline__ uint32_t lane_val(uint32_t v, uint32_t k) {
    return __builtin_amdgcn_readlane(v, k);
}

__device__ __forceinline__ const uint32_t *lane_ptr(const uint32_t *p, uint32_t k) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    return reinterpret_cast<const uint32_t *>(join64(lane_val(uint32_t(v), k), lane_val(uint32_t(v >> 32), k)));
}

// One pair's lists with X = S's object when `xs`, else R's.
template <class Args>
__device__ __forceinline__ PairLists pair_lists(const Args &a, bool xs, uint64_t ar0, uint32_t nar,
                                                uint64_t fr0, uint32_t nfr, uint64_t as0, uint32_t nas,
                                                uint64_t fs0, uint32_t nfs) {
    PairLists L;
    const uint32_t *ras = a.Ar.s + ar0, *rae = a.Ar.e + ar0, *rfs = a.Fr.s + fr0, *rfe = a.Fr.e + fr0;
    const uint32_t *sas = a.As.s + as0, *sae = a.As.e + as0, *sfs = a.Fs.s + fs0, *sfe = a.Fs.e + fs0;
    L.xas = xs ? sas : ras; L.xae = xs ? sae : rae; L.xfs = xs ? sfs : rfs; L.xfe = xs ? sfe : rfe;
    L.yas = xs ? ras : sas; L.yae = xs ? rae : sae; L.yfs = xs ? rfs : sfs; L.yfe = xs ? rfe : sfe;
    L.nxa = xs ? nas : nar; L.nxf = xs ? nfs : nfr;
    L.nya = xs ? nar : nas; L.nyf = xs ? nfr : nfs;
    return L;
}

// The pair lane k holds, as the whole wave sees it (scalar registers).
__device__ __forceinline__ PairLists lane_pair(const PairLists &m, uint32_t k) {
    PairLists L;
    L.xas = lane_ptr(m.xas, k); L.xae = lane_ptr(m.xae, k); L.xfs = lane_ptr(m.xfs, k); L.xfe = lane_ptr(m.xfe, k);
    L.yas = lane_ptr(m.yas, k); L.yae = lane_ptr(m.yae, k); L.yfs = lane_ptr(m.yfs, k); L.yfe = lane_ptr(m.yfe, k);
    L.nxa = lane_val(m.nxa, k); L.nxf = lane_val(m.nxf, k);
    L.nya = lane_val(m.nya, k); L.nyf = lane_val(m.nyf, k);
    return L;
}

// The end of a wave of a persistent kernel, for APRIL_WAVE_TIMES: t[0] and
// t[1] take the earliest and the latest end (the call's start is taken by
// the zeroing kernel that precedes the launches).  Lane 0 only.
__device__ __forceinline__ void wave_ended(unsigned long long *t) {
    const unsigned long long now = __builtin_amdgcn_s_memrealtime();
    atomicMin(&t[0], now);
    atomicMax(&t[1], now);
}

// The workgroup bin: a persistent kernel whose workgroups take the queued
// pairs, each XCD's workgroups from that XCD range's queue first, then the
// others'.  It runs before the wave kernel (same stream), so the longest
// joins start first.
template <int TILE, int C>
__global__ __launch_bounds__(kBlock) void k_wg(BatchArgs b) {
    __shared__ uint32_t lds_words[kWavesPerBlock * 4 * TILE];
    __shared__ WgShared wg_sh;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = uniform(threadIdx.x >> 6);
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;
    const uint32_t xcds = b.xcds;
    const uint32_t my_xcd = blockIdx.x % xcds;
    {
        constexpr int TW = kWavesPerBlock * TILE;
        Resident wres;
        wres.ae = lds_words;   // one tile of TW per list: A.end, A.start, F.end, F.start
        wres.as = wres.ae + TW;
        wres.fe = wres.as + TW;
        wres.fs = wres.fe + TW;
        wres.na = wres.nf = 0;
        for (uint32_t k = 0; k < xcds; k++) {
            typedef const __attribute__((address_space(4))) BatchArgs *KArgs;
            KArgs pb = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
            asm volatile("" : "+s"(pb));
            const uint32_t seg = (my_xcd + k) % xcds;
            // (every wave reads the same count: the binning pass has ended;
            // the grab is one thread's, passed on through LDS, so that all
            // four waves take the same branches and reach every barrier)
            const uint32_t nq = uniform(min(pb->qfill[seg * kCtrStride], pb->qcap));
            for (;;) {
                __syncthreads();   // the last pair's shared words are no longer read
                if (threadIdx.x == 0) wg_sh.grab = atomicAdd(&pb->qhead[seg * kCtrStride], 1u);
                __syncthreads();
                const uint32_t q = uniform(wg_sh.grab);
                if (q >= nq) break;
                const __attribute__((address_space(4))) FilterArgs &a = pb->f;
                const uint64_t p = pb->queue[uint64_t(seg) * pb->qcap + q];
                const uint32_t r = uniform(gload32(a.r, p)), s = uniform(gload32(a.s, p));
                const uint64_t ar0 = gload64(a.Ar.off, r), fr0 = gload64(a.Fr.off, r);
                const uint64_t as0 = gload64(a.As.off, s), fs0 = gload64(a.Fs.off, s);
                const uint32_t nar = uint32_t(gload64(a.Ar.off, r + 1) - ar0);
                const uint32_t nfr = uint32_t(gload64(a.Fr.off, r + 1) - fr0);
                const uint32_t nas = uint32_t(gload64(a.As.off, s + 1) - as0);
                const uint32_t nfs = uint32_t(gload64(a.Fs.off, s + 1) - fs0);
                const bool xs = max(nas, nfs) < max(nar, nfr);   // the shorter object is cut into pieces
                const PairLists L = pair_lists(a, xs, ar0, nar, fr0, nfr, as0, nas, fs0, nfs);
                const uint32_t v = wg_pair<TW, C>(wres, L, pb->search_min, w, lane, &wg_sh);
                if (threadIdx.x == 0) {
                    pb->f.verdict[p] = uint8_t(v);
                    c_tn += v == APRIL_TN;
                    c_th += v == APRIL_TH;
                    c_ind += v == APRIL_INDECISIVE;
                }
            }
        }
        __syncthreads();   // the shared tile is free for the waves' own tiles
    }
    if (b.f.counts) {
        for (int off = 32; off > 0; off >>= 1) {
            c_tn += __shfl_down(c_tn, off);
            c_th += __shfl_down(c_th, off);
            c_ind += __shfl_down(c_ind, off);
        }
        const unsigned long long v[3] = {c_tn, c_th, c_ind};
        if (lane == 0) add_totals(b.xhead, blockIdx.x * kWavesPerBlock + w, v, 3);
    }
    if (b.times && lane == 0) wave_ended(b.times + 3);
}

template <int TILE, int C, int MODE>
// Register budget: 8 waves per SIMD where LDS allows it (TILE <= 256).
// The hardware allocates SGPRs in blocks of 16, and above 80 SGPRs fewer
// waves fit than the compiler's occupancy estimate says: the kernel at 97
// SGPRs ran 5 waves per SIMD (2.42 ms at scale), capped to 80 SGPRs and 64
// VGPRs (16 bytes of spill) it runs 8 (2.11 ms).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8), amdgpu_num_sgpr(80)))
void k_batched(BatchArgs b) {
    __shared__ uint32_t lds_words[kWavesPerBlock * 4 * TILE];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = uniform(threadIdx.x >> 6);
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;
    const uint32_t xcds = b.xcds;
    const uint32_t my_xcd = blockIdx.x % xcds;


    Resident res;
    res.ae = lds_words + w * 4 * TILE;   // layout: A.end, A.start, F.end, F.start
    res.as = res.ae + TILE;
    res.fe = res.as + TILE;
    res.fs = res.fe + TILE;
    res.na = res.nf = 0;
    uint32_t cached = kNone;   // resident object id | side bit
    uint32_t pcached = kNone;  // object whose piece is resident (512-interval Alg. 2 instance)
    __shared__ uint32_t piece_words[kWavesPerBlock][8];

    // ---- pairs in input order: each XCD drains its own contiguous range,
    // then helps the others
    uint32_t grab = b.grab;
    for (uint32_t k = 0; k < xcds; k++) {
        const uint32_t seg = (my_xcd + k) % xcds;
        const uint64_t lo = b.f.n_pairs * seg / xcds, hi = b.f.n_pairs * (seg + 1) / xcds;
        if (k > 0) {
            typedef const __attribute__((address_space(4))) BatchArgs *KArgs;
            KArgs pb = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
            asm volatile("" : "+s"(pb));
            if (range_drained(pb->xhead, seg, lo, hi, lane)) continue;
        }
        for (;;) {
            // The arguments are read afresh for every grab (through a pointer
            // the compiler cannot see through), so they hold no scalar
            // registers while the grab's pairs are processed.
            typedef const __attribute__((address_space(4))) BatchArgs *KArgs;
            KArgs pb = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
            asm volatile("" : "+s"(pb));
            const __attribute__((address_space(4))) FilterArgs &a = pb->f;
            unsigned int got = 0;
            if (lane == 0) got = atomicAdd(&pb->xhead[seg * kCtrStride], grab);
            const uint64_t g0 = lo + uniform(__shfl(got, 0));
            if (g0 >= hi) break;
            const uint64_t g1 = min(hi, g0 + grab);
            if (hi - g1 < pb->tail_pairs) grab = pb->tail_grab;
            const uint64_t p = g0 + lane;
            bool seq = false, wave = false;
            // lane k's verdict for pair g0 + k, stored once per grab (a
            // store per pair would make each pair wait for the last one's)
            uint32_t vv = APRIL_BAD_PAIR;
            // lane k's pair: its lists with X the object to keep resident
            PairLists m{};
            uint32_t key = kNone;
            bool mine = p < g1;   // false for a pair the workgroup bin answers
            if (p < g1) {
                const uint32_t r = gload32(a.r, p), s = gload32(a.s, p);
                if ((r < a.n_r) & (s < a.n_s)) {
                    const uint64_t ar0 = gload64(a.Ar.off, r), fr0 = gload64(a.Fr.off, r);
                    const uint64_t as0 = gload64(a.As.off, s), fs0 = gload64(a.Fs.off, s);
                    const uint32_t nar = uint32_t(gload64(a.Ar.off, r + 1) - ar0);
                    const uint32_t nfr = uint32_t(gload64(a.Fr.off, r + 1) - fr0);
                    const uint32_t nas = uint32_t(gload64(a.As.off, s + 1) - as0);
                    const uint32_t nfs = uint32_t(gload64(a.Fs.off, s + 1) - fs0);
                    const uint32_t mr = max(nar, nfr), ms = max(nas, nfs);
                    if (MODE == kAlg2 && wg_bin(mr, ms, TILE, pb->wg_min) &&
                        ((const uint8_t __attribute__((address_space(1))) *)a.verdict)[p] != kOverflow)
                        mine = false;
                    // R resident when its lists fit a tile; else S when its
                    // do or when neither does and S's are shorter
                    // (mixed orders: the coarser side, whose lists stay
                    // sorted and disjoint; within joins: s, the container;
                    // linestrings: the polygon)
                    const bool xs = MODE == kMixedOrders ? pb->shift_r != 0
                                    : MODE == kWithinJoin ? true
                                    : MODE == kLinestrings ? false
                                                           : !(mr < TILE) && (ms < TILE || ms < mr);
                    if (!mine) {
                    } else if (MODE == kAlg2 && max(mr, ms) <= pb->thread_max) seq = true;
                    else wave = true;
                    m = pair_lists(a, xs, ar0, nar, fr0, nfr, as0, nas, fs0, nfs);
                    key = (xs ? s : r) | (xs ? kSideS : 0u);
                }
            }
            // one pair after another, the wave cooperating
            uint64_t todo = __ballot(wave);
            const uint32_t search_min = pb->search_min;
            while (todo) {
                const uint32_t k2 = uint32_t(__builtin_ctzll(todo));
                todo &= todo - 1;
                const PairLists L = lane_pair(m, k2);
                const uint32_t kk = lane_val(key, k2);
                const uint32_t sh = MODE == kMixedOrders ? ((kk & kSideS) ? pb->shift_r : pb->shift_s) : 0;
                const uint32_t v =
                    wave_pair<TILE, C, MODE>(res, cached, kk, L, search_min, lane, sh, pcached, piece_words[w]);
                vv = lane == k2 ? v : vv;
            }
            // very short lists: every such lane runs Alg. 2 on its own pair
            // (X and Y stand for R and S in either order; the verdict is
            // symmetric)
            if (seq) {
                uint32_t x, y;
                uint32_t v;
                if (!seq_join(m.xas, m.xae, m.nxa, m.yas, m.yae, m.nya, &x, &y))
                    v = APRIL_TN;
                else if (seq_join(m.xas, m.xae, m.nxa, m.yfs, m.yfe, m.nyf, &x, &y) ||
                         seq_join(m.xfs, m.xfe, m.nxf, m.yas, m.yae, m.nya, &x, &y))
                    v = APRIL_TH;
                else
                    v = APRIL_INDECISIVE;
                vv = v;
            }
            if (mine) {
                pb->f.verdict[p] = uint8_t(vv);
                c_tn += vv == APRIL_TN;
                c_th += vv == APRIL_TH;
                c_ind += vv == APRIL_INDECISIVE;
            }
        }
    }

    if (b.f.counts) {
        for (int off = 32; off > 0; off >>= 1) {
            c_tn += __shfl_down(c_tn, off);
            c_th += __shfl_down(c_th, off);
            c_ind += __shfl_down(c_ind, off);
        }
        const unsigned long long v[3] = {c_tn, c_th, c_ind};
        if (lane == 0) add_totals(b.xhead, blockIdx.x * kWavesPerBlock + w, v, 3);
    }
    if (b.times && lane == 0) wave_ended(b.times + 1);
}


template <int TILE, int C, int MODE = kAlg2>
int launch_tc(const BatchArgs &b, int cus, uint32_t waves, hipStream_t stream) {
    static int per_cu = 0;   // resident workgroups per CU (same on every gfx950 device)
    if (!per_cu) {
        int q = 0;
        APRIL_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_batched<TILE, C, MODE>, kBlock, 0));
        per_cu = q < 1 ? 1 : q;
    }
    // default residency (measured on the at-scale join): 4 waves per SIMD
    // with 512-interval tiles, as many as fit (8) with 256 and 128
    const int dflt = TILE >= 512 ? 4 : per_cu;
    uint64_t blocks = uint64_t(cus) * std::min(per_cu, dflt);
    if (waves) blocks = std::max<uint64_t>(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
    // a range is near its end once its waves have about two full grabs each left
    BatchArgs bb = b;
    bb.tail_pairs = 2ull * b.grab * kWavesPerBlock * ((blocks + b.xcds - 1) / b.xcds);
    if (MODE == kAlg2 && b.wg_min != kNone) {
        const uint64_t bin_blocks = std::min<uint64_t>((b.f.n_pairs + 255) / 256, uint64_t(cus) * 8);
        k_bin<<<dim3(uint32_t(bin_blocks)), dim3(256), 0, stream>>>(bb, TILE);
        APRIL_HIP_TRY(hipGetLastError());
        static int wg_per_cu = 0;   // resident workgroups per CU
        if (!wg_per_cu) {
            int q = 0;
            APRIL_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_wg<TILE, C>, kBlock, 0));
            wg_per_cu = q < 1 ? 1 : q;
        }
        k_wg<TILE, C><<<dim3(uint32_t(uint64_t(cus) * wg_per_cu)), dim3(kBlock), 0, stream>>>(bb);
        APRIL_HIP_TRY(hipGetLastError());
    }
    k_batched<TILE, C, MODE><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(bb);
    APRIL_HIP_TRY(hipGetLastError());
    if (b.f.counts) {
        k_sum_totals<<<1, 64, 0, stream>>>(b.xhead, b.f.counts, 3);
        APRIL_HIP_TRY(hipGetLastError());
    }
    return APRIL_OK;
}

template <int TILE>
int launch_t(const BatchArgs &b, uint32_t chunk, int cus, uint32_t waves, hipStream_t stream) {
    switch (chunk) {
        case 1: return launch_tc<TILE, 1>(b, cus, waves, stream);
        case 2: return launch_tc<TILE, 2>(b, cus, waves, stream);
        case 4: return launch_tc<TILE, 4>(b, cus, waves, stream);
    }
    return fail(APRIL_E_INVALID, "chunk must be 1, 2 or 4");
}

}  // namespace

// Workspace of the batched schedule: the counters and count slots
// (kCtrBytes), the workgroup queues' fill and head counters (two regions of
// kMaxCtrs slots, 128 bytes apart), then the queues: kBigQueueCap pair
// indices shared evenly by the XCD ranges.
constexpr uint64_t kQueueCtrBytes = 2ull * kMaxCtrs * kCtrStride * sizeof(unsigned int);
static_assert(kCtrBytes + kQueueCtrBytes + 4ull * kBigQueueCap <= kStaticWorkspaceBytes,
              "the static scratch holds a batched workspace");

uint64_t batched_workspace_bytes(uint64_t) { return kCtrBytes + kQueueCtrBytes + 4ull * kBigQueueCap; }

// Wave times (APRIL_WAVE_TIMES) sit in the last fill-counter slot, which no
// XCD range uses (xcd_count stays below kMaxCtrs).
constexpr uint64_t kTimesOffset = kCtrBytes + uint64_t(kMaxCtrs - 1) * kCtrStride * sizeof(unsigned int);
static_assert(kTimesOffset == APRIL_WAVE_TIMES_OFFSET, "wave times offset");

__global__ void k_zero_queue_ctrs(unsigned int *qctr) {
    const uint32_t t = threadIdx.x;
    if (t < 2 * kMaxCtrs && t != kMaxCtrs - 1) qctr[t * kCtrStride] = 0;
    if (t == kMaxCtrs - 1) {
        // the launch's start (the kernels that follow on the stream begin
        // after this one), then the two end times
        unsigned long long *times = reinterpret_cast<unsigned long long *>(qctr + (kMaxCtrs - 1) * kCtrStride);
        times[0] = __builtin_amdgcn_s_memrealtime();
        times[1] = times[3] = ~0ull;
        times[2] = times[4] = 0;
    }
}

int xcd_count(int cus) { return (cus >= 64 && cus % 32 == 0) ? std::min<int>(cus / 32, kMaxCtrs - 1) : 1; }

__global__ void k_zero_ctrs(unsigned int *ctr) {
    const uint32_t t = threadIdx.x;
    if (t < kMaxCtrs) {
        ctr[t * kCtrStride] = 0;
        unsigned long long *slot = reinterpret_cast<unsigned long long *>(ctr + kMaxCtrs * kCtrStride) + t * kSlotWords;
        slot[0] = slot[1] = slot[2] = 0;
    }
}

__global__ void k_sum_totals(const unsigned int *ctr, unsigned long long *totals, uint32_t n) {
    const uint32_t t = threadIdx.x;   // one wave of 64 = kMaxCtrs lanes
    const unsigned long long *slot =
        reinterpret_cast<const unsigned long long *>(ctr + kMaxCtrs * kCtrStride) + t * kSlotWords;
    for (uint32_t k = 0; k < n; k++) {
        unsigned long long v = slot[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if (t == 0) totals[k] = v;
    }
}

void batched_defaults(april_filter_opts_t &o, const BatchedShape &shape) {
    // default tile: 256 intervals when a typical A-list fits it (more waves
    // per CU), else 512 (fewer pieces, and the probe join for short objects
    // spread over a wide key range).  Measured: 6% faster at 256 on the
    // at-scale join (mean 177 intervals); 11% faster at 512 on the skewed
    // one (mean 990; 75.7 against 84.9 ms).
    if (!o.tile) o.tile = shape.intervals_a <= 256 * shape.objects ? 256 : 512;
    // the workgroup bin needs two objects of at least max(tile, wg_min)
    // intervals: without such objects on both sides, no binning pass
    if (!o.wg_min) o.wg_min = kDefaultWgMin;
    const uint64_t need_len = std::max(o.tile, o.wg_min);
    if (shape.max_len_r < need_len || shape.max_len_s < need_len) o.wg_min = kNone;
}

// Workgroup-bin fields of the arguments: off (kNone) or on, with the queues
// in the workspace after the counters.
static void set_wg_bin(BatchArgs &b, uint32_t wg_min, void *workspace) {
    unsigned int *qctr = reinterpret_cast<unsigned int *>(static_cast<char *>(workspace) + kCtrBytes);
    b.wg_min = wg_min;
    b.qfill = qctr;
    b.qhead = qctr + kMaxCtrs * kCtrStride;
    b.queue = reinterpret_cast<uint32_t *>(static_cast<char *>(workspace) + kCtrBytes + kQueueCtrBytes);
    b.qcap = uint32_t(kBigQueueCap / b.xcds);
    b.times = nullptr;
}

int launch_batched(const FilterArgs &a, const april_filter_opts_t &o, int cus, void *workspace,
                   hipStream_t stream) {
    const uint32_t tile = o.tile ? o.tile : 256;
    // default chunk: 2 elements per lane per step (with chunk skipping, also
    // the best for 512-interval tiles: skewed workload 61.5 against 64.5 ms
    // with 4, partitioned raw join 118.5 against 123.5 ms)
    const uint32_t chunk = o.chunk ? o.chunk : 2;
    BatchArgs b;
    b.f = a;
    b.xhead = static_cast<unsigned int *>(workspace);
    b.xcds = uint32_t(xcd_count(cus));
    b.thread_max = o.thread_max ? o.thread_max : 8;
    b.search_min = o.search_min ? o.search_min : 512;
    // workgroup bin: pairs whose shorter object spans kDefaultWgMin
    // intervals or more (0 = that default, 0xFFFFFFFF = no workgroup bin);
    // pair indices in the queues are 32-bit
    uint32_t wg_min = o.wg_min ? o.wg_min : kDefaultWgMin;
    if (a.n_pairs >= (1ull << 32)) wg_min = kNone;
    set_wg_bin(b, wg_min, workspace);
    // Grabs of 32 pairs: an XCD's waves then hold about 32k consecutive
    // pairs at once, whose S objects' lists about fill its L2 (4 MB); with
    // 64 the at-scale join ran 4% slower (2.13 vs 2.05 ms), with 16 no faster.
    b.grab = 32;
    b.tail_grab = 8;
    b.shift_r = b.shift_s = 0;
    if (b.thread_max >= tile) return fail(APRIL_E_INVALID, "thread_max must be below tile");
    k_zero_ctrs<<<1, 64, 0, stream>>>(b.xhead);
    APRIL_HIP_TRY(hipGetLastError());
    if (o.flags & APRIL_WAVE_TIMES)
        b.times = reinterpret_cast<unsigned long long *>(static_cast<char *>(workspace) + kTimesOffset);
    if (wg_min != kNone || b.times) {
        k_zero_queue_ctrs<<<1, 2 * kMaxCtrs, 0, stream>>>(b.qfill);
        APRIL_HIP_TRY(hipGetLastError());
    }
    switch (tile) {
        case 128: return launch_t<128>(b, chunk, cus, o.waves, stream);
        case 256: return launch_t<256>(b, chunk, cus, o.waves, stream);
        case 512: return launch_t<512>(b, chunk, cus, o.waves, stream);
    }
    return fail(APRIL_E_INVALID, "tile must be 128, 256 or 512");
}

int launch_batched_mixed(const FilterArgs &a, uint32_t shift_r, uint32_t shift_s, int cus, void *workspace,
                         hipStream_t stream) {
    if ((shift_r == 0) == (shift_s == 0)) return fail(APRIL_E_INVALID, "exactly one side must be finer");
    BatchArgs b;
    b.f = a;
    b.xhead = static_cast<unsigned int *>(workspace);
    b.xcds = uint32_t(xcd_count(cus));
    b.thread_max = 0;   // unused: every pair by the wave
    b.search_min = 512;
    b.grab = 32;
    b.tail_grab = 8;
    b.shift_r = shift_r;
    b.shift_s = shift_s;
    set_wg_bin(b, kNone, workspace);
    k_zero_ctrs<<<1, 64, 0, stream>>>(b.xhead);
    APRIL_HIP_TRY(hipGetLastError());
    return launch_tc<256, 2, kMixedOrders>(b, cus, 0, stream);
}

int launch_batched_within(const FilterArgs &a, int cus, void *workspace, hipStream_t stream) {
    BatchArgs b;
    b.f = a;
    b.xhead = static_cast<unsigned int *>(workspace);
    b.xcds = uint32_t(xcd_count(cus));
    b.thread_max = 0;   // unused: every pair by the wave
    b.search_min = 512;
    b.grab = 32;
    b.tail_grab = 8;
    b.shift_r = b.shift_s = 0;
    set_wg_bin(b, kNone, workspace);
    k_zero_ctrs<<<1, 64, 0, stream>>>(b.xhead);
    APRIL_HIP_TRY(hipGetLastError());
    return launch_tc<256, 2, kWithinJoin>(b, cus, 0, stream);
}

int launch_batched_linestrings(const FilterArgs &a, int cus, void *workspace, hipStream_t stream) {
    BatchArgs b;
    b.f = a;
    b.xhead = static_cast<unsigned int *>(workspace);
    b.xcds = uint32_t(xcd_count(cus));
    b.thread_max = 0;   // unused: every pair by the wave
    b.search_min = 512;
    b.grab = 32;
    b.tail_grab = 8;
    b.shift_r = b.shift_s = 0;
    set_wg_bin(b, kNone, workspace);
    k_zero_ctrs<<<1, 64, 0, stream>>>(b.xhead);
    APRIL_HIP_TRY(hipGetLastError());
    return launch_tc<256, 2, kLinestrings>(b, cus, 0, stream);
}

}  // namespace april
