// Batched schedule of the APRIL filter: length binning + one persistent kernel.
//
// Join kernel used here.  For sorted, disjoint interval lists X and Y,
// IntervalJoin of Alg. 2 returns true iff some X_i overlaps some Y_j.  That
// predicate can be decided from Y's side alone: for Y_j let i*(j) be the
// first i with X_i.end > Y_j.start; then
//     some X_i overlaps Y_j   <=>   i*(j) exists and X_{i*(j)}.start < Y_j.end.
// (<=: the pair is an overlap.  =>: an overlapping X_i has X_i.end >
// Y_j.start, so i*(j) <= i and X_{i*(j)}.start <= X_i.start < Y_j.end.)
// So one list X is kept in LDS and every lane takes elements of the other
// list Y, read in coalesced chunks, and binary-searches X for i*(j); a
// ballot gives the join's result after each chunk (early exit).  Elements of
// Y that end before X starts or start after X ends cannot overlap; long
// streamed lists are first cut to that window by a 64-ary search.  When X is
// longer than LDS it is processed tile by tile; an overlap (X_i, Y_j) is
// found in the tile holding X_i, because Y_j lies in that tile's window.
//
// The three joins of Alg. 2 (AA, AF = A(r) x F(s), FA = F(r) x A(s)) are
// symmetric in r and s, so the LDS side can be either object: with X the
// resident object and Y the streamed one, the joins are X.A x Y.A, then
// X.A x Y.F and X.F x Y.A.  The verdict is Alg. 2's: no AA overlap -> true
// negative; else an overlap in either of the other two -> true hit; else
// indecisive.
//
// Bins (chosen per pair by the binning kernel):
//   THREAD  all four lists short: one lane runs Alg. 2 sequentially;
//   WAVE    one side's A- and F-lists fit the per-wave LDS tile: that side
//           is resident (reused by consecutive pairs on the same object),
//           the other streamed, one wavefront per pair;
//   BLOCK   both sides longer: the shorter side is resident in the whole
//           workgroup's LDS, tile by tile, and the four wavefronts stream
//           the other side's window together.
// The persistent kernel drains BLOCK, then WAVE, then THREAD (largest work
// first); queues are filled once per call, so every wave exits when they
// are empty.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

constexpr uint32_t kSideS = 0x80000000u;   // queue entry: resident side is S
enum { Q_THREAD = 0, Q_WAVE = 1, Q_BLOCK = 2 };

struct BatchArgs {
    FilterArgs f;
    uint32_t *queue[3];          // pair index | kSideS (only the workgroup queue is used)
    unsigned int *tail;          // [3] entries per queue (binning kernel)
    unsigned int *head;          // [3] entries taken (persistent kernel)
    unsigned int *xhead;         // [xcds] pairs taken from each XCD's range
    uint32_t xcds;
    uint32_t thread_max;
    uint32_t search_min;
    uint32_t grab;
};

// rank of this lane among the set lanes of `mask` below it
__device__ __forceinline__ uint32_t rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(256) void k_zero_batch(unsigned int *ctr, unsigned long long *counts) {
    if (threadIdx.x < 64) ctr[threadIdx.x] = 0;
    if (counts && threadIdx.x < 3) counts[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_bin(BatchArgs b, uint32_t tile) {
    const FilterArgs &a = b.f;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t base = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); base < a.n_pairs;
         base += stride) {
        const uint64_t p = base + lane;
        bool big = false;
        uint32_t entry = uint32_t(p);
        if (p < a.n_pairs) {
            const uint32_t r = a.r[p], s = a.s[p];
            if (r >= a.n_r || s >= a.n_s) {
                a.verdict[p] = APRIL_BAD_PAIR;
            } else {
                const uint64_t nar = a.Ar.off[r + 1] - a.Ar.off[r], nfr = a.Fr.off[r + 1] - a.Fr.off[r];
                const uint64_t nas = a.As.off[s + 1] - a.As.off[s], nfs = a.Fs.off[s + 1] - a.Fs.off[s];
                const uint64_t mr = nar > nfr ? nar : nfr, ms = nas > nfs ? nas : nfs;
                // neither side fits a wavefront's LDS: workgroup queue, the
                // shorter side resident
                if ((mr > ms ? mr : ms) > b.thread_max && mr > tile && ms > tile) {
                    big = true;
                    if (ms < mr) entry |= kSideS;
                }
            }
        }
        const uint64_t mask = __ballot(big);
        if (mask) {
            const uint32_t leader = __builtin_ctzll(mask);
            unsigned int pos = 0;
            if (lane == leader) pos = atomicAdd(&b.tail[Q_BLOCK], unsigned(__popcll(mask)));
            pos = __shfl(pos, leader);
            if (big) b.queue[Q_BLOCK][pos + rank_in(mask)] = entry;
        }
    }
}

// ------------------------------------------------------------ join pieces

// first j in [0, m) with ye[j] > key (m if none): wave-cooperative 64-ary
// search, one global round trip per factor of 64
__device__ uint32_t wave_first_end_after(const uint32_t *__restrict__ ye, uint32_t m, uint32_t key,
                                         uint32_t lane) {
    uint32_t lo = 0, hi = m;
    while (hi - lo > 64) {
        const uint64_t step = (uint64_t(hi - lo) + 63) >> 6;
        const uint64_t probe = lo + (lane + 1) * step - 1;
        const bool pred = probe >= hi ? true : (ye[probe] > key);
        const uint64_t mask = __ballot(pred);
        if (!mask) { lo = hi; break; }
        const uint64_t f = __builtin_ctzll(mask);
        const uint64_t pf = lo + (f + 1) * step - 1;
        const uint32_t nlo = uint32_t(lo + f * step);
        hi = pf < hi ? uint32_t(pf) : hi;
        lo = nlo;
    }
    if (hi - lo == 0) return lo;
    const uint32_t j = lo + lane;
    const bool pred = j >= hi ? true : (ye[j] > key);
    const uint64_t mask = __ballot(pred);
    return mask ? lo + uint32_t(__builtin_ctzll(mask)) : hi;
}

// For C streamed elements per lane: does Y[j] overlap the resident list X
// (n entries in LDS, sorted)?  Branch-free lower bound on X.end.
template <int C>
__device__ __forceinline__ bool probe_resident(const uint2 *X, uint32_t n, const uint32_t (&ys)[C],
                                               const uint32_t (&ye)[C], const bool (&valid)[C]) {
    uint32_t pos[C];
#pragma unroll
    for (int c = 0; c < C; c++) pos[c] = 0;
    for (uint32_t step = 1u << (31 - __builtin_clz(n)); step; step >>= 1) {
#pragma unroll
        for (int c = 0; c < C; c++) {
            const uint32_t q = pos[c] + step;
            if (q <= n && X[q - 1].y <= ys[c]) pos[c] = q;
        }
    }
    bool hit = false;
#pragma unroll
    for (int c = 0; c < C; c++) hit |= valid[c] && pos[c] < n && X[pos[c]].x < ye[c];
    return hit;
}

// Stream Y[j_begin..) against X (LDS, n > 0) until an overlap is seen, Y is
// exhausted, or Y starts at/after x_hi.  `stride`/`first` let several waves
// share one Y window (chunk k of this wave is first + k * stride chunks).
template <int C>
__device__ __forceinline__ bool stream_overlap(const uint2 *X, uint32_t n, uint32_t x_hi,
                               const uint32_t *__restrict__ ys, const uint32_t *__restrict__ ye,
                               uint32_t m, uint32_t j_begin, uint32_t first, uint32_t stride,
                               uint32_t lane, const volatile int *stop) {
    constexpr uint32_t CH = 64 * C;
    for (uint32_t base = j_begin + first * CH; base < m; base += stride * CH) {
        if (stop && *stop) return false;
        uint32_t s[C], e[C];
        bool valid[C];
#pragma unroll
        for (int c = 0; c < C; c++) {
            const uint32_t j = base + c * 64 + lane;
            valid[c] = j < m;
            s[c] = valid[c] ? ys[j] : 0xffffffffu;
            e[c] = valid[c] ? ye[j] : 0u;
        }
        if (__any(probe_resident<C>(X, n, s, e, valid))) return true;
        // the chunk's first element already starts at or after X's end
        if (uniform(__shfl(s[0], 0)) >= x_hi) return false;
    }
    return false;
}

// X resident in this wave's LDS (n entries), Y global (m entries).
template <int C>
__device__ __forceinline__ bool wave_overlap(const uint2 *X, uint32_t n, const uint32_t *__restrict__ ys,
                             const uint32_t *__restrict__ ye, uint32_t m, uint32_t search_min,
                             uint32_t lane) {
    if (n == 0 || m == 0) return false;
    const uint32_t x_lo = X[0].x, x_hi = X[n - 1].y;
    const uint32_t j0 = m > search_min ? wave_first_end_after(ye, m, x_lo, lane) : 0;
    return stream_overlap<C>(X, n, x_hi, ys, ye, m, j0, 0, 1, lane, nullptr);
}

struct Side {
    uint64_t a0, na, f0, nf;
};

__device__ __forceinline__ Side side_of(const ListView &A, const ListView &F, uint32_t o) {
    Side s;
    s.a0 = A.off[o];
    s.na = A.off[o + 1] - s.a0;
    s.f0 = F.off[o];
    s.nf = F.off[o + 1] - s.f0;
    return s;
}

// wave-cooperative copy of n intervals into LDS
__device__ __forceinline__ void load_resident(uint2 *dst, const uint32_t *__restrict__ s,
                                              const uint32_t *__restrict__ e, uint32_t n,
                                              uint32_t lane, uint32_t width) {
    for (uint32_t t = lane; t < n; t += width) dst[t] = make_uint2(s[t], e[t]);
}

// ------------------------------------------------------------- persistent

// first i in [0, n) with E[i] > key (n if none), E sorted, in LDS
__device__ __forceinline__ uint32_t first_end_after(const uint32_t *E, uint32_t n, uint32_t key) {
    uint32_t pos = 0;
    for (uint32_t step = n ? 1u << (31 - __builtin_clz(n)) : 0u; step; step >>= 1) {
        const uint32_t q = pos + step;
        if (q <= n && E[q - 1] <= key) pos = q;
    }
    return pos;
}

// Resident lists of one wave, SoA in LDS: A.start, A.end, F.start, F.end.
struct Resident {
    uint32_t *as, *ae, *fs, *fe;
    uint32_t na, nf;
};

// Join of the resident list (RS, RE, n) with the streamed list Y: true iff
// some Y element overlaps some resident element.  With `fs`/`fe` set, Y is
// an A-list and every Y element that overlaps the resident A-list is also
// tested against the resident F-list; *th reports an F overlap (then the
// loop stops: the pair is a true hit).
template <int C>
__device__ __forceinline__ bool stream_join_resident(const uint32_t *RS, const uint32_t *RE, uint32_t n,
                                                     const uint32_t *FS, const uint32_t *FE, uint32_t nf,
                                                     const uint32_t *__restrict__ ys,
                                                     const uint32_t *__restrict__ ye, uint32_t m,
                                                     uint32_t search_min, uint32_t lane, bool *th) {
    if (n == 0 || m == 0) return false;
    const uint32_t x_lo = RS[0], x_hi = RE[n - 1];
    uint32_t j = m > search_min ? wave_first_end_after(ye, m, x_lo, lane) : 0;
    bool any_hit = false;
    for (; j < m; j += 64 * C) {
        uint32_t s[C], e[C];
#pragma unroll
        for (int c = 0; c < C; c++) {
            const uint32_t k = j + c * 64 + lane;
            const bool v = k < m;
            s[c] = v ? ys[k] : 0xffffffffu;
            e[c] = v ? ye[k] : 0u;
        }
        uint32_t pos[C];
#pragma unroll
        for (int c = 0; c < C; c++) pos[c] = 0;
        for (uint32_t step = 1u << (31 - __builtin_clz(n)); step; step >>= 1) {
#pragma unroll
            for (int c = 0; c < C; c++) {
                const uint32_t q = pos[c] + step;
                if (q <= n && RE[q - 1] <= s[c]) pos[c] = q;
            }
        }
        bool hit = false, fhit = false;
#pragma unroll
        for (int c = 0; c < C; c++) {
            const bool h = pos[c] < n && RS[pos[c]] < e[c];
            hit |= h;
            if (FS && h) {
                const uint32_t pf = first_end_after(FE, nf, s[c]);
                fhit |= pf < nf && FS[pf] < e[c];
            }
        }
        if (FS) {
            if (__any(fhit)) { *th = true; return true; }
            any_hit |= __any(hit);
        } else if (__any(hit)) {
            return true;
        }
        if (uniform(__shfl(s[0], 0)) >= x_hi) break;
    }
    return any_hit;
}

// Per-pair metadata a lane holds for its pair of the current grab.
struct PairMeta {
    uint32_t p, r, s;
    uint32_t ar0lo, ar0hi, nar, fr0lo, fr0hi, nfr;   // offsets split in 32-bit halves
    uint32_t as0lo, as0hi, nas, fs0lo, fs0hi, nfs;
};

__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) { return (uint64_t(hi) << 32) | lo; }

__device__ __forceinline__ uint32_t lane_val(uint32_t v, uint32_t k) {
    return __builtin_amdgcn_readlane(v, k);
}

template <int TILE, int C>
__global__ __launch_bounds__(kBlock) void k_batched(BatchArgs b) {
    // wave mode: wave w owns 4*TILE words: A.start, A.end, F.start, F.end
    // block mode: the whole array is one uint2 tile of 8*TILE entries
    __shared__ uint32_t lds_words[kWavesPerBlock * 4 * TILE];
    __shared__ unsigned int sh_item;
    __shared__ int sh_found;
    __shared__ uint32_t sh_j0;
    uint2 *lds = reinterpret_cast<uint2 *>(lds_words);
    const FilterArgs &a = b.f;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = uniform(threadIdx.x >> 6);
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;

    // ---- BLOCK queue: the workgroup takes one pair at a time (the three
    // joins of Alg. 2 one after the other, resident side tiled through LDS)
    const unsigned int n_block = b.tail[Q_BLOCK];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh_item = atomicAdd(&b.head[Q_BLOCK], 1u);
        __syncthreads();
        const unsigned int item = sh_item;
        if (item >= n_block) break;
        const uint32_t entry = b.queue[Q_BLOCK][item];
        const uint32_t p = entry & ~kSideS;
        const bool xs_is_s = entry & kSideS;
        const uint32_t r = a.r[p], s = a.s[p];
        const Side sr = side_of(a.Ar, a.Fr, r), ss = side_of(a.As, a.Fs, s);
        const Side X = xs_is_s ? ss : sr, Y = xs_is_s ? sr : ss;
        const ListView &XA = xs_is_s ? a.As : a.Ar, &XF = xs_is_s ? a.Fs : a.Fr;
        const ListView &YA = xs_is_s ? a.Ar : a.As, &YF = xs_is_s ? a.Fr : a.Fs;
        uint8_t v = APRIL_INDECISIVE;
        for (int jn = 0; jn < 3; jn++) {
            // jn 0: X.A x Y.A   jn 1: X.A x Y.F   jn 2: X.F x Y.A
            const ListView &XL = jn == 2 ? XF : XA;
            const ListView &YL = jn == 1 ? YF : YA;
            const uint64_t x0 = jn == 2 ? X.f0 : X.a0, nx = jn == 2 ? X.nf : X.na;
            const uint64_t y0 = jn == 1 ? Y.f0 : Y.a0, ny = jn == 1 ? Y.nf : Y.na;
            bool found = false;
            constexpr uint32_t TB = kWavesPerBlock * 2 * TILE;
            for (uint64_t t0 = 0; t0 < nx && ny > 0 && !found; t0 += TB) {
                const uint32_t nt = uint32_t(nx - t0 < TB ? nx - t0 : TB);
                __syncthreads();
                load_resident(lds, XL.s + x0 + t0, XL.e + x0 + t0, nt, threadIdx.x, kBlock);
                if (threadIdx.x == 0) sh_found = 0;
                __syncthreads();
                const uint32_t x_lo = lds[0].x, x_hi = lds[nt - 1].y;
                if (w == 0) {
                    const uint32_t j0 = uint32_t(ny) > b.search_min
                                            ? wave_first_end_after(YL.e + y0, uint32_t(ny), x_lo, lane)
                                            : 0;
                    if (lane == 0) sh_j0 = j0;
                }
                __syncthreads();
                if (stream_overlap<C>(lds, nt, x_hi, YL.s + y0, YL.e + y0, uint32_t(ny), sh_j0, w,
                                      kWavesPerBlock, lane, &sh_found)) {
                    if (lane == 0) sh_found = 1;
                }
                __syncthreads();
                found = sh_found;
            }
            if (jn == 0 && !found) { v = APRIL_TN; break; }
            if (jn > 0 && found) { v = APRIL_TH; break; }
        }
        if (threadIdx.x == 0) {
            a.verdict[p] = v;
            c_tn += v == APRIL_TN;
            c_th += v == APRIL_TH;
            c_ind += v == APRIL_INDECISIVE;
        }
    }

    // ---- pairs in input order: each XCD drains its own contiguous range
    // (pairs close in the input share lists in that XCD's L2), then helps the
    // others.  A wave takes 64 pairs at a time, one lane per pair's metadata.
    Resident res;
    res.as = lds_words + w * 4 * TILE;
    res.ae = res.as + TILE;
    res.fs = res.ae + TILE;
    res.fe = res.fs + TILE;
    res.na = res.nf = 0;
    uint32_t cached = 0xffffffffu;   // resident object id | side bit
    const uint32_t xcds = b.xcds;
    const uint32_t my_xcd = blockIdx.x % xcds;
    for (uint32_t k = 0; k < xcds; k++) {
        const uint32_t seg = (my_xcd + k) % xcds;
        const uint64_t lo = a.n_pairs * seg / xcds, hi = a.n_pairs * (seg + 1) / xcds;
        for (;;) {
            unsigned int got = 0;
            if (lane == 0) got = atomicAdd(&b.xhead[seg], 64u);
            const uint64_t g0 = lo + uniform(__shfl(got, 0));
            if (g0 >= hi) break;
            const uint64_t p = g0 + lane;
            int bin = -1;
            bool side_s = false;
            PairMeta m{};
            if (p < hi) {
                m.p = uint32_t(p);
                m.r = a.r[p];
                m.s = a.s[p];
                if (m.r < a.n_r && m.s < a.n_s) {
                    const uint64_t ar0 = a.Ar.off[m.r], ar1 = a.Ar.off[m.r + 1];
                    const uint64_t fr0 = a.Fr.off[m.r], fr1 = a.Fr.off[m.r + 1];
                    const uint64_t as0 = a.As.off[m.s], as1 = a.As.off[m.s + 1];
                    const uint64_t fs0 = a.Fs.off[m.s], fs1 = a.Fs.off[m.s + 1];
                    m.ar0lo = uint32_t(ar0); m.ar0hi = uint32_t(ar0 >> 32); m.nar = uint32_t(ar1 - ar0);
                    m.fr0lo = uint32_t(fr0); m.fr0hi = uint32_t(fr0 >> 32); m.nfr = uint32_t(fr1 - fr0);
                    m.as0lo = uint32_t(as0); m.as0hi = uint32_t(as0 >> 32); m.nas = uint32_t(as1 - as0);
                    m.fs0lo = uint32_t(fs0); m.fs0hi = uint32_t(fs0 >> 32); m.nfs = uint32_t(fs1 - fs0);
                    const uint32_t mr = max(m.nar, m.nfr), ms = max(m.nas, m.nfs);
                    if (max(mr, ms) <= b.thread_max) bin = Q_THREAD;
                    else if (mr <= TILE) bin = Q_WAVE;
                    else if (ms <= TILE) { bin = Q_WAVE; side_s = true; }
                    // else: workgroup queue, done above
                }
            }
            // wave bin: one pair after another, the wave cooperating
            uint64_t todo = __ballot(bin == Q_WAVE);
            const uint64_t sides = __ballot(side_s);
            while (todo) {
                const uint32_t k2 = uint32_t(__builtin_ctzll(todo));
                todo &= todo - 1;
                const bool xs = (sides >> k2) & 1;
                const uint32_t pp = lane_val(m.p, k2);
                const uint32_t xo = lane_val(xs ? m.s : m.r, k2);
                const uint64_t xa0 = join64(lane_val(xs ? m.as0lo : m.ar0lo, k2), lane_val(xs ? m.as0hi : m.ar0hi, k2));
                const uint32_t nxa = lane_val(xs ? m.nas : m.nar, k2);
                const uint64_t xf0 = join64(lane_val(xs ? m.fs0lo : m.fr0lo, k2), lane_val(xs ? m.fs0hi : m.fr0hi, k2));
                const uint32_t nxf = lane_val(xs ? m.nfs : m.nfr, k2);
                const uint64_t ya0 = join64(lane_val(xs ? m.ar0lo : m.as0lo, k2), lane_val(xs ? m.ar0hi : m.as0hi, k2));
                const uint32_t nya = lane_val(xs ? m.nar : m.nas, k2);
                const uint64_t yf0 = join64(lane_val(xs ? m.fr0lo : m.fs0lo, k2), lane_val(xs ? m.fr0hi : m.fs0hi, k2));
                const uint32_t nyf = lane_val(xs ? m.nfr : m.nfs, k2);
                const ListView &XA = xs ? a.As : a.Ar, &XF = xs ? a.Fs : a.Fr;
                const ListView &YA = xs ? a.Ar : a.As, &YF = xs ? a.Fr : a.Fs;
                const uint32_t key = xo | (xs ? kSideS : 0u);
                if (key != cached) {
                    wave_lds_sync();
                    for (uint32_t t = lane; t < nxa; t += 64) { res.as[t] = XA.s[xa0 + t]; res.ae[t] = XA.e[xa0 + t]; }
                    for (uint32_t t = lane; t < nxf; t += 64) { res.fs[t] = XF.s[xf0 + t]; res.fe[t] = XF.e[xf0 + t]; }
                    wave_lds_sync();
                    res.na = nxa;
                    res.nf = nxf;
                    cached = key;
                }
                // AA, with FA on every AA-overlapping element (F inside A)
                bool th = false;
                const bool aa = stream_join_resident<C>(res.as, res.ae, res.na, res.fs, res.fe, res.nf,
                                                        YA.s + ya0, YA.e + ya0, nya, b.search_min, lane,
                                                        &th);
                uint8_t v;
                if (!aa) v = APRIL_TN;
                else if (th) v = APRIL_TH;
                else if (stream_join_resident<C>(res.as, res.ae, res.na, nullptr, nullptr, 0,
                                                 YF.s + yf0, YF.e + yf0, nyf, b.search_min, lane,
                                                 &th))
                    v = APRIL_TH;
                else v = APRIL_INDECISIVE;
                if (lane == 0) {
                    a.verdict[pp] = v;
                    c_tn += v == APRIL_TN;
                    c_th += v == APRIL_TH;
                    c_ind += v == APRIL_INDECISIVE;
                }
            }
            // thread bin: every such lane runs Alg. 2 on its own pair
            if (bin == Q_THREAD) {
                const uint64_t ar0 = join64(m.ar0lo, m.ar0hi), fr0 = join64(m.fr0lo, m.fr0hi);
                const uint64_t as0 = join64(m.as0lo, m.as0hi), fs0 = join64(m.fs0lo, m.fs0hi);
                uint32_t x, y;
                uint8_t v;
                if (!seq_join(a.Ar.s + ar0, a.Ar.e + ar0, m.nar, a.As.s + as0, a.As.e + as0, m.nas, &x, &y))
                    v = APRIL_TN;
                else if (seq_join(a.Ar.s + ar0, a.Ar.e + ar0, m.nar, a.Fs.s + fs0, a.Fs.e + fs0, m.nfs, &x, &y) ||
                         seq_join(a.Fr.s + fr0, a.Fr.e + fr0, m.nfr, a.As.s + as0, a.As.e + as0, m.nas, &x, &y))
                    v = APRIL_TH;
                else
                    v = APRIL_INDECISIVE;
                a.verdict[m.p] = v;
                c_tn += v == APRIL_TN;
                c_th += v == APRIL_TH;
                c_ind += v == APRIL_INDECISIVE;
            }
        }
    }

    if (a.counts) {
        for (int off = 32; off > 0; off >>= 1) {
            c_tn += __shfl_down(c_tn, off);
            c_th += __shfl_down(c_th, off);
            c_ind += __shfl_down(c_ind, off);
        }
        if (lane == 0) {
            if (c_tn) atomicAdd(&a.counts[0], c_tn);
            if (c_th) atomicAdd(&a.counts[1], c_th);
            if (c_ind) atomicAdd(&a.counts[2], c_ind);
        }
    }
}

constexpr uint64_t kCtrBytes = 256;

template <int TILE, int C>
int launch_tc(const BatchArgs &b, int cus, uint32_t waves, hipStream_t stream) {
    static int per_cu = 0;   // resident workgroups per CU (same on every gfx950 device)
    if (!per_cu) {
        int q = 0;
        APRIL_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_batched<TILE, C>, kBlock, 0));
        per_cu = q < 1 ? 1 : q;
    }
    uint64_t blocks = uint64_t(cus) * per_cu;
    if (waves) blocks = std::max<uint64_t>(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
    k_batched<TILE, C><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(b);
    APRIL_HIP_TRY(hipGetLastError());
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

uint64_t batched_workspace_bytes(uint64_t n_pairs) { return kCtrBytes + 4 * (n_pairs ? n_pairs : 1); }

int xcd_count(int cus) { return (cus >= 64 && cus % 32 == 0) ? cus / 32 : 1; }

int launch_batched(const FilterArgs &a, const april_filter_opts_t &o, int cus, void *workspace,
                   hipStream_t stream) {
    const uint32_t tile = o.tile ? o.tile : 512;
    const uint32_t chunk = o.chunk ? o.chunk : 1;
    BatchArgs b;
    b.f = a;
    char *ws = static_cast<char *>(workspace);
    b.tail = reinterpret_cast<unsigned int *>(ws);
    b.head = b.tail + 3;
    b.xhead = b.tail + 6;
    b.xcds = uint32_t(xcd_count(cus));
    b.queue[Q_THREAD] = b.queue[Q_WAVE] = nullptr;
    b.queue[Q_BLOCK] = reinterpret_cast<uint32_t *>(ws + kCtrBytes);
    b.thread_max = o.thread_max ? o.thread_max : 8;
    b.search_min = o.search_min ? o.search_min : 512;
    b.grab = 64;
    if (b.thread_max >= tile) return fail(APRIL_E_INVALID, "thread_max must be below tile");
    k_zero_batch<<<1, 64, 0, stream>>>(b.tail, a.counts);
    APRIL_HIP_TRY(hipGetLastError());
    const uint64_t bin_blocks = std::min<uint64_t>((a.n_pairs + 255) / 256, uint64_t(cus) * 8);
    k_bin<<<dim3(uint32_t(std::max<uint64_t>(bin_blocks, 1))), dim3(256), 0, stream>>>(b, tile);
    APRIL_HIP_TRY(hipGetLastError());
    switch (tile) {
        case 128: return launch_t<128>(b, chunk, cus, o.waves, stream);
        case 256: return launch_t<256>(b, chunk, cus, o.waves, stream);
        case 512: return launch_t<512>(b, chunk, cus, o.waves, stream);
    }
    return fail(APRIL_E_INVALID, "tile must be 128, 256 or 512");
}

}  // namespace april
