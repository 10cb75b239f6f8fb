// The filter on delta + VByte compressed lists (Sec. 5.1: join while
// decoding, so an early exit leaves the rest of a list undecoded).
//
// One wavefront per pair, pairs taken 64 at a time from per-XCD contiguous
// ranges like the raw batched schedule.  The three joins of Alg. 2 run in
// order: X.A x Y.A, then X.A x Y.F and X.F x Y.A.  X is the R object when its
// lists fit the wave's decode cache: its A-list is decoded once, into the
// cache, for a run of pairs that share it (its F-list when a X.F x Y.A join
// first needs it, which few pairs reach), and each join copies its tiles
// from there into LDS (skipping the copy when LDS already holds that tile).
// Otherwise X is the side with the shorter lists, decoded tile by tile into
// LDS by each join.  Tiles are padded to TILE entries.  For each tile, the Y
// intervals that can meet it are decoded window by window into a small LDS
// buffer: a short Y from its start; a longer one only in the 64-interval
// blocks (from its block index) whose key range meets a tile interval.
// Every lane searches the tile for its Y intervals (the overlap test of the
// raw batched kernel).  A ballot after each window ends the join early.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "internal.hpp"
#include "vbyte.hpp"

namespace april {
namespace {

struct CList {
    const uint64_t *off, *boff, *blk;
    const uint8_t *bytes;
    const uint32_t *bval, *bpos;
};

struct CArgs {
    CList Ar, Fr, As, Fs;
    const uint32_t *r, *s;
    uint64_t n_pairs, n_r, n_s;
    uint8_t *verdict;
    unsigned long long *counts;
    unsigned int *xhead;
    uint32_t xcds;
    uint32_t search_min;
    uint32_t first_cap;   // X intervals decoded before a join's first test (at most TILE)
    // decode cache: per wave, R's A and F lists of up to cache_cap intervals
    // each, decoded once per run of pairs that share the R object (nullptr:
    // no cache)
    uint32_t *cache;
    uint32_t cache_cap;
};

__device__ __forceinline__ uint32_t first_gt(const uint32_t *__restrict__ arr, uint32_t m, uint32_t key,
                                             uint32_t lane) {
    // first j in [0, m) with arr[j] > key (m if none): 64-ary search
    uint32_t lo = 0, hi = m;
    while (hi - lo > 64) {
        const uint64_t step = (uint64_t(hi - lo) + 63) >> 6;
        const uint64_t probe = lo + (lane + 1) * step - 1;
        const bool pred = probe >= hi ? true : (arr[probe] > key);
        const uint64_t mask = __ballot(pred);
        if (!mask) { lo = hi; break; }
        const uint64_t f = __builtin_ctzll(mask);
        const uint64_t pf = lo + (f + 1) * step - 1;
        const uint32_t nlo = uint32_t(lo + f * step);
        hi = pf < hi ? uint32_t(pf) : hi;
        lo = nlo;
    }
    if (hi == lo) return lo;
    const uint32_t j = lo + lane;
    const bool pred = j >= hi ? true : (arr[j] > key);
    const uint64_t mask = __ballot(pred);
    return mask ? lo + uint32_t(__builtin_ctzll(mask)) : hi;
}

// A list of one object: its collection's arrays stay in the kernel's
// argument segment (read with scalar loads where they are used), so that a
// reference costs two scalar registers, not twelve.
typedef const __attribute__((address_space(4))) CList KList;
typedef const __attribute__((address_space(4))) CArgs KArgs;

struct ListRef {
    KList *L;
    uint32_t obj, n;
};

__device__ __forceinline__ VCursor cursor_at(const ListRef &x) {
    return vcursor(x.L->bytes, x.L->boff[x.obj], x.L->boff[x.obj + 1], x.n);
}

// Pad the X tile's entries nt .. TILE-1 with 0xFFFFFFFF (start and end): a
// padding end lies above every start, so a search of the tile's ends stops
// at index nt at most, and a padding start meets no interval.
template <int TILE>
__device__ __forceinline__ void pad_tile(uint32_t *ts, uint32_t *te, uint32_t nt, uint32_t lane) {
    for (uint32_t i = nt + lane; i < TILE; i += 64) {
        ts[i] = 0xffffffffu;
        te[i] = 0xffffffffu;
    }
}

// The first entry of the padded tile's ends above `key` (as an address;
// the matching start lies TILE entries below): log2(TILE) fixed rounds, no
// bounds tests, as in the raw batched kernel.
template <int TILE>
__device__ __forceinline__ const uint32_t *tile_first_above(const uint32_t *te, uint32_t key) {
    const uint32_t *p = te;
#pragma unroll
    for (uint32_t S = TILE / 2; S > 0; S >>= 1) p = p[S - 1] <= key ? p + S : p;
    return p;
}

// Decode Y window by window from cursor cy until cy.g reaches `gend` (or the
// list ends), testing every decoded interval against the tile: 1 = an
// overlap, 2 = the decoded intervals have passed the tile's end (nothing
// later can meet it), 0 = neither.
template <int TILE>
__device__ __forceinline__ uint32_t scan_windows(VCursor &cy, uint32_t gend, const uint32_t *te, uint32_t x_lo,
                                                 uint32_t x_hi, uint32_t *ys, uint32_t *ye, uint32_t lane) {
    while (cy.g < gend) {
        wave_lds_sync();
        const uint32_t k = vdecode_window(cy, ys, ye, true, lane);
        wave_lds_sync();
        // a window completes at most 128 intervals: lane l tests intervals l
        // and l + 64, both searches interleaved; one outside [x_lo, x_hi)
        // cannot meet the tile and is empty
        const bool v0 = lane < k, v1 = lane + 64 < k;
        uint32_t s0 = v0 ? ys[lane] : 0u, e0 = v0 ? ye[lane] : 0u;
        uint32_t s1 = v1 ? ys[lane + 64] : 0u, e1 = v1 ? ye[lane + 64] : 0u;
        if (e0 <= x_lo || s0 >= x_hi) e0 = s0 = 0;
        if (e1 <= x_lo || s1 >= x_hi) e1 = s1 = 0;
        const uint32_t *p0 = te, *p1 = te;
#pragma unroll
        for (uint32_t S = TILE / 2; S > 0; S >>= 1) {
            const uint32_t u0 = p0[S - 1], u1 = p1[S - 1];
            p0 = u0 <= s0 ? p0 + S : p0;
            p1 = u1 <= s1 ? p1 + S : p1;
        }
        const bool hit = (p0[-TILE] < e0) || (p1[-TILE] < e1);   // the matching starts
        if (__any(hit)) return 1;
        // every later Y interval starts after this tile ends
        if (k == 0 || ys[k - 1] >= x_hi) return 2;
    }
    return 0;
}

// Does Y (compressed, streamed) overlap the X tile ts/te (0 < nt < TILE
// sorted, disjoint intervals in LDS, padded to TILE entries; te = ts +
// TILE)?  A short Y is decoded from its start.  A longer one is taken block
// by block (64 intervals, whose starts the block index holds): the blocks
// from the last one starting at or before the tile's first start to the
// last one starting below its end are tested against the tile 64 at a time,
// a lane per block (its intervals lie in [its first start, the next
// block's first start), and only a tile interval meeting that range can
// meet one of them), and only the blocks that pass are decoded, window by
// window from their block-index entry (or onward from where the previous
// window stopped).
template <int TILE>
__device__ __forceinline__ bool probe_tile(const uint32_t *ts, const uint32_t *te, uint32_t nt, const ListRef &Y,
                                           uint32_t *ys, uint32_t *ye, uint32_t search_min, uint32_t lane) {
    const uint64_t yb0 = Y.L->boff[Y.obj], yb1 = Y.L->boff[Y.obj + 1];
    const uint64_t yblk = Y.L->blk[Y.obj];
    const uint32_t ynblk = uint32_t(Y.L->blk[Y.obj + 1] - yblk);
    const uint32_t x_lo = ts[0], x_hi = te[nt - 1];
    VCursor cy = vcursor(Y.L->bytes, yb0, yb1, Y.n);
    if (Y.n <= search_min || ynblk <= 1) return scan_windows<TILE>(cy, cy.nvals, te, x_lo, x_hi, ys, ye, lane) == 1;
    const uint32_t *bval = Y.L->bval + yblk, *bpos = Y.L->bpos + yblk;
    uint32_t b0 = first_gt(bval, ynblk, x_lo, lane);
    b0 = b0 ? b0 - 1 : 0;
    const uint32_t b1 = first_gt(bval, ynblk, x_hi - 1, lane);   // the first block starting at or after x_hi
    bool started = false;
    for (uint32_t bb = b0; bb < b1; bb += 64) {
        const uint32_t b = bb + lane;
        bool need = false;
        uint32_t bv = 0, bp = 0;
        if (b < b1) {
            bv = bval[b];
            bp = bpos[b];
            const uint32_t bn = b + 1 < ynblk ? bval[b + 1] : 0xffffffffu;
            need = tile_first_above<TILE>(te, bv)[-TILE] < bn;
        }
        uint64_t mask = __ballot(need);
        while (mask) {
            const uint32_t jl = uint32_t(__builtin_ctzll(mask));
            mask &= mask - 1;
            const uint32_t blk = bb + jl;
            const uint32_t gend = min(cy.nvals, 2 * 64 * (blk + 1));   // values through the block's last end
            if (started && cy.g >= gend) continue;                     // an earlier window decoded it
            if (!started || cy.g < 2 * 64 * blk) {
                cy = vcursor_block(Y.L->bytes, yb0, yb1, Y.n, blk, __builtin_amdgcn_readlane(bv, jl),
                                   __builtin_amdgcn_readlane(bp, jl));
                started = true;
            }
            const uint32_t r = scan_windows<TILE>(cy, gend, te, x_lo, x_hi, ys, ye, lane);
            if (r) return r == 1;
        }
    }
    return false;
}

// Any overlap between list X (compressed, decoded tile by tile into LDS) and
// list Y (compressed, streamed)?
template <int TILE>
__device__ bool cjoin(const ListRef &X, const ListRef &Y, uint32_t *ts, uint32_t *te, uint32_t *ys,
                      uint32_t *ye, uint32_t search_min, uint32_t first_cap, uint32_t lane) {
    if (X.n == 0 || Y.n == 0) return false;
    VCursor cx = cursor_at(X);
    uint32_t cap = first_cap;   // a short first tile: a join that ends early decodes less of X
    while (cx.g < cx.nvals) {
        // fill the tile window by window (a window completes at most 128
        // intervals and may leave one start pending after them)
        uint32_t nt = 0;
        while (cx.g < cx.nvals && nt + 130 <= cap) {
            wave_lds_sync();
            nt += vdecode_window(cx, ts + nt, te + nt, false, lane);
        }
        wave_lds_sync();
        // a start decoded after the tile's last full interval opens the next
        // tile (taken before the padding covers it)
        const uint32_t pend = (cx.g & 1u) ? ts[nt] : 0u;
        wave_lds_sync();
        pad_tile<TILE>(ts, te, nt, lane);
        wave_lds_sync();
        if (nt && probe_tile<TILE>(ts, te, nt, Y, ys, ye, search_min, lane)) return true;
        cap = TILE;
        if (cx.g & 1u) {
            wave_lds_sync();
            if (lane == 0) ts[0] = pend;
        }
    }
    return false;
}

// Which tile of the cached R object the LDS tile holds: (first interval << 1)
// | list (0: A, 1: F), or kNoTile.
constexpr uint32_t kNoTile = 0xffffffffu;

// The same join with X already decoded: nx intervals xs/xe in global memory
// (the wave's decode cache, list `list` of the cached R object), copied into
// LDS a tile at a time unless the LDS tile already holds that tile (*held).
template <int TILE>
__device__ bool rjoin(const uint32_t *xs, const uint32_t *xe, uint32_t nx, uint32_t list, uint32_t *held,
                      const ListRef &Y, uint32_t *ts, uint32_t *te, uint32_t *ys, uint32_t *ye,
                      uint32_t search_min, uint32_t lane) {
    if (nx == 0 || Y.n == 0) return false;
    // tiles of TILE - 1 intervals, so that every tile has a padding entry;
    // any order finds an overlap, so the join starts with the tile LDS
    // already holds (where the previous join on this list stopped) and
    // wraps around
    const uint32_t ntiles = (nx + TILE - 2) / (TILE - 1);
    const uint32_t first = (*held != kNoTile && (*held & 1u) == list) ? (*held >> 1) / (TILE - 1) : 0u;
    for (uint32_t n = 0; n < ntiles; n++) {
        const uint32_t t0 = (first + n < ntiles ? first + n : first + n - ntiles) * (TILE - 1);
        const uint32_t nt = min(uint32_t(TILE - 1), nx - t0);
        const uint32_t key = (t0 << 1) | list;
        if (*held != key) {
            wave_lds_sync();
            for (uint32_t i = lane; i < TILE; i += 64) {
                ts[i] = i < nt ? xs[t0 + i] : 0xffffffffu;
                te[i] = i < nt ? xe[t0 + i] : 0xffffffffu;
            }
            wave_lds_sync();
            *held = key;
        }
        if (probe_tile<TILE>(ts, te, nt, Y, ys, ye, search_min, lane)) return true;
    }
    return false;
}

// Decode a whole list into xs/xe (global memory, room for X.n intervals).
__device__ __forceinline__ void decode_all(const ListRef &X, uint32_t *xs, uint32_t *xe, uint32_t lane) {
    if (X.n == 0) return;
    VCursor c = cursor_at(X);
    while (c.g < c.nvals) {
        const uint32_t got = vdecode_window(c, xs, xe, false, lane);
        xs += got;
        xe += got;
    }
}

template <int TILE>
__global__ __launch_bounds__(kBlock) void k_filter_vbyte(CArgs a) {
    __shared__ uint32_t lds[kWavesPerBlock][2 * TILE + 2 * 132];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = uniform(threadIdx.x >> 6);
    uint32_t *ts = lds[w], *te = ts + TILE, *ys = te + TILE, *ye = ys + 132;
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;
    // this wave's decode cache: R's A-list (cas, cae) and F-list (cfs, cfe)
    const uint32_t cap = a.cache ? a.cache_cap : 0u;
    uint32_t *cas = a.cache + uint64_t(blockIdx.x * kWavesPerBlock + w) * 4 * cap;
    uint32_t *cae = cas + cap, *cfs = cae + cap, *cfe = cfs + cap;
    uint32_t cached = 0xffffffffu;   // the R object whose A-list is held there
    bool cached_f = false;           // its F-list too (decoded when a FA join first needs it)
    uint32_t held = kNoTile;         // its tile in ts/te
    const uint32_t my_xcd = blockIdx.x % a.xcds;
    for (uint32_t k = 0; k < a.xcds; k++) {
        const uint32_t seg = (my_xcd + k) % a.xcds;
        const uint64_t lo = a.n_pairs * seg / a.xcds, hi = a.n_pairs * (seg + 1) / a.xcds;
        if (k > 0 && range_drained(a.xhead, seg, lo, hi, lane)) continue;
        for (;;) {
            unsigned int got = 0;
            if (lane == 0) got = atomicAdd(&a.xhead[seg * kCtrStride], 64u);
            const uint64_t g0 = lo + uniform(__shfl(got, 0));
            if (g0 >= hi) break;
            const uint32_t cnt = uint32_t(min<uint64_t>(64, hi - g0));
            for (uint32_t i = 0; i < cnt; i++) {
                const uint64_t p = g0 + i;
                // the list arrays are read from the argument segment through a
                // pointer the compiler cannot see through, so they hold no
                // scalar registers between their uses
                KArgs *pa = (KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
                asm volatile("" : "+s"(pa));
                const uint32_t r = uniform(a.r[p]), s = uniform(a.s[p]);
                if (r >= a.n_r || s >= a.n_s) {
                    if (lane == 0) a.verdict[p] = APRIL_BAD_PAIR;
                    continue;
                }
                const uint32_t nar = uint32_t(a.Ar.off[r + 1] - a.Ar.off[r]);
                const uint32_t nfr = uint32_t(a.Fr.off[r + 1] - a.Fr.off[r]);
                const uint32_t nas = uint32_t(a.As.off[s + 1] - a.As.off[s]);
                const uint32_t nfs = uint32_t(a.Fs.off[s + 1] - a.Fs.off[s]);
                uint8_t v;
                if (max(nar, nfr) <= cap) {
                    // R from the decode cache (decoded once while consecutive
                    // pairs share it), S streamed
                    if (r != cached) {
                        decode_all(ListRef{&pa->Ar, r, nar}, cas, cae, lane);
                        __threadfence_block();   // the wave's stores, visible to all its lanes
                        cached = r;
                        cached_f = false;
                        held = kNoTile;
                    }
                    const ListRef SA{&pa->As, s, nas}, SF{&pa->Fs, s, nfs};
                    if (!rjoin<TILE>(cas, cae, nar, 0, &held, SA, ts, te, ys, ye, a.search_min, lane)) {
                        v = APRIL_TN;
                    } else if (rjoin<TILE>(cas, cae, nar, 0, &held, SF, ts, te, ys, ye, a.search_min, lane)) {
                        v = APRIL_TH;
                    } else {
                        // the FA join, which few pairs reach: R's F-list is
                        // decoded into the cache on first use
                        if (!cached_f) {
                            decode_all(ListRef{&pa->Fr, r, nfr}, cfs, cfe, lane);
                            __threadfence_block();
                            cached_f = true;
                        }
                        v = rjoin<TILE>(cfs, cfe, nfr, 1, &held, SA, ts, te, ys, ye, a.search_min, lane)
                                ? APRIL_TH
                                : APRIL_INDECISIVE;
                    }
                    if (lane == 0) {
                        a.verdict[p] = v;
                        c_tn += v == APRIL_TN;
                        c_th += v == APRIL_TH;
                        c_ind += v == APRIL_INDECISIVE;
                    }
                    continue;
                }
                const bool xs = max(nas, nfs) < max(nar, nfr);
                const ListRef XA{xs ? &pa->As : &pa->Ar, xs ? s : r, xs ? nas : nar};
                const ListRef XF{xs ? &pa->Fs : &pa->Fr, xs ? s : r, xs ? nfs : nfr};
                const ListRef YA{xs ? &pa->Ar : &pa->As, xs ? r : s, xs ? nar : nas};
                const ListRef YF{xs ? &pa->Fr : &pa->Fs, xs ? r : s, xs ? nfr : nfs};
                held = kNoTile;   // the decoding joins overwrite ts/te
                if (!cjoin<TILE>(XA, YA, ts, te, ys, ye, a.search_min, a.first_cap, lane)) v = APRIL_TN;
                else if (cjoin<TILE>(XA, YF, ts, te, ys, ye, a.search_min, a.first_cap, lane) ||
                         cjoin<TILE>(XF, YA, ts, te, ys, ye, a.search_min, a.first_cap, lane))
                    v = APRIL_TH;
                else v = APRIL_INDECISIVE;
                if (lane == 0) {
                    a.verdict[p] = v;
                    c_tn += v == APRIL_TN;
                    c_th += v == APRIL_TH;
                    c_ind += v == APRIL_INDECISIVE;
                }
            }
        }
    }
    if (a.counts && lane == 0) {
        const unsigned long long v[3] = {c_tn, c_th, c_ind};
        add_totals(a.xhead, blockIdx.x * kWavesPerBlock + w, v, 3);
    }
}


// Alg. 2's data movement on compressed lists, one lane per pair: the joins
// run sequentially as in Alg. 2 (AA; then AF, then FA), each list decoded
// value by value from its start, and the bytes of each list's consumed
// prefix are counted (the longest prefix over the joins that read it).
struct SeqReader {
    const uint8_t *p;
    uint32_t prev;   // last value decoded
    uint32_t left;   // intervals not yet decoded
    uint64_t used;   // bytes consumed
    uint32_t s, e;   // current interval
};

__device__ __forceinline__ uint32_t seq_value(SeqReader &c) {
    uint32_t d = 0, sh = 0, b;
    do {
        b = *c.p++;
        d |= (b & 0x7fu) << sh;
        sh += 7;
        c.used++;
    } while (b & 0x80u);
    c.prev = c.prev + d + 1u;
    return c.prev;
}

__device__ __forceinline__ bool seq_next(SeqReader &c) {
    if (!c.left) return false;
    c.left--;
    c.s = seq_value(c);
    c.e = seq_value(c);
    return true;
}

__device__ __forceinline__ SeqReader seq_open(const CList &L, uint32_t k) {
    SeqReader c;
    c.p = L.bytes + L.boff[k];
    c.prev = 0xffffffffu;
    c.left = uint32_t(L.off[k + 1] - L.off[k]);
    c.used = 0;
    c.s = c.e = 0;
    return c;
}

// IntervalJoin of Alg. 2 on two compressed lists; *bx, *by: bytes of each
// list consumed (the elements read, decoded in order).
__device__ bool seq_join_vbyte(const CList &X, uint32_t kx, const CList &Y, uint32_t ky, uint64_t *bx,
                               uint64_t *by) {
    SeqReader x = seq_open(X, kx), y = seq_open(Y, ky);
    bool found = false;
    if (seq_next(x) && seq_next(y)) {
        for (;;) {
            if (x.s < y.e && y.s < x.e) { found = true; break; }
            if (x.e <= y.e) { if (!seq_next(x)) break; }
            else if (!seq_next(y)) break;
        }
    }
    *bx = x.used;
    *by = y.used;
    return found;
}

__global__ void k_alg2_vbyte_bytes(CArgs a, unsigned long long *bytes) {
    for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < a.n_pairs;
         p += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t r = a.r[p], s = a.s[p];
        if (r >= a.n_r || s >= a.n_s) { bytes[p] = 0; continue; }
        uint64_t bar, bas, bfr = 0, bfs = 0, x, y, lists = 2;
        if (seq_join_vbyte(a.Ar, r, a.As, s, &bar, &bas)) {
            lists++;
            const bool af = seq_join_vbyte(a.Ar, r, a.Fs, s, &x, &bfs);
            bar = max(bar, x);
            if (!af) {
                lists++;
                seq_join_vbyte(a.Fr, r, a.As, s, &bfr, &y);
                bas = max(bas, y);
            }
        }
        bytes[p] = 8ull + 16ull * lists + bar + bas + bfr + bfs + 1ull;
    }
}

// One wave per list: decode it whole into raw start/end arrays.
__global__ __launch_bounds__(256) void k_decode_lists(const uint8_t *bytes, const uint64_t *boff,
                                                      const uint64_t *off, uint64_t n, uint32_t *out_s,
                                                      uint32_t *out_e) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t waves = uint64_t(gridDim.x) * (blockDim.x / 64);
    for (uint64_t k = uint64_t(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6); k < n; k += waves) {
        const uint32_t cnt = uint32_t(off[k + 1] - off[k]);
        VCursor c = vcursor(bytes, boff[k], boff[k + 1], cnt);
        uint32_t *s = out_s + off[k], *e = out_e + off[k];
        while (c.g < c.nvals) {
            const uint32_t got = vdecode_window(c, s, e, false, lane);
            s += got;
            e += got;
        }
    }
}

CList clist(const april_lists_t *L, bool f) {
    CList c;
    c.off = f ? L->d.off_f : L->d.off_a;
    c.boff = f ? L->d.boff_f : L->d.boff_a;
    c.blk = f ? L->d.blk_f : L->d.blk_a;
    c.bytes = f ? L->d.bytes_f : L->d.bytes_a;
    c.bval = f ? L->d.bval_f : L->d.bval_a;
    c.bpos = f ? L->d.bpos_f : L->d.bpos_a;
    return c;
}

}  // namespace

uint64_t vbyte_workspace_bytes() { return kCtrBytes; }

// Intervals per list in a wave's decode cache (R objects with longer lists
// decode per pair): 4 lists x 4 B x 4096 = 64 KiB per wave.
constexpr uint32_t kCacheCap = 4096;
// Blocks of the compressed filter's grid per CU.
constexpr uint64_t kVbyteBlocksPerCu = 8;

uint64_t vbyte_cache_bytes(int cus) {
    return uint64_t(cus) * kVbyteBlocksPerCu * kWavesPerBlock * 4ull * kCacheCap * sizeof(uint32_t);
}

// the counters first, the cache 256-byte aligned after them
uint64_t vbyte_cache_offset() { return (kCtrBytes + 255) & ~uint64_t(255); }

int launch_filter_vbyte(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r, const uint32_t *d_s,
                        uint64_t n_pairs, uint8_t *d_verdict, unsigned long long *counts,
                        const april_filter_opts_t &o, int cus, void *workspace, hipStream_t stream) {
    CArgs a;
    a.Ar = clist(R, false);
    a.Fr = clist(R, true);
    a.As = clist(S, false);
    a.Fs = clist(S, true);
    a.r = d_r;
    a.s = d_s;
    a.n_pairs = n_pairs;
    a.n_r = R->n;
    a.n_s = S->n;
    a.verdict = d_verdict;
    a.counts = counts;
    a.xhead = static_cast<unsigned int *>(workspace);
    a.xcds = uint32_t(xcd_count(cus));
    // S is searched from its block index for each tile of R whenever it
    // spans more than one block (R's tiles come from the decode cache, so S
    // may be the shorter side)
    a.search_min = o.search_min ? o.search_min : 64;
    k_zero_ctrs<<<1, 64, 0, stream>>>(a.xhead);
    APRIL_HIP_TRY(hipGetLastError());
    const uint32_t tile = o.tile ? o.tile : 512;
    // chunk: windows (up to 130 intervals each) in a join's first tile
    if (o.chunk > 4) return fail(APRIL_E_INVALID, "compressed lists: chunk must be 0 to 4");
    // (one by default: most joins of overlapping objects end within it)
    a.first_cap = std::min<uint32_t>(tile, 130u * (o.chunk ? o.chunk : 1u));
    const uint64_t blocks = uint64_t(cus) * kVbyteBlocksPerCu;
    // decode cache: cache_cap intervals per list for every wave of the grid,
    // from the caller's workspace (APRIL_WS_DECODE_CACHE) or stream-ordered;
    // without one (allocation refused) every pair decodes both objects
    a.cache_cap = kCacheCap;
    a.cache = nullptr;
    const uint64_t cache_bytes = vbyte_cache_bytes(cus);
    bool own_cache = false;
    if (o.flags & APRIL_WS_DECODE_CACHE) {
        if (!o.d_workspace || o.workspace_bytes < vbyte_cache_offset() + cache_bytes)
            return fail(APRIL_E_INVALID, "workspace too small for the decode cache");
        a.cache = reinterpret_cast<uint32_t *>(static_cast<char *>(o.d_workspace) + vbyte_cache_offset());
    } else if (hipMallocAsync(reinterpret_cast<void **>(&a.cache), cache_bytes, stream) == hipSuccess) {
        own_cache = true;
    } else {
        (void)hipGetLastError();
        a.cache = nullptr;
    }
    switch (tile) {
        case 256: k_filter_vbyte<256><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(a); break;
        case 512: k_filter_vbyte<512><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(a); break;
        case 1024: k_filter_vbyte<1024><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(a); break;
        default:
            if (own_cache) (void)hipFreeAsync(a.cache, stream);
            return fail(APRIL_E_INVALID, "compressed lists: tile must be 256, 512 or 1024");
    }
    const hipError_t e = hipGetLastError();
    if (own_cache) APRIL_HIP_TRY(hipFreeAsync(a.cache, stream));
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("compressed filter launch: ") + hipGetErrorString(e));
    if (counts) {
        k_sum_totals<<<1, 64, 0, stream>>>(a.xhead, counts, 3);
        APRIL_HIP_TRY(hipGetLastError());
    }
    return APRIL_OK;
}

int launch_alg2_vbyte_bytes(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                            const uint32_t *d_s, uint64_t n_pairs, unsigned long long *d_bytes, int cus,
                            hipStream_t stream) {
    CArgs a{};
    a.Ar = clist(R, false);
    a.Fr = clist(R, true);
    a.As = clist(S, false);
    a.Fs = clist(S, true);
    a.r = d_r;
    a.s = d_s;
    a.n_pairs = n_pairs;
    a.n_r = R->n;
    a.n_s = S->n;
    const uint64_t blocks = std::min<uint64_t>((n_pairs + 255) / 256, uint64_t(cus) * 16);
    k_alg2_vbyte_bytes<<<dim3(uint32_t(blocks)), dim3(256), 0, stream>>>(a, d_bytes);
    APRIL_HIP_TRY(hipGetLastError());
    return APRIL_OK;
}

int launch_decode_lists(const april_lists_t *L, bool f, uint32_t *out_s, uint32_t *out_e, hipStream_t stream) {
    const uint64_t n = L->n;
    if (n == 0) return APRIL_OK;
    const uint64_t blocks = std::min<uint64_t>((n + 3) / 4, 65535);
    k_decode_lists<<<dim3(uint32_t(blocks)), dim3(256), 0, stream>>>(f ? L->d.bytes_f : L->d.bytes_a,
                                                                    f ? L->d.boff_f : L->d.boff_a,
                                                                    f ? L->d.off_f : L->d.off_a, n, out_s, out_e);
    APRIL_HIP_TRY(hipGetLastError());
    return APRIL_OK;
}

}  // namespace april
