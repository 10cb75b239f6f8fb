// Wave-cooperative decoding of delta + VByte interval lists (Sec. 5.1).
//
// A list's stream holds the values s_0 < e_0 < s_1 < e_1 < ... as
// varint(v_t - v_{t-1} - 1) with v_{-1} = 2^32 - 1 (so the first value is
// stored as itself), 7 bits per byte, low bits first, high bit set on all but
// a value's last byte.  A wave decodes the stream in aligned 256-byte
// windows: lane l holds the window's word l and sees word l+1, so every value
// that starts in its four bytes (at most 5 bytes long) lies in its 8-byte
// view.  A byte starts a value when the byte before it ends one; the number
// of values before a lane (wave prefix sum) and the running sum of
// (delta + 1) give every value's index and absolute value; values with even
// index are starts, odd ones ends.  The next window begins right after the
// last value that started in this one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace april {

typedef const __attribute__((address_space(1))) uint32_t *GWords;   // global memory

// Decoder state of one list (wave-uniform, but for the prefetched words).
struct VCursor {
    const uint8_t *base;   // the list's stream
    uint32_t nbytes;       // stream length
    uint32_t nvals;        // 2 x intervals
    uint32_t pos;          // first byte of the next value
    uint32_t prev;         // last absolute value decoded
    uint32_t g;            // values decoded so far
    // The aligned 256 bytes that follow the window being decoded, loaded
    // while it is decoded: lane l holds word l of the block at byte pfo of
    // the stream, lane 63 also words 64 and 65.  The next window starts at
    // pfo or pfo + 4, so its words are these.  Window starts are aligned
    // addresses, all congruent mod 4 as stream offsets: a pfo of another
    // residue marks that nothing is loaded.
    uint32_t pfo;
    uint32_t pw, px0, px1;
};

// Cross-lane steps on DPP (VALU operand routing, no trip through the LDS
// unit): every lane of the wave must be active.
//
// Inclusive prefix sum over the wave: a scan within each row of 16 lanes by
// shifts of 1, 2, 4 and 8 lanes (lanes shifted in from outside the row read
// 0), then lane 15 of a row added to the row above it (rows 1 and 3), and
// lane 31 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, true);    // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, true);    // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, true);    // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, true);    // row_shr:8
    x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return x;
}

// Lane l receives lane l - 1's value (lane 0 receives 0).
__device__ __forceinline__ uint32_t from_lane_below(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xf, 0xf, false);   // wave_shr:1
}

// Lane l receives lane l + 1's value (lane 63 receives 0).
__device__ __forceinline__ uint32_t from_lane_above(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xf, 0xf, false);   // wave_shl:1
}

// Cursor at interval 0 of a list.
__device__ __forceinline__ VCursor vcursor(const uint8_t *bytes, uint64_t b0, uint64_t b1, uint32_t n) {
    VCursor c;
    c.base = bytes + b0;
    c.nbytes = uint32_t(b1 - b0);
    c.nvals = 2 * n;
    c.pos = 0;
    c.prev = 0xffffffffu;
    c.g = 0;
    c.pfo = 1u - uint32_t(reinterpret_cast<uintptr_t>(c.base) & 3u);   // no window starts there
    c.pw = c.px0 = c.px1 = 0u;
    return c;
}

// Cursor at interval 64*b of a list (block entry b): its start is known,
// decoding resumes at its end.
__device__ __forceinline__ VCursor vcursor_block(const uint8_t *bytes, uint64_t b0, uint64_t b1, uint32_t n,
                                                 uint32_t blk, uint32_t bval, uint32_t bpos) {
    VCursor c = vcursor(bytes, b0, b1, n);
    c.pos = bpos;
    c.prev = bval;
    c.g = 2 * 64 * blk + 1;
    return c;
}

// The values that start in one lane's four bytes of a window.
struct LaneVals {
    uint32_t starts;     // bit k: a value starts at byte k of the lane's word
    uint32_t nval;       // number of such values
    uint32_t local;      // sum of (delta + 1) over them
    uint32_t last_end;   // window byte of the last one's last byte
    uint32_t cum[4];     // cum[k]: the running sum up to and including byte k's value
};

// Per-lane part of a window's decoding, branch-free arithmetic (also built
// for the host).  w is the lane's word (window bytes 4 lane .. 4 lane + 3),
// wn the next word and wprev the one before; the window's values start at
// window byte `first` and the stream ends before window byte `stop`.
__host__ __device__ __forceinline__ LaneVals vdecode_lane(uint32_t w, uint32_t wn, uint32_t wprev, uint32_t lane,
                                                          uint32_t first, uint32_t stop) {
    const uint64_t x = uint64_t(w) | (uint64_t(wn) << 32);
    // bit 8k + 7: byte k - 1 (for k = 0, byte 3 of the word before) has its
    // high bit clear, i.e. ends a value, so byte k starts one
    const uint32_t after_end = ((~w & 0x80808080u) << 8) | ((~wprev & 0x80000000u) >> 24);
    LaneVals r{0u, 0u, 0u, 0u, {0u, 0u, 0u, 0u}};
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t b = 4 * lane + uint32_t(k);
        const bool st = (b >= first) & (b < stop) & ((b == first) | bool((after_end >> (8 * k + 7)) & 1u));
        // the value at byte k: 7-bit groups of bytes k .. k + 4, low group
        // first, cut after its first byte with the high bit clear (byte t)
        const uint32_t y = uint32_t(x >> (8 * k));
        const uint32_t y4 = uint32_t(x >> (8 * k + 32)) & 0xffu;
        uint32_t v = (y & 0x7fu) | ((y >> 1) & 0x3f80u) | ((y >> 2) & 0x1fc000u) | ((y >> 3) & 0xfe00000u) |
                     (y4 << 28);
        const uint32_t term = ~y & 0x80808080u;
        const uint32_t t = term ? uint32_t(__builtin_ctz(term)) >> 3 : 4u;
        if (t < 4) v &= (1u << (7 * t + 7)) - 1u;
        // selects, not branches: every byte position is worked out
        r.local += st ? v + 1u : 0u;
        r.cum[k] = r.local;
        r.last_end = st ? b + t : r.last_end;
        r.starts |= uint32_t(st) << k;
        r.nval += uint32_t(st);
    }
    return r;
}

// Decode one window.  Interval t of the window (t = 0 is the interval whose
// start was pending, if any) goes to (bs[t], be[t]); returns the number of
// intervals completed, k (their ends are all written).  The start of the
// pending interval k (if the window ends on a start) is written to bs[k].
// With `write_pending` the pending start carried in from the previous window
// is written to bs[0] (needed when bs is reused; not when the caller
// advances bs by k between windows).  bs/be must hold 130 entries.
//
// Unless the stream ends within the window, the last value that starts in
// its 256 bytes ends at window byte 256 to 260, so the next window begins at
// byte 256 or 260 of this one: the call loads those bytes for the next call
// before it decodes, and the next call finds its words already in registers
// (the loads stay within the 512 bytes that follow a stream's end).
__device__ __forceinline__ uint32_t vdecode_window(VCursor &c, uint32_t *bs, uint32_t *be, bool write_pending,
                                                   uint32_t lane) {
    if (c.g >= c.nvals) return 0;
    const uint8_t *p = c.base + c.pos;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p) & ~uintptr_t(3);
    const uint32_t skip = uint32_t(reinterpret_cast<uintptr_t>(p) - a);     // bytes before the value start
    const uint32_t *wp = reinterpret_cast<const uint32_t *>(a);
    const GWords gw = (GWords)wp;
    const uint32_t wofs = c.pos - skip;   // the window's stream offset
    uint32_t w, wn;
    if (wofs == c.pfo) {
        w = c.pw;
        wn = from_lane_above(w);
        if (lane == 63) wn = c.px0;
    } else if (wofs == c.pfo + 4u) {
        w = from_lane_above(c.pw);
        if (lane == 63) w = c.px0;
        wn = from_lane_above(w);
        if (lane == 63) wn = c.px1;
    } else {
        w = gw[lane];
        wn = from_lane_above(w);
        if (lane == 63) wn = gw[64];
    }
    // a window spans 256 bytes (+4 seen by lane 63)
    const uint32_t avail = c.nbytes - c.pos;
    const uint32_t wprev = from_lane_below(w);
    const LaneVals L = vdecode_lane(w, wn, wprev, lane, skip, skip + (avail < 512u ? avail : 512u));
    // issued once w and wn are in registers (the empty asm takes them, and
    // no memory access moves across it), so that no wait for them waits
    // for these loads too
    asm volatile("" ::"v"(w), "v"(wn) : "memory");
    if (avail > 260u) {
        c.pfo = wofs + 256u;
        c.pw = gw[64 + lane];
        if (lane == 63) {
            c.px0 = gw[128];
            c.px1 = gw[129];
        }
    } else {
        c.pfo = wofs + 1u;
    }
    const uint32_t inc_vals = wave_incl_scan(L.nval), inc_sum = wave_incl_scan(L.local);
    const uint32_t before_vals = inc_vals - L.nval, before_sum = inc_sum - L.local;
    const uint32_t V = __builtin_amdgcn_readlane(inc_vals, 63);
    const uint32_t total = __builtin_amdgcn_readlane(inc_sum, 63);
    const uint32_t g0 = c.g, i0 = g0 >> 1;
    if (write_pending && lane == 0 && (g0 & 1u)) bs[0] = c.prev;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((L.starts >> k) & 1u) {
            const uint32_t gv = g0 + before_vals + uint32_t(__builtin_popcount(L.starts & ((1u << k) - 1u)));
            const uint32_t absv = c.prev + before_sum + L.cum[k];
            const uint32_t i = (gv >> 1) - i0;
            if (gv & 1u) be[i] = absv;
            else bs[i] = absv;
        }
    }
    // one past the window byte where the last value ends: values in higher
    // lanes end later, so the highest lane holding a value has it
    const uint64_t holds = __ballot(L.nval != 0);
    const uint32_t end_byte =
        holds ? __builtin_amdgcn_readlane(L.last_end + 1, 63 - __builtin_clzll(holds)) : 0u;   // window-relative
    c.pos += end_byte - skip;
    c.prev += total;
    c.g += V;
    return ((g0 + V) >> 1) - i0;
}

}  // namespace april
