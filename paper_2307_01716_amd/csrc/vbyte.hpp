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

// Wave-uniform decoder state of one list.
struct VCursor {
    const uint8_t *base;   // the list's stream
    uint32_t nbytes;       // stream length
    uint32_t nvals;        // 2 x intervals
    uint32_t pos;          // first byte of the next value
    uint32_t prev;         // last absolute value decoded
    uint32_t g;            // values decoded so far
};

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t lane) {
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= uint32_t(d)) x += y;
    }
    return x - v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d));
    return v;
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

// Decode one window.  Interval t of the window (t = 0 is the interval whose
// start was pending, if any) goes to (bs[t], be[t]); returns the number of
// intervals completed, k (their ends are all written).  The start of the
// pending interval k (if the window ends on a start) is written to bs[k].
// With `write_pending` the pending start carried in from the previous window
// is written to bs[0] (needed when bs is reused; not when the caller
// advances bs by k between windows).  bs/be must hold 130 entries.
__device__ __forceinline__ uint32_t vdecode_window(VCursor &c, uint32_t *bs, uint32_t *be, bool write_pending,
                                                   uint32_t lane) {
    if (c.g >= c.nvals) return 0;
    const uint8_t *p = c.base + c.pos;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p) & ~uintptr_t(3);
    const uint32_t skip = uint32_t(reinterpret_cast<uintptr_t>(p) - a);     // bytes before the value start
    const uint32_t *wp = reinterpret_cast<const uint32_t *>(a);
    const uint32_t w = wp[lane];
    uint32_t wn = __shfl_down(w, 1);
    if (lane == 63) wn = wp[64];
    const uint32_t wprev = __shfl_up(w, 1);
    const uint64_t x = uint64_t(w) | (uint64_t(wn) << 32);
    // byte positions relative to the value start p: 4*lane + k - skip
    uint32_t starts = 0;   // bit k: a value starts at byte k of this lane's word
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int rel = int(4 * lane + k) - int(skip);
        const bool valid = rel >= 0 && uint32_t(rel) < c.nbytes - c.pos;
        uint32_t before;
        if (k > 0) before = (w >> (8 * (k - 1))) & 0xffu;
        else before = (wprev >> 24) & 0xffu;
        const bool st = valid && (rel == 0 || before < 0x80u);
        starts |= uint32_t(st) << k;
    }
    // decode the values that start here
    uint32_t vals[4], nval = 0, last_end = 0, local = 0;
    uint32_t cum[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        if ((starts >> k) & 1u) {
            uint32_t v = 0, t = 0;
#pragma unroll
            for (int u = 0; u < 5; u++) {
                const uint32_t b = uint32_t(x >> (8 * (k + u))) & 0xffu;
                if (u == t) {
                    v |= (b & 0x7fu) << (7 * u);
                    if (b >= 0x80u) t++;
                }
            }
            last_end = 4 * lane + k + t;     // window byte of the value's last byte
            local += v + 1u;
            vals[nval] = v;
            cum[nval] = local;
            nval++;
        }
    }
    (void)vals;
    const uint32_t before_vals = wave_excl_scan(nval, lane);
    const uint32_t V = wave_sum(nval);
    const uint32_t before_sum = wave_excl_scan(local, lane);
    const uint32_t total = wave_sum(local);
    const uint32_t g0 = c.g, i0 = g0 >> 1;
    if (write_pending && lane == 0 && (g0 & 1u)) bs[0] = c.prev;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        if (uint32_t(j) < nval) {
            const uint32_t gv = g0 + before_vals + j;
            const uint32_t absv = c.prev + before_sum + cum[j];
            const uint32_t i = (gv >> 1) - i0;
            if (gv & 1u) be[i] = absv;
            else bs[i] = absv;
        }
    }
    const uint32_t end_byte = wave_max(nval ? last_end + 1 : 0u);   // window-relative
    c.pos += end_byte - skip;
    c.prev += total;
    c.g += V;
    return ((g0 + V) >> 1) - i0;
}

}  // namespace april
