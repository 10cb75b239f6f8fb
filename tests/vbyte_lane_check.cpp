// Host check of the device VByte decoder's per-lane arithmetic
// (vdecode_lane): one wave of 64 lanes is emulated on the CPU over random
// lists, encoded here from the format's definition (delta + VByte, Sec. 5.1:
// values s0 < e0 < s1 < ..., each stored as value - previous - 1 in 7-bit
// groups, low group first, high bit set on all but the last byte), and the
// decoded values must equal the encoded ones.  Lanes are combined as the
// device does: running counts and sums over lanes give each value's index
// and absolute value, and the next window starts after the last value that
// started in this one.  Exit status 0 iff every value matches.
#include "vbyte.hpp"

#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

using april::LaneVals;
using april::vdecode_lane;

int main() {
    std::mt19937_64 rng(5);
    long bad = 0, lists = 0, vals = 0;
    for (int trial = 0; trial < 2000; trial++) {
        const int n = 1 + int(rng() % (trial < 1000 ? 300 : 3000));
        const int spread = trial % 4;   // gaps: 1-3, up to 300, up to 1e5, up to 3e7
        std::vector<uint32_t> v;
        uint64_t cur = rng() % 1000;
        for (int i = 0; i < 2 * n; i++) {
            uint64_t gap = 1 + (spread == 0   ? rng() % 3
                                : spread == 1 ? rng() % 300
                                : spread == 2 ? rng() % 100000
                                              : rng() % 30000000);
            if (trial % 97 == 0 && i == 0) gap = 0xfffff000u;   // five-byte values near 2^32
            if (cur + gap >= 0xffffffffull) break;
            cur += gap;
            v.push_back(uint32_t(cur));
        }
        if (v.size() % 2) v.pop_back();
        if (v.empty()) continue;
        std::vector<uint8_t> by;
        const size_t lead = rng() % 4;   // the stream starts 0-3 bytes into a word
        for (size_t i = 0; i < lead; i++) by.push_back(uint8_t(0x80 | (rng() & 0x7f)));
        uint32_t prev = 0xffffffffu;
        for (uint32_t x : v) {
            uint32_t d = x - prev - 1u;
            while (d >= 0x80u) {
                by.push_back(uint8_t(d | 0x80u));
                d >>= 7;
            }
            by.push_back(uint8_t(d));
            prev = x;
        }
        const uint32_t nbytes = uint32_t(by.size() - lead);
        for (int i = 0; i < 600; i++) by.push_back(uint8_t(rng()));   // whatever follows the stream
        uint32_t pos = 0, pv = 0xffffffffu, g = 0;
        const uint32_t nv = uint32_t(v.size());
        std::vector<uint32_t> out(v.size() + 600, 0xdeadbeefu);
        while (g < nv) {
            const size_t p = lead + pos, a = p & ~size_t(3);
            const uint32_t skip = uint32_t(p - a);
            uint32_t W[65];
            for (int l = 0; l < 65; l++) memcpy(&W[l], by.data() + a + 4 * l, 4);
            const uint32_t avail = nbytes - pos;
            uint32_t before_vals = 0, before_sum = 0, end_byte = 0;
            for (uint32_t l = 0; l < 64; l++) {
                const LaneVals L = vdecode_lane(W[l], W[l + 1], l ? W[l - 1] : 0u, l, skip,
                                                skip + (avail < 512u ? avail : 512u));
                for (int k = 0; k < 4; k++)
                    if ((L.starts >> k) & 1u) {
                        const uint32_t gv = g + before_vals + uint32_t(__builtin_popcount(L.starts & ((1u << k) - 1u)));
                        if (gv < out.size()) out[gv] = pv + before_sum + L.cum[k];
                        else bad++;
                    }
                before_vals += L.nval;
                before_sum += L.local;
                if (L.nval) end_byte = L.last_end + 1;
            }
            if (before_vals == 0) {   // no progress
                bad++;
                break;
            }
            pos += end_byte - skip;
            pv += before_sum;
            g += before_vals;
        }
        lists++;
        bad += g != nv;
        for (uint32_t i = 0; i < nv; i++) bad += out[i] != v[i];
        vals += nv;
    }
    printf("vdecode_lane: %ld lists, %ld values, %ld mismatches\n", lists, vals, bad);
    return bad ? 1 : 0;
}
