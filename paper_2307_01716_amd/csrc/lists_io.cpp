// List files: host lists saved to and loaded from a versioned binary file
// sealed with a SHA-256 digest, so a collection's approximations are built
// once and reused (the paper precomputes and stores the A- and F-lists,
// Sec. 4.1 and Sec. 6).
//
// Layout (little-endian, no padding):
//   off  size  field
//     0     8  magic "APRILLST"
//     8     4  version (1)
//    12     4  header bytes (88)
//    16    24  grid x0, y0, side (float64)
//    40     4  grid order (uint32)
//    44     4  grid flags (uint32)
//    48     8  partition key (uint64; 0 for one grid)
//    56     8  n objects
//    64     8  n A intervals
//    72     8  n F intervals
//    80     8  reserved, 0
//    88        off_a[n+1] u64, start_a[n_a] u32, end_a[n_a] u32,
//              off_f[n+1] u64, start_f[n_f] u32, end_f[n_f] u32
//   end-32 32  SHA-256 of every byte before it
//
// SHA-256 follows FIPS 180-4 (message padding, the 64-word schedule, 64
// rounds per 512-bit block).  Its constants are defined there as the first
// 32 fractional bits of the square roots (initial hash) and cube roots
// (round constants) of the first primes; they are derived here from that
// definition with exact integer roots instead of being tabulated.
#include <sys/stat.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.hpp"

static_assert(__BYTE_ORDER__ == __ORDER_LITTLE_ENDIAN__, "list files are written little-endian");

namespace april {
namespace {

constexpr char kMagic[8] = {'A', 'P', 'R', 'I', 'L', 'L', 'S', 'T'};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 88;

// ------------------------------------------------------------- SHA-256

typedef unsigned __int128 u128;

// floor(p^(1/k) * 2^32) for k = 2 or 3, exactly: the largest m with
// m^k <= p * 2^(32k), found from a floating-point estimate by stepping.
uint64_t root_bits(uint64_t p, int k) {
    const u128 target = u128(p) << (32 * k);
    auto pw = [k](u128 m) { return k == 2 ? m * m : m * m * m; };
    long double est = (k == 2 ? sqrtl((long double)p) : cbrtl((long double)p)) * 4294967296.0L;
    u128 m = u128(est);
    while (pw(m) > target) m--;
    while (pw(m + 1) <= target) m++;
    return uint64_t(m);
}

struct Constants {
    uint32_t k[64], h0[8];
    Constants() {
        uint32_t primes[64];
        int n = 0;
        for (uint32_t c = 2; n < 64; c++) {
            bool prime = true;
            for (int i = 0; i < n && primes[i] * primes[i] <= c; i++)
                if (c % primes[i] == 0) { prime = false; break; }
            if (prime) primes[n++] = c;
        }
        for (int i = 0; i < 64; i++) k[i] = uint32_t(root_bits(primes[i], 3));   // low 32 bits = fraction
        for (int i = 0; i < 8; i++) h0[i] = uint32_t(root_bits(primes[i], 2));
    }
};

const Constants &constants() {
    static const Constants c;
    return c;
}

inline uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

class Sha256 {
  public:
    Sha256() : c_(constants()) { std::memcpy(h_, c_.h0, sizeof h_); }

    void update(const void *data, size_t len) {
        const uint8_t *p = static_cast<const uint8_t *>(data);
        total_ += len;
        if (fill_) {
            size_t take = std::min(len, size_t(64) - fill_);
            std::memcpy(buf_ + fill_, p, take);
            fill_ += take; p += take; len -= take;
            if (fill_ < 64) return;
            block(buf_);
            fill_ = 0;
        }
        for (; len >= 64; p += 64, len -= 64) block(p);
        std::memcpy(buf_, p, len);
        fill_ = len;
    }

    void finish(uint8_t out[32]) {
        const uint64_t bits = total_ * 8;
        uint8_t pad[72] = {0x80};
        size_t npad = (fill_ < 56 ? 56 : 120) - fill_;
        for (int i = 0; i < 8; i++) pad[npad + i] = uint8_t(bits >> (56 - 8 * i));
        update(pad, npad + 8);
        for (int i = 0; i < 8; i++)
            for (int b = 0; b < 4; b++) out[4 * i + b] = uint8_t(h_[i] >> (24 - 8 * b));
    }

  private:
    void block(const uint8_t *m) {
        uint32_t w[64];
        for (int t = 0; t < 16; t++)
            w[t] = uint32_t(m[4 * t]) << 24 | uint32_t(m[4 * t + 1]) << 16 | uint32_t(m[4 * t + 2]) << 8 |
                   uint32_t(m[4 * t + 3]);
        for (int t = 16; t < 64; t++) {
            uint32_t s0 = rotr(w[t - 15], 7) ^ rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
            uint32_t s1 = rotr(w[t - 2], 17) ^ rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
            w[t] = s1 + w[t - 7] + s0 + w[t - 16];
        }
        uint32_t a = h_[0], b = h_[1], c = h_[2], d = h_[3], e = h_[4], f = h_[5], g = h_[6], h = h_[7];
        for (int t = 0; t < 64; t++) {
            uint32_t t1 = h + (rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25)) + ((e & f) ^ (~e & g)) + c_.k[t] + w[t];
            uint32_t t2 = (rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22)) + ((a & b) ^ (a & c) ^ (b & c));
            h = g; g = f; f = e; e = d + t1;
            d = c; c = b; b = a; a = t1 + t2;
        }
        h_[0] += a; h_[1] += b; h_[2] += c; h_[3] += d;
        h_[4] += e; h_[5] += f; h_[6] += g; h_[7] += h;
    }

    const Constants &c_;
    uint32_t h_[8];
    uint8_t buf_[64];
    size_t fill_ = 0;
    uint64_t total_ = 0;
};

// --------------------------------------------------------------- files

struct Writer {
    FILE *f;
    Sha256 sha;
    bool ok = true;
    void put(const void *p, size_t n) {
        if (!n) return;
        sha.update(p, n);
        ok = ok && std::fwrite(p, 1, n, f) == n;
    }
};

struct Reader {
    FILE *f;
    Sha256 sha;
    bool get(void *p, size_t n) {
        if (!n) return true;
        if (std::fread(p, 1, n, f) != n) return false;
        sha.update(p, n);
        return true;
    }
};

template <class T> void put_le(uint8_t *dst, T v) { std::memcpy(dst, &v, sizeof v); }
template <class T> T get_le(const uint8_t *src) {
    T v;
    std::memcpy(&v, src, sizeof v);
    return v;
}

}  // namespace
}  // namespace april

using namespace april;

extern "C" {

int april_lists_save(const april_lists_t *L, const char *path) {
    clear_error();
    if (!L || !path) return fail(APRIL_E_INVALID, "NULL argument");
    if (L->device >= 0) return fail(APRIL_E_INVALID, "save needs host lists (download device lists first)");
    uint8_t hdr[kHeaderBytes] = {};
    std::memcpy(hdr, kMagic, 8);
    put_le<uint32_t>(hdr + 8, kVersion);
    put_le<uint32_t>(hdr + 12, kHeaderBytes);
    put_le<double>(hdr + 16, L->grid.x0);
    put_le<double>(hdr + 24, L->grid.y0);
    put_le<double>(hdr + 32, L->grid.side);
    put_le<uint32_t>(hdr + 40, L->grid.order);
    put_le<uint32_t>(hdr + 44, L->grid.flags);
    put_le<uint64_t>(hdr + 48, L->partition_key);
    put_le<uint64_t>(hdr + 56, L->n);
    put_le<uint64_t>(hdr + 64, L->n_a);
    put_le<uint64_t>(hdr + 72, L->n_f);

    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(APRIL_E_IO, "cannot create " + tmp + ": " + std::strerror(errno));
    Writer w{f};
    w.put(hdr, sizeof hdr);
    w.put(L->off_a.data(), L->off_a.size() * 8);
    w.put(L->start_a.data(), L->start_a.size() * 4);
    w.put(L->end_a.data(), L->end_a.size() * 4);
    w.put(L->off_f.data(), L->off_f.size() * 8);
    w.put(L->start_f.data(), L->start_f.size() * 4);
    w.put(L->end_f.data(), L->end_f.size() * 4);
    uint8_t digest[32];
    w.sha.finish(digest);
    bool ok = w.ok && std::fwrite(digest, 1, 32, f) == 32;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(APRIL_E_IO, std::string("cannot write ") + path + ": " + std::strerror(errno));
    }
    return APRIL_OK;
}

int april_lists_load(const char *path, int validate, april_lists_t **out) {
    clear_error();
    if (!path || !out) return fail(APRIL_E_INVALID, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(APRIL_E_IO, std::string("cannot open ") + path + ": " + std::strerror(errno));
    struct stat st;
    if (fstat(fileno(f), &st) != 0) {
        std::fclose(f);
        return fail(APRIL_E_IO, std::string("cannot stat ") + path);
    }
    const uint64_t size = uint64_t(st.st_size);
    auto corrupt = [&](const std::string &why) {
        std::fclose(f);
        return fail(APRIL_E_CORRUPT, std::string(path) + ": " + why);
    };
    Reader r{f};
    uint8_t hdr[kHeaderBytes];
    if (size < kHeaderBytes + 32 || !r.get(hdr, sizeof hdr)) return corrupt("shorter than a header");
    if (std::memcmp(hdr, kMagic, 8) != 0) return corrupt("not a list file");
    if (get_le<uint32_t>(hdr + 8) != kVersion) return corrupt("unsupported version");
    if (get_le<uint32_t>(hdr + 12) != kHeaderBytes || get_le<uint64_t>(hdr + 80) != 0)
        return corrupt("bad header");
    april_grid_t grid{get_le<double>(hdr + 16), get_le<double>(hdr + 24), get_le<double>(hdr + 32),
                      get_le<uint32_t>(hdr + 40), get_le<uint32_t>(hdr + 44)};
    const uint64_t key = get_le<uint64_t>(hdr + 48), n = get_le<uint64_t>(hdr + 56),
                   na = get_le<uint64_t>(hdr + 64), nf = get_le<uint64_t>(hdr + 72);
    // every count is bounded by the file size before it sizes anything
    if (n >= size / 16 || na >= size / 8 || nf >= size / 8 ||
        kHeaderBytes + 16 * (n + 1) + 8 * (na + nf) + 32 != size)
        return corrupt("size does not match the header");

    auto *L = new (std::nothrow) april_lists;
    if (!L) {
        std::fclose(f);
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    try {
        L->off_a.resize(n + 1); L->off_f.resize(n + 1);
        L->start_a.resize(na); L->end_a.resize(na);
        L->start_f.resize(nf); L->end_f.resize(nf);
    } catch (...) {
        delete L;
        std::fclose(f);
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    uint8_t digest[32], stored[32];
    bool ok = r.get(L->off_a.data(), (n + 1) * 8) && r.get(L->start_a.data(), na * 4) &&
              r.get(L->end_a.data(), na * 4) && r.get(L->off_f.data(), (n + 1) * 8) &&
              r.get(L->start_f.data(), nf * 4) && r.get(L->end_f.data(), nf * 4);
    ok = ok && std::fread(stored, 1, 32, f) == 32;
    if (!ok) {
        delete L;
        return corrupt("short read");
    }
    r.sha.finish(digest);
    if (std::memcmp(digest, stored, 32) != 0) {
        delete L;
        return corrupt("SHA-256 mismatch");
    }
    std::fclose(f);
    LatticeGrid lg;
    int rc = lattice_grid(&grid, &lg);
    if (!rc && (L->off_a[n] != na || L->off_f[n] != nf)) rc = fail(APRIL_E_CORRUPT, "offsets do not end at the counts");
    if (!rc) rc = check_lists(n, L->off_a.data(), L->start_a.data(), L->end_a.data(), L->off_f.data(),
                              L->start_f.data(), L->end_f.data(), validate != 0);
    if (rc) {
        delete L;
        return fail(APRIL_E_CORRUPT, std::string(path) + ": " + april_last_error());
    }
    L->grid = grid;
    L->partition_key = key;
    L->n = n; L->n_a = na; L->n_f = nf;
    *out = L;
    return APRIL_OK;
}

}  // extern "C"
