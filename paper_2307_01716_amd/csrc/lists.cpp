// Host/device list containers, errors, grid checks, Hilbert numbering,
// device info and the host MBR join.
#include <hip/hip_runtime_api.h>
#include <sched.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace april {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }

// Host worker threads: APRIL_HOST_THREADS if set, else the CPUs this
// process may run on, capped by OMP_NUM_THREADS when that is set, and by 64.
int host_threads() {
    const char *e = getenv("APRIL_HOST_THREADS");
    if (e && atoi(e) > 0) return atoi(e);
    int n = 0;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof set, &set) == 0) n = CPU_COUNT(&set);
    if (n <= 0) n = int(std::thread::hardware_concurrency());
    if (n <= 0) n = 4;
    const char *omp = getenv("OMP_NUM_THREADS");
    if (omp && atoi(omp) > 0) n = std::min(n, atoi(omp));
    return std::min(n, 64);
}

bool same_grid(const april_grid_t &a, const april_grid_t &b) {
    return a.x0 == b.x0 && a.y0 == b.y0 && a.side == b.side && a.order == b.order && a.flags == b.flags;
}

int lattice_grid(const april_grid_t *g, LatticeGrid *out) {
    if (!g) return fail(APRIL_E_INVALID, "grid is NULL");
    if (g->order < 1 || g->order > 16) return fail(APRIL_E_GRID, "grid order must be 1..16");
    if (g->flags & ~APRIL_GRID_PARTITIONED) return fail(APRIL_E_INVALID, "unknown grid flags");
    const double sl = g->side * 1073741824.0;
    const int64_t cells = int64_t(1) << g->order;
    if (!(sl >= cells) || sl > 9.0e15) return fail(APRIL_E_GRID, "grid side out of range");
    const int64_t w = int64_t(sl) / cells;
    if (double(w * cells) != sl) return fail(APRIL_E_GRID, "side*2^30 is not a multiple of 2^order");
    for (double v : {g->x0, g->y0}) {
        double q = v * 1073741824.0;
        if (!(std::fabs(q) < 4.0e15) || q != std::floor(q))
            return fail(APRIL_E_GRID, "grid origin is not a lattice point");
    }
    *out = LatticeGrid{g->x0, g->y0, w, int(g->order), cells};
    return APRIL_OK;
}

// --------------------------------------------------------------- Hilbert
//
// The curve of order n is four copies of the order n-1 curve, one per
// quadrant, visited lower-left, upper-left, upper-right, lower-right; the
// first copy is transposed, the last one reflected in the anti-diagonal.
// A state is the symmetry (identity, transpose, anti-transpose, half turn)
// that maps the current quadrant's curve onto the base curve; these four
// form the Klein group, so composing symmetries is XOR of their codes.
namespace {
constexpr uint8_t kIdent = 0, kTranspose = 1, kAnti = 2;  // half turn = 3
// digit of a canonical quadrant (qx, qy): (0,0)->0 (0,1)->1 (1,1)->2 (1,0)->3
constexpr uint8_t kDigit[2][2] = {{0, 1}, {3, 2}};
constexpr uint8_t kQuadX[4] = {0, 0, 1, 1};
constexpr uint8_t kQuadY[4] = {0, 1, 1, 0};
// symmetry of the sub-curve in quadrant `digit`, relative to its parent
constexpr uint8_t kChild[4] = {kTranspose, kIdent, kIdent, kAnti};

}  // namespace

// Apply a symmetry to the top bits (bx, by) of a cell's coordinates.
//   identity: (x, y); transpose: (y, x); anti-transpose: (1-y, 1-x); half turn: (1-x, 1-y)
static inline void sym(uint8_t s, uint32_t bx, uint32_t by, uint32_t *ox, uint32_t *oy) {
    switch (s) {
        case 0: *ox = bx; *oy = by; break;
        case 1: *ox = by; *oy = bx; break;
        case 2: *ox = 1u - by; *oy = 1u - bx; break;
        default: *ox = 1u - bx; *oy = 1u - by; break;
    }
}

uint64_t hilbert_xy2d(int order, uint32_t x, uint32_t y) {
    uint8_t state = 0;
    uint64_t d = 0;
    for (int lvl = order - 1; lvl >= 0; lvl--) {
        uint32_t qx, qy;
        sym(state, (x >> lvl) & 1u, (y >> lvl) & 1u, &qx, &qy);
        const uint8_t digit = kDigit[qx][qy];
        d = (d << 2) | digit;
        state ^= kChild[digit];
    }
    return d;
}

void hilbert_d2xy(int order, uint64_t d, uint32_t *x, uint32_t *y) {
    uint8_t state = 0;
    uint32_t X = 0, Y = 0;
    for (int lvl = order - 1; lvl >= 0; lvl--) {
        const uint8_t digit = uint8_t((d >> (2 * lvl)) & 3u);
        uint32_t bx, by;
        sym(state, kQuadX[digit], kQuadY[digit], &bx, &by);   // every symmetry is its own inverse
        X = (X << 1) | bx;
        Y = (Y << 1) | by;
        state ^= kChild[digit];
    }
    *x = X;
    *y = Y;
}

uint64_t vbyte_encode(const uint32_t *s, const uint32_t *e, uint64_t n, std::vector<uint8_t> &out,
                      std::vector<uint32_t> &bval, std::vector<uint32_t> &bpos) {
    const size_t base = out.size();
    uint32_t prev = 0xffffffffu;   // so that the first value is stored as itself
    auto put = [&](uint32_t d) {
        while (d >= 0x80u) {
            out.push_back(uint8_t(d | 0x80u));
            d >>= 7;
        }
        out.push_back(uint8_t(d));
    };
    for (uint64_t i = 0; i < n; i++) {
        put(s[i] - prev - 1u);   // first value: s_0 (prev + 1 wraps to 0)
        prev = s[i];
        if (i % kVbyteBlock == 0) {
            bval.push_back(s[i]);
            bpos.push_back(uint32_t(out.size() - base));
        }
        put(e[i] - prev - 1u);
        prev = e[i];
    }
    return out.size() - base;
}

// Offsets start at 0 and never decrease; with `full`, every list is sorted,
// disjoint and non-empty per interval, and every F interval lies inside one
// A interval (a Full cell is a cell of the polygon, Sec. 4.1).
int check_lists(uint64_t n, const uint64_t *off_a, const uint32_t *start_a, const uint32_t *end_a,
                const uint64_t *off_f, const uint32_t *start_f, const uint32_t *end_f, bool full) {
    if (off_a[0] != 0 || off_f[0] != 0) return fail(APRIL_E_INVALID, "offsets must start at 0");
    for (uint64_t k = 0; k < n; k++)
        if (off_a[k + 1] < off_a[k] || off_f[k + 1] < off_f[k])
            return fail(APRIL_E_INVALID, "offsets must be non-decreasing");
    if (full) {
        auto check = [&](const uint64_t *off, const uint32_t *s, const uint32_t *e) -> bool {
            for (uint64_t k = 0; k < n; k++)
                for (uint64_t t = off[k]; t < off[k + 1]; t++) {
                    if (s[t] >= e[t]) return false;
                    if (t + 1 < off[k + 1] && e[t] > s[t + 1]) return false;
                }
            return true;
        };
        if (!check(off_a, start_a, end_a) || !check(off_f, start_f, end_f))
            return fail(APRIL_E_CORRUPT, "interval lists are not sorted and disjoint");
        // every F interval lies inside one A interval (Full cells are cells
        // of the polygon)
        for (uint64_t k = 0; k < n; k++) {
            uint64_t t = off_a[k];
            for (uint64_t q = off_f[k]; q < off_f[k + 1]; q++) {
                while (t < off_a[k + 1] && end_a[t] < end_f[q]) t++;
                if (t == off_a[k + 1] || start_a[t] > start_f[q])
                    return fail(APRIL_E_CORRUPT, "F-list not contained in the A-list");
            }
        }
    }
    return APRIL_OK;
}

}  // namespace april

using namespace april;

extern "C" {

const char *april_last_error(void) { return april::g_last_error.c_str(); }

int april_lists_from_arrays(const april_grid_t *grid, uint64_t n, const uint64_t *off_a,
                            const uint32_t *start_a, const uint32_t *end_a, const uint64_t *off_f,
                            const uint32_t *start_f, const uint32_t *end_f, int validate,
                            april_lists_t **out) {
    clear_error();
    if (!grid || !out || !off_a || !off_f) return fail(APRIL_E_INVALID, "NULL argument");
    LatticeGrid lg;
    if (int rc = lattice_grid(grid, &lg)) return rc;
    const uint64_t na = off_a[n], nf = off_f[n];
    if ((na && (!start_a || !end_a)) || (nf && (!start_f || !end_f)))
        return fail(APRIL_E_INVALID, "NULL interval arrays");
    if (int rc = check_lists(n, off_a, start_a, end_a, off_f, start_f, end_f, validate != 0)) return rc;
    auto *L = new (std::nothrow) april_lists;
    if (!L) return fail(APRIL_E_NOMEM, "out of host memory");
    try {
        L->grid = *grid;
        L->n = n; L->n_a = na; L->n_f = nf;
        L->off_a.assign(off_a, off_a + n + 1);
        L->off_f.assign(off_f, off_f + n + 1);
        L->start_a.assign(start_a, start_a + na);
        L->end_a.assign(end_a, end_a + na);
        L->start_f.assign(start_f, start_f + nf);
        L->end_f.assign(end_f, end_f + nf);
    } catch (...) {
        delete L;
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    *out = L;
    return APRIL_OK;
}

int april_lists_info(const april_lists_t *L, april_lists_info_t *info) {
    if (!L || !info) return fail(APRIL_E_INVALID, "NULL argument");
    info->n_objects = L->n;
    info->n_a = L->n_a;
    info->n_f = L->n_f;
    info->device_bytes = L->device >= 0 ? L->d.bytes : 0;
    info->on_device = L->device;
    info->codec = L->codec;
    return APRIL_OK;
}

int april_lists_export(const april_lists_t *L, uint64_t *off_a, uint32_t *start_a, uint32_t *end_a,
                       uint64_t *off_f, uint32_t *start_f, uint32_t *end_f) {
    clear_error();
    if (!L) return fail(APRIL_E_INVALID, "NULL lists");
    if (L->device >= 0) return fail(APRIL_E_INVALID, "export needs host lists");
    std::copy(L->off_a.begin(), L->off_a.end(), off_a);
    std::copy(L->off_f.begin(), L->off_f.end(), off_f);
    std::copy(L->start_a.begin(), L->start_a.end(), start_a);
    std::copy(L->end_a.begin(), L->end_a.end(), end_a);
    std::copy(L->start_f.begin(), L->start_f.end(), start_f);
    std::copy(L->end_f.begin(), L->end_f.end(), end_f);
    return APRIL_OK;
}

int april_lists_to_device(const april_lists_t *h, uint32_t codec, void *stream,
                          april_lists_t **out) {
    clear_error();
    if (!h || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (h->device >= 0) return fail(APRIL_E_INVALID, "lists are already on a device");
    if (codec != APRIL_CODEC_RAW && codec != APRIL_CODEC_VBYTE) return fail(APRIL_E_INVALID, "unknown codec");
    int dev = 0;
    APRIL_HIP_TRY(hipGetDevice(&dev));
    auto *L = new (std::nothrow) april_lists;
    if (!L) return fail(APRIL_E_NOMEM, "out of host memory");
    L->grid = h->grid;
    L->partition_key = h->partition_key;
    L->n = h->n; L->n_a = h->n_a; L->n_f = h->n_f;
    L->device = dev;
    L->codec = codec;
    uint64_t longest = 0;
    for (uint64_t k = 0; k < h->n; k++)
        longest = std::max({longest, h->off_a[k + 1] - h->off_a[k], h->off_f[k + 1] - h->off_f[k]});
    L->max_len = uint32_t(std::min<uint64_t>(longest, 0xfffffffeull));
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const uint64_t n = h->n;
    const size_t b_off = up(8 * (n + 1));
    // host staging for the compressed form (kept alive in L until freed)
    std::vector<uint64_t> boff_a, boff_f, blk_a, blk_f;
    std::vector<uint8_t> bytes_a, bytes_f;
    std::vector<uint32_t> bval_a, bpos_a, bval_f, bpos_f;
    size_t total = 2 * b_off;
    size_t b_a = 0, b_f = 0, b_ba = 0, b_bf = 0, b_va = 0, b_vf = 0;
    if (codec == APRIL_CODEC_RAW) {
        b_a = up(4 * std::max<uint64_t>(h->n_a, 1));
        b_f = up(4 * std::max<uint64_t>(h->n_f, 1));
        total += 2 * b_a + 2 * b_f;
    } else {
        try {
            for (int t = 0; t < 2; t++) {
                const auto &off = t ? h->off_f : h->off_a;
                const auto &st = t ? h->start_f : h->start_a;
                const auto &en = t ? h->end_f : h->end_a;
                auto &bo = t ? boff_f : boff_a;
                auto &bk = t ? blk_f : blk_a;
                auto &by = t ? bytes_f : bytes_a;
                auto &bv = t ? bval_f : bval_a;
                auto &bp = t ? bpos_f : bpos_a;
                bo.resize(n + 1);
                bk.resize(n + 1);
                by.reserve(size_t((off[n]) * 3));
                for (uint64_t k = 0; k < n; k++) {
                    bo[k] = by.size();
                    bk[k] = bv.size();
                    vbyte_encode(st.data() + off[k], en.data() + off[k], off[k + 1] - off[k], by, bv, bp);
                }
                bo[n] = by.size();
                bk[n] = bv.size();
                if (bv.size() != bp.size()) return fail(APRIL_E_INVALID, "block index mismatch");
                // the decoder reads whole aligned 256-byte windows (+4 bytes)
                for (uint32_t pad = 0; pad < 512; pad++) by.push_back(0);
            }
        } catch (...) {
            delete L;
            return fail(APRIL_E_NOMEM, "out of host memory");
        }
        b_ba = up(bytes_a.size());
        b_bf = up(bytes_f.size());
        b_va = up(4 * std::max<size_t>(bval_a.size(), 1));
        b_vf = up(4 * std::max<size_t>(bval_f.size(), 1));
        total += 4 * b_off + b_ba + b_bf + 2 * b_va + 2 * b_vf;
    }
    hipError_t e = hipMalloc(&L->d.block, total);
    if (e != hipSuccess) {
        delete L;
        return fail(APRIL_E_NOMEM, std::string("hipMalloc lists: ") + hipGetErrorString(e));
    }
    char *p = static_cast<char *>(L->d.block);
    L->d.off_a = reinterpret_cast<uint64_t *>(p); p += b_off;
    L->d.off_f = reinterpret_cast<uint64_t *>(p); p += b_off;
    if (codec == APRIL_CODEC_RAW) {
        L->d.start_a = reinterpret_cast<uint32_t *>(p); p += b_a;
        L->d.end_a = reinterpret_cast<uint32_t *>(p); p += b_a;
        L->d.start_f = reinterpret_cast<uint32_t *>(p); p += b_f;
        L->d.end_f = reinterpret_cast<uint32_t *>(p);
    } else {
        L->d.boff_a = reinterpret_cast<uint64_t *>(p); p += b_off;
        L->d.boff_f = reinterpret_cast<uint64_t *>(p); p += b_off;
        L->d.blk_a = reinterpret_cast<uint64_t *>(p); p += b_off;
        L->d.blk_f = reinterpret_cast<uint64_t *>(p); p += b_off;
        L->d.bytes_a = reinterpret_cast<uint8_t *>(p); p += b_ba;
        L->d.bytes_f = reinterpret_cast<uint8_t *>(p); p += b_bf;
        L->d.bval_a = reinterpret_cast<uint32_t *>(p); p += b_va;
        L->d.bpos_a = reinterpret_cast<uint32_t *>(p); p += b_va;
        L->d.bval_f = reinterpret_cast<uint32_t *>(p); p += b_vf;
        L->d.bpos_f = reinterpret_cast<uint32_t *>(p);
        L->d.n_bytes_a = boff_a[n];
        L->d.n_bytes_f = boff_f[n];
        L->d.n_blk_a = bval_a.size();
        L->d.n_blk_f = bval_f.size();
    }
    L->d.bytes = total;
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto cp = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    hipError_t rc = cp(L->d.off_a, h->off_a.data(), 8 * (n + 1));
    if (rc == hipSuccess) rc = cp(L->d.off_f, h->off_f.data(), 8 * (n + 1));
    if (codec == APRIL_CODEC_RAW) {
        if (rc == hipSuccess) rc = cp(L->d.start_a, h->start_a.data(), 4 * h->n_a);
        if (rc == hipSuccess) rc = cp(L->d.end_a, h->end_a.data(), 4 * h->n_a);
        if (rc == hipSuccess) rc = cp(L->d.start_f, h->start_f.data(), 4 * h->n_f);
        if (rc == hipSuccess) rc = cp(L->d.end_f, h->end_f.data(), 4 * h->n_f);
    } else {
        // the staging vectors die with this call: copy synchronously
        if (rc == hipSuccess) rc = cp(L->d.boff_a, boff_a.data(), 8 * (n + 1));
        if (rc == hipSuccess) rc = cp(L->d.boff_f, boff_f.data(), 8 * (n + 1));
        if (rc == hipSuccess) rc = cp(L->d.blk_a, blk_a.data(), 8 * (n + 1));
        if (rc == hipSuccess) rc = cp(L->d.blk_f, blk_f.data(), 8 * (n + 1));
        if (rc == hipSuccess) rc = cp(L->d.bytes_a, bytes_a.data(), bytes_a.size());
        if (rc == hipSuccess) rc = cp(L->d.bytes_f, bytes_f.data(), bytes_f.size());
        if (rc == hipSuccess) rc = cp(L->d.bval_a, bval_a.data(), 4 * bval_a.size());
        if (rc == hipSuccess) rc = cp(L->d.bpos_a, bpos_a.data(), 4 * bpos_a.size());
        if (rc == hipSuccess) rc = cp(L->d.bval_f, bval_f.data(), 4 * bval_f.size());
        if (rc == hipSuccess) rc = cp(L->d.bpos_f, bpos_f.data(), 4 * bpos_f.size());
        if (rc == hipSuccess) rc = hipStreamSynchronize(s);
    }
    if (rc != hipSuccess) {
        (void)hipFree(L->d.block);
        delete L;
        return fail(APRIL_E_HIP, std::string("upload: ") + hipGetErrorString(rc));
    }
    *out = L;
    return APRIL_OK;
}

int april_lists_download(const april_lists_t *d, void *stream, april_lists_t **out) {
    clear_error();
    if (!d || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (d->device < 0) return fail(APRIL_E_INVALID, "lists are not on a device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto *L = new (std::nothrow) april_lists;
    if (!L) return fail(APRIL_E_NOMEM, "out of host memory");
    try {
        L->grid = d->grid;
        L->partition_key = d->partition_key;
        L->n = d->n; L->n_a = d->n_a; L->n_f = d->n_f;
        L->off_a.resize(d->n + 1);
        L->off_f.resize(d->n + 1);
        L->start_a.resize(d->n_a); L->end_a.resize(d->n_a);
        L->start_f.resize(d->n_f); L->end_f.resize(d->n_f);
    } catch (...) {
        delete L;
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    void *tmp = nullptr;
    const uint32_t *sa = d->d.start_a, *ea = d->d.end_a, *sf = d->d.start_f, *ef = d->d.end_f;
    int rc = APRIL_OK;
    if (d->codec == APRIL_CODEC_VBYTE) {
        const size_t na = std::max<uint64_t>(d->n_a, 1), nf = std::max<uint64_t>(d->n_f, 1);
        if (hipMalloc(&tmp, 4 * (2 * na + 2 * nf)) != hipSuccess) {
            delete L;
            return fail(APRIL_E_NOMEM, "download: device scratch");
        }
        uint32_t *t = static_cast<uint32_t *>(tmp);
        uint32_t *ta = t, *tea = t + na, *tf = t + 2 * na, *tef = t + 2 * na + nf;
        rc = launch_decode_lists(d, false, ta, tea, s);
        if (!rc) rc = launch_decode_lists(d, true, tf, tef, s);
        sa = ta; ea = tea; sf = tf; ef = tef;
    }
    auto cp = [&](void *dst, const void *src, size_t b) {
        return b ? hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, s) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    if (!rc) {
        e = cp(L->off_a.data(), d->d.off_a, 8 * (d->n + 1));
        if (e == hipSuccess) e = cp(L->off_f.data(), d->d.off_f, 8 * (d->n + 1));
        if (e == hipSuccess) e = cp(L->start_a.data(), sa, 4 * d->n_a);
        if (e == hipSuccess) e = cp(L->end_a.data(), ea, 4 * d->n_a);
        if (e == hipSuccess) e = cp(L->start_f.data(), sf, 4 * d->n_f);
        if (e == hipSuccess) e = cp(L->end_f.data(), ef, 4 * d->n_f);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (tmp) (void)hipFree(tmp);
    if (rc || e != hipSuccess) {
        delete L;
        return rc ? rc : fail(APRIL_E_HIP, std::string("download: ") + hipGetErrorString(e));
    }
    *out = L;
    return APRIL_OK;
}

void april_lists_free(april_lists_t *L) {
    if (!L) return;
    if (L->device >= 0 && L->d.block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != L->device) (void)hipSetDevice(L->device);
        (void)hipFree(L->d.block);
        if (cur != L->device) (void)hipSetDevice(cur);
    }
    delete L;
}

int april_device_info(april_device_info_t *info) {
    clear_error();
    if (!info) return fail(APRIL_E_INVALID, "NULL argument");
    memset(info, 0, sizeof(*info));
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(APRIL_E_NODEV, "no HIP device");
    int dev = 0;
    APRIL_HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t p;
    APRIL_HIP_TRY(hipGetDeviceProperties(&p, dev));
    info->device = dev;
    info->compute_units = p.multiProcessorCount;
    info->wavefront_size = p.warpSize;
    info->hbm_bytes = p.totalGlobalMem;
    snprintf(info->arch, sizeof(info->arch), "%s", p.gcnArchName);
    snprintf(info->name, sizeof(info->name), "%s", p.name);
    return APRIL_OK;
}

// ------------------------------------------------------------- MBR join
//
// Uniform grid over the joint extent; every S box is registered in the grid
// cells it overlaps; each R box probes its cells and reports (r, s) from the
// cell that holds the lower-left corner of the two boxes' intersection, so
// every pair is found exactly once.
int april_mbr_join(const double *br, uint64_t nr, const double *bs, uint64_t ns, uint32_t *r_out,
                   uint32_t *s_out, uint64_t capacity, uint64_t *n_out) {
    clear_error();
    if (!n_out || (nr && !br) || (ns && !bs)) return fail(APRIL_E_INVALID, "NULL argument");
    if (nr > 0xffffffffull || ns > 0xffffffffull) return fail(APRIL_E_INVALID, "too many boxes");
    *n_out = 0;
    if (nr == 0 || ns == 0) return APRIL_OK;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    double sum_w = 0, sum_h = 0;
    for (const double *b : {br, bs}) {
        const uint64_t n = (b == br) ? nr : ns;
        for (uint64_t k = 0; k < n; k++) {
            const double *q = b + 4 * k;
            if (!(q[0] <= q[2] && q[1] <= q[3])) return fail(APRIL_E_INVALID, "box with min > max");
            lo[0] = std::min(lo[0], q[0]); lo[1] = std::min(lo[1], q[1]);
            hi[0] = std::max(hi[0], q[2]); hi[1] = std::max(hi[1], q[3]);
            sum_w += q[2] - q[0]; sum_h += q[3] - q[1];
        }
    }
    const double ext = std::max(hi[0] - lo[0], hi[1] - lo[1]);
    const double mean_side = std::max(sum_w, sum_h) / double(nr + ns);
    int64_t G = ext > 0 && mean_side > 0 ? int64_t(ext / (2.0 * mean_side)) : 1;
    G = std::max<int64_t>(1, std::min<int64_t>(G, 2048));
    const double cs = ext > 0 ? ext / double(G) : 1.0;
    auto cell = [&](double v, int axis) -> int64_t {
        int64_t c = int64_t((v - lo[axis]) / cs);
        return std::min<int64_t>(std::max<int64_t>(c, 0), G - 1);
    };
    // CSR of S ids per grid cell
    std::vector<uint64_t> cnt(size_t(G * G) + 1, 0);
    for (uint64_t k = 0; k < ns; k++) {
        const double *q = bs + 4 * k;
        for (int64_t cy = cell(q[1], 1); cy <= cell(q[3], 1); cy++)
            for (int64_t cx = cell(q[0], 0); cx <= cell(q[2], 0); cx++) cnt[cy * G + cx + 1]++;
    }
    for (size_t c = 1; c < cnt.size(); c++) cnt[c] += cnt[c - 1];
    std::vector<uint32_t> ids(cnt.back());
    {
        std::vector<uint64_t> pos(cnt.begin(), cnt.end() - 1);
        for (uint64_t k = 0; k < ns; k++) {
            const double *q = bs + 4 * k;
            for (int64_t cy = cell(q[1], 1); cy <= cell(q[3], 1); cy++)
                for (int64_t cx = cell(q[0], 0); cx <= cell(q[2], 0); cx++)
                    ids[pos[cy * G + cx]++] = uint32_t(k);
        }
    }
    const int T = host_threads();
    std::vector<std::vector<uint32_t>> per_r(nr);
    std::atomic<uint64_t> next{0};
    parallel(T, [&](int) {
        std::vector<uint32_t> tmp;
        for (;;) {
            const uint64_t r = next.fetch_add(1);
            if (r >= nr) break;
            const double *a = br + 4 * r;
            tmp.clear();
            for (int64_t cy = cell(a[1], 1); cy <= cell(a[3], 1); cy++)
                for (int64_t cx = cell(a[0], 0); cx <= cell(a[2], 0); cx++) {
                    const int64_t c = cy * G + cx;
                    for (uint64_t t = cnt[c]; t < cnt[c + 1]; t++) {
                        const uint32_t s = ids[t];
                        const double *b = bs + 4 * s;
                        if (!(a[0] <= b[2] && b[0] <= a[2] && a[1] <= b[3] && b[1] <= a[3])) continue;
                        // report from the cell of the intersection's lower-left corner
                        const double ix = std::max(a[0], b[0]), iy = std::max(a[1], b[1]);
                        if (cell(ix, 0) == cx && cell(iy, 1) == cy) tmp.push_back(s);
                    }
                }
            std::sort(tmp.begin(), tmp.end());
            per_r[r] = tmp;
        }
    });
    uint64_t total = 0;
    for (auto &v : per_r) total += v.size();
    *n_out = total;
    if (total > capacity) return fail(APRIL_E_NOMEM, "pair capacity too small");
    if (total && (!r_out || !s_out)) return fail(APRIL_E_INVALID, "NULL output arrays");
    // emit r objects in the Z-order of their MBR centres, so that pairs that
    // are close in the output are close in space (their lists are shared)
    std::vector<std::pair<uint64_t, uint32_t>> order(nr);
    const double inv = ext > 0 ? 65535.0 / ext : 0.0;
    for (uint64_t r = 0; r < nr; r++) {
        const double *a = br + 4 * r;
        const uint32_t qx = uint32_t(std::min(65535.0, std::max(0.0, ((a[0] + a[2]) * 0.5 - lo[0]) * inv)));
        const uint32_t qy = uint32_t(std::min(65535.0, std::max(0.0, ((a[1] + a[3]) * 0.5 - lo[1]) * inv)));
        uint64_t z = 0;
        for (int b = 15; b >= 0; b--) z = (z << 2) | (uint64_t((qy >> b) & 1u) << 1) | ((qx >> b) & 1u);
        order[r] = {z, uint32_t(r)};
    }
    std::sort(order.begin(), order.end());
    uint64_t t = 0;
    for (const auto &o : order)
        for (uint32_t s : per_r[o.second]) { r_out[t] = o.second; s_out[t] = s; t++; }
    return APRIL_OK;
}

}  // extern "C"
