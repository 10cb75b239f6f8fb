// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "april.h"

namespace april {

// ------------------------------------------------------------------ errors
int fail(int code, const std::string &msg);   // records msg for april_last_error
void clear_error();

#define APRIL_HIP_TRY(expr)                                                          \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::april::fail(APRIL_E_HIP, std::string(#expr) + ": " +           \
                                                  hipGetErrorString(e_));            \
    } while (0)

// ------------------------------------------------------------------- lists
// Compressed (delta + VByte) form of one list type (A or F) of a collection.
// List k is the value sequence s_0 < e_0 < s_1 < e_1 < ...; its byte stream
// holds varint(s_0) and then varint(v_t - v_{t-1} - 1) for t >= 1, 7 bits per
// byte, low bits first, high bit set on every byte but a value's last.
// Every kVbyteBlock intervals a block entry stores the absolute value of the
// block's first start and the byte offset just after that value's varint,
// so decoding can begin at any block.
constexpr uint32_t kVbyteBlock = 64;
struct DeviceArrays {
    uint64_t *off_a = nullptr, *off_f = nullptr;   // n+1 each
    uint32_t *start_a = nullptr, *end_a = nullptr;  // n_a each (raw codec)
    uint32_t *start_f = nullptr, *end_f = nullptr;  // n_f each (raw codec)
    // VByte codec
    uint64_t *boff_a = nullptr, *boff_f = nullptr;  // n+1 each: byte offsets
    uint64_t *blk_a = nullptr, *blk_f = nullptr;    // n+1 each: first block entry
    uint8_t *bytes_a = nullptr, *bytes_f = nullptr;
    uint32_t *bval_a = nullptr, *bval_f = nullptr;  // per block: absolute start value
    uint32_t *bpos_a = nullptr, *bpos_f = nullptr;  // per block: byte offset within the list
    uint64_t n_bytes_a = 0, n_bytes_f = 0, n_blk_a = 0, n_blk_f = 0;
    void *block = nullptr;                          // one allocation holding all of the above
    size_t bytes = 0;
};

// Encode one list (n intervals) into `out` (appended); block entries into
// bval/bpos (appended).  Returns the number of bytes written.
uint64_t vbyte_encode(const uint32_t *s, const uint32_t *e, uint64_t n, std::vector<uint8_t> &out,
                      std::vector<uint32_t> &bval, std::vector<uint32_t> &bpos);

}  // namespace april

struct april_lists {
    april_grid_t grid{};
    uint64_t partition_key = 0;      // partitioned collections: hash of all partition grids
    uint64_t n = 0, n_a = 0, n_f = 0;
    int device = -1;                 // -1: host lists
    uint32_t codec = APRIL_CODEC_RAW;
    // device lists uploaded from host lists: the most intervals in one
    // object's A- or F-list (0xffffffff: not known), which tells the filter
    // whether any pair can reach its workgroup bin
    uint32_t max_len = 0xffffffffu;
    // host copy (empty for device lists)
    std::vector<uint64_t> off_a, off_f;
    std::vector<uint32_t> start_a, end_a, start_f, end_f;
    // device copy
    april::DeviceArrays d;
};

// Linestring cell lists (Sec. 4.3.3): per linestring the sorted ids of the
// cells its segments meet.
struct april_cells {
    april_grid_t grid{};
    uint64_t n = 0, n_ids = 0;
    int device = -1;                 // -1: host
    std::vector<uint64_t> off;       // host cells: CSR offsets and sorted ids
    std::vector<uint32_t> ids;
    // device cells: each list's ids as maximal runs of consecutive ids,
    // [start, end) (run CSR offsets, starts, ends; one allocation; the host
    // vectors run_* hold what was uploaded until the free)
    std::vector<uint64_t> run_off;
    std::vector<uint32_t> run_start, run_end;
    uint64_t n_runs = 0;
    uint64_t *d_off = nullptr;
    uint32_t *d_start = nullptr, *d_end = nullptr;
    void *d_block = nullptr;
};

namespace april {

bool same_grid(const april_grid_t &a, const april_grid_t &b);

// Exact grid in lattice units (multiples of 2^-30).
struct LatticeGrid {
    double x0, y0;
    int64_t w;       // cell side, lattice units
    int order;
    int64_t cells;   // 2^order
};
int lattice_grid(const april_grid_t *g, LatticeGrid *out);

// Hilbert position <-> cell, table-driven (state = one of the four
// symmetries of the square that map the curve of a quadrant onto the base
// curve); both directions walk the levels from the top.
uint64_t hilbert_xy2d(int order, uint32_t x, uint32_t y);
void hilbert_d2xy(int order, uint64_t d, uint32_t *x, uint32_t *y);

// Run fn(worker_index) on `threads` host threads.
template <class F>
void parallel(int threads, F fn) {
    if (threads <= 1) { fn(0); return; }
    std::vector<std::thread> th;
    th.reserve(threads);
    for (int t = 0; t < threads; t++) th.emplace_back(fn, t);
    for (auto &t : th) t.join();
}
int host_threads();

// Offsets start at 0 and never decrease (APRIL_E_INVALID); with `full`, the
// lists are sorted, disjoint and every F interval lies inside an A interval
// (APRIL_E_CORRUPT).  Reads n + 1 offsets and the intervals they span.
int check_lists(uint64_t n, const uint64_t *off_a, const uint32_t *start_a, const uint32_t *end_a,
                const uint64_t *off_f, const uint32_t *start_f, const uint32_t *end_f, bool full);
// april_build_lists with at most max_threads host threads (polygons in
// parallel, or one large polygon split over them)
int build_lists_threads(const april_grid_t *grid, const double *xy, const uint64_t *vtx_off, uint64_t n,
                        uint32_t flags, int max_threads, april_lists_t **out);

// Per-device state of the filter, created on first use on each device (with
// that device current): compute-unit count, the device address of this
// device's static scratch (april_filter_pairs_static's workspace), and the
// one-word flag of index validation inside it.
struct DeviceState {
    int cus = 0;
    void *scratch = nullptr;
    unsigned int *flag = nullptr;
};
int device_state(DeviceState **out);

// One query of a served batch: its MBR and the grid cells the MBR covers.
struct ProbeQuery {
    double x0, y0, x1, y1;
    uint32_t cx0, cy0, cx1, cy1;
};
// Decode the A (f = false) or F lists of compressed device lists into raw
// device arrays (one wavefront per list).
int launch_decode_lists(const april_lists_t *L, bool f, uint32_t *out_s, uint32_t *out_e, hipStream_t stream);
// The filter on compressed lists (compressed.hip); `workspace` holds the
// work counters (kCtrBytes).
// The compressed filter's decode cache: its size for a device of `cus` CUs,
// and where it starts in a workspace that holds it.
uint64_t vbyte_cache_bytes(int cus);
uint64_t vbyte_cache_offset();
int launch_filter_vbyte(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r, const uint32_t *d_s,
                        uint64_t n_pairs, uint8_t *d_verdict, unsigned long long *counts,
                        const april_filter_opts_t &o, int cus, void *workspace, hipStream_t stream);
// Alg. 2's bytes per pair on compressed lists (april_alg2_bytes).
int launch_alg2_vbyte_bytes(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                            const uint32_t *d_s, uint64_t n_pairs, unsigned long long *d_bytes, int cus,
                            hipStream_t stream);
// Candidate pairs (batch query index, S id) of a batch of queries against
// the uniform MBR grid of S; *count receives the number found (pairs beyond
// `cap` are not written).
int launch_probe(const ProbeQuery *d_q, uint32_t n_q, const uint32_t *cell_off, const uint32_t *cell_ids,
                 const double *boxes, const uint16_t *cells, uint32_t G, uint32_t *pr, uint32_t *ps,
                 uint32_t cap, unsigned int *count, hipStream_t stream);

}  // namespace april
