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
struct DeviceArrays {
    uint64_t *off_a = nullptr, *off_f = nullptr;   // n+1 each
    uint32_t *start_a = nullptr, *end_a = nullptr;  // n_a each
    uint32_t *start_f = nullptr, *end_f = nullptr;  // n_f each
    void *block = nullptr;                          // one allocation holding all of the above
    size_t bytes = 0;
};

}  // namespace april

struct april_lists {
    april_grid_t grid{};
    uint64_t n = 0, n_a = 0, n_f = 0;
    int device = -1;                 // -1: host lists
    uint32_t codec = APRIL_CODEC_RAW;
    // host copy (empty for device lists)
    std::vector<uint64_t> off_a, off_f;
    std::vector<uint32_t> start_a, end_a, start_f, end_f;
    // device copy
    april::DeviceArrays d;
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

// Per-device state of the filter: compute-unit count and a one-word flag
// used by index validation.  Created on first use on each device.
struct DeviceState {
    int cus = 0;
    unsigned int *flag = nullptr;
};
int device_state(DeviceState **out);

}  // namespace april
