// Linestring cell lists (Sec. 4.3.3): upload (as runs of consecutive ids),
// export, free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "internal.hpp"

using namespace april;

extern "C" int april_cells_to_device(const april_cells_t *h, void *hip_stream, april_cells_t **out) {
    clear_error();
    if (!h || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (h->device >= 0) return fail(APRIL_E_INVALID, "cells are already on a device");
    auto *C = new (std::nothrow) april_cells;
    if (!C) return fail(APRIL_E_NOMEM, "out of host memory");
    C->grid = h->grid;
    C->n = h->n;
    C->n_ids = h->n_ids;
    // runs of consecutive ids: a run meets an interval exactly when one of
    // its cells does, so the joins give the same verdicts on fewer elements
    try {
        C->run_off.assign(h->n + 1, 0);
        for (uint64_t k = 0; k < h->n; k++) {
            for (uint64_t t = h->off[k]; t < h->off[k + 1]; t++) {
                if (t == h->off[k] || h->ids[t] != h->ids[t - 1] + 1) {
                    C->run_start.push_back(h->ids[t]);
                    C->run_end.push_back(h->ids[t] + 1);
                } else {
                    C->run_end.back() = h->ids[t] + 1;
                }
            }
            C->run_off[k + 1] = C->run_start.size();
        }
    } catch (const std::bad_alloc &) {
        delete C;
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    C->n_runs = C->run_start.size();
    const size_t b_off = (8 * (h->n + 1) + 255) & ~size_t(255);
    const size_t b_run = (4 * std::max<uint64_t>(C->n_runs, 1) + 255) & ~size_t(255);
    if (hipGetDevice(&C->device) != hipSuccess || hipMalloc(&C->d_block, b_off + 2 * b_run) != hipSuccess) {
        delete C;
        return fail(APRIL_E_NOMEM, "device allocation of the cells failed");
    }
    C->d_off = static_cast<uint64_t *>(C->d_block);
    C->d_start = reinterpret_cast<uint32_t *>(static_cast<char *>(C->d_block) + b_off);
    C->d_end = reinterpret_cast<uint32_t *>(static_cast<char *>(C->d_block) + b_off + b_run);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(C->d_off, C->run_off.data(), 8 * (h->n + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && C->n_runs)
        e = hipMemcpyAsync(C->d_start, C->run_start.data(), 4 * C->n_runs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && C->n_runs)
        e = hipMemcpyAsync(C->d_end, C->run_end.data(), 4 * C->n_runs, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        (void)hipFree(C->d_block);
        delete C;
        return fail(APRIL_E_HIP, std::string("cells upload: ") + hipGetErrorString(e));
    }
    *out = C;
    return APRIL_OK;
}

extern "C" int april_cells_info(const april_cells_t *C, uint64_t *n, uint64_t *n_ids) {
    clear_error();
    if (!C) return fail(APRIL_E_INVALID, "NULL cells");
    if (n) *n = C->n;
    if (n_ids) *n_ids = C->n_ids;
    return APRIL_OK;
}

extern "C" int april_cells_export(const april_cells_t *C, uint64_t *off, uint32_t *ids) {
    clear_error();
    if (!C || !off || (!ids && C->n_ids)) return fail(APRIL_E_INVALID, "NULL argument");
    if (C->device >= 0) return fail(APRIL_E_INVALID, "cells are on a device");
    std::memcpy(off, C->off.data(), 8 * (C->n + 1));
    if (C->n_ids) std::memcpy(ids, C->ids.data(), 4 * C->n_ids);
    return APRIL_OK;
}

extern "C" void april_cells_free(april_cells_t *C) {
    if (!C) return;
    if (C->device >= 0 && C->d_block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != C->device) (void)hipSetDevice(C->device);
        (void)hipFree(C->d_block);
        if (cur != C->device) (void)hipSetDevice(cur);
    }
    delete C;
}
