// Entry points of the filter's query variants, all on the filter's batched
// kernel (csrc/batched.hip):
//   within joins (Sec. 4.3.2): AA, then every A(r) interval inside one F(s)
//     interval;
//   polygon-linestring joins (Sec. 4.3.3): A(p) and F(p) against the
//     linestring's cell ids taken as intervals [c, c+1), consecutive ids
//     merged into one run;
//   different granularity (Sec. 5.3): the finer side's A mapped to the
//     coarser grid, a' = [a_s >> n, ((a_e - 1) >> n) + 1), then AA and the
//     coarser side's F only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

int check_device(const april_lists_t *L) {
    if (!L) return fail(APRIL_E_INVALID, "NULL lists");
    if (L->device < 0) return fail(APRIL_E_INVALID, "lists must be on a device");
    if (L->codec != APRIL_CODEC_RAW) return fail(APRIL_E_INVALID, "query variants take raw lists");
    int cur = 0;
    APRIL_HIP_TRY(hipGetDevice(&cur));
    if (cur != L->device) return fail(APRIL_E_INVALID, "current device does not hold the lists");
    return APRIL_OK;
}

enum class Variant { kWithin, kLinestrings, kMixed };

// A variant on the filter's batched kernel, with a stream-ordered workspace.
int run_batched(const FilterArgs &fa, int device, Variant v, uint32_t shift_r, uint32_t shift_s,
                hipStream_t stream) {
    if (fa.n_pairs >= (1ull << 32)) return fail(APRIL_E_INVALID, "fewer than 2^32 pairs per call");
    DeviceState *st = nullptr;
    if (int rc = device_state(&st)) return rc;
    int cur = 0;
    APRIL_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) return fail(APRIL_E_INVALID, "current device does not hold the lists");
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, batched_workspace_bytes(fa.n_pairs), stream);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
    const int rc = v == Variant::kWithin        ? launch_batched_within(fa, st->cus, ws, stream)
                   : v == Variant::kLinestrings ? launch_batched_linestrings(fa, st->cus, ws, stream)
                                                : launch_batched_mixed(fa, shift_r, shift_s, st->cus, ws, stream);
    APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    return rc;
}

}  // namespace
}  // namespace april

using namespace april;

extern "C" int april_filter_within(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                                   const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict,
                                   uint64_t *d_counts, void *hip_stream) {
    clear_error();
    if (int rc = check_device(R)) return rc;
    if (int rc = check_device(S)) return rc;
    if (R->device != S->device) return fail(APRIL_E_INVALID, "lists on different devices");
    if (!same_grid(R->grid, S->grid) || R->partition_key != S->partition_key)
        return fail(APRIL_E_GRID, "R and S lists use different grids");
    if (n_pairs && (!d_r || !d_s || !d_verdict)) return fail(APRIL_E_INVALID, "NULL pair/verdict array");
    const FilterArgs fa =
        make_args(R, S, d_r, d_s, n_pairs, d_verdict, reinterpret_cast<unsigned long long *>(d_counts));
    return run_batched(fa, R->device, Variant::kWithin, 0, 0, static_cast<hipStream_t>(hip_stream));
}

extern "C" int april_filter_linestrings(const april_lists_t *P, const april_cells_t *L, const uint32_t *d_p,
                                        const uint32_t *d_l, uint64_t n_pairs, uint8_t *d_verdict,
                                        uint64_t *d_counts, void *hip_stream) {
    clear_error();
    if (int rc = check_device(P)) return rc;
    if (!L) return fail(APRIL_E_INVALID, "NULL cells");
    if (L->device != P->device) return fail(APRIL_E_INVALID, "cells must be on the lists' device");
    if (!same_grid(P->grid, L->grid) || P->partition_key != 0)
        return fail(APRIL_E_GRID, "polygons and linestrings use different grids");
    if (n_pairs && (!d_p || !d_l || !d_verdict)) return fail(APRIL_E_INVALID, "NULL pair/verdict array");
    // R: the polygons; S: the linestrings, their runs of cell ids in the A view
    FilterArgs fa = make_args(P, P, d_p, d_l, n_pairs, d_verdict, reinterpret_cast<unsigned long long *>(d_counts));
    fa.As = {L->d_off, L->d_start, L->d_end};
    fa.Fs = fa.As;
    fa.n_s = L->n;
    return run_batched(fa, P->device, Variant::kLinestrings, 0, 0, static_cast<hipStream_t>(hip_stream));
}

extern "C" int april_filter_mixed(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                                  const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict, uint64_t *d_counts,
                                  void *hip_stream) {
    clear_error();
    if (int rc = check_device(R)) return rc;
    if (int rc = check_device(S)) return rc;
    if (R->device != S->device) return fail(APRIL_E_INVALID, "lists on different devices");
    const april_grid_t &g = R->grid, &h = S->grid;
    if (g.x0 != h.x0 || g.y0 != h.y0 || g.side != h.side || g.flags != h.flags || R->partition_key ||
        S->partition_key)
        return fail(APRIL_E_GRID, "R and S must cover one data space (same origin and side)");
    if (n_pairs && (!d_r || !d_s || !d_verdict)) return fail(APRIL_E_INVALID, "NULL pair/verdict array");
    const uint32_t shift_r = g.order > h.order ? 2 * (g.order - h.order) : 0;
    const uint32_t shift_s = h.order > g.order ? 2 * (h.order - g.order) : 0;
    if (shift_r == 0 && shift_s == 0) {   // one order: Alg. 2 itself
        april_filter_opts_t o{};
        o.schedule = APRIL_SCHED_BATCHED;
        return april_filter_pairs(R, S, d_r, d_s, n_pairs, d_verdict, d_counts, &o, hip_stream);
    }
    const FilterArgs fa =
        make_args(R, S, d_r, d_s, n_pairs, d_verdict, reinterpret_cast<unsigned long long *>(d_counts));
    return run_batched(fa, R->device, Variant::kMixed, shift_r, shift_s, static_cast<hipStream_t>(hip_stream));
}
