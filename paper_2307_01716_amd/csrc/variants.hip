// The filter's query variants on the GPU.
//
// Within joins (Sec. 4.3.2: AA, then every A(r) interval inside one F(s)
// interval) and different granularity (Sec. 5.3: the finer side's A mapped
// to the coarser grid, a' = [a_s >> n, ((a_e - 1) >> n) + 1), then AA and the
// coarser side's F only) run on the filter's batched kernel; their entry
// points are here.
//
// Polygon-linestring joins (Sec. 4.3.3: A(p) and F(p) against the
// linestring's cell ids taken as intervals [c, c+1)) run on k_linestrings:
// one wave per pair, pairs dealt to waves in order (wave w takes pairs w,
// w + W, ...).  The linestring's cells are copied into the wave's LDS when
// there are at most 1,024 of them (else read from global memory), the
// polygon's A- and then F-list is streamed, 64 elements per step, one per
// lane, and each lane binary-searches the cells for the first one at or after
// its element's start: the element meets a cell iff that cell is below its
// end.  A ballot per step ends a join on its first hit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

struct VList {
    const uint32_t *s, *e;   // interval starts / ends; e == nullptr: cell ids, e = s + 1
    uint32_t n;
};

struct VArgs {
    // the polygons' lists
    const uint64_t *offAr, *offFr;
    const uint32_t *sAr, *eAr, *sFr, *eFr;
    // the linestrings' cell ids
    const uint64_t *offAs;
    const uint32_t *sAs;
    const uint32_t *r, *s;
    uint64_t n_pairs, n_r, n_s;
    uint8_t *verdict;
    unsigned int *ctr;   // count slots (totals), or nullptr
};

__device__ __forceinline__ uint32_t gl(const uint32_t *p, uint64_t i) {
    return ((const uint32_t __attribute__((address_space(1))) *)p)[i];
}

// Cells kept in a wave's LDS (at most 4 * kTile ids).
constexpr uint32_t kTile = 256;

// Does any interval of Y overlap a cell of the sorted cell-id list C (as
// [c, c+1))?  The first cell >= y0 decides for element [y0, y1).  C is in
// LDS (in_lds) or global memory.  Whole wave.
template <bool LDS>
__device__ __forceinline__ bool cell_hit(const uint32_t *c, uint32_t n, uint32_t y0, uint32_t y1) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((LDS ? c[mid] : gl(c, mid)) < y0) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && (LDS ? c[lo] : gl(c, lo)) < y1;
}

__device__ bool any_cell_overlap(const uint32_t *c, uint32_t n, bool in_lds, const VList &Y, uint32_t lane) {
    if (n == 0) return false;
    for (uint32_t j0 = 0; j0 < Y.n; j0 += 64) {
        const uint32_t j = j0 + lane;
        bool h = false;
        if (j < Y.n) {
            const uint32_t y0 = gl(Y.s, j), y1 = gl(Y.e, j);
            h = in_lds ? cell_hit<true>(c, n, y0, y1) : cell_hit<false>(c, n, y0, y1);
        }
        if (__any(h)) return true;
    }
    return false;
}

__device__ __forceinline__ VList list_of(const uint64_t *off, const uint32_t *s, const uint32_t *e, uint32_t k) {
    const uint64_t a = ((const uint64_t __attribute__((address_space(1))) *)off)[k];
    const uint64_t b = ((const uint64_t __attribute__((address_space(1))) *)off)[k + 1];
    return VList{s + a, e ? e + a : nullptr, uint32_t(b - a)};
}

__global__ __launch_bounds__(kBlock) void k_linestrings(VArgs a) {
    __shared__ uint32_t lds_all[kWavesPerBlock][4 * kTile];
    const uint32_t lane = threadIdx.x & 63;
    uint32_t *lds = lds_all[threadIdx.x >> 6];
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;
    for (uint64_t p = wave; p < a.n_pairs; p += waves) {
        const uint32_t r = uniform(gl(a.r, p)), s = uniform(gl(a.s, p));
        uint8_t v;
        if (r >= a.n_r || s >= a.n_s) {
            v = APRIL_BAD_PAIR;
        } else {
            // the linestring's cells searched (in LDS when at most 4 kTile
            // of them: a linestring has more cells than a polygon has
            // intervals); the polygon's A- and F-lists streamed
            const VList Cl = list_of(a.offAs, a.sAs, nullptr, s);
            const bool in_lds = Cl.n <= 4 * kTile;
            if (in_lds) {
                wave_lds_sync();
                for (uint32_t i = lane; i < Cl.n; i += 64) lds[i] = gl(Cl.s, i);
                wave_lds_sync();
            }
            const uint32_t *c = in_lds ? lds : Cl.s;
            v = !any_cell_overlap(c, Cl.n, in_lds, list_of(a.offAr, a.sAr, a.eAr, r), lane) ? APRIL_TN
                : any_cell_overlap(c, Cl.n, in_lds, list_of(a.offFr, a.sFr, a.eFr, r), lane) ? APRIL_TH
                                                                                             : APRIL_INDECISIVE;
        }
        if (lane == 0) {
            a.verdict[p] = v;
            c_tn += v == APRIL_TN;
            c_th += v == APRIL_TH;
            c_ind += v == APRIL_INDECISIVE;
        }
    }
    if (a.ctr && lane == 0) {
        const unsigned long long t[3] = {c_tn, c_th, c_ind};
        add_totals(a.ctr, uint32_t(wave), t, 3);
    }
}

int launch_linestrings(VArgs a, unsigned long long *counts, hipStream_t stream) {
    DeviceState *st = nullptr;
    if (int rc = device_state(&st)) return rc;
    void *ws = nullptr;
    if (counts) {
        hipError_t e = hipMallocAsync(&ws, kCtrBytes, stream);
        if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("variant scratch: ") + hipGetErrorString(e));
        a.ctr = static_cast<unsigned int *>(ws);
        k_zero_ctrs<<<1, 64, 0, stream>>>(a.ctr);
    } else {
        a.ctr = nullptr;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && a.n_pairs) {
        const uint64_t waves = std::min<uint64_t>(a.n_pairs, uint64_t(st->cus) * 32);
        const uint32_t blocks = uint32_t((waves + kWavesPerBlock - 1) / kWavesPerBlock);
        k_linestrings<<<blocks, kBlock, 0, stream>>>(a);
        e = hipGetLastError();
    }
    if (e == hipSuccess && counts) {
        k_sum_totals<<<1, 64, 0, stream>>>(a.ctr, counts, 3);
        e = hipGetLastError();
    }
    if (ws) APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("variant launch: ") + hipGetErrorString(e));
    return APRIL_OK;
}

int check_device(const april_lists_t *L) {
    if (!L) return fail(APRIL_E_INVALID, "NULL lists");
    if (L->device < 0) return fail(APRIL_E_INVALID, "lists must be on a device");
    if (L->codec != APRIL_CODEC_RAW) return fail(APRIL_E_INVALID, "query variants take raw lists");
    int cur = 0;
    APRIL_HIP_TRY(hipGetDevice(&cur));
    if (cur != L->device) return fail(APRIL_E_INVALID, "current device does not hold the lists");
    return APRIL_OK;
}

VArgs base_args(const april_lists_t *R, const uint32_t *d_r, const uint32_t *d_s, uint64_t n, uint8_t *d_v) {
    VArgs a{};
    a.offAr = R->d.off_a;
    a.offFr = R->d.off_f;
    a.sAr = R->d.start_a;
    a.eAr = R->d.end_a;
    a.sFr = R->d.start_f;
    a.eFr = R->d.end_f;
    a.r = d_r;
    a.s = d_s;
    a.n_pairs = n;
    a.n_r = R->n;
    a.verdict = d_v;
    return a;
}

// Within joins and mixed orders on the filter's batched kernel, with a
// stream-ordered workspace.
int run_batched(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r, const uint32_t *d_s,
                uint64_t n_pairs, uint8_t *d_verdict, uint64_t *d_counts, hipStream_t stream, uint32_t shift_r,
                uint32_t shift_s, bool within) {
    if (n_pairs >= (1ull << 32)) return fail(APRIL_E_INVALID, "fewer than 2^32 pairs per call");
    DeviceState *st = nullptr;
    if (int rc = device_state(&st)) return rc;
    int cur = 0;
    APRIL_HIP_TRY(hipGetDevice(&cur));
    if (cur != R->device) return fail(APRIL_E_INVALID, "current device does not hold the lists");
    const FilterArgs fa =
        make_args(R, S, d_r, d_s, n_pairs, d_verdict, reinterpret_cast<unsigned long long *>(d_counts));
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, batched_workspace_bytes(n_pairs), stream);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
    const int rc = within ? launch_batched_within(fa, st->cus, ws, stream)
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
    return run_batched(R, S, d_r, d_s, n_pairs, d_verdict, d_counts, static_cast<hipStream_t>(hip_stream), 0, 0,
                       true);
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
    VArgs a = base_args(P, d_p, d_l, n_pairs, d_verdict);
    a.offAs = L->d_off;
    a.sAs = L->d_ids;
    a.n_s = L->n;
    return launch_linestrings(a, reinterpret_cast<unsigned long long *>(d_counts),
                          static_cast<hipStream_t>(hip_stream));
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
    return run_batched(R, S, d_r, d_s, n_pairs, d_verdict, d_counts, static_cast<hipStream_t>(hip_stream), shift_r,
                       shift_s, false);
}
