// Device-side pieces shared by the filter kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "april.h"

namespace april {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

struct ListView {
    const uint64_t *off;
    const uint32_t *s;
    const uint32_t *e;
};

struct FilterArgs {
    ListView Ar, Fr, As, Fs;
    const uint32_t *r;
    const uint32_t *s;
    uint64_t n_pairs;
    uint64_t n_r, n_s;
    uint8_t *verdict;
    unsigned long long *counts;
};

// Make this wave's LDS writes visible to its own later LDS reads (and keep
// the compiler from moving LDS accesses across this point).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Scratch of the persistent kernels (the caller's workspace, or a
// stream-ordered allocation), two regions of kMaxCtrs slots, 128 bytes each:
//  * work counters, one per XCD range: counter k is ctr[k * kCtrStride];
//  * totals (verdict counts): each wave adds its sums to slot (wave id mod
//    kMaxCtrs), and k_sum_totals writes the slots' sum to the caller's array.
// Atomics on one cache line are serialized: with every counter in one line
// the grabs of the whole chip queued behind each other (the at-scale join ran
// 17% slower), and the end-of-kernel additions of 5,000 waves into one line
// took 0.14 ms of a 2.5 ms launch.
constexpr uint32_t kCtrStride = 32;    // uint32 words per slot
constexpr uint32_t kMaxCtrs = 64;
constexpr uint32_t kSlotWords = 16;    // uint64 words per slot
constexpr uint64_t kCtrBytes = 2ull * kMaxCtrs * kCtrStride * sizeof(unsigned int);
// Pairs the batched schedule can queue for its workgroup bin in one call
// (the rest of that bin runs on single waves).
constexpr uint64_t kBigQueueCap = 1ull << 20;
// Default workgroup-bin threshold: pairs whose shorter object spans at
// least this many intervals (and neither object fits a tile) run on a
// workgroup.  On the skewed workload 2048 and 4096 time the same; on the
// at-scale one (longest list 3,588 intervals) 4096 leaves the bin empty, so
// the binning pass is skipped.
constexpr uint32_t kDefaultWgMin = 4096;
// Workspace part of the static scratch (april_filter_pairs_static): enough
// for any filter call's scratch on raw lists.
constexpr uint64_t kStaticWorkspaceBytes = (4ull << 20) + (64ull << 10);

// zero both regions
__global__ void k_zero_ctrs(unsigned int *ctr);
// totals[0 .. n) = sums over the slots (n <= 3)
__global__ void k_sum_totals(const unsigned int *ctr, unsigned long long *totals, uint32_t n);

// Add a wave's sums v[0 .. n) (already reduced over the wave) into its slot;
// lane 0 only.
__device__ __forceinline__ void add_totals(unsigned int *ctr, uint32_t wave_id, const unsigned long long *v,
                                           uint32_t n) {
    unsigned long long *slot =
        reinterpret_cast<unsigned long long *>(ctr + kMaxCtrs * kCtrStride) + (wave_id % kMaxCtrs) * kSlotWords;
    for (uint32_t k = 0; k < n; k++)
        if (v[k]) atomicAdd(&slot[k], v[k]);
}

// Has XCD range `seg` ([lo, hi)) been drained?  A plain read, for waves
// about to help another range: without it, waves that finish together all
// line up on the drained range's counter.  Whole wave, lane 0 reads.
__device__ __forceinline__ bool range_drained(const unsigned int *ctr, uint32_t seg, uint64_t lo, uint64_t hi,
                                              uint32_t lane) {
    unsigned int taken = 0;
    if (lane == 0) taken = __hip_atomic_load(&ctr[seg * kCtrStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return lo + uniform(__shfl(taken, 0)) >= hi;
}

// Alg. 2's IntervalJoin run sequentially by one lane; *rx, *ry receive how
// many leading elements of X and Y the loop read.
__device__ inline bool seq_join(const uint32_t *__restrict__ xs, const uint32_t *__restrict__ xe,
                         uint32_t n, const uint32_t *__restrict__ ys,
                         const uint32_t *__restrict__ ye, uint32_t m, uint32_t *rx, uint32_t *ry) {
    uint32_t i = 0, j = 0, ri = 0, rj = 0;
    bool found = false;
    while (i < n && j < m) {
        ri = i + 1;
        rj = j + 1;
        const uint32_t a = xs[i], b = xe[i], c = ys[j], d = ye[j];
        if (a < d && c < b) { found = true; break; }
        if (b <= d) i++;
        else j++;
    }
    *rx = ri;
    *ry = rj;
    return found;
}


// Batched schedule (batched.hip): scratch bytes for n_pairs, the library's
// default settings for a call (filled into the zero fields of `o`), and the
// launch of its binning and persistent kernels on `workspace`.
uint64_t batched_workspace_bytes(uint64_t n_pairs);
struct BatchedShape {
    uint64_t intervals_a;   // A-list intervals of both collections
    uint64_t objects;       // objects of both collections
    uint32_t max_len_r, max_len_s;   // longest list of one object (0xffffffff: unknown)
};
void batched_defaults(april_filter_opts_t &o, const BatchedShape &shape);
// XCDs of a device with `cus` compute units (32 CUs each on gfx950)
int xcd_count(int cus);
int launch_batched(const FilterArgs &a, const april_filter_opts_t &o, int cus, void *workspace,
                   hipStream_t stream);
// Kernel arguments of a filter call on device lists R and S (raw codec).
FilterArgs make_args(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r, const uint32_t *d_s,
                     uint64_t n_pairs, uint8_t *d_verdict, unsigned long long *counts);
// The batched schedule for lists on two orders of one data space (Sec. 5.3):
// exactly one of shift_r, shift_s is non-zero (2 * the order difference);
// the coarser side is kept resident and the finer side's A-list is mapped
// to its grid while streamed; true hits come from the coarser side's F only.
int launch_batched_mixed(const FilterArgs &a, uint32_t shift_r, uint32_t shift_s, int cus, void *workspace,
                         hipStream_t stream);
// The batched schedule for within joins (Sec. 4.3.2): s resident, A(r)
// streamed for AA, then tested for lying inside F(s).
int launch_batched_within(const FilterArgs &a, int cus, void *workspace, hipStream_t stream);
// The batched schedule for polygon-linestring joins (Sec. 4.3.3): R are the
// polygons (resident), S the linestrings, As their cell ids as runs of
// consecutive ids [start, end) (the F views are not read).
int launch_batched_linestrings(const FilterArgs &a, int cus, void *workspace, hipStream_t stream);

}  // namespace april
