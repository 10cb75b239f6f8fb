// The APRIL intermediate filter on gfx950 (Sec. 4.2, Alg. 2).
//
// Plain schedule: one wavefront per candidate pair.  The wave reads the
// pair's ids and the CSR bounds of its four lists, then runs the three
// interval joins of Alg. 2 in order (AA; then AF; then FA) with early exit.
//
// A join of sorted, disjoint lists X and Y is done wave-cooperatively as a
// merge path.  Alg. 2's merge loop visits states (i, j); the state after t
// steps is the point of the merge path on diagonal i + j = t, where the
// merged order takes X_i before Y_j iff X_i.end <= Y_j.end (Alg. 2 advances
// i on ties).  A tile of 64*K consecutive diagonals is processed at once:
// both lists' next 64*K intervals are staged in LDS, lane l binary-searches
// its start state on diagonal l*K, then runs K steps of Alg. 2's loop from
// there.  The lanes together perform exactly the comparisons of Alg. 2 over
// the tile, so "some lane saw an overlap" equals "Alg. 2 returns true within
// these steps"; a ballot decides, and the state on the tile's last diagonal
// (lane 63's end state) starts the next tile.  The join ends as soon as one
// list is exhausted, like Alg. 2.
//
// Interval lists are SoA uint32 start[] / end[] arrays in HBM with uint64
// CSR offsets per object; tile loads are coalesced 4-byte loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace april {
// Static scratch: the work counters and count slots of a filter call made
// through april_filter_pairs_static (which allocates nothing), then the
// one-word flag of index validation at kStaticFlagOffset (used by every
// validating filter call).  One copy per device, held until the process
// ends; all calls on a device share it.
constexpr uint64_t kStaticFlagOffset = kStaticWorkspaceBytes;
constexpr uint64_t kStaticScratchBytes = kStaticWorkspaceBytes + 256;
}  // namespace april

static __device__ __align__(256) unsigned char scratch[april::kStaticScratchBytes];

namespace april {
namespace {

// One wave's LDS tiles: the two lists' starts and ends, each its own array
// of 64*K words at t, t + 64K, t + 128K, t + 192K (X starts, X ends, Y starts,
// Y ends).  A lane's merge-path search reads ends only, so these reads fall
// on consecutive words rather than every other word of interleaved
// (start, end) pairs: LDS bank conflict cycles per LDS instruction fell
// from 2.5 to 1.5 at scale, and the kernel from 6.09-6.11 to 6.02-6.06 ms.
// (Padding one word per 64, against the remaining two-way conflicts of lanes
// two elements apart, and a first tile of 64 intervals, against loads past
// an early overlap, each made it slower: 6.32 and 6.49 ms against 6.07 ms
// in the same runs.)

// One tile of the merge: both lists' next 64*K intervals from (i0, j0) are
// staged in LDS, every lane runs K steps of Alg. 2's loop from its
// diagonal's merge-path point; true iff some lane saw an overlap, else
// (i0, j0) advance to the tile's last diagonal.
template <int K>
__device__ __forceinline__ bool merge_tile(const uint32_t *__restrict__ xs, const uint32_t *__restrict__ xe,
                                           uint32_t n, const uint32_t *__restrict__ ys,
                                           const uint32_t *__restrict__ ye, uint32_t m, uint32_t *t,
                                           uint32_t &i0, uint32_t &j0, uint32_t lane) {
    constexpr uint32_t T = kWave * K;
    uint32_t *const txs = t, *const txe = t + T, *const tys = t + 2 * T, *const tye = t + 3 * T;
    const uint32_t nx = min(T, n - i0), ny = min(T, m - j0);
    // all of this wave's reads of the previous tile are done before the
    // tile is overwritten
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint32_t q = lane + k * kWave;
        if (q < nx) {
            txs[q] = xs[i0 + q];
            txe[q] = xe[i0 + q];
        }
        if (q < ny) {
            tys[q] = ys[j0 + q];
            tye[q] = ye[j0 + q];
        }
    }
    wave_lds_sync();
    // start state of this lane: merge-path point on diagonal d
    const uint32_t d = lane * K;
    uint32_t lo = d > ny ? d - ny : 0, hi = min(d, nx);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (txe[mid] <= tye[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo, j = d - lo;   // i > nx only past the end of both lists
    bool found = false;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (!found && i < nx && j < ny) {
            const uint32_t a = txs[i], b = txe[i], c = tys[j], e = tye[j];
            if (a < e && c < b) found = true;
            else if (b <= e) i++;
            else j++;
        }
    }
    if (__any(found)) return true;
    i0 += uniform(__shfl(i, kWave - 1));
    j0 += uniform(__shfl(j, kWave - 1));
    return false;
}

// Any overlap between X = [xs, xe)[0..n) and Y = [ys, ye)[0..m)?  Result is
// the one Alg. 2's IntervalJoin returns.
template <int K>
__device__ __forceinline__ bool wave_join(const uint32_t *__restrict__ xs, const uint32_t *__restrict__ xe,
                                          uint32_t n, const uint32_t *__restrict__ ys,
                                          const uint32_t *__restrict__ ye, uint32_t m, uint32_t *t,
                                          uint32_t lane) {
    uint32_t i0 = 0, j0 = 0;
    while (i0 < n && j0 < m)
        if (merge_tile<K>(xs, xe, n, ys, ye, m, t, i0, j0, lane)) return true;
    return false;
}

// Workgroups are dealt to the XCDs round-robin, so workgroup b runs on XCD
// b % xcds; each XCD takes one contiguous range of the pairs, keeping pairs
// that are close in the input (and share lists) in one L2.
struct PlainArgs {
    FilterArgs f;
    unsigned int *ctr;   // scratch slots that sum the counts
    uint32_t xcds;
};

// 80 SGPRs at most: the hardware allocates SGPRs in blocks of 16, and
// above 80 fewer than 8 waves per SIMD fit (at 81 SGPRs the kernel ran 1.6x
// longer with a grid of 8 waves per SIMD: part of it ran as a second round).
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_num_sgpr(80))) void k_filter_plain(PlainArgs pa) {
    const FilterArgs &a = pa.f;
    const uint32_t xcds = pa.xcds;
    __shared__ uint32_t lds[kWavesPerBlock][4 * kWave * K];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t w = uniform(threadIdx.x / kWave);
    uint32_t *const lt = lds[w];
    const uint32_t xcd = blockIdx.x % xcds, bx = blockIdx.x / xcds, nbx = gridDim.x / xcds;
    const uint64_t lo = a.n_pairs * xcd / xcds, hi = a.n_pairs * (xcd + 1) / xcds;
    const uint64_t n_waves = uint64_t(nbx) * kWavesPerBlock;
    unsigned long long c_tn = 0, c_th = 0, c_ind = 0;
    for (uint64_t p = lo + uint64_t(bx) * kWavesPerBlock + w; p < hi; p += n_waves) {
        const uint32_t r = uniform(a.r[p]), s = uniform(a.s[p]);
        uint8_t v;
        if (r >= a.n_r || s >= a.n_s) {
            v = APRIL_BAD_PAIR;
        } else {
            const uint64_t ar0 = a.Ar.off[r], ar1 = a.Ar.off[r + 1];
            const uint64_t as0 = a.As.off[s], as1 = a.As.off[s + 1];
            const uint64_t fr0 = a.Fr.off[r], fr1 = a.Fr.off[r + 1];
            const uint64_t fs0 = a.Fs.off[s], fs1 = a.Fs.off[s + 1];
            const uint32_t nar = uint32_t(ar1 - ar0), nas = uint32_t(as1 - as0);
            const uint32_t nfr = uint32_t(fr1 - fr0), nfs = uint32_t(fs1 - fs0);
            if (!wave_join<K>(a.Ar.s + ar0, a.Ar.e + ar0, nar, a.As.s + as0, a.As.e + as0, nas,
                              lt, lane)) {
                v = APRIL_TN;
            } else if (wave_join<K>(a.Ar.s + ar0, a.Ar.e + ar0, nar, a.Fs.s + fs0, a.Fs.e + fs0,
                                    nfs, lt, lane) ||
                       wave_join<K>(a.Fr.s + fr0, a.Fr.e + fr0, nfr, a.As.s + as0, a.As.e + as0,
                                    nas, lt, lane)) {
                v = APRIL_TH;
            } else {
                v = APRIL_INDECISIVE;
            }
        }
        if (lane == 0) a.verdict[p] = v;
        c_tn += (v == APRIL_TN);
        c_th += (v == APRIL_TH);
        c_ind += (v == APRIL_INDECISIVE);
    }
    if (a.counts && lane == 0) {
        // the slot pointer is read from the kernel arguments only here, so
        // it holds no scalar registers during the loop (two more SGPRs cost
        // this kernel a third of its resident waves)
        typedef const __attribute__((address_space(4))) PlainArgs *KArgs;
        KArgs pk = (KArgs)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(pk));
        const unsigned long long v[3] = {c_tn, c_th, c_ind};
        add_totals(pk->ctr, blockIdx.x * kWavesPerBlock + w, v, 3);
    }
}

// One lane per pair: the verdict of Alg. 2 and the bytes it moves --
// 8 for the pair's ids, 16 per list whose CSR bounds it reads, 8 per distinct
// interval it reads (two uint32 endpoints), 1 for the verdict.
__global__ void k_alg2_bytes(FilterArgs a, unsigned long long *bytes) {
    for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < a.n_pairs;
         p += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t r = a.r[p], s = a.s[p];
        if (r >= a.n_r || s >= a.n_s) { bytes[p] = 0; continue; }
        const uint64_t ar0 = a.Ar.off[r], nar = a.Ar.off[r + 1] - ar0;
        const uint64_t as0 = a.As.off[s], nas = a.As.off[s + 1] - as0;
        uint32_t x, y, ax_r, ax_s, nfs = 0, nfr = 0, lists = 2;
        if (seq_join(a.Ar.s + ar0, a.Ar.e + ar0, uint32_t(nar), a.As.s + as0, a.As.e + as0,
                     uint32_t(nas), &x, &y)) {
            ax_r = x;
            ax_s = y;
            const uint64_t fs0 = a.Fs.off[s], nf = a.Fs.off[s + 1] - fs0;
            lists++;
            const bool af = seq_join(a.Ar.s + ar0, a.Ar.e + ar0, uint32_t(nar), a.Fs.s + fs0,
                                     a.Fs.e + fs0, uint32_t(nf), &x, &y);
            ax_r = max(ax_r, x);
            nfs = y;
            if (!af) {
                const uint64_t fr0 = a.Fr.off[r], nfr_ = a.Fr.off[r + 1] - fr0;
                lists++;
                seq_join(a.Fr.s + fr0, a.Fr.e + fr0, uint32_t(nfr_), a.As.s + as0, a.As.e + as0,
                         uint32_t(nas), &x, &y);
                nfr = x;
                ax_s = max(ax_s, y);
            }
        } else {
            ax_r = x;
            ax_s = y;
        }
        bytes[p] = 8ull + 16ull * lists + 8ull * (uint64_t(ax_r) + ax_s + nfs + nfr) + 1ull;
    }
}

__global__ void k_zero_counts(unsigned long long *c) {
    if (threadIdx.x < 3) c[threadIdx.x] = 0;
}

__global__ void k_clear_flag(unsigned int *f) { *f = 0; }

__global__ void k_check_pairs(const uint32_t *r, const uint32_t *s, uint64_t n, uint64_t n_r,
                              uint64_t n_s, unsigned int *bad) {
    for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
         p += uint64_t(gridDim.x) * blockDim.x)
        if (r[p] >= n_r || s[p] >= n_s) atomicOr(bad, 1u);
}

}  // namespace

int device_state(DeviceState **out) {
    static DeviceState states[64];
    static std::mutex mu;
    int dev = 0;
    APRIL_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(APRIL_E_NODEV, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(mu);
    DeviceState &st = states[dev];
    if (!st.cus) {
        hipDeviceProp_t p;
        APRIL_HIP_TRY(hipGetDeviceProperties(&p, dev));
        if (std::string(p.gcnArchName).rfind("gfx950", 0) != 0)
            return fail(APRIL_E_NODEV, std::string("library built for gfx950, device is ") + p.gcnArchName);
        // this device's copy of the static scratch (its own address on
        // every device); host code uses only this address, never the
        // array's name
        void *ptr = nullptr;
        APRIL_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        st.scratch = ptr;
        st.flag = reinterpret_cast<unsigned int *>(static_cast<char *>(ptr) + kStaticFlagOffset);
        st.cus = p.multiProcessorCount;
    }
    *out = &st;
    return APRIL_OK;
}

}  // namespace april

using namespace april;

static int check_lists(const april_lists_t *R, const april_lists_t *S) {
    if (!R || !S) return fail(APRIL_E_INVALID, "NULL lists");
    if (R->device < 0 || S->device < 0) return fail(APRIL_E_INVALID, "lists must be on a device");
    if (R->device != S->device) return fail(APRIL_E_INVALID, "lists on different devices");
    if (!same_grid(R->grid, S->grid) || R->partition_key != S->partition_key)
        return fail(APRIL_E_GRID, "R and S lists use different grids");
    int cur = 0;
    APRIL_HIP_TRY(hipGetDevice(&cur));
    if (cur != R->device) return fail(APRIL_E_INVALID, "current device does not hold the lists");
    return APRIL_OK;
}

namespace april {
FilterArgs make_args(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r, const uint32_t *d_s,
                     uint64_t n_pairs, uint8_t *d_verdict, unsigned long long *counts) {
    FilterArgs a;
    a.Ar = {R->d.off_a, R->d.start_a, R->d.end_a};
    a.Fr = {R->d.off_f, R->d.start_f, R->d.end_f};
    a.As = {S->d.off_a, S->d.start_a, S->d.end_a};
    a.Fs = {S->d.off_f, S->d.start_f, S->d.end_f};
    a.r = d_r;
    a.s = d_s;
    a.n_pairs = n_pairs;
    a.n_r = R->n;
    a.n_s = S->n;
    a.verdict = d_verdict;
    a.counts = counts;
    return a;
}
}  // namespace april

extern "C" int april_alg2_bytes(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                                const uint32_t *d_s, uint64_t n_pairs, uint64_t *d_bytes,
                                void *hip_stream) {
    clear_error();
    if (int rc = check_lists(R, S)) return rc;
    if (R->codec != S->codec) return fail(APRIL_E_INVALID, "R and S lists use different codecs");
    if (n_pairs == 0) return APRIL_OK;
    if (!d_r || !d_s || !d_bytes) return fail(APRIL_E_INVALID, "NULL pair/bytes array");
    DeviceState *st;
    if (int rc = device_state(&st)) return rc;
    if (R->codec == APRIL_CODEC_VBYTE)
        return launch_alg2_vbyte_bytes(R, S, d_r, d_s, n_pairs, reinterpret_cast<unsigned long long *>(d_bytes),
                                       st->cus, static_cast<hipStream_t>(hip_stream));
    FilterArgs a = make_args(R, S, d_r, d_s, n_pairs, nullptr, nullptr);
    const uint64_t blocks = std::min<uint64_t>((n_pairs + 255) / 256, uint64_t(st->cus) * 16);
    k_alg2_bytes<<<dim3(uint32_t(blocks)), dim3(256), 0, static_cast<hipStream_t>(hip_stream)>>>(
        a, reinterpret_cast<unsigned long long *>(d_bytes));
    APRIL_HIP_TRY(hipGetLastError());
    return APRIL_OK;
}

extern "C" int april_filter_pairs(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                                  const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict,
                                  uint64_t *d_counts, const april_filter_opts_t *opts,
                                  void *hip_stream) {
    clear_error();
    if (int rc = check_lists(R, S)) return rc;
    if (n_pairs && (!d_r || !d_s || !d_verdict)) return fail(APRIL_E_INVALID, "NULL pair/verdict array");
    april_filter_opts_t o{};
    if (opts) o = *opts;
    if (o.schedule != APRIL_SCHED_PLAIN && o.schedule != APRIL_SCHED_BATCHED)
        return fail(APRIL_E_INVALID, "unknown schedule");
    if (R->n >= 0x7fffffffull || S->n >= 0x7fffffffull)
        return fail(APRIL_E_INVALID, "collections must hold fewer than 2^31 - 1 objects");
    DeviceState *st;
    if (int rc = device_state(&st)) return rc;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    auto *counts = reinterpret_cast<unsigned long long *>(d_counts);
    if (n_pairs == 0) {
        if (counts) {
            k_zero_counts<<<1, 64, 0, stream>>>(counts);
            APRIL_HIP_TRY(hipGetLastError());
        }
        return APRIL_OK;
    }
    if (o.flags & APRIL_VALIDATE) {
        k_clear_flag<<<1, 1, 0, stream>>>(st->flag);
        APRIL_HIP_TRY(hipGetLastError());
        k_check_pairs<<<1024, 256, 0, stream>>>(d_r, d_s, n_pairs, R->n, S->n, st->flag);
        APRIL_HIP_TRY(hipGetLastError());
        unsigned int bad = 0;
        APRIL_HIP_TRY(hipMemcpyAsync(&bad, st->flag, sizeof(bad), hipMemcpyDeviceToHost, stream));
        APRIL_HIP_TRY(hipStreamSynchronize(stream));
        if (bad) return fail(APRIL_E_INVALID, "pair index out of range");
    }
    if (R->codec != S->codec) return fail(APRIL_E_INVALID, "R and S lists use different codecs");
    if (R->codec == APRIL_CODEC_VBYTE) {
        if (o.schedule != APRIL_SCHED_BATCHED)
            return fail(APRIL_E_INVALID, "compressed lists need the batched schedule");
        if (o.d_workspace) {
            if (o.workspace_bytes < kCtrBytes) return fail(APRIL_E_INVALID, "workspace too small");
            return launch_filter_vbyte(R, S, d_r, d_s, n_pairs, d_verdict, counts, o, st->cus, o.d_workspace,
                                       stream);
        }
        void *ws = nullptr;
        hipError_t e = hipMallocAsync(&ws, kCtrBytes, stream);
        if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
        const int rc = launch_filter_vbyte(R, S, d_r, d_s, n_pairs, d_verdict, counts, o, st->cus, ws, stream);
        APRIL_HIP_TRY(hipFreeAsync(ws, stream));
        return rc;
    }
    FilterArgs a = make_args(R, S, d_r, d_s, n_pairs, d_verdict, counts);
    if (o.schedule == APRIL_SCHED_BATCHED) {
        batched_defaults(o, BatchedShape{R->n_a + S->n_a, R->n + S->n, R->max_len, S->max_len});
        const uint64_t need = batched_workspace_bytes(n_pairs);
        if (o.d_workspace) {
            if (o.workspace_bytes < need) return fail(APRIL_E_INVALID, "workspace too small");
            return launch_batched(a, o, st->cus, o.d_workspace, stream);
        }
        void *ws = nullptr;
        hipError_t e = hipMallocAsync(&ws, need, stream);
        if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
        const int rc = launch_batched(a, o, st->cus, ws, stream);
        APRIL_HIP_TRY(hipFreeAsync(ws, stream));
        return rc;
    }
    // the counts are summed through the scratch slots (the caller's
    // workspace, else a stream-ordered allocation)
    void *ws = nullptr;
    if (counts) {
        if (o.d_workspace) {
            if (o.workspace_bytes < kCtrBytes) return fail(APRIL_E_INVALID, "workspace too small");
            ws = o.d_workspace;
        } else {
            hipError_t e = hipMallocAsync(&ws, kCtrBytes, stream);
            if (e != hipSuccess) return fail(APRIL_E_NOMEM, std::string("workspace: ") + hipGetErrorString(e));
        }
        k_zero_ctrs<<<1, 64, 0, stream>>>(static_cast<unsigned int *>(ws));
    }
    static int per_cu = 0;   // resident workgroups per CU (same on every gfx950 device)
    if (!per_cu) {
        int q = 0;
        APRIL_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k_filter_plain<4>, kBlock, 0));
        per_cu = q < 1 ? 1 : q;
    }
    // one resident wave per slot: a second round of waves would run the
    // statically assigned pairs after the first
    uint64_t waves = o.waves ? o.waves : uint64_t(st->cus) * per_cu * kWavesPerBlock;
    waves = std::min<uint64_t>(waves, n_pairs);
    const uint32_t xcds = uint32_t(xcd_count(st->cus));
    uint64_t blocks = std::max<uint64_t>(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
    blocks = (blocks + xcds - 1) / xcds * xcds;   // every XCD gets the same number of workgroups
    PlainArgs pa{a, static_cast<unsigned int *>(ws), xcds};
    k_filter_plain<4><<<dim3(uint32_t(blocks)), dim3(kBlock), 0, stream>>>(pa);
    hipError_t e = hipGetLastError();
    if (counts) {
        if (e == hipSuccess) {
            k_sum_totals<<<1, 64, 0, stream>>>(static_cast<unsigned int *>(ws), counts, 3);
            e = hipGetLastError();
        }
        if (!o.d_workspace) APRIL_HIP_TRY(hipFreeAsync(ws, stream));
    }
    if (e != hipSuccess) return fail(APRIL_E_HIP, std::string("filter launch: ") + hipGetErrorString(e));
    return APRIL_OK;
}

extern "C" int april_filter_pairs_static(const april_lists_t *R, const april_lists_t *S, const uint32_t *d_r,
                                         const uint32_t *d_s, uint64_t n_pairs, uint8_t *d_verdict,
                                         uint64_t *d_counts, const april_filter_opts_t *opts,
                                         void *hip_stream) {
    clear_error();
    april_filter_opts_t o{};
    if (opts) o = *opts;
    if (o.d_workspace || o.workspace_bytes)
        return fail(APRIL_E_INVALID, "april_filter_pairs_static takes no workspace (it uses the static scratch)");
    if (o.flags & APRIL_WS_DECODE_CACHE)
        return fail(APRIL_E_INVALID, "april_filter_pairs_static has no decode cache");
    if ((R && R->codec != APRIL_CODEC_RAW) || (S && S->codec != APRIL_CODEC_RAW))
        return fail(APRIL_E_INVALID,
                    "april_filter_pairs_static takes raw lists only (compressed lists need a decode cache)");
    const uint64_t need = batched_workspace_bytes(n_pairs);
    if (need > kStaticWorkspaceBytes)
        return fail(APRIL_E_INVALID, "this call needs " + std::to_string(need) + " bytes of scratch; the static "
                                     "scratch holds " + std::to_string(kStaticWorkspaceBytes));
    DeviceState *st;
    if (int rc = device_state(&st)) return rc;
    o.d_workspace = st->scratch;
    o.workspace_bytes = kStaticWorkspaceBytes;
    return april_filter_pairs(R, S, d_r, d_s, n_pairs, d_verdict, d_counts, &o, hip_stream);
}

extern "C" int april_filter_workspace_size(uint64_t n_pairs, const april_filter_opts_t *opts,
                                           uint64_t *bytes) {
    clear_error();
    if (!bytes) return fail(APRIL_E_INVALID, "NULL argument");
    *bytes = batched_workspace_bytes(n_pairs);   // plain: the scratch that sums the counts
    if (opts && (opts->flags & APRIL_WS_DECODE_CACHE)) {
        DeviceState *st;
        if (int rc = device_state(&st)) return rc;
        *bytes = vbyte_cache_offset() + vbyte_cache_bytes(st->cus);
    }
    return APRIL_OK;
}
