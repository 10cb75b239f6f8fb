// Served selection queries (Sec. 4.3.1) with continuous batching.
//
// A query polygon QP is answered against a device-resident collection S:
// its A-/F-lists are built on the host (one-step intervalization), the MBR
// grid index of S gives the candidate pairs (QP, s) on the device, and the
// intermediate filter classifies them.  Requests flow through three stages:
//
//   submit -> builder threads (lists, MBR cell range, pair upper bound;
//             large queries: one device thread builds all those queued in
//             one call)
//          -> dispatcher: packs ready requests into the next free slot while
//             the slot's device memory (pairs, intervals, queries) suffices
//             -> slot phase A on its stream: H2D of the batch's lists and MBRs,
//                probe kernel, D2H of the pair count
//             -> slot phase B: filter (batched schedule, slot workspace), D2H
//                of pairs and verdicts
//          -> results split per request, sorted by S id, ticket ready.
//
// Several slots are in flight at once on their own streams, so requests that
// arrive while others are on the GPU are admitted as soon as a slot frees up
// and their work overlaps on the device.  A request whose lists or pair
// bound alone exceed a slot's capacity fails with APRIL_E_NOMEM.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>

#include "internal.hpp"

namespace {

using april::fail;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum ReqState { RQ_QUEUED, RQ_BUILT, RQ_RUNNING, RQ_DONE, RQ_FAILED };

// A request is shared by whoever holds it: the ticket table, a queue, a
// builder thread, a slot's batch, and callers blocked in april_serve_wait.
// It is freed with the last of them, so a cancel or a release never frees a
// request another thread still reads.  Every field is read and written under
// the server's mutex, except the query and the lists, which only the thread
// holding the request in its stage touches.
struct Req {
    uint64_t ticket = 0;
    std::vector<double> xy;
    april::ProbeQuery q{};
    april_lists_t *lists = nullptr;   // host lists of the query (1 object)
    uint64_t pair_bound = 0;
    int state = RQ_QUEUED;
    int rc = APRIL_OK;
    bool cancelled = false;           // cancelled: no longer in the ticket table
    double t_submit = 0, t_built = 0, t_done = 0;
    std::vector<uint32_t> s_ids;
    std::vector<uint8_t> verdict;
    uint64_t counts[3] = {0, 0, 0};
    ~Req() {
        if (lists) april_lists_free(lists);
    }
};
using ReqPtr = std::shared_ptr<Req>;

enum SlotState { SL_FREE, SL_PROBING, SL_FILTERING };

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int state = SL_FREE;      // written by the dispatcher under the server's mutex
    std::vector<ReqPtr> batch;
    uint64_t n_pairs = 0;
    // device
    void *d_block = nullptr;
    april::ProbeQuery *d_q = nullptr;
    uint32_t *d_pr = nullptr, *d_ps = nullptr;
    uint8_t *d_v = nullptr;
    uint64_t *d_counts = nullptr;
    unsigned int *d_n = nullptr;
    void *d_ws = nullptr;
    uint64_t ws_bytes = 0;
    april_lists Q;   // device view of the batch's query lists (no ownership)
    // pinned host staging
    void *h_block = nullptr;
    april::ProbeQuery *h_q = nullptr;
    uint64_t *h_offa = nullptr, *h_offf = nullptr;
    uint32_t *h_sa = nullptr, *h_ea = nullptr, *h_sf = nullptr, *h_ef = nullptr;
    uint32_t *h_pr = nullptr, *h_ps = nullptr;
    uint8_t *h_v = nullptr;
    unsigned int *h_n = nullptr;
};

}  // namespace

struct april_server {
    const april_lists_t *S = nullptr;
    int device = 0;
    april_filter_opts_t fopts{};
    double cell_lattice = 1;       // grid cell side of S, lattice units
    double gpu_build_cells = 0;    // queries spanning this many cells or more build on the GPU
    // MBR grid index of S
    uint32_t G = 0;
    double lo[2] = {0, 0}, cs = 1;
    std::vector<uint64_t> sat;   // (G+1)^2 summed-area table of cell entry counts
    void *d_index = nullptr;
    uint32_t *d_cell_off = nullptr, *d_cell_ids = nullptr;
    double *d_boxes = nullptr;
    uint16_t *d_cells = nullptr;
    // slot capacities
    uint64_t cap_pairs = 0, cap_intervals = 0, cap_queries = 0;
    std::vector<Slot> slots;
    // requests
    std::mutex mu;
    std::condition_variable cv_build, cv_gpu, cv_dispatch, cv_done;   // host builders, device builder,
                                                                      // dispatcher, waiters
    std::deque<ReqPtr> to_build, to_gpu, ready;   // host builds, device builds, built
    std::map<uint64_t, ReqPtr> reqs;   // live tickets (not released, not cancelled)
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> builders;
    std::thread gpu_builder;
    int builders_busy = 0;        // builder threads with a request in hand (under mu)
    std::thread dispatcher;
    int dispatcher_rc = APRIL_OK;
};

namespace {

uint32_t cell_of(const april_server *sv, double v, int axis) {
    double c = std::floor((v - sv->lo[axis]) / sv->cs);
    if (c < 0) c = 0;
    if (c > double(sv->G - 1)) c = double(sv->G - 1);
    return uint32_t(c);
}

uint64_t sat_sum(const april_server *sv, uint32_t x0, uint32_t y0, uint32_t x1, uint32_t y1) {
    const uint64_t W = sv->G + 1;
    auto at = [&](uint32_t x, uint32_t y) { return sv->sat[uint64_t(y) * W + x]; };
    return at(x1 + 1, y1 + 1) - at(x0, y1 + 1) - at(x1 + 1, y0) + at(x0, y0);
}

// Boundary cells of a query, estimated from its edges' extents (in cells).
double est_cells(const april_server *sv, const std::vector<double> &xy) {
    const size_t nv = xy.size() / 2;
    double cells = 0;
    for (size_t v = 0; v < nv; v++) {
        const size_t v2 = v + 1 == nv ? 0 : v + 1;
        cells += (std::fabs(xy[2 * v2] - xy[2 * v]) + std::fabs(xy[2 * v2 + 1] - xy[2 * v + 1])) * 1073741824.0 /
                     sv->cell_lattice + 2;
    }
    return cells;
}

// A query's lists are built (rc, L): its MBR and grid-cell range, the
// upper bound of its pairs, the capacity checks, then ready for a slot (or
// failed).  Takes the server's mutex.
void finish_build(april_server *sv, const ReqPtr &q, april_lists_t *L, int rc) {
    const uint64_t nv = q->xy.size() / 2;
    if (rc == APRIL_OK) {
        double b[4] = {q->xy[0], q->xy[1], q->xy[0], q->xy[1]};
        for (uint64_t k = 1; k < nv; k++) {
            b[0] = std::min(b[0], q->xy[2 * k]);
            b[1] = std::min(b[1], q->xy[2 * k + 1]);
            b[2] = std::max(b[2], q->xy[2 * k]);
            b[3] = std::max(b[3], q->xy[2 * k + 1]);
        }
        q->q = april::ProbeQuery{b[0], b[1], b[2], b[3], cell_of(sv, b[0], 0), cell_of(sv, b[1], 1),
                                 cell_of(sv, b[2], 0), cell_of(sv, b[3], 1)};
        q->pair_bound = sat_sum(sv, q->q.cx0, q->q.cy0, q->q.cx1, q->q.cy1);
        if (L->n_a + L->n_f > sv->cap_intervals || q->pair_bound > sv->cap_pairs) rc = APRIL_E_NOMEM;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    q->lists = L;
    q->t_built = now_s();
    if (q->cancelled) return;   // cancelled while being built: dropped with the last holder
    if (rc != APRIL_OK) {
        q->rc = rc;
        q->state = RQ_FAILED;
        q->t_done = q->t_built;
        sv->cv_done.notify_all();
    } else {
        q->state = RQ_BUILT;
        sv->ready.push_back(q);
        sv->cv_dispatch.notify_one();
    }
}

// Builder threads: the lists of small queries, on the host.
void builder_main(april_server *sv) {
    for (;;) {
        ReqPtr q;
        int threads = 1;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_build.wait(lk, [&] { return sv->stop || !sv->to_build.empty(); });
            if (sv->stop) return;
            q = sv->to_build.front();
            sv->to_build.pop_front();
            q->state = RQ_BUILT;   // held by this builder from now on
            // a large query may use the builders that are idle with nothing
            // queued; under load every query is built on its own thread
            threads = sv->to_build.empty() ? int(sv->builders.size()) - sv->builders_busy : 1;
            sv->builders_busy++;
        }
        const uint64_t off[2] = {0, q->xy.size() / 2};
        april_lists_t *L = nullptr;
        const int rc = april::build_lists_threads(&sv->S->grid, q->xy.data(), off, 1, 0, std::max(1, threads), &L);
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->builders_busy--;
        }
        finish_build(sv, q, L, rc);
    }
}

// The lists of the queued large queries, built on the device in one call
// (all of them at once, so the call's synchronizations and launches are
// shared), read back, split per query.  On error the batch's queries are
// built one by one on the host, so that each gets its own result.
void gpu_build_batch(april_server *sv, std::vector<ReqPtr> &batch, hipStream_t stream) {
    std::vector<double> xy;
    std::vector<uint64_t> off(1, 0);
    for (const ReqPtr &q : batch) {
        xy.insert(xy.end(), q->xy.begin(), q->xy.end());
        off.push_back(off.back() + q->xy.size() / 2);
    }
    april_lists_t *Ld = nullptr, *L = nullptr;
    int rc = april_build_lists_gpu(&sv->S->grid, xy.data(), off.data(), batch.size(), 0, stream, &Ld);
    if (rc == APRIL_OK) rc = april_lists_download(Ld, stream, &L);
    if (Ld) april_lists_free(Ld);
    for (size_t k = 0; k < batch.size(); k++) {
        april_lists_t *Lq = nullptr;
        int rq = rc;
        if (rc == APRIL_OK) {
            const uint64_t a0 = L->off_a[k], a1 = L->off_a[k + 1], f0 = L->off_f[k], f1 = L->off_f[k + 1];
            const uint64_t oa[2] = {0, a1 - a0}, of[2] = {0, f1 - f0};
            rq = april_lists_from_arrays(&sv->S->grid, 1, oa, L->start_a.data() + a0, L->end_a.data() + a0, of,
                                         L->start_f.data() + f0, L->end_f.data() + f0, 0, &Lq);
        } else {
            const uint64_t o1[2] = {0, batch[k]->xy.size() / 2};
            rq = april::build_lists_threads(&sv->S->grid, batch[k]->xy.data(), o1, 1, 0, 1, &Lq);
        }
        finish_build(sv, batch[k], Lq, rq);
    }
    if (L) april_lists_free(L);
}

// The device builder thread: takes every large query queued (up to
// kGpuBuildVertices vertices) and builds them in one device call.  (Batches
// capped at 4M grid cells on two such threads served 2,564 queries/s at
// saturation against 4,159: the calls' fixed costs, paid per batch, then
// bound the build rate.)
constexpr uint64_t kGpuBuildVertices = 4u << 20;

void gpu_builder_main(april_server *sv) {
    hipStream_t stream = nullptr;
    if (hipSetDevice(sv->device) != hipSuccess ||
        hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess)
        stream = nullptr;
    for (;;) {
        std::vector<ReqPtr> batch;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_gpu.wait(lk, [&] { return sv->stop || !sv->to_gpu.empty(); });
            if (sv->stop) break;
            uint64_t nv = 0;
            while (!sv->to_gpu.empty() &&
                   (batch.empty() || nv + sv->to_gpu.front()->xy.size() / 2 <= kGpuBuildVertices)) {
                batch.push_back(sv->to_gpu.front());
                sv->to_gpu.pop_front();
                batch.back()->state = RQ_BUILT;   // held by this thread from now on
                nv += batch.back()->xy.size() / 2;
            }
        }
        if (stream) {
            gpu_build_batch(sv, batch, stream);
        } else {
            for (const ReqPtr &q : batch) finish_build(sv, q, nullptr, fail(APRIL_E_HIP, "builder stream"));
        }
    }
    if (stream) (void)hipStreamDestroy(stream);
}

// Phase A: stage the batch, probe the MBR grid, read back the pair count.
int slot_phase_a(april_server *sv, Slot &sl) {
    const uint64_t nq = sl.batch.size();
    uint64_t na = 0, nf = 0;
    for (uint64_t k = 0; k < nq; k++) {
        const april_lists_t *L = sl.batch[k]->lists;
        sl.h_q[k] = sl.batch[k]->q;
        sl.h_offa[k] = na;
        sl.h_offf[k] = nf;
        std::copy(L->start_a.begin(), L->start_a.end(), sl.h_sa + na);
        std::copy(L->end_a.begin(), L->end_a.end(), sl.h_ea + na);
        std::copy(L->start_f.begin(), L->start_f.end(), sl.h_sf + nf);
        std::copy(L->end_f.begin(), L->end_f.end(), sl.h_ef + nf);
        na += L->n_a;
        nf += L->n_f;
    }
    sl.h_offa[nq] = na;
    sl.h_offf[nq] = nf;
    april_lists &Q = sl.Q;
    Q.n = nq;
    Q.n_a = na;
    Q.n_f = nf;
    auto h2d = [&](void *d, const void *h, size_t b) {
        return b ? hipMemcpyAsync(d, h, b, hipMemcpyHostToDevice, sl.stream) : hipSuccess;
    };
    APRIL_HIP_TRY(h2d(sl.d_q, sl.h_q, sizeof(april::ProbeQuery) * nq));
    APRIL_HIP_TRY(h2d(Q.d.off_a, sl.h_offa, 8 * (nq + 1)));
    APRIL_HIP_TRY(h2d(Q.d.off_f, sl.h_offf, 8 * (nq + 1)));
    APRIL_HIP_TRY(h2d(Q.d.start_a, sl.h_sa, 4 * na));
    APRIL_HIP_TRY(h2d(Q.d.end_a, sl.h_ea, 4 * na));
    APRIL_HIP_TRY(h2d(Q.d.start_f, sl.h_sf, 4 * nf));
    APRIL_HIP_TRY(h2d(Q.d.end_f, sl.h_ef, 4 * nf));
    APRIL_HIP_TRY(hipMemsetAsync(sl.d_n, 0, sizeof(unsigned int), sl.stream));
    if (int rc = april::launch_probe(sl.d_q, uint32_t(nq), sv->d_cell_off, sv->d_cell_ids, sv->d_boxes,
                                     sv->d_cells, sv->G, sl.d_pr, sl.d_ps, uint32_t(sv->cap_pairs), sl.d_n,
                                     sl.stream))
        return rc;
    APRIL_HIP_TRY(hipMemcpyAsync(sl.h_n, sl.d_n, sizeof(unsigned int), hipMemcpyDeviceToHost, sl.stream));
    APRIL_HIP_TRY(hipEventRecord(sl.ev, sl.stream));
    std::lock_guard<std::mutex> lk(sv->mu);
    sl.state = SL_PROBING;
    return APRIL_OK;
}

// Phase B: filter the batch's pairs, read back pairs and verdicts.
int slot_phase_b(april_server *sv, Slot &sl) {
    sl.n_pairs = std::min<uint64_t>(*sl.h_n, sv->cap_pairs);
    if (sl.n_pairs) {
        april_filter_opts_t o = sv->fopts;
        o.schedule = APRIL_SCHED_BATCHED;
        o.d_workspace = sl.d_ws;
        o.workspace_bytes = sl.ws_bytes;
        if (int rc = april_filter_pairs(&sl.Q, sv->S, sl.d_pr, sl.d_ps, sl.n_pairs, sl.d_v, sl.d_counts, &o,
                                        sl.stream))
            return rc;
        APRIL_HIP_TRY(hipMemcpyAsync(sl.h_pr, sl.d_pr, 4 * sl.n_pairs, hipMemcpyDeviceToHost, sl.stream));
        APRIL_HIP_TRY(hipMemcpyAsync(sl.h_ps, sl.d_ps, 4 * sl.n_pairs, hipMemcpyDeviceToHost, sl.stream));
        APRIL_HIP_TRY(hipMemcpyAsync(sl.h_v, sl.d_v, sl.n_pairs, hipMemcpyDeviceToHost, sl.stream));
    }
    APRIL_HIP_TRY(hipEventRecord(sl.ev, sl.stream));
    std::lock_guard<std::mutex> lk(sv->mu);
    sl.state = SL_FILTERING;
    return APRIL_OK;
}

// Split a finished batch into per-request results (sorted by S id).
void slot_finish(april_server *sv, Slot &sl) {
    const uint64_t nq = sl.batch.size();
    std::vector<uint64_t> cnt(nq + 1, 0);
    for (uint64_t t = 0; t < sl.n_pairs; t++) cnt[sl.h_pr[t] + 1]++;
    for (uint64_t k = 0; k < nq; k++) cnt[k + 1] += cnt[k];
    std::vector<uint64_t> idx(sl.n_pairs);
    {
        std::vector<uint64_t> pos(cnt.begin(), cnt.end() - 1);
        for (uint64_t t = 0; t < sl.n_pairs; t++) idx[pos[sl.h_pr[t]]++] = t;
    }
    const double t = now_s();
    std::lock_guard<std::mutex> lk(sv->mu);
    for (uint64_t k = 0; k < nq; k++) {
        Req *q = sl.batch[k].get();
        std::vector<std::pair<uint32_t, uint8_t>> sv_pairs;
        sv_pairs.reserve(cnt[k + 1] - cnt[k]);
        for (uint64_t u = cnt[k]; u < cnt[k + 1]; u++) sv_pairs.emplace_back(sl.h_ps[idx[u]], sl.h_v[idx[u]]);
        std::sort(sv_pairs.begin(), sv_pairs.end());
        q->s_ids.resize(sv_pairs.size());
        q->verdict.resize(sv_pairs.size());
        q->counts[0] = q->counts[1] = q->counts[2] = 0;
        for (size_t u = 0; u < sv_pairs.size(); u++) {
            q->s_ids[u] = sv_pairs[u].first;
            q->verdict[u] = sv_pairs[u].second;
            if (sv_pairs[u].second <= APRIL_INDECISIVE) q->counts[sv_pairs[u].second]++;
        }
        april_lists_free(q->lists);
        q->lists = nullptr;
        q->state = RQ_DONE;
        q->t_done = t;
    }
    sl.batch.clear();   // cancelled requests are freed here, unless a waiter still holds one
    sl.state = SL_FREE;
    sv->cv_done.notify_all();
}

void fail_batch(april_server *sv, Slot &sl, int rc) {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (const ReqPtr &q : sl.batch) {
        q->rc = rc;
        q->state = RQ_FAILED;
        q->t_done = now_s();
        if (q->lists) { april_lists_free(q->lists); q->lists = nullptr; }
    }
    sl.batch.clear();
    sl.state = SL_FREE;
    sv->cv_done.notify_all();
}

void dispatcher_main(april_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        bool progressed = false;
        // advance slots whose stream work has completed
        for (Slot &sl : sv->slots) {
            if (sl.state == SL_FREE) continue;
            const hipError_t e = hipEventQuery(sl.ev);
            if (e == hipErrorNotReady) continue;
            progressed = true;
            if (e != hipSuccess) { fail_batch(sv, sl, APRIL_E_HIP); continue; }
            if (sl.state == SL_PROBING) {
                if (int rc = slot_phase_b(sv, sl)) fail_batch(sv, sl, rc);
            } else {
                slot_finish(sv, sl);
            }
        }
        // admit ready requests into a free slot
        Slot *free_slot = nullptr;
        for (Slot &sl : sv->slots)
            if (sl.state == SL_FREE) { free_slot = &sl; break; }
        if (free_slot) {
            std::unique_lock<std::mutex> lk(sv->mu);
            uint64_t pairs = 0, ivs = 0;
            while (!sv->ready.empty() && free_slot->batch.size() < sv->cap_queries) {
                ReqPtr q = sv->ready.front();
                if (q->cancelled) { sv->ready.pop_front(); continue; }
                const uint64_t qi = q->lists->n_a + q->lists->n_f;
                if (!free_slot->batch.empty() &&
                    (pairs + q->pair_bound > sv->cap_pairs || ivs + qi > sv->cap_intervals))
                    break;   // the slot is full: the request waits for the next one
                pairs += q->pair_bound;
                ivs += qi;
                q->state = RQ_RUNNING;
                free_slot->batch.push_back(q);
                sv->ready.pop_front();
            }
            lk.unlock();
            if (!free_slot->batch.empty()) {
                progressed = true;
                if (int rc = slot_phase_a(sv, *free_slot)) fail_batch(sv, *free_slot, rc);
            }
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stop) {
            bool busy = false;
            for (Slot &sl : sv->slots) busy |= sl.state != SL_FREE;
            if (!busy) return;
        }
        if (!progressed) {
            bool busy = false;
            for (Slot &sl : sv->slots) busy |= sl.state != SL_FREE;
            // poll in-flight slots often; sleep until work arrives otherwise
            if (busy) sv->cv_dispatch.wait_for(lk, std::chrono::microseconds(50));
            else sv->cv_dispatch.wait_for(lk, std::chrono::milliseconds(5),
                                          [&] { return sv->stop || !sv->ready.empty(); });
        }
    }
}

int alloc_slot(april_server *sv, Slot &sl) {
    const uint64_t P = sv->cap_pairs, I = sv->cap_intervals, NQ = sv->cap_queries;
    sl.ws_bytes = 0;
    april_filter_opts_t o{};
    o.schedule = APRIL_SCHED_BATCHED;
    if (int rc = april_filter_workspace_size(P, &o, &sl.ws_bytes)) return rc;
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    const uint64_t b_q = up(sizeof(april::ProbeQuery) * NQ), b_off = up(8 * (NQ + 1)), b_i = up(4 * I),
                   b_p = up(4 * P), b_v = up(P), b_c = up(24), b_n = up(4), b_ws = up(sl.ws_bytes);
    const uint64_t dev_total = b_q + 2 * b_off + 4 * b_i + 2 * b_p + b_v + b_c + b_n + b_ws;
    hipError_t e = hipMalloc(&sl.d_block, dev_total);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, "server slot: device memory");
    char *d = static_cast<char *>(sl.d_block);
    sl.d_q = reinterpret_cast<april::ProbeQuery *>(d); d += b_q;
    sl.Q.d.off_a = reinterpret_cast<uint64_t *>(d); d += b_off;
    sl.Q.d.off_f = reinterpret_cast<uint64_t *>(d); d += b_off;
    sl.Q.d.start_a = reinterpret_cast<uint32_t *>(d); d += b_i;
    sl.Q.d.end_a = reinterpret_cast<uint32_t *>(d); d += b_i;
    sl.Q.d.start_f = reinterpret_cast<uint32_t *>(d); d += b_i;
    sl.Q.d.end_f = reinterpret_cast<uint32_t *>(d); d += b_i;
    sl.d_pr = reinterpret_cast<uint32_t *>(d); d += b_p;
    sl.d_ps = reinterpret_cast<uint32_t *>(d); d += b_p;
    sl.d_v = reinterpret_cast<uint8_t *>(d); d += b_v;
    sl.d_counts = reinterpret_cast<uint64_t *>(d); d += b_c;
    sl.d_n = reinterpret_cast<unsigned int *>(d); d += b_n;
    sl.d_ws = d;
    sl.Q.grid = sv->S->grid;
    sl.Q.device = sv->device;
    sl.Q.codec = APRIL_CODEC_RAW;
    sl.Q.d.block = nullptr;
    const uint64_t host_total = b_q + 2 * b_off + 4 * b_i + 2 * b_p + b_v + b_n;
    e = hipHostMalloc(&sl.h_block, host_total, hipHostMallocDefault);
    if (e != hipSuccess) return fail(APRIL_E_NOMEM, "server slot: pinned host memory");
    char *h = static_cast<char *>(sl.h_block);
    sl.h_q = reinterpret_cast<april::ProbeQuery *>(h); h += b_q;
    sl.h_offa = reinterpret_cast<uint64_t *>(h); h += b_off;
    sl.h_offf = reinterpret_cast<uint64_t *>(h); h += b_off;
    sl.h_sa = reinterpret_cast<uint32_t *>(h); h += b_i;
    sl.h_ea = reinterpret_cast<uint32_t *>(h); h += b_i;
    sl.h_sf = reinterpret_cast<uint32_t *>(h); h += b_i;
    sl.h_ef = reinterpret_cast<uint32_t *>(h); h += b_i;
    sl.h_pr = reinterpret_cast<uint32_t *>(h); h += b_p;
    sl.h_ps = reinterpret_cast<uint32_t *>(h); h += b_p;
    sl.h_v = reinterpret_cast<uint8_t *>(h); h += b_v;
    sl.h_n = reinterpret_cast<unsigned int *>(h);
    APRIL_HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    APRIL_HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    return APRIL_OK;
}

void destroy(april_server *sv) {
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_build.notify_all();
    sv->cv_gpu.notify_all();
    sv->cv_dispatch.notify_all();
    for (auto &t : sv->builders)
        if (t.joinable()) t.join();
    if (sv->gpu_builder.joinable()) sv->gpu_builder.join();
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    for (Slot &sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.d_block) (void)hipFree(sl.d_block);
        if (sl.h_block) (void)hipHostFree(sl.h_block);
    }
    if (sv->d_index) (void)hipFree(sv->d_index);
    delete sv;   // frees the requests no caller holds any more
}

}  // namespace

using namespace april;

extern "C" {

int april_serve_create(const april_lists_t *S, const double *boxes, const april_serve_opts_t *opts,
                       april_server_t **out) {
    clear_error();
    if (!S || !boxes || !out) return fail(APRIL_E_INVALID, "NULL argument");
    if (S->device < 0) return fail(APRIL_E_INVALID, "S must be device-resident");
    if (S->n == 0 || S->n > 0x7ffffffeull) return fail(APRIL_E_INVALID, "S size out of range");
    april_serve_opts_t o{};
    if (opts) o = *opts;
    const uint32_t G = o.mbr_grid ? o.mbr_grid : 1024;
    if (G > 65535) return fail(APRIL_E_INVALID, "mbr_grid must be at most 65535");
    const uint32_t nslots = o.slots ? o.slots : 3;
    const uint64_t budget = o.mem_budget ? o.mem_budget : (uint64_t(2) << 30);
    auto *sv = new (std::nothrow) april_server;
    if (!sv) return fail(APRIL_E_NOMEM, "out of host memory");
    sv->S = S;
    sv->device = S->device;
    sv->fopts = o.filter;
    sv->G = G;
    {
        april::LatticeGrid lg;
        if (int rc = april::lattice_grid(&S->grid, &lg)) {
            delete sv;
            return rc;
        }
        sv->cell_lattice = double(lg.w);
        sv->gpu_build_cells = o.gpu_build_cells == 0xFFFFFFFFu ? 1e300
                              : o.gpu_build_cells ? double(o.gpu_build_cells) : 262144.0;
    }
    if (o.reserved) {
        delete sv;
        return fail(APRIL_E_INVALID, "reserved option must be 0");
    }
    // per-slot capacities: 70% of a slot's share for pairs (13 bytes each:
    // two ids, a verdict, a queue entry), 30% for query intervals (8 bytes)
    const uint64_t per_slot = budget / nslots;
    sv->cap_pairs = std::max<uint64_t>(1024, per_slot * 7 / 10 / 13);
    sv->cap_pairs = std::min<uint64_t>(sv->cap_pairs, 0x7fffffffull);
    sv->cap_intervals = std::max<uint64_t>(1024, per_slot * 3 / 10 / 8);
    sv->cap_queries = o.max_batch ? o.max_batch : 8192;
    // uniform MBR grid over S's extent
    const uint64_t n = S->n;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (uint64_t k = 0; k < n; k++) {
        const double *b = boxes + 4 * k;
        if (!(b[0] <= b[2] && b[1] <= b[3])) { delete sv; return fail(APRIL_E_INVALID, "box with min > max"); }
        lo[0] = std::min(lo[0], b[0]); lo[1] = std::min(lo[1], b[1]);
        hi[0] = std::max(hi[0], b[2]); hi[1] = std::max(hi[1], b[3]);
    }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], 1e-300});
    sv->lo[0] = lo[0];
    sv->lo[1] = lo[1];
    sv->cs = ext / G;
    std::vector<uint16_t> cells(4 * n);
    std::vector<uint64_t> cnt(uint64_t(G) * G + 1, 0);
    for (uint64_t k = 0; k < n; k++) {
        const double *b = boxes + 4 * k;
        uint16_t *c = &cells[4 * k];
        c[0] = uint16_t(cell_of(sv, b[0], 0));
        c[1] = uint16_t(cell_of(sv, b[1], 1));
        c[2] = uint16_t(cell_of(sv, b[2], 0));
        c[3] = uint16_t(cell_of(sv, b[3], 1));
        for (uint32_t y = c[1]; y <= c[3]; y++)
            for (uint32_t x = c[0]; x <= c[2]; x++) cnt[uint64_t(y) * G + x + 1]++;
    }
    // summed-area table of entry counts for pair upper bounds
    sv->sat.assign(uint64_t(G + 1) * (G + 1), 0);
    for (uint32_t y = 0; y < G; y++)
        for (uint32_t x = 0; x < G; x++)
            sv->sat[uint64_t(y + 1) * (G + 1) + x + 1] = cnt[uint64_t(y) * G + x + 1] +
                                                          sv->sat[uint64_t(y) * (G + 1) + x + 1] +
                                                          sv->sat[uint64_t(y + 1) * (G + 1) + x] -
                                                          sv->sat[uint64_t(y) * (G + 1) + x];
    for (uint64_t c = 1; c < cnt.size(); c++) cnt[c] += cnt[c - 1];
    if (cnt.back() > 0xffffffffull) { delete sv; return fail(APRIL_E_NOMEM, "MBR index too large"); }
    std::vector<uint32_t> off(cnt.begin(), cnt.end()), ids(cnt.back());
    {
        std::vector<uint64_t> pos(cnt.begin(), cnt.end() - 1);
        for (uint64_t k = 0; k < n; k++) {
            const uint16_t *c = &cells[4 * k];
            for (uint32_t y = c[1]; y <= c[3]; y++)
                for (uint32_t x = c[0]; x <= c[2]; x++) ids[pos[uint64_t(y) * G + x]++] = uint32_t(k);
        }
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != sv->device) (void)hipSetDevice(sv->device);
    auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
    const uint64_t b_off = up(4 * off.size()), b_ids = up(4 * std::max<size_t>(ids.size(), 1)),
                   b_box = up(8 * 4 * n), b_cell = up(2 * 4 * n);
    if (hipMalloc(&sv->d_index, b_off + b_ids + b_box + b_cell) != hipSuccess) {
        delete sv;
        return fail(APRIL_E_NOMEM, "MBR index: device memory");
    }
    char *d = static_cast<char *>(sv->d_index);
    sv->d_cell_off = reinterpret_cast<uint32_t *>(d); d += b_off;
    sv->d_cell_ids = reinterpret_cast<uint32_t *>(d); d += b_ids;
    sv->d_boxes = reinterpret_cast<double *>(d); d += b_box;
    sv->d_cells = reinterpret_cast<uint16_t *>(d);
    hipError_t e = hipMemcpy(sv->d_cell_off, off.data(), 4 * off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ids.empty()) e = hipMemcpy(sv->d_cell_ids, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sv->d_boxes, boxes, 8 * 4 * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(sv->d_cells, cells.data(), 2 * 4 * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy(sv);
        return fail(APRIL_E_HIP, std::string("MBR index upload: ") + hipGetErrorString(e));
    }
    sv->slots.resize(nslots);
    for (Slot &sl : sv->slots) {
        if (int rc = alloc_slot(sv, sl)) {
            const std::string msg = april_last_error();
            destroy(sv);
            return fail(rc, msg);
        }
    }
    const int nb = o.host_threads ? int(o.host_threads) : std::max(1, host_threads() - 2);
    for (int t = 0; t < nb; t++) sv->builders.emplace_back(builder_main, sv);
    sv->gpu_builder = std::thread(gpu_builder_main, sv);
    sv->dispatcher = std::thread(dispatcher_main, sv);
    *out = sv;
    return APRIL_OK;
}

int april_serve_submit(april_server_t *sv, const double *xy, uint64_t n_vertices, uint64_t *ticket) {
    clear_error();
    if (!sv || !xy || !ticket) return fail(APRIL_E_INVALID, "NULL argument");
    if (n_vertices < 3) return fail(APRIL_E_INVALID, "query with < 3 vertices");
    ReqPtr q;
    try {
        q = std::make_shared<Req>();
        q->xy.assign(xy, xy + 2 * n_vertices);
    } catch (const std::bad_alloc &) {
        return fail(APRIL_E_NOMEM, "out of host memory");
    }
    q->t_submit = now_s();
    std::lock_guard<std::mutex> lk(sv->mu);
    q->ticket = sv->next_ticket++;
    sv->reqs[q->ticket] = q;
    if (est_cells(sv, q->xy) >= sv->gpu_build_cells) {
        sv->to_gpu.push_back(q);
        sv->cv_gpu.notify_one();
    } else {
        sv->to_build.push_back(q);
        sv->cv_build.notify_one();
    }
    *ticket = q->ticket;
    return APRIL_OK;
}

static void fill_result(const Req *q, april_result_t *out) {
    memset(out, 0, sizeof(*out));
    out->t_submit = q->t_submit;
    out->t_built = q->t_built;
    out->t_done = q->t_done;
    if (q->state == RQ_FAILED) { out->status = q->rc; return; }
    if (q->state != RQ_DONE) { out->status = APRIL_PENDING; return; }
    out->status = APRIL_OK;
    out->n_pairs = q->s_ids.size();
    out->s_ids = q->s_ids.data();
    out->verdict = q->verdict.data();
    for (int k = 0; k < 3; k++) out->counts[k] = q->counts[k];
}

int april_serve_poll(april_server_t *sv, uint64_t ticket, april_result_t *out) {
    clear_error();
    if (!sv || !out) return fail(APRIL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(APRIL_E_INVALID, "unknown ticket");
    fill_result(it->second.get(), out);
    if (out->status < 0) fail(out->status, "request failed");
    return out->status;
}

int april_serve_wait(april_server_t *sv, uint64_t ticket, double timeout_s, april_result_t *out) {
    clear_error();
    if (!sv || !out) return fail(APRIL_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(APRIL_E_INVALID, "unknown ticket");
    const ReqPtr q = it->second;   // held while waiting: a cancel or release cannot free it
    sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                         [&] { return q->cancelled || q->state == RQ_DONE || q->state == RQ_FAILED; });
    if (q->cancelled || !sv->reqs.count(ticket)) return fail(APRIL_E_INVALID, "request cancelled or released");
    fill_result(q.get(), out);
    if (out->status < 0) fail(out->status, "request failed");
    return out->status;
}

int april_serve_release(april_server_t *sv, uint64_t ticket) {
    clear_error();
    if (!sv) return fail(APRIL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(APRIL_E_INVALID, "unknown ticket");
    const Req *q = it->second.get();
    if (q->state != RQ_DONE && q->state != RQ_FAILED) return fail(APRIL_E_INVALID, "request still pending");
    sv->reqs.erase(it);   // freed with the last holder
    return APRIL_OK;
}

int april_serve_cancel(april_server_t *sv, uint64_t ticket) {
    clear_error();
    if (!sv) return fail(APRIL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(APRIL_E_INVALID, "unknown ticket");
    const ReqPtr q = it->second;
    // out of the ticket table and the queues; a builder or a slot holding it
    // drops it when its stage ends, a waiter wakes and reports the cancel
    q->cancelled = true;
    for (auto *dq : {&sv->to_build, &sv->to_gpu, &sv->ready}) {
        auto f = std::find(dq->begin(), dq->end(), q);
        if (f != dq->end()) dq->erase(f);
    }
    sv->reqs.erase(it);
    sv->cv_done.notify_all();
    return APRIL_OK;
}

int april_serve_stats(april_server_t *sv, april_serve_stats_t *st) {
    clear_error();
    if (!sv || !st) return fail(APRIL_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    memset(st, 0, sizeof(*st));
    st->slots = uint32_t(sv->slots.size());
    for (const Slot &sl : sv->slots) st->slots_busy += sl.state != SL_FREE;
    st->queued = sv->to_build.size() + sv->to_gpu.size();
    st->ready = sv->ready.size();
    st->cap_pairs = sv->cap_pairs;
    st->cap_intervals = sv->cap_intervals;
    st->cap_queries = sv->cap_queries;
    return APRIL_OK;
}

void april_serve_destroy(april_server_t *sv) {
    if (sv) destroy(sv);
}

}  // extern "C"
