// MBR filter of the served form (Sec. 4.3.1: a query polygon's MBR selects
// the data polygons whose MBRs intersect it, then the intermediate filter
// runs on those pairs).
//
// S is indexed by a uniform G x G grid over its extent: every S object is
// registered in each grid cell its MBR overlaps (CSR cell -> ids), and its
// integer cell range is stored beside its box.  A query probes the cells its
// MBR overlaps and reports (q, s) only from the cell holding the lower-left
// corner of the two MBRs' intersection -- that cell is (max(qcx0, scx0),
// max(qcy0, scy0)) because the cell map is monotone -- so each pair appears
// exactly once.  One workgroup per query; pairs are appended with one atomic
// per wavefront.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "internal.hpp"

namespace april {
namespace {

__global__ __launch_bounds__(256) void k_probe(const ProbeQuery *__restrict__ q, uint32_t n_q,
                                               const uint32_t *__restrict__ cell_off,
                                               const uint32_t *__restrict__ cell_ids,
                                               const double *__restrict__ boxes,
                                               const uint16_t *__restrict__ cells, uint32_t G,
                                               uint32_t *pr, uint32_t *ps, uint32_t cap,
                                               unsigned int *count) {
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t k = blockIdx.x; k < n_q; k += gridDim.x) {
        const ProbeQuery Q = q[k];
        const uint32_t ncx = Q.cx1 - Q.cx0 + 1, ncy = Q.cy1 - Q.cy0 + 1;
        const uint64_t ncell = uint64_t(ncx) * ncy;
        // every thread walks cells; the entries of a cell are read by one thread
        for (uint64_t c = threadIdx.x; c < ncell; c += blockDim.x) {
            const uint32_t cx = Q.cx0 + uint32_t(c % ncx);
            const uint32_t cy = Q.cy0 + uint32_t(c / ncx);
            const uint32_t cell = cy * G + cx;
            uint32_t b = cell_off[cell];
            const uint32_t e = cell_off[cell + 1];
            for (;;) {
                bool emit = false;
                uint32_t s = 0;
                if (b < e) {
                    s = cell_ids[b++];
                    const double *sb = boxes + 4 * uint64_t(s);
                    const uint16_t *sc = cells + 4 * uint64_t(s);
                    const bool meet = Q.x0 <= sb[2] && sb[0] <= Q.x1 && Q.y0 <= sb[3] && sb[1] <= Q.y1;
                    const uint32_t rx = max(Q.cx0, uint32_t(sc[0])), ry = max(Q.cy0, uint32_t(sc[1]));
                    emit = meet && rx == cx && ry == cy;
                }
                // ballot over the lanes still active in this loop
                const uint64_t mask = __ballot(emit);
                if (mask) {
                    const uint32_t leader = __builtin_ctzll(mask);
                    unsigned int pos = 0;
                    if (lane == leader) pos = atomicAdd(count, unsigned(__popcll(mask)));
                    pos = __shfl(pos, leader);
                    const uint32_t at = pos + __builtin_amdgcn_mbcnt_hi(
                                                  uint32_t(mask >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
                    if (emit && at < cap) {
                        pr[at] = k;
                        ps[at] = s;
                    }
                }
                if (!__any(b < e)) break;
            }
        }
    }
}

}  // namespace

int launch_probe(const ProbeQuery *d_q, uint32_t n_q, const uint32_t *cell_off, const uint32_t *cell_ids,
                 const double *boxes, const uint16_t *cells, uint32_t G, uint32_t *pr, uint32_t *ps,
                 uint32_t cap, unsigned int *count, hipStream_t stream) {
    if (n_q == 0) return APRIL_OK;
    const uint32_t blocks = n_q < 4096 ? n_q : 4096;
    k_probe<<<dim3(blocks), dim3(256), 0, stream>>>(d_q, n_q, cell_off, cell_ids, boxes, cells, G, pr, ps,
                                                    cap, count);
    APRIL_HIP_TRY(hipGetLastError());
    return APRIL_OK;
}

}  // namespace april
