// Batched exact distance queries (the 2-hop query of Section 2.1):
// Dis(u,v) = min over common hubs h of d(u,h) + d(h,v), found by merging the
// two hub-rank-sorted label lists.  Labels are packed (hub rank << 8) | dist.
#include "pll_internal.h"

namespace {

constexpr int kBlock = 256;

// One lane per pair: two-pointer merge.
__global__ void __launch_bounds__(kBlock) k_query_lane(const uint64_t* __restrict__ off,
                                                       const uint32_t* __restrict__ ent, uint64_t count,
                                                       const uint32_t* __restrict__ qu,
                                                       const uint32_t* __restrict__ qv, uint32_t* __restrict__ out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = qu[i], v = qv[i];
        uint64_t a = off[u], ae = off[u + 1], b = off[v], be = off[v + 1];
        uint32_t best = PLL_DIST_INF;
        if (a < ae && b < be) {
            uint32_t ea = ent[a], eb = ent[b];
            for (;;) {
                const uint32_t ha = ea >> 8, hb = eb >> 8;
                if (ha == hb) {
                    best = min(best, (ea & 255u) + (eb & 255u));
                    if (++a == ae || ++b == be) break;
                    ea = ent[a];
                    eb = ent[b];
                } else if (ha < hb) {
                    if (++a == ae) break;
                    ea = ent[a];
                } else {
                    if (++b == be) break;
                    eb = ent[b];
                }
            }
        }
        out[i] = best;
    }
}

}  // namespace

int pll_query_launch(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v,
                     uint32_t* d_out, hipStream_t stream) {
    if (count == 0) return PLL_OK;
    uint64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    k_query_lane<<<(uint32_t)blocks, kBlock, 0, stream>>>(idx->d_off, idx->d_ent, count, d_u, d_v, d_out);
    return hipGetLastError() == hipSuccess ? PLL_OK : PLL_EDEVICE;
}
