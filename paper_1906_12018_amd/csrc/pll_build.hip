// Label construction on gfx950: BVC-PLL (Algorithm 4 of the paper) as
// vertex-centric rounds inside rank-ordered batches.
//
// Per build:   input checks -> relabel to rank space -> batches -> finalize.
// Per batch i (ranks [ib, ib+bs)):
//   k_batch_init   append (u,0) to L(u), spread L(u) into the distance table T
//                  (the paper's H(u), Section 4.1), seed the active list
//   rounds j = 1, 2, ... until no vertex accepts anything:
//     k_push       scatter: OR delta L(a) of every active a into msgs(v) of its
//                  neighbours v ranked below the batch hubs, minus C(v)
//                  (the scatter step of Algorithm 4); collect the receivers
//     k_check      gather: cand(v) = msgs(v); C(v) |= cand(v); a candidate
//                  u_k survives iff no (h, d) in L(v) with d < j has
//                  T[h][k] + d <= j (its distance check); append survivors
//                  with distance j, write T for batch vertices, build the
//                  next active list
//   k_batch_end    clear C(v) over the touched vertices (the batch's last step,
//                  Section 5.2 bitmap + queue), optional recheck (Section 5.1), sort each
//                  touched vertex's batch segment by hub rank
//   k_clear_table  reset T and its row masks for the next batch
//
// A round-j candidate can only be pruned by entries of distance < j, and
// entries accepted in round j can never prune a round-j candidate, so the
// concurrent T and label writes of k_check do not change any decision.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "pll_internal.h"
#include "pll_phases.h"

namespace {

constexpr int kBlock = 256;              // 4 waves
constexpr int kWavesPerBlock = kBlock / PLL_WAVE;
constexpr uint32_t kMaxBlocks = 4096;
constexpr uint32_t kHotRows = 4096;        // top-ranked table rows whose row masks stay all ones
constexpr uint64_t kPullFrac = 2;          // a round with at least n / 2 receivers pulls the next one
constexpr uint64_t kPullFrac1 = 8;         // ... and a batch's first round with at least n / 8
constexpr uint32_t kPullMinN = 16384;      // smaller graphs always push (the pull's set-up outweighs it)
constexpr uint64_t kPackMin = 16384;       // receivers from which a fused round checks four per wave

inline uint32_t blocks_for_waves(uint64_t waves) {
    uint64_t b = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (uint32_t)b;
}

inline uint32_t blocks_for_threads(uint64_t threads) {
    uint64_t b = (threads + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (uint32_t)b;
}

__device__ inline uint32_t global_wave() { return (blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ inline uint32_t num_waves() { return (gridDim.x * blockDim.x) >> 6; }

// ---- exclusive scan (uint32 -> uint64, n+1 outputs) ---------------------------------------------

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ uint64_t block_excl_scan(uint64_t x, uint64_t* total) {
    __shared__ uint64_t wsum[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t s = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(s, o, 64);
        if (lane >= (uint32_t)o) s += y;
    }
    if (lane == 63) wsum[wave] = s;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
        uint64_t ws = wsum[w];
        if (w < (int)wave) pre += ws;
        tot += ws;
    }
    __syncthreads();
    *total = tot;
    return pre + s - x;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t* in, uint64_t n, uint64_t* bsum) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) acc += in[base + i];
    uint64_t tot;
    block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kBlock) k_scan_sums(uint64_t* bsum, uint32_t nb) {
    uint64_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kBlock) {
        uint32_t i = base + threadIdx.x;
        uint64_t x = i < nb ? bsum[i] : 0;
        uint64_t tot;
        uint64_t e = block_excl_scan(x, &tot);
        if (i < nb) bsum[i] = carry + e;
        carry += tot;
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const uint32_t* in, uint64_t n, const uint64_t* bsum,
                                                       uint64_t* out) {
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0u;
        acc += v[i];
    }
    uint64_t tot;
    uint64_t run = bsum[blockIdx.x] + block_excl_scan(acc, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) {
            out[base + i] = run;
            run += v[i];
            if (base + i == n - 1) out[n] = run;
        }
    }
}

// out[0..n] = exclusive prefix sums of in[0..n-1]; scratch holds >= ceil(n / kScanTile) words.
hipError_t scan_u32_to_u64(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* scratch, hipStream_t s) {
    if (n == 0) return hipMemsetAsync(out, 0, sizeof(uint64_t), s);
    uint32_t nb = (uint32_t)((n + kScanTile - 1) / kScanTile);
    k_scan_reduce<<<nb, kBlock, 0, s>>>(in, n, scratch);
    k_scan_sums<<<1, kBlock, 0, s>>>(scratch, nb);
    k_scan_apply<<<nb, kBlock, 0, s>>>(in, n, scratch, out);
    return hipGetLastError();
}

// ---- input checks and relabelling ---------------------------------------------------------------

__global__ void k_check_rowptr(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, DevCounters* ctr) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v <= n; v += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t a = row_ptr[v];
        bool bad = (v == 0 && a != 0) || (v == n && a != nnz) || (v < n && a > row_ptr[v + 1]) || a > nnz;
        if (bad) atomicOr(&ctr->error, PLL_ERR_BOUNDS);
    }
}

__global__ void k_check_cols(uint32_t n, uint64_t nnz, const uint32_t* col, DevCounters* ctr) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x)
        if (col[e] >= n) atomicOr(&ctr->error, PLL_ERR_BOUNDS);
}

__global__ void k_count_order(uint32_t n, const uint32_t* order, uint32_t* cnt, DevCounters* ctr) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        uint32_t o = order[k];
        if (o >= n)
            atomicOr(&ctr->error, PLL_ERR_ORDER);
        else
            atomicAdd(&cnt[o], 1u);
    }
}

__global__ void k_check_order_counts(uint32_t n, const uint32_t* cnt, DevCounters* ctr) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        if (cnt[v] != 1u) atomicOr(&ctr->error, PLL_ERR_ORDER);
}

// Full CSR check (flag PLL_FLAG_VALIDATE): each row strictly ascending, no
// self-loop, and (`symmetric`, undirected graphs) every edge present in both
// directions.  Runs only after the row pointers and column ids passed the
// bounds checks.
__global__ void __launch_bounds__(kBlock) k_check_csr(uint32_t n, const uint64_t* row_ptr, const uint32_t* col,
                                                      uint32_t symmetric, const uint8_t* w, DevCounters* ctr) {
    const uint32_t lane = lane_id();
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint64_t beg = row_ptr[v], end = row_ptr[v + 1];
        bool bad = false;
        for (uint64_t e = beg + lane; e < end; e += 64) {
            uint32_t c = col[e];
            if (c == v) bad = true;
            if (e > beg && col[e - 1] >= c) bad = true;
            if (!symmetric) continue;
            uint64_t lo = row_ptr[c], hi = row_ptr[c + 1];
            while (lo < hi) {
                uint64_t mid = (lo + hi) >> 1;
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= row_ptr[c + 1] || col[lo] != v) bad = true;
            else if (w && w[lo] != w[e]) bad = true;  // both arcs of an edge carry one weight
        }
        if (ballot64(bad) && lane == 0) atomicOr(&ctr->error, PLL_ERR_CSR);
    }
}

__global__ void k_make_rank(uint32_t n, const uint32_t* order, uint32_t* rank) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) rank[order[k]] = k;
}

__global__ void k_rank_degrees(uint32_t n, const uint32_t* order, const uint64_t* row_ptr, uint32_t* deg) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        uint32_t v = order[k];
        deg[k] = (uint32_t)(row_ptr[v + 1] - row_ptr[v]);
    }
}

// Row k of the rank-space CSR is the row of vertex order[k], with every
// neighbour replaced by its rank (neighbour order kept).
__global__ void __launch_bounds__(kBlock) k_relabel_cols(uint32_t n, const uint32_t* order, const uint64_t* row_ptr,
                                                         const uint32_t* col, const uint32_t* rank,
                                                         const uint64_t* rrow, uint32_t* rcol) {
    const uint32_t lane = lane_id();
    for (uint32_t k = global_wave(); k < n; k += num_waves()) {
        const uint32_t v = order[k];
        const uint64_t src = row_ptr[v], dst = rrow[k];
        const uint32_t deg = (uint32_t)(row_ptr[v + 1] - src);
        for (uint32_t i = lane; i < deg; i += 64) rcol[dst + i] = rank[col[src + i]];
    }
}

// In-arcs of a directed graph in rank space: heads count their in-arcs,
// the counts are scanned into row pointers, then every arc r -> c claims a
// slot of row c.  Rows come out in no particular order, which the rounds do
// not need.
__global__ void k_count_heads(uint64_t nnz, const uint32_t* rcol, uint32_t* cnt) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[rcol[e]], 1u);
}

__global__ void __launch_bounds__(kBlock) k_fill_transpose(uint32_t n, const uint64_t* rrow, const uint32_t* rcol,
                                                           const uint64_t* irow, uint32_t* cursor, uint32_t* icol) {
    const uint32_t lane = lane_id();
    for (uint32_t r = global_wave(); r < n; r += num_waves()) {
        const uint64_t beg = rrow[r], end = rrow[r + 1];
        for (uint64_t e = beg + lane; e < end; e += 64) {
            const uint32_t c = rcol[e];
            icol[irow[c] + atomicAdd(&cursor[c], 1u)] = r;
        }
    }
}

// ---- batch kernels (whole-grid wrappers over the phases of pll_phases.h) ---------------------------

using pll::kHeavy;
using pll::PhaseStats;

__device__ inline uint32_t my_shard() { return blockIdx.x % PLL_SHARDS; }

// The whole grid runs a phase; queue counters are the 32 global shards.
__device__ inline pll::Exec grid_exec(const BuildArgs& A) {
    pll::Exec X;
    X.w = global_wave();
    X.nw = num_waves();
    X.qs = A.ctr->sh;
    X.nq = PLL_SHARDS;
    X.my = my_shard();
    X.seg = A.n;
    X.zero_i = blockIdx.x == 0 ? threadIdx.x : ~0u;
    X.arena_sh = X.my;
    return X;
}

// Per-lane statistics summed over the workgroup, then one atomic per value
// into the workgroup's shard.  Every thread of the block must call this.
template <int N>
__device__ inline void block_add_stats(DevCounters* ctr, const unsigned long long (&v)[N], const int (&which)[N]) {
    static_assert(N <= 10, "at most 10 statistics per call");
    __shared__ unsigned long long s_part[kWavesPerBlock][10];
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const unsigned long long t = wave_sum64(v[k]);
        if (lane == 0) s_part[wv][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)N) {
        unsigned long long t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += s_part[w][threadIdx.x];
        if (t) atomicAdd(&ctr->sh[my_shard()].stat[which[threadIdx.x]], t);
    }
}

// Capacities of the compacted lists: 16 entries for isolated vertices, 32
// for the others before the first batch; afterwards the current length plus
// half of it (at least 16 more), rounded to 16 entries.
__global__ void k_list_caps(uint32_t n, const uint64_t* rrow, const uint32_t* llen, uint32_t first, uint32_t* cap) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        if (first) {
            cap[r] = rrow[r + 1] == rrow[r] ? 16u : 32u;
        } else {
            const uint32_t l = llen[r];
            cap[r] = (l + max(l / 2u, 16u) + 15u) & ~15u;
        }
    }
}

// Move every list to its compacted position in a new arena.
__global__ void __launch_bounds__(kBlock) k_compact(uint32_t n, const uint64_t* old_off, const uint32_t* llen,
                                                    const uint32_t* old_arena, const uint64_t* new_off,
                                                    uint32_t* new_arena) {
    const uint32_t lane = lane_id();
    for (uint32_t r = global_wave(); r < n; r += num_waves()) {
        const uint64_t src = old_off[r], dst = new_off[r];
        const uint32_t len = llen[r];
        for (uint32_t i = lane; i < len; i += 64) new_arena[dst + i] = old_arena[src + i];
    }
}

__global__ void k_batch_prep(DevCounters* ctr) {
    if (threadIdx.x < PLL_SHARDS) {
        Shard& sh = ctr->sh[threadIdx.x];
        sh.recv[0] = sh.recv[1] = sh.recv[2] = 0;
        sh.hq[0] = sh.hq[1] = 0;
        sh.touched = 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_batch_init(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t bstamp) {
    pll::phase_batch_init(A, grid_exec(A), ib, bs, bstamp);
}

__global__ void __launch_bounds__(kBlock) k_push(BuildArgs A, uint32_t ib, uint32_t p, uint32_t nact, uint32_t rstamp,
                                                 uint32_t bstamp) {
    PhaseStats st;
    pll::phase_push(A, grid_exec(A), ib, p, nact, rstamp, bstamp, st);
    const unsigned long long v[1] = {st.edges};
    const int which[1] = {PLL_ST_EDGES};
    block_add_stats<1>(A.ctr, v, which);
}

template <int WM, bool BP>
__global__ void __launch_bounds__(kBlock) k_check(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t j, uint32_t p,
                                                  uint32_t relaxed) {
    PhaseStats st;
    pll::phase_check<WM, BP>(A, grid_exec(A), ib, bs, j, p, relaxed != 0, st);
    const unsigned long long v[7] = {st.cand, st.acc, st.read, st.table, st.cost_pos, st.cost_neg, st.bp};
    const int which[7] = {PLL_ST_CAND,     PLL_ST_ACC,      PLL_ST_READ, PLL_ST_TABLE,
                          PLL_ST_COST_POS, PLL_ST_COST_NEG, PLL_ST_BP};
    block_add_stats<7>(A.ctr, v, which);
}

// Round j's check fused with round j+1's push (NextRound in pll_phases.h).
// SMALLT: every prune threshold of round j is at most pll::kSmallT (j <= kSmallT),
// so the scans take the cheaper byte compare.  The packed check is only
// instantiated with it.
template <int WM, bool BP, bool PACK = false, bool SMALLT = false>
__device__ inline void check_push_body(const BuildArgs& A, const pll::Exec& X, uint32_t ib, uint32_t bs, uint32_t j,
                                       const pll::NextRound& nr, uint32_t relaxed) {
    PhaseStats st;
    if (PACK && !BP)
        pll::phase_check4<WM, SMALLT>(A, X, ib, bs, j, relaxed != 0, st, nr);
    else
        pll::phase_check<WM, BP, true, false, SMALLT && !BP>(A, X, ib, bs, j, nr.rin, relaxed != 0, st, &nr);
    const unsigned long long v[9] = {st.cand,     st.acc, st.read,  st.table,          st.cost_pos,
                                     st.cost_neg, st.bp,  st.edges + st.pulled, st.edges};
    const int which[9] = {PLL_ST_CAND,     PLL_ST_ACC, PLL_ST_READ,  PLL_ST_TABLE,      PLL_ST_COST_POS,
                          PLL_ST_COST_NEG, PLL_ST_BP,  PLL_ST_EDGES, PLL_ST_FUSED_EDGES};
    block_add_stats<9>(A.ctr, v, which);
}

// at most 128 VGPRs, i.e. 4 waves per SIMD, like the unfused check
template <int WM, bool PACK, bool SMALLT>
__global__ void __launch_bounds__(kBlock, 4) k_check_push(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t j,
                                                          pll::NextRound nr, uint32_t relaxed) {
    check_push_body<WM, false, PACK, SMALLT>(A, grid_exec(A), ib, bs, j, nr, relaxed);
}

// The blocks [b0, b0 + nb) of the grid run a phase on their own: queue
// counters are the build's 32 shards, the first block clears them.
__device__ inline pll::Exec side_exec(const BuildArgs& A, uint32_t b0, uint32_t nb) {
    pll::Exec X;
    X.w = ((blockIdx.x - b0) * blockDim.x + threadIdx.x) >> 6;
    X.nw = (nb * blockDim.x) >> 6;
    X.qs = A.ctr->sh;
    X.nq = PLL_SHARDS;
    X.my = (blockIdx.x - b0) % PLL_SHARDS;
    X.seg = A.n;
    X.zero_i = blockIdx.x == b0 ? threadIdx.x : ~0u;
    X.arena_sh = X.my;
    return X;
}

// Directed graphs: both sides' fused rounds in one launch, blocks [0, nb0)
// on the forward side and the rest on the backward side.
template <int WM, bool SMALLT>
__global__ void __launch_bounds__(kBlock, 4) k_check_push2(BuildArgs A0, pll::NextRound nr0, BuildArgs A1,
                                                           pll::NextRound nr1, uint32_t ib, uint32_t bs, uint32_t j,
                                                           uint32_t nb0) {
    if (blockIdx.x < nb0)
        check_push_body<WM, false, false, SMALLT>(A0, side_exec(A0, 0, nb0), ib, bs, j, nr0, 0);
    else
        check_push_body<WM, false, false, SMALLT>(A1, side_exec(A1, nb0, gridDim.x - nb0), ib, bs, j, nr1, 0);
}

// with bit-parallel labels (no register cap: it would spill)
template <int WM>
__global__ void __launch_bounds__(kBlock) k_check_push_bp(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t j,
                                                          pll::NextRound nr, uint32_t relaxed) {
    check_push_body<WM, true>(A, grid_exec(A), ib, bs, j, nr, relaxed);
}

// Pulled rounds: the (vertex, segment) items, once per build, and a round.
__global__ void __launch_bounds__(kBlock) k_pull_items(BuildArgs A, uint2* items, uint32_t* nitems) {
    pll::phase_pull_items(A, grid_exec(A), items, nitems);
}

__global__ void __launch_bounds__(kBlock) k_pull(BuildArgs A, uint32_t ib, const uint2* items, const uint32_t* nitems,
                                                 uint32_t q, pll::NextRound nr) {
    pll::phase_pull4(A, grid_exec(A), ib, items, nitems, q, nr);
}

// The heavy rows the fused round queued, pushed for the next round.
__global__ void __launch_bounds__(kBlock) k_push_heavy(BuildArgs A, uint32_t ib, uint32_t hp, uint32_t rq,
                                                       uint64_t* msgs, uint32_t* recv, uint32_t rstamp,
                                                       uint32_t bstamp) {
    PhaseStats st;
    pll::phase_push_heavy(A, grid_exec(A), ib, hp, rq, msgs, recv, rstamp, bstamp, st);
    const unsigned long long v[1] = {st.edges};
    const int which[1] = {PLL_ST_EDGES};
    block_add_stats<1>(A.ctr, v, which);
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_batch_end(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t recheck) {
    __shared__ uint64_t s_pres[kWavesPerBlock][PLL_WMAX];
    __shared__ uint8_t s_dist[kWavesPerBlock][PLL_BMAX];
    const uint32_t wv = threadIdx.x >> 6;
    PhaseStats st;
    pll::phase_batch_end<WM>(A, grid_exec(A), ib, bs, recheck != 0, s_pres[wv], s_dist[wv], nullptr, st);
    const unsigned long long v[3] = {st.removed, st.read, st.table};
    const int which[3] = {PLL_ST_RECHECK, PLL_ST_READ, PLL_ST_TABLE};
    block_add_stats<3>(A.ctr, v, which);
}

// ---- weighted batch kernels (Section 5.1) ----

__global__ void __launch_bounds__(kBlock) k_push_w(BuildArgs A, uint32_t ib, uint32_t p, uint32_t nact,
                                                   uint32_t rstamp, uint32_t bstamp) {
    PhaseStats st;
    pll::phase_push_w(A, grid_exec(A), ib, p, nact, rstamp, bstamp, st);
    const unsigned long long v[1] = {st.edges};
    const int which[1] = {PLL_ST_EDGES};
    block_add_stats<1>(A.ctr, v, which);
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_check_w(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t p) {
    __shared__ uint4 s_thr[kWavesPerBlock][4 * PLL_WMAX];
    PhaseStats st;
    pll::phase_check_w<WM>(A, grid_exec(A), ib, bs, p, s_thr[threadIdx.x >> 6], st);
    const unsigned long long v[6] = {st.cand, st.acc, st.read, st.table, st.cost_pos, st.cost_neg};
    const int which[6] = {PLL_ST_CAND, PLL_ST_ACC, PLL_ST_READ, PLL_ST_TABLE, PLL_ST_COST_POS, PLL_ST_COST_NEG};
    block_add_stats<6>(A.ctr, v, which);
}

template <int WM>
__global__ void __launch_bounds__(kBlock) k_batch_end_w(BuildArgs A, uint32_t ib, uint32_t bs) {
    __shared__ uint64_t s_pres[kWavesPerBlock][PLL_WMAX];
    __shared__ uint8_t s_dist[kWavesPerBlock][PLL_BMAX];
    __shared__ uint32_t s_pos[kWavesPerBlock][PLL_BMAX];
    const uint32_t wv = threadIdx.x >> 6;
    PhaseStats st;
    pll::phase_batch_end<WM, true>(A, grid_exec(A), ib, bs, true, s_pres[wv], s_dist[wv], s_pos[wv], st);
    const unsigned long long v[3] = {st.removed, st.read, st.table};
    const int which[3] = {PLL_ST_RECHECK, PLL_ST_READ, PLL_ST_TABLE};
    block_add_stats<3>(A.ctr, v, which);
}

// Weights follow their CSR entries into rank space.
__global__ void __launch_bounds__(kBlock) k_relabel_weights(uint32_t n, const uint32_t* order, const uint64_t* row_ptr,
                                                            const uint8_t* w, const uint64_t* rrow, uint8_t* rw) {
    const uint32_t lane = lane_id();
    for (uint32_t k = global_wave(); k < n; k += num_waves()) {
        const uint32_t v = order[k];
        const uint64_t src = row_ptr[v], dst = rrow[k];
        const uint32_t deg = (uint32_t)(row_ptr[v + 1] - src);
        for (uint32_t i = lane; i < deg; i += 64) rw[dst + i] = w[src + i];
    }
}

__global__ void k_check_weights(uint64_t nnz, const uint8_t* w, DevCounters* ctr) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x)
        if (w[e] == 0) atomicOr(&ctr->error, PLL_ERR_BOUNDS);
}

// With `prep` set it also does k_batch_prep's reset for the next batch (the
// batch end, which reads the touched counts, has finished by then).
__global__ void __launch_bounds__(kBlock) k_clear_table(BuildArgs A, uint32_t ib, uint32_t bs, DevCounters* prep) {
    if (prep && blockIdx.x == 0 && threadIdx.x < PLL_SHARDS) {
        Shard& sh = prep->sh[threadIdx.x];
        sh.recv[0] = sh.recv[1] = sh.recv[2] = 0;
        sh.hq[0] = sh.hq[1] = 0;
        sh.touched = 0;
    }
    pll::phase_clear_table(A, grid_exec(A), ib, bs);
}

// ---- bit-parallel labels (Section 5.2) ------------------------------------------------------------

// Choose up to t_req BP roots in rank space (one workgroup of 1,024
// threads): the root is the smallest unused rank; its neighbour set is its
// (up to) 64 smallest unused neighbour ranks, found by an 8-bit radix
// select over the 24-bit ranks (three histogram passes over the row), then
// ordered by counting.  The root and the set become used.
constexpr int kSelBlock = 1024;

__global__ void __launch_bounds__(kSelBlock) k_bp_select(uint32_t n, uint32_t t_req, const uint64_t* rrow,
                                                         const uint32_t* rcol, uint8_t* used, uint32_t* roots,
                                                         uint32_t* nbrs, uint32_t* t_out /* [2]: roots, used */) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_sel[64];
    __shared__ uint32_t s_next, s_cnt, s_prefix, s_kth;
    const uint32_t tid = threadIdx.x;
    uint32_t cursor = 0, t = 0, nused = 0;
    for (; t < t_req; ++t) {
        if (tid == 0) s_next = 0xFFFFFFFFu;
        __syncthreads();
        uint32_t r = 0xFFFFFFFFu;
        for (uint32_t base = cursor; base < n; base += kSelBlock) {
            const uint32_t x = base + tid;
            if (x < n && !used[x]) atomicMin(&s_next, x);
            __syncthreads();
            r = s_next;
            __syncthreads();  // every thread has read s_next before the next chunk writes it
            if (r != 0xFFFFFFFFu) break;
        }
        if (r == 0xFFFFFFFFu) break;
        cursor = r + 1;
        const uint64_t beg = rrow[r], end = rrow[r + 1];
        if (tid == 0) {
            used[r] = 1;
            s_cnt = 0;
        }
        __syncthreads();
        uint32_t c = 0;
        for (uint64_t e = beg + tid; e < end; e += kSelBlock) c += used[rcol[e]] ? 0u : 1u;
        if (c) atomicAdd(&s_cnt, c);
        __syncthreads();
        const uint32_t cnt = s_cnt;
        uint32_t limit = 0xFFFFFFFFu;  // largest rank taken
        if (cnt > 64) {
            if (tid == 0) {
                s_prefix = 0;
                s_kth = 64;
            }
            for (int shift = 16; shift >= 0; shift -= 8) {
                for (uint32_t b = tid; b < 256; b += kSelBlock) s_hist[b] = 0;
                __syncthreads();
                const uint32_t prefix = s_prefix;
                for (uint64_t e = beg + tid; e < end; e += kSelBlock) {
                    const uint32_t x = rcol[e];
                    if (!used[x] && (x >> (shift + 8)) == (prefix >> (shift + 8)))
                        atomicAdd(&s_hist[(x >> shift) & 255u], 1u);
                }
                __syncthreads();
                if (tid == 0) {
                    uint32_t cum = 0, kth = s_kth;
                    for (uint32_t b = 0; b < 256; ++b) {
                        if (cum + s_hist[b] >= kth) {
                            s_prefix = prefix | (b << shift);
                            s_kth = kth - cum;
                            break;
                        }
                        cum += s_hist[b];
                    }
                }
                __syncthreads();
            }
            limit = s_prefix;  // the 64th smallest unused neighbour rank
        }
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        for (uint64_t e = beg + tid; e < end; e += kSelBlock) {
            const uint32_t x = rcol[e];
            if (!used[x] && x <= limit) {
                const uint32_t slot = atomicAdd(&s_cnt, 1u);
                if (slot < 64) s_sel[slot] = x;  // more only with duplicate neighbours (an invalid CSR)
            }
        }
        __syncthreads();
        const uint32_t m = min(s_cnt, 64u);
        if (tid < 64) {
            uint32_t pos = tid;
            if (tid < m) {
                const uint32_t x = s_sel[tid];
                pos = 0;
                for (uint32_t q = 0; q < m; ++q) pos += s_sel[q] < x ? 1u : 0u;
                nbrs[t * 64 + pos] = x;
            } else {
                nbrs[t * 64 + tid] = 0xFFFFFFFFu;
            }
        }
        if (tid == 0) {
            roots[t] = r;
            nused += 1 + m;
        }
        __syncthreads();
        if (tid < m) used[s_sel[tid]] = 1;
        __syncthreads();
    }
    if (tid == 0) {
        t_out[0] = t;
        t_out[1] = nused;
    }
}

// Level 0 and the neighbour sets at level 1 of every BP root (block i = root i).
__global__ void k_bp_seed(uint32_t t, const uint32_t* roots, const uint32_t* nbrs, uint8_t* bp_dist,
                          ulonglong2* bp_sets) {
    const uint32_t i = blockIdx.x, j = threadIdx.x;
    if (j == 64) {
        bp_dist[(size_t)roots[i] * t + i] = 0;
    } else if (j < 64) {
        const uint32_t s = nbrs[i * 64 + j];
        if (s != 0xFFFFFFFFu) {
            bp_dist[(size_t)s * t + i] = 1;
            bp_sets[(size_t)s * t + i] = make_ulonglong2(1ull << j, 0ull);
        }
    }
}

// Level L+1 of every BP root, pushed from the vertices at level L: a
// neighbour that is unreached, or already reached at L+1 in this launch,
// is at L+1 and ORs in the vertex's S^-1 and S^0 (a member s of S_r at
// distance L - 1 or L from a parent is at distance L or L + 1 from the
// child).  The sets of level L are final here and nothing at level L is
// written, so the pushes of one launch do not interfere.
__global__ void __launch_bounds__(kBlock) k_bp_push(uint32_t n, uint32_t t, uint32_t L, const uint64_t* rrow,
                                                    const uint32_t* rcol, uint8_t* bp_dist, ulonglong2* bp_sets,
                                                    DevCounters* ctr) {
    const uint32_t lane = lane_id();
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint64_t at_l = ballot64(lane < t && bp_dist[(size_t)v * t + lane] == L);
        if (!at_l) continue;
        if (L + 1 >= PLL_INF8) {
            if (lane == 0) atomicOr(&ctr->error, PLL_ERR_DIST);
            continue;
        }
        const uint64_t beg = rrow[v], end = rrow[v + 1];
        uint64_t todo = at_l;
        while (todo) {
            const uint32_t i = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const ulonglong2 sv = bp_sets[(size_t)v * t + i];
            for (uint64_t e = beg + lane; e < end; e += 64) {
                const uint32_t w = rcol[e];
                uint8_t* dw = &bp_dist[(size_t)w * t + i];
                const uint32_t d = *dw;
                if (d != PLL_INF8 && d != L + 1) continue;
                if (d == PLL_INF8) *dw = (uint8_t)(L + 1);
                ulonglong2* sw = &bp_sets[(size_t)w * t + i];
                if (sv.x) atomicOr((unsigned long long*)&sw->x, (unsigned long long)sv.x);
                if (sv.y) atomicOr((unsigned long long*)&sw->y, (unsigned long long)sv.y);
            }
        }
    }
}

// Siblings at level L: S^0(v) gains S^-1 of every neighbour at the same
// level, then drops what S^-1(v) holds.  Counts the (vertex, root) pairs at
// level L into the first shard's receiver counter (the loop stops at 0).
__global__ void __launch_bounds__(kBlock) k_bp_sibling(uint32_t n, uint32_t t, uint32_t L, const uint64_t* rrow,
                                                       const uint32_t* rcol, const uint8_t* bp_dist,
                                                       ulonglong2* bp_sets, DevCounters* ctr) {
    const uint32_t lane = lane_id();
    uint32_t seen = 0;
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint64_t at_l = ballot64(lane < t && bp_dist[(size_t)v * t + lane] == L);
        if (!at_l) continue;
        seen += (uint32_t)__builtin_popcountll(at_l);
        const uint64_t beg = rrow[v], end = rrow[v + 1];
        uint64_t todo = at_l;
        while (todo) {
            const uint32_t i = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            uint64_t acc = 0;
            for (uint64_t e = beg + lane; e < end; e += 64) {
                const uint32_t w = rcol[e];
                if (bp_dist[(size_t)w * t + i] == L) acc |= bp_sets[(size_t)w * t + i].x;
            }
            acc = wave_or64(acc);
            if (lane == 0) {
                ulonglong2* p = &bp_sets[(size_t)v * t + i];
                p->y = (p->y | acc) & ~p->x;
            }
        }
    }
    if (lane == 0 && seen) atomicAdd(&ctr->sh[0].recv[0], seen);
}

// Transposed copy of the batch vertices' BP data (root-major, so that the
// check's lanes over batch vertices read consecutive addresses).
__global__ void k_bp_batch_stage(BuildArgs A, uint32_t ib, uint32_t bs) {
    const uint32_t t = A.bp_t;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < t * bs; x += gridDim.x * blockDim.x) {
        const uint32_t i = x / bs, k = x % bs;
        const size_t src = (size_t)(ib + k) * t + i;
        A.bpb_dist[(size_t)i * A.bstride + k] = A.bp_dist[src];
        A.bpb_sets[(size_t)i * A.bstride + k] = A.bp_sets[src];
    }
}

// BP data by vertex id for the index, and the roots and sets as vertex ids.
__global__ void k_bp_by_vertex(uint32_t n, uint32_t t, const uint32_t* rank, const uint8_t* bp_dist,
                               const ulonglong2* bp_sets, uint8_t* out_dist, ulonglong2* out_sets) {
    const uint64_t total = (uint64_t)n * t;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(x / t), i = (uint32_t)(x % t);
        const size_t src = (size_t)rank[v] * t + i;
        out_dist[x] = bp_dist[src];
        out_sets[x] = bp_sets[src];
    }
}

__global__ void k_bp_ids(uint32_t t, const uint32_t* order, const uint32_t* roots, const uint32_t* nbrs,
                         uint32_t* out_roots, uint32_t* out_nbrs) {
    for (uint32_t x = threadIdx.x; x < t * 64; x += blockDim.x) {
        const uint32_t s = nbrs[x];
        out_nbrs[x] = s == 0xFFFFFFFFu ? s : order[s];
        if (x < t) out_roots[x] = order[roots[x]];
    }
}

// 1 + the highest rank with an edge, into ctr->edge_end.  A batch whose
// roots all rank at or above it has isolated roots only: each root's label is
// its self entry, and no other label holds it, so such batches need no run.
__global__ void __launch_bounds__(kBlock) k_edge_end(uint32_t n, const uint64_t* rrow, DevCounters* ctr) {
    uint32_t m = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        if (rrow[r + 1] > rrow[r]) m = r + 1;
    m = wave_max32(m);
    if (lane_id() == 0 && m) atomicMax(&ctr->edge_end, m);
}

// ---- finalize -----------------------------------------------------------------------------------

// Lists of ranks r >= self_from were never batch roots (their batches held
// isolated vertices only): each gets its self entry (r, 0) here, after any
// entries it holds (none, for an isolated vertex).

__global__ void __launch_bounds__(kBlock) k_final_lens(uint32_t n, const uint32_t* rank, const uint32_t* llen,
                                                       uint32_t self_from, uint32_t* lens, DevCounters* ctr) {
    __shared__ uint32_t smax[kWavesPerBlock];
    uint32_t ml = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t r = rank[v];
        const uint32_t l = llen[r] + (r >= self_from ? 1u : 0u);
        lens[v] = l;
        ml = max(ml, l);
    }
    ml = wave_max32(ml);
    if (lane_id() == 0) smax[threadIdx.x >> 6] = ml;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWavesPerBlock; ++w) ml = max(ml, smax[w]);
        atomicMax(&ctr->max_label, ml);
    }
}

__global__ void __launch_bounds__(kBlock) k_final_copy(uint32_t n, const uint32_t* rank, const uint64_t* loff,
                                                       const uint32_t* llen, const uint32_t* arena,
                                                       uint32_t self_from, const uint64_t* off, uint32_t* ent,
                                                       uint2* lb, DevCounters* ctr) {
    __shared__ uint32_t smax[kWavesPerBlock];
    const uint32_t lane = lane_id();
    uint32_t md = 0;
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint32_t r = rank[v];
        const uint64_t src = loff[r], dst = off[v];
        const uint32_t len = llen[r];
        for (uint32_t i = lane; i < len; i += 64) {
            const uint32_t e = arena[src + i];
            ent[dst + i] = e;
            md = max(md, e & 255u);
        }
        if (lane == 0) {
            if (r >= self_from) {
                ent[dst + len] = pll_pack(r, 0);
                lb[v] = make_uint2(len ? arena[src] >> 8 : r, r);
            } else {
                lb[v] = len ? make_uint2(arena[src] >> 8, arena[src + len - 1] >> 8) : make_uint2(0xFFFFFFFFu, 0u);
            }
        }
    }
    md = wave_max32(md);
    if (lane == 0) smax[threadIdx.x >> 6] = md;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWavesPerBlock; ++w) md = max(md, smax[w]);
        atomicMax(&ctr->max_dist, md);
    }
}

// ---- host driver --------------------------------------------------------------------------------

// Buffers of one build: workspace from the caching allocator (returned once
// the stream has drained), outputs from hipMalloc (kept with forget()).
//
// With `fixed` set, every block (outputs included) is carved in order out of
// one region the caller provides and nothing is allocated or freed: blocks
// live until the region is reused, and a request past its end fails with
// hipErrorOutOfMemory.
struct DevAllocs {
    std::vector<void*> ws, outs;
    hipStream_t s = nullptr;
    hipError_t err = hipSuccess;
    char* fixed = nullptr;
    size_t fixed_cap = 0, fixed_used = 0;
    void* carve(size_t bytes) {
        const size_t at = (fixed_used + 255) & ~size_t(255);
        if (at + bytes > fixed_cap) {
            err = hipErrorOutOfMemory;
            return nullptr;
        }
        fixed_used = at + bytes;
        return fixed + at;
    }
    template <class T>
    T* get(size_t count) {
        if (err != hipSuccess) return nullptr;
        if (fixed) return static_cast<T*>(carve(std::max<size_t>(count * sizeof(T), 256)));
        void* p = nullptr;
        err = pll_ws_alloc(&p, std::max<size_t>(count * sizeof(T), 256));
        if (err != hipSuccess) return nullptr;
        ws.push_back(p);
        return static_cast<T*>(p);
    }
    template <class T>
    T* get_out(size_t count) {
        if (err != hipSuccess) return nullptr;
        if (fixed) return static_cast<T*>(carve(std::max<size_t>(count * sizeof(T), 256)));
        void* p = nullptr;
        err = hipMalloc(&p, std::max<size_t>(count * sizeof(T), 256));
        if (err != hipSuccess) return nullptr;
        outs.push_back(p);
        return static_cast<T*>(p);
    }
    void forget(void* p) {
        for (auto& q : outs)
            if (q == p) q = nullptr;
    }
    // return a workspace block early (the stream must have drained)
    void drop(void* p) {
        for (auto& q : ws)
            if (q == p) {
                pll_ws_free(q);
                q = nullptr;
            }
    }
    ~DevAllocs() {
        (void)hipStreamSynchronize(s);
        for (void* p : ws)
            if (p) pll_ws_free(p);
        for (void* p : outs)
            if (p) (void)hipFree(p);
    }
};

// A fixed device region and host counter record for a build that allocates
// nothing (pll_build_labels_noalloc).
struct FixedWs {
    void* base = nullptr;
    size_t bytes = 0;
    DevCounters* host_ctr = nullptr;
};

inline int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? PLL_ENOMEM : PLL_EDEVICE; }

#define TRY_HIP(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return status_of(_e);    \
    } while (0)

struct HostCounters {
    DevCounters* p = nullptr;
    bool own = true;
    ~HostCounters() {
        if (p && own) pll_pinned_free(p);
    }
};

// Per-phase device time from HIP events on the build stream (PLL_FLAG_PROFILE).
// Spans are resolved at the host sync points the build already has.
struct PhaseProfiler {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> all, pool;
    struct Span {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Span> pending;
    double ms[PLL_NUM_PHASES] = {};
    uint64_t launches[PLL_NUM_PHASES] = {};

    hipEvent_t mark() {
        if (!on) return nullptr;
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else {
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            all.push_back(e);
        }
        if (hipEventRecord(e, s) != hipSuccess) {
            pool.push_back(e);
            return nullptr;
        }
        return e;
    }
    void span(int phase, hipEvent_t a, hipEvent_t b, uint64_t nlaunch) {
        if (!on) return;
        launches[phase] += nlaunch;
        if (a && b) pending.push_back({phase, a, b});
    }
    // Call only after the stream has been synchronised.
    void resolve() {
        std::vector<hipEvent_t> done;
        for (const Span& sp : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, sp.a, sp.b) == hipSuccess) ms[sp.phase] += t;
            done.push_back(sp.a);
            done.push_back(sp.b);
        }
        pending.clear();
        // an event may close one span and open the next: recycle it once
        std::sort(done.begin(), done.end());
        done.erase(std::unique(done.begin(), done.end()), done.end());
        pool.insert(pool.end(), done.begin(), done.end());
    }
    ~PhaseProfiler() {
        for (hipEvent_t e : all) (void)hipEventDestroy(e);
    }
};

int read_counters(const DevCounters* d, DevCounters* h, hipStream_t s) {
    TRY_HIP(hipMemcpyAsync(h, d, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    return PLL_OK;
}

int device_error_status(uint32_t err) {
    if (err & PLL_ERR_TIMEOUT) return PLL_EDEVICE;
    if (err & (PLL_ERR_BOUNDS | PLL_ERR_CSR | PLL_ERR_ORDER)) return PLL_EINVAL;
    if (err & PLL_ERR_DIST) return PLL_EDIST;
    if (err & PLL_ERR_ARENA) return PLL_ENOSPC;
    return PLL_OK;
}

template <int WM>
void launch_check(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t j,
                  uint32_t p, uint32_t relaxed) {
    if (A.bp_t)
        k_check<WM, true><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, p, relaxed);
    else
        k_check<WM, false><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, p, relaxed);
}

template <int WM>
void launch_batch_end(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t recheck) {
    k_batch_end<WM><<<blocks, kBlock, 0, s>>>(A, ib, bs, recheck);
}

// Kernels are instantiated for 1, 2, 4, 8 and 16 candidate words.
inline int words_class(uint32_t W) { return W <= 1 ? 1 : W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16; }

void dispatch_check(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t j,
                    uint32_t p, uint32_t relaxed) {
    switch (words_class(A.W)) {
        case 1: launch_check<1>(blocks, s, A, ib, bs, j, p, relaxed); break;
        case 2: launch_check<2>(blocks, s, A, ib, bs, j, p, relaxed); break;
        case 4: launch_check<4>(blocks, s, A, ib, bs, j, p, relaxed); break;
        case 8: launch_check<8>(blocks, s, A, ib, bs, j, p, relaxed); break;
        default: launch_check<16>(blocks, s, A, ib, bs, j, p, relaxed); break;
    }
}

template <int WM>
void launch_check_push(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t j,
                       const pll::NextRound& nr, uint32_t relaxed, bool pack) {
    if (A.bp_t)
        k_check_push_bp<WM><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, nr, relaxed);
    else if (pack)  // only in rounds j <= kSmallT
        k_check_push<WM, true, true><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, nr, relaxed);
    else if (j <= pll::kSmallT)
        k_check_push<WM, false, true><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, nr, relaxed);
    else
        k_check_push<WM, false, false><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, nr, relaxed);
}

template <bool SMALLT>
void launch_check_push2(uint32_t nb0, uint32_t nb1, hipStream_t s, const BuildArgs& A0, const pll::NextRound& nr0,
                        const BuildArgs& A1, const pll::NextRound& nr1, uint32_t ib, uint32_t bs, uint32_t j) {
    const uint32_t g = nb0 + nb1;
    switch (words_class(A0.W)) {
        case 1: k_check_push2<1, SMALLT><<<g, kBlock, 0, s>>>(A0, nr0, A1, nr1, ib, bs, j, nb0); break;
        case 2: k_check_push2<2, SMALLT><<<g, kBlock, 0, s>>>(A0, nr0, A1, nr1, ib, bs, j, nb0); break;
        case 4: k_check_push2<4, SMALLT><<<g, kBlock, 0, s>>>(A0, nr0, A1, nr1, ib, bs, j, nb0); break;
        case 8: k_check_push2<8, SMALLT><<<g, kBlock, 0, s>>>(A0, nr0, A1, nr1, ib, bs, j, nb0); break;
        default: k_check_push2<16, SMALLT><<<g, kBlock, 0, s>>>(A0, nr0, A1, nr1, ib, bs, j, nb0); break;
    }
}

void dispatch_check_push2(uint32_t nb0, uint32_t nb1, hipStream_t s, const BuildArgs& A0, const pll::NextRound& nr0,
                          const BuildArgs& A1, const pll::NextRound& nr1, uint32_t ib, uint32_t bs, uint32_t j) {
    if (j <= pll::kSmallT)
        launch_check_push2<true>(nb0, nb1, s, A0, nr0, A1, nr1, ib, bs, j);
    else
        launch_check_push2<false>(nb0, nb1, s, A0, nr0, A1, nr1, ib, bs, j);
}

void dispatch_check_push(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t j,
                         const pll::NextRound& nr, uint32_t relaxed, bool pack) {
    switch (words_class(A.W)) {
        case 1: launch_check_push<1>(blocks, s, A, ib, bs, j, nr, relaxed, pack); break;
        case 2: launch_check_push<2>(blocks, s, A, ib, bs, j, nr, relaxed, pack); break;
        case 4: launch_check_push<4>(blocks, s, A, ib, bs, j, nr, relaxed, pack); break;
        case 8: launch_check_push<8>(blocks, s, A, ib, bs, j, nr, relaxed, pack); break;
        default: launch_check_push<16>(blocks, s, A, ib, bs, j, nr, relaxed, pack); break;
    }
}

void dispatch_batch_end(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs,
                        uint32_t recheck) {
    switch (words_class(A.W)) {
        case 1: launch_batch_end<1>(blocks, s, A, ib, bs, recheck); break;
        case 2: launch_batch_end<2>(blocks, s, A, ib, bs, recheck); break;
        case 4: launch_batch_end<4>(blocks, s, A, ib, bs, recheck); break;
        case 8: launch_batch_end<8>(blocks, s, A, ib, bs, recheck); break;
        default: launch_batch_end<16>(blocks, s, A, ib, bs, recheck); break;
    }
}

void dispatch_check_w(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t p) {
    switch (words_class(A.W)) {
        case 1: k_check_w<1><<<blocks, kBlock, 0, s>>>(A, ib, bs, p); break;
        case 2: k_check_w<2><<<blocks, kBlock, 0, s>>>(A, ib, bs, p); break;
        case 4: k_check_w<4><<<blocks, kBlock, 0, s>>>(A, ib, bs, p); break;
        case 8: k_check_w<8><<<blocks, kBlock, 0, s>>>(A, ib, bs, p); break;
        default: k_check_w<16><<<blocks, kBlock, 0, s>>>(A, ib, bs, p); break;
    }
}

void dispatch_batch_end_w(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs) {
    switch (words_class(A.W)) {
        case 1: k_batch_end_w<1><<<blocks, kBlock, 0, s>>>(A, ib, bs); break;
        case 2: k_batch_end_w<2><<<blocks, kBlock, 0, s>>>(A, ib, bs); break;
        case 4: k_batch_end_w<4><<<blocks, kBlock, 0, s>>>(A, ib, bs); break;
        case 8: k_batch_end_w<8><<<blocks, kBlock, 0, s>>>(A, ib, bs); break;
        default: k_batch_end_w<16><<<blocks, kBlock, 0, s>>>(A, ib, bs); break;
    }
}

// Keeps the stream busy for `ticks` of the device wall clock (bounded).
// Profiled builds run it ahead of each timed launch so that the host has
// queued the launch before its start event is stamped: the event span is
// then the kernel's run, not the host's launch overhead.
__global__ void k_delay(uint64_t ticks) {
    const uint64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(2);
}

__global__ void k_reset_tops(DevCounters* ctr) {
    if (threadIdx.x < PLL_SHARDS) ctr->sh[threadIdx.x].arena_top = 0;
}

unsigned long long sum_stat(const DevCounters* h, int k) {
    unsigned long long t = 0;
    for (int s = 0; s < PLL_SHARDS; ++s) t += h->sh[s].stat[k];
    return t;
}

uint32_t sum_recv(const DevCounters* h, uint32_t p) {
    uint32_t t = 0;
    for (int s = 0; s < PLL_SHARDS; ++s) t += h->sh[s].recv[p];
    return t;
}

uint32_t sum_hq(const DevCounters* h, uint32_t p) {
    uint32_t t = 0;
    for (int s = 0; s < PLL_SHARDS; ++s) t += h->sh[s].hq[p];
    return t;
}

uint32_t sum_touched(const DevCounters* h) {
    uint32_t t = 0;
    for (int s = 0; s < PLL_SHARDS; ++s) t += h->sh[s].touched;
    return t;
}

unsigned long long max_top(const DevCounters* h) {
    unsigned long long t = 0;
    for (int s = 0; s < PLL_SHARDS; ++s) t = std::max(t, h->sh[s].arena_top);
    return t;
}

// Lay every label list out back to back in a fresh arena with headroom
// (capacities from k_list_caps), followed by PLL_SHARDS empty bump regions
// of region_cap entries each.  `first` builds the initial layout.
int relayout_arena(DevAllocs& M, BuildArgs& A, uint64_t*& spare_off, uint32_t* caps, uint64_t* scan_scratch,
                   bool first, uint64_t region_cap, uint64_t fixed_total, hipStream_t s) {
    const uint32_t n = A.n;
    k_list_caps<<<blocks_for_threads(n), kBlock, 0, s>>>(n, A.rrow, A.llen, first ? 1u : 0u, caps);
    TRY_HIP(scan_u32_to_u64(caps, n, spare_off, scan_scratch, s));
    uint64_t lists = 0;
    TRY_HIP(hipMemcpyAsync(&lists, spare_off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    const uint64_t base = (lists + 63) & ~63ull;
    if (fixed_total) {
        if (fixed_total < base + PLL_SHARDS * 16ull) return PLL_ENOSPC;
        region_cap = (fixed_total - base) / PLL_SHARDS;
    }
    uint32_t* na = M.get<uint32_t>(base + PLL_SHARDS * region_cap);
    if (!na) return status_of(M.err);
    if (!first)
        k_compact<<<blocks_for_waves(n), kBlock, 0, s>>>(n, A.loff, A.llen, A.arena, spare_off, na);
    TRY_HIP(hipMemcpyAsync(A.lcap, caps, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    k_reset_tops<<<1, 64, 0, s>>>(A.ctr);
    TRY_HIP(hipGetLastError());
    TRY_HIP(hipStreamSynchronize(s));
    if (A.arena) M.drop(A.arena);
    std::swap(A.loff, spare_off);
    A.arena = na;
    A.region_base = base;
    A.region_cap = region_cap;
    return PLL_OK;
}

// Input checks (bounds always; the full CSR structure under
// PLL_FLAG_VALIDATE, symmetry only for undirected graphs) and the rank-space
// CSR of the given rows.
struct RankCsr {
    uint32_t* rank = nullptr;
    uint32_t* tmp32 = nullptr;  // n+1 scratch counts
    uint64_t* scan_scratch = nullptr;
    uint64_t* rrow = nullptr;
    uint32_t* rcol = nullptr;
    uint8_t* rw = nullptr;  // weighted graphs only
};

int prepare_rank_csr(DevAllocs& M, DevCounters* ctr, DevCounters* h, uint32_t n, uint64_t nnz,
                     const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order, uint32_t flags,
                     bool symmetric, hipStream_t s, RankCsr* R, const uint8_t* w = nullptr) {
    R->rank = M.get<uint32_t>(n);
    R->tmp32 = M.get<uint32_t>((size_t)n + 1);
    R->scan_scratch = M.get<uint64_t>((n + 1) / kScanTile + 2);
    R->rrow = M.get<uint64_t>((size_t)n + 1);
    R->rcol = M.get<uint32_t>(nnz ? nnz : 1);
    if (M.err != hipSuccess) return status_of(M.err);
    uint32_t* tmp32 = R->tmp32;
    k_check_rowptr<<<blocks_for_threads((uint64_t)n + 1), kBlock, 0, s>>>(n, nnz, row_ptr, ctr);
    TRY_HIP(hipMemsetAsync(tmp32, 0, sizeof(uint32_t) * n, s));
    k_count_order<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, tmp32, ctr);
    k_check_order_counts<<<blocks_for_threads(n), kBlock, 0, s>>>(n, tmp32, ctr);
    TRY_HIP(hipGetLastError());
    int rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return PLL_EINVAL;
    if (nnz) k_check_cols<<<blocks_for_threads(nnz), kBlock, 0, s>>>(n, nnz, col, ctr);
    if (nnz && w) k_check_weights<<<blocks_for_threads(nnz), kBlock, 0, s>>>(nnz, w, ctr);
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return PLL_EINVAL;
    if (flags & PLL_FLAG_VALIDATE) {
        k_check_csr<<<blocks_for_waves(n), kBlock, 0, s>>>(n, row_ptr, col, symmetric ? 1u : 0u, w, ctr);
        rc = read_counters(ctr, h, s);
        if (rc) return rc;
        if (h->error) return PLL_EINVAL;
    }
    // rank space (a0)
    k_make_rank<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, R->rank);
    k_rank_degrees<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, row_ptr, tmp32);
    TRY_HIP(scan_u32_to_u64(tmp32, n, R->rrow, R->scan_scratch, s));
    k_relabel_cols<<<blocks_for_waves(n), kBlock, 0, s>>>(n, order, row_ptr, col, R->rank, R->rrow, R->rcol);
    if (w) {
        R->rw = M.get<uint8_t>(nnz ? nnz : 1);
        if (M.err != hipSuccess) return status_of(M.err);
        k_relabel_weights<<<blocks_for_waves(n), kBlock, 0, s>>>(n, order, row_ptr, w, R->rrow, R->rw);
    }
    TRY_HIP(hipGetLastError());
    return PLL_OK;
}

// Working buffers of the batch phases over the rank-space CSR (rrow, rcol);
// the pruning checks read the build's own table until the caller says
// otherwise.  The row masks of the first hot_rows table rows stay all ones.
// Returns the spare offsets array of the arena relayout.
int init_state(DevAllocs& M, BuildArgs& A, uint32_t n, uint64_t nnz, uint32_t W, const uint64_t* rrow,
               const uint32_t* rcol, DevCounters* ctr, hipStream_t s, uint64_t** spare_off,
               uint32_t hot_rows = kHotRows) {
    A = BuildArgs{};
    A.n = n;
    A.W = W;
    A.bstride = 64 * W;
    A.rrow = rrow;
    A.rcol = rcol;
    A.loff = M.get<uint64_t>((size_t)n + 1);
    *spare_off = M.get<uint64_t>((size_t)n + 1);
    A.llen = M.get<uint32_t>(n);
    A.lcap = M.get<uint32_t>(n);
    A.C = M.get<uint64_t>((size_t)n * W);
    A.msgs = M.get<uint64_t>((size_t)n * W);
    A.T = M.get<uint8_t>((size_t)n * A.bstride);
    A.rowmask = M.get<uint64_t>(n);
    A.Tchk = A.T;
    A.rmchk = A.rowmask;
    A.hq_seg = 2 * (nnz / pll::kHeavyItem) + 64;
    for (int q = 0; q < 2; ++q) {
        A.act_v[q] = M.get<uint32_t>(n);
        A.act_delta[q] = M.get<uint64_t>((size_t)n * W);
        A.hq[q] = M.get<uint2>(PLL_SHARDS * A.hq_seg);
    }
    A.recv = M.get<uint32_t>((size_t)PLL_SHARDS * n);
    A.recv_stamp = M.get<uint32_t>(n);
    A.touched = M.get<uint32_t>((size_t)PLL_SHARDS * n);
    A.tstart = M.get<uint32_t>((size_t)PLL_SHARDS * n);
    A.touch_stamp = M.get<uint32_t>(n);
    A.ctr = ctr;
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(A.llen, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.C, 0, sizeof(uint64_t) * n * W, s));
    TRY_HIP(hipMemsetAsync(A.msgs, 0, sizeof(uint64_t) * n * W, s));
    TRY_HIP(hipMemsetAsync(A.T, 0xFF, (size_t)n * A.bstride, s));
    A.hot = std::min<uint32_t>(n, hot_rows);
    TRY_HIP(hipMemsetAsync(A.rowmask, 0xFF, sizeof(uint64_t) * A.hot, s));
    TRY_HIP(hipMemsetAsync(A.rowmask + A.hot, 0, sizeof(uint64_t) * (n - A.hot), s));
    TRY_HIP(hipMemsetAsync(A.recv_stamp, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.touch_stamp, 0, sizeof(uint32_t) * n, s));
    return PLL_OK;
}

// Final label CSR of one build, by vertex id with hubs as ranks (a8):
// lengths, their scan, then the copy out of the arena.  The entry array is
// padded to whole 4-entry chunks: the query kernel reads labels in aligned
// 16-byte loads.
int finalize_labels(DevAllocs& M, const BuildArgs& A, const uint32_t* rank, uint32_t* tmp32,
                    uint64_t* scan_scratch, hipStream_t s, uint64_t** d_off, uint32_t** d_ent, uint2** d_lb,
                    uint64_t* total, uint32_t self_from) {
    const uint32_t n = A.n;
    k_final_lens<<<blocks_for_threads(n), kBlock, 0, s>>>(n, rank, A.llen, self_from, tmp32, A.ctr);
    *d_off = M.get_out<uint64_t>((size_t)n + 1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(scan_u32_to_u64(tmp32, n, *d_off, scan_scratch, s));
    TRY_HIP(hipMemcpyAsync(total, *d_off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    *d_ent = M.get_out<uint32_t>(std::max<uint64_t>((*total + 3) & ~3ull, 4));
    *d_lb = M.get_out<uint2>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    k_final_copy<<<std::min<uint32_t>(blocks_for_waves(n), 1024), kBlock, 0, s>>>(
        n, rank, A.loff, A.llen, A.arena, self_from, *d_off, *d_ent, *d_lb, A.ctr);
    TRY_HIP(hipGetLastError());
    return PLL_OK;
}

// One complete build attempt with a given initial arena size.
// Bit-parallel labels of up to t_req roots in rank space (Section 5.2):
// choose the roots and their sets, then grow every root's levels together,
// one push and one sibling launch per level, until a level is empty.
struct BpState {
    uint32_t t = 0, used_count = 0;
    uint8_t* used = nullptr;
    uint32_t* roots = nullptr;
    uint32_t* nbrs = nullptr;
    uint8_t* dist = nullptr;
    ulonglong2* sets = nullptr;
};

int build_bp(DevAllocs& M, uint32_t n, uint32_t t_req, const uint64_t* rrow, const uint32_t* rcol, DevCounters* ctr,
             DevCounters* h, hipStream_t s, BpState* B) {
    B->used = M.get<uint8_t>(n);
    B->roots = M.get<uint32_t>(64);
    B->nbrs = M.get<uint32_t>(64 * 64);
    uint32_t* tcount = M.get<uint32_t>(2);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(B->used, 0, n, s));
    k_bp_select<<<1, kSelBlock, 0, s>>>(n, t_req, rrow, rcol, B->used, B->roots, B->nbrs, tcount);
    TRY_HIP(hipGetLastError());
    uint32_t th[2] = {0, 0};
    TRY_HIP(hipMemcpyAsync(th, tcount, sizeof(th), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    B->t = th[0];
    B->used_count = th[1];
    const uint32_t t = B->t;
    if (t == 0) return PLL_OK;
    B->dist = M.get<uint8_t>((size_t)n * t);
    B->sets = M.get<ulonglong2>((size_t)n * t);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(B->dist, 0xFF, (size_t)n * t, s));
    TRY_HIP(hipMemsetAsync(B->sets, 0, sizeof(ulonglong2) * n * t, s));
    k_bp_seed<<<t, 65, 0, s>>>(t, B->roots, B->nbrs, B->dist, B->sets);
    for (uint32_t L = 1; L < PLL_INF8; ++L) {
        k_bp_push<<<blocks_for_waves(n), kBlock, 0, s>>>(n, t, L - 1, rrow, rcol, B->dist, B->sets, ctr);
        TRY_HIP(hipMemsetAsync(&ctr->sh[0].recv[0], 0, sizeof(uint32_t), s));
        k_bp_sibling<<<blocks_for_waves(n), kBlock, 0, s>>>(n, t, L, rrow, rcol, B->dist, B->sets, ctr);
        TRY_HIP(hipGetLastError());
        int rc = read_counters(ctr, h, s);
        if (rc) return rc;
        if (h->error) return device_error_status(h->error);
        if (h->sh[0].recv[0] == 0) break;
    }
    TRY_HIP(hipMemsetAsync(&ctr->sh[0].recv[0], 0, sizeof(uint32_t), s));
    return PLL_OK;
}

int build_attempt(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                  uint32_t b, uint32_t flags, uint64_t arena_hint, bool arena_fixed, uint32_t max_workgroups,
                  uint32_t bp_req, hipStream_t s, pll_index* idx, uint64_t* used_arena, const FixedWs* fw = nullptr) {
    DevAllocs M;
    M.s = s;
    HostCounters HC;
    PhaseProfiler P;
    P.on = (flags & PLL_FLAG_PROFILE) != 0;
    P.s = s;
    if (fw) {
        M.fixed = static_cast<char*>(fw->base);
        M.fixed_cap = fw->bytes;
        HC.p = fw->host_ctr;
        HC.own = false;
    } else {
        TRY_HIP(pll_pinned_alloc((void**)&HC.p, sizeof(DevCounters)));
    }
    DevCounters* h = HC.p;
    const uint32_t W = (b + 63) / 64;

    DevCounters* ctr = M.get<DevCounters>(1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(ctr, 0, sizeof(DevCounters), s));
    hipEvent_t e_prep = P.mark();
    RankCsr RC;
    int rc = prepare_rank_csr(M, ctr, h, n, nnz, row_ptr, col, order, flags, true, s, &RC);
    if (rc) return rc;
    uint32_t* rank = RC.rank;
    uint32_t* tmp32 = RC.tmp32;
    uint64_t* scan_scratch = RC.scan_scratch;

    // --- build state
    BuildArgs A{};
    uint64_t* spare_off = nullptr;
    // bit-parallel roots take the top-ranked vertices out of the labels, which
    // leaves the top rows sparse: their masks are kept exact then
    rc = init_state(M, A, n, nnz, W, RC.rrow, RC.rcol, ctr, s, &spare_off, bp_req ? 0u : kHotRows);
    if (rc) return rc;
    // the round-2 neighbour check needs every higher-ranked neighbour to be a
    // hub, which bit-parallel roots (taken out of the labels) break
    A.nbr_hubs = bp_req ? 0u : 1u;
    BpState BP;
    if (bp_req) {
        rc = build_bp(M, n, bp_req, RC.rrow, RC.rcol, ctr, h, s, &BP);
        if (rc) return rc;
        A.bp_t = BP.t;
        A.bp_used = BP.used;
        A.bp_dist = BP.dist;
        A.bp_sets = BP.sets;
        if (BP.t) {
            A.bpb_dist = M.get<uint8_t>((size_t)BP.t * A.bstride);
            A.bpb_sets = M.get<ulonglong2>((size_t)BP.t * A.bstride);
            if (M.err != hipSuccess) return status_of(M.err);
        }
    }
    // initial label layout: capacities 16/32, then the bump regions
    uint64_t region_cap = std::max<uint64_t>(4096, arena_hint / PLL_SHARDS);
    rc = relayout_arena(M, A, spare_off, tmp32, scan_scratch, true, region_cap, arena_fixed ? arena_hint : 0, s);
    if (rc) return rc;
    P.span(PLL_PHASE_PREP, e_prep, P.mark(), (flags & PLL_FLAG_VALIDATE) ? 14 : 13);

    const uint32_t recheck = (flags & PLL_FLAG_RECHECK) ? 1u : 0u;
    const uint32_t relaxed = (flags & PLL_FLAG_RELAXED) ? 1u : 0u;
    uint32_t rstamp = 0, bstamp = 0;
    uint64_t rounds = 0, batches = 0, accepted_seen = 0;
    // PLL_TRACE=1 prints one line per round to stderr (with PLL_FLAG_PROFILE: kernel times too)
    const char* trace_env = std::getenv("PLL_TRACE");
    const bool trace = trace_env && trace_env[0] == '1';
    unsigned long long last[PLL_NUM_ST] = {};

    // --- batches (a1-a7): one launch per phase with a read-back per round,
    // or (PLL_FLAG_PERSISTENT) one persistent launch that hands back to the
    // host only for arena compaction
    uint32_t grid_workgroups = 0;
    // profiled builds: 30 us of device wall clock ahead of each timed check
    uint64_t delay_ticks = 0;
    if (P.on) {
        int khz = 0, dev = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            delay_ticks = (uint64_t)khz * 30 / 1000;
    }
    // the second message buffer and receiver list of the fused rounds:
    // round j's messages and receivers live in mbuf[j & 1] and rbuf[j & 1]
    uint64_t* mbuf[2] = {A.msgs, nullptr};
    uint32_t* rbuf[2] = {A.recv, nullptr};
    // pulled rounds: a round whose receivers number at least n / kPullFrac
    // (the active vertices of the next round are among them) gathers at
    // every vertex instead of scattering atomics along every active edge
    uint2* pull_items = nullptr;
    uint32_t* pull_n = nullptr;
    uint64_t pull_cap = 0;
    const bool pull_ok = !(flags & PLL_FLAG_PERSISTENT) && n >= kPullMinN;
    if (!(flags & PLL_FLAG_PERSISTENT)) {
        mbuf[1] = M.get<uint64_t>((size_t)n * W);
        rbuf[1] = M.get<uint32_t>((size_t)PLL_SHARDS * n);
        if (M.err != hipSuccess) return status_of(M.err);
        TRY_HIP(hipMemsetAsync(mbuf[1], 0, sizeof(uint64_t) * n * W, s));
    }
    if (pull_ok) {
        pull_cap = (uint64_t)n + nnz / pll::kPullSeg + 1;
        pull_items = M.get<uint2>(pull_cap);
        pull_n = M.get<uint32_t>(1);
        A.act_at = M.get<uint64_t>(n);
        if (M.err != hipSuccess) return status_of(M.err);
        TRY_HIP(hipMemsetAsync(pull_n, 0, sizeof(uint32_t), s));
        TRY_HIP(hipMemsetAsync(A.act_at, 0, sizeof(uint64_t) * n, s));
        k_pull_items<<<blocks_for_waves((n + 63) / 64), kBlock, 0, s>>>(A, pull_items, pull_n);
        TRY_HIP(hipGetLastError());
    }
    if (flags & PLL_FLAG_PERSISTENT) {
        TRY_HIP(hipStreamSynchronize(s));
        P.resolve();
        for (uint32_t ib = 0; ib < n;) {
            BatchRun R{};
            hipEvent_t l0 = P.mark(), l1 = P.mark();  // recorded again around the launch
            rc = pll_run_batches(A, ib, b, flags, &bstamp, &rstamp, !arena_fixed, max_workgroups, s, l0, l1, &R);
            if (rc) return rc;
            P.span(PLL_PHASE_LOOP, l0, l1, 1);
            P.resolve();
            rc = read_counters(ctr, h, s);
            if (rc) return rc;
            if (h->error) return device_error_status(h->error);
            rounds += R.rounds;
            batches += R.batches;
            grid_workgroups = R.grid;
            for (int ph = PLL_PHASE_INIT; ph <= PLL_PHASE_END && P.on; ++ph) {
                P.ms[ph] += R.ms[ph];
                P.launches[ph] += R.counts[ph];
            }
            if (R.next_ib <= ib) return PLL_EDEVICE;  // no progress: cannot happen
            ib = R.next_ib;
            if (ib < n) {
                rc = relayout_arena(M, A, spare_off, tmp32, scan_scratch, false, A.region_cap * 2, 0, s);
                if (rc) return rc;
            }
        }
    }
    // Batches from skip_from on hold isolated roots only (k_edge_end); they
    // are not run: each counts as one batch of one round (the round in which
    // nobody receives), and finalize writes its roots' self entries.  The
    // bound is known from the first read-back on.  Not with bit-parallel
    // roots, whose vertices (isolated ones among them) store no self entry.
    uint32_t skip_from = n;
    bool skip_known = (flags & PLL_FLAG_PERSISTENT) || A.bp_t;
    if (!skip_known) {
        k_edge_end<<<std::min<uint32_t>(blocks_for_threads(n), 1024), kBlock, 0, s>>>(n, A.rrow, ctr);
        TRY_HIP(hipGetLastError());
    }
    // round 1's receivers (the neighbours of the batch) are only counted
    // after its launch; its grid is sized by the previous batch's count,
    // which falls from batch to batch in rank order (a grid-stride loop
    // covers any excess)
    uint64_t r1_est = n;
    for (uint32_t ib = 0; !(flags & PLL_FLAG_PERSISTENT) && ib < n; ib += b) {
        if (ib >= skip_from) {
            const uint64_t left = (n - ib + b - 1) / b;
            batches += left;
            rounds += left;
            break;
        }
        const uint32_t bs = std::min(b, n - ib);
        ++bstamp;
        ++batches;
        hipEvent_t e0 = P.mark();
        // later batches have the counters reset by the previous batch's
        // table clear
        if (ib == 0) k_batch_prep<<<1, 64, 0, s>>>(ctr);
        if (A.bp_t) k_bp_batch_stage<<<blocks_for_threads((uint64_t)A.bp_t * bs), kBlock, 0, s>>>(A, ib, bs);
        k_batch_init<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs, bstamp);
        P.span(PLL_PHASE_INIT, e0, P.mark(), (A.bp_t ? 2 : 1) + (ib == 0 ? 1 : 0));
        // round 1's push from the batch vertices (active list 0) into
        // receiver queue 0 and message buffer 1; afterwards every round j is
        // one fused launch (check of round j, push of round j+1 into buffer
        // (j+1) & 1), plus a launch for heavy rows when there are any
        ++rstamp;
        {
            BuildArgs A1 = A;
            A1.msgs = mbuf[1];
            A1.recv = rbuf[1];
            hipEvent_t r0 = P.mark();
            k_push<<<blocks_for_waves((uint64_t)bs + 1024), kBlock, 0, s>>>(A1, ib, 0, bs, rstamp, bstamp);
            P.span(PLL_PHASE_PUSH, r0, P.mark(), 1);
        }
        uint64_t next_est = r1_est;
        for (uint32_t j = 1;; ++j) {
            ++rounds;
            // the first round's receivers push the batch's densest deltas along
            // high-degree rows, so gathering pays off from fewer of them
            const uint32_t pull = pull_ok && next_est * (j == 1 ? kPullFrac1 : kPullFrac) >= n ? 1u : 0u;
            const pll::NextRound nr{mbuf[(j + 1) & 1u], rbuf[(j + 1) & 1u], (j - 1) % 3, j % 3, (j + 1) % 3, j & 1u,
                                    rstamp + 1, bstamp, pull};
            ++rstamp;
            BuildArgs Aj = A;
            Aj.msgs = mbuf[j & 1u];
            Aj.recv = rbuf[j & 1u];
            if (P.on) k_delay<<<1, 1, 0, s>>>(delay_ticks);
            hipEvent_t r1 = P.mark();
            // rounds with many receivers check four per wave (phase_check4)
            const bool pack = ((flags & PLL_FLAG_PACK4) || next_est >= kPackMin) && j <= pll::kSmallT;
            const uint64_t waves = pack ? next_est / 4 + 512 : next_est + 2048;
            dispatch_check_push(blocks_for_waves(std::min<uint64_t>(n, waves)), s, Aj, ib, bs, j, nr, relaxed, pack);
            P.span(PLL_PHASE_CHECK, r1, P.mark(), 1);
            TRY_HIP(hipGetLastError());
            if (pull) {
                hipEvent_t r3 = P.mark();
                k_pull<<<blocks_for_waves(pull_cap), kBlock, 0, s>>>(A, ib, pull_items, pull_n, nr.hout, nr);
                P.span(PLL_PHASE_PUSH, r3, P.mark(), 1);
                TRY_HIP(hipGetLastError());
            }
            const double check_ms0 = P.ms[PLL_PHASE_CHECK];
            rc = read_counters(ctr, h, s);
            if (rc) return rc;
            P.resolve();
            if (!skip_known) {  // this batch runs: skipping starts after it
                skip_known = true;
                const uint64_t from = std::max<uint64_t>(((uint64_t)h->edge_end + b - 1) / b * b, (uint64_t)ib + b);
                if (from < n) skip_from = (uint32_t)from;
            }
            const unsigned long long acc_now = sum_stat(h, PLL_ST_ACC);
            if (j == 1) r1_est = std::max<uint64_t>(bs, sum_recv(h, nr.rin));
            if (trace) {
                unsigned long long cur[PLL_NUM_ST];
                for (int k = 0; k < PLL_NUM_ST; ++k) cur[k] = sum_stat(h, k);
                std::fprintf(stderr,
                             "pll-trace batch=%u round=%u recv=%u next=%u heavy=%u cand=%llu acc=%llu read=%llu "
                             "table=%llu grow=%llu check_us=%.1f\n",
                             (unsigned)(ib / b), j, sum_recv(h, nr.rin), sum_recv(h, nr.rout), sum_hq(h, nr.hout),
                             cur[PLL_ST_CAND] - last[PLL_ST_CAND], cur[PLL_ST_ACC] - last[PLL_ST_ACC],
                             cur[PLL_ST_READ] - last[PLL_ST_READ], cur[PLL_ST_TABLE] - last[PLL_ST_TABLE],
                             cur[PLL_ST_GROW] - last[PLL_ST_GROW], (P.ms[PLL_PHASE_CHECK] - check_ms0) * 1e3);
                for (int k = 0; k < PLL_NUM_ST; ++k) last[k] = cur[k];
            }
            if (h->error) return device_error_status(h->error);
            if (acc_now == accepted_seen) break;  // nobody accepted anything: the batch is done
            accepted_seen = acc_now;
            const uint32_t nh = sum_hq(h, nr.hout);
            if (nh) {
                hipEvent_t r2 = P.mark();
                k_push_heavy<<<blocks_for_waves(nh), kBlock, 0, s>>>(A, ib, nr.hout, nr.rout, nr.msgs, nr.recv,
                                                                     nr.rstamp, bstamp);
                P.span(PLL_PHASE_PUSH, r2, P.mark(), 1);
            }
            next_est = (uint64_t)sum_recv(h, nr.rout) + 1024ull * nh;
            if (next_est == 0) {  // nobody receives in round j+1: it would accept nothing
                ++rounds;
                break;
            }
        }
        hipEvent_t e1 = P.mark();
        dispatch_batch_end(blocks_for_waves(sum_touched(h)), s, A, ib, bs, recheck);
        k_clear_table<<<blocks_for_waves(4ull * bs), kBlock, 0, s>>>(A, ib, bs, ctr);
        P.span(PLL_PHASE_END, e1, P.mark(), 2);
        TRY_HIP(hipGetLastError());
        // compact the lists into a larger arena once a bump region is half used
        if (!arena_fixed && ib + b < n && max_top(h) * 2 > A.region_cap) {
            rc = relayout_arena(M, A, spare_off, tmp32, scan_scratch, false, A.region_cap * 2, 0, s);
            if (rc) return rc;
        }
    }

    // --- finalize (a8): CSR by vertex id, hubs as ranks
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return device_error_status(h->error);
    P.resolve();
    hipEvent_t e_fin = P.mark();
    uint64_t* d_off = nullptr;
    uint32_t* d_ent = nullptr;
    uint2* d_lb = nullptr;
    uint64_t total = 0;
    rc = finalize_labels(M, A, rank, tmp32, scan_scratch, s, &d_off, &d_ent, &d_lb, &total, skip_from);
    if (rc) return rc;
    uint32_t* d_order = M.get_out<uint32_t>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemcpyAsync(d_order, order, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    if (BP.t) {
        idx->d_bp_roots = M.get_out<uint32_t>(BP.t);
        idx->d_bp_nbrs = M.get_out<uint32_t>((size_t)BP.t * 64);
        idx->d_bp_dist = M.get_out<uint8_t>((size_t)n * BP.t);
        idx->d_bp_sets = M.get_out<ulonglong2>((size_t)n * BP.t);
        if (M.err != hipSuccess) return status_of(M.err);
        k_bp_by_vertex<<<blocks_for_threads((uint64_t)n * BP.t), kBlock, 0, s>>>(n, BP.t, RC.rank, BP.dist, BP.sets,
                                                                                 idx->d_bp_dist, idx->d_bp_sets);
        k_bp_ids<<<1, kBlock, 0, s>>>(BP.t, order, BP.roots, BP.nbrs, idx->d_bp_roots, idx->d_bp_nbrs);
    }
    TRY_HIP(hipGetLastError());
    P.span(PLL_PHASE_FINAL, e_fin, P.mark(), 5);
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    P.resolve();

    idx->n = n;
    idx->total = total;
    idx->d_off = d_off;
    idx->d_ent = d_ent;
    idx->d_lb = d_lb;
    idx->d_order = d_order;
    M.forget(d_off);
    M.forget(d_ent);
    M.forget(d_lb);
    M.forget(d_order);
    M.forget(idx->d_bp_roots);
    M.forget(idx->d_bp_nbrs);
    M.forget(idx->d_bp_dist);
    M.forget(idx->d_bp_sets);
    pll_index_info& I = idx->info;
    I.n = n;
    I.batch_size = b;
    I.total_entries = total;
    I.in_entries = total;
    I.out_entries = total;
    I.bp_roots = BP.t;
    I.bp_vertices = BP.used_count;
    I.bp_pruned = sum_stat(h, PLL_ST_BP);
    I.check_push_edges = sum_stat(h, PLL_ST_FUSED_EDGES);
    I.label_bytes = total * sizeof(uint32_t) + ((uint64_t)n + 1) * sizeof(uint64_t) + (uint64_t)n * sizeof(uint2);
    I.max_dist = h->max_dist;
    I.max_label = h->max_label;
    I.batches = batches;
    I.rounds = rounds;
    I.candidates = sum_stat(h, PLL_ST_CAND);
    I.accepted = sum_stat(h, PLL_ST_ACC);
    I.edges_scanned = sum_stat(h, PLL_ST_EDGES);
    I.recheck_removed = sum_stat(h, PLL_ST_RECHECK);
    I.gang = grid_workgroups ? grid_workgroups : 1;
    I.check_entries_read = sum_stat(h, PLL_ST_READ);
    I.check_table_reads = sum_stat(h, PLL_ST_TABLE);
    I.check_cost_pos = sum_stat(h, PLL_ST_COST_POS);
    I.check_cost_neg = sum_stat(h, PLL_ST_COST_NEG);
    for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
        I.phase_ms[ph] = P.ms[ph];
        I.phase_launches[ph] = P.launches[ph];
    }
    *used_arena = A.region_base + PLL_SHARDS * A.region_cap;
    return PLL_OK;
}

// Weighted graphs (Section 5.1).  The rounds of a batch become
// Bellman-Ford iterations restricted to vertices ranked below the roots:
// a vertex that accepted entries in round j-1 pushes each of them along its
// edges with distance d + w_e; a candidate passes the D filter only if it
// lowers the best distance that reached the vertex in this batch, and the
// pruning check compares each candidate with its own distance.  A batch
// ends when a round accepts nothing.  Entries accepted on the way can be
// non-canonical (a shorter path through a higher-ranked hub may arrive in a
// later round); the batch end keeps each hub's last (shortest) entry and
// rechecks every entry of the batch against the batch's tables, which
// leaves exactly the canonical labels.  Distances stay uint8: a candidate
// path of 255 or more fails the build with PLL_EDIST.
int build_attempt_weighted(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col, const uint8_t* w,
                           const uint32_t* order, uint32_t b, uint32_t flags, uint64_t arena_hint, bool arena_fixed,
                           hipStream_t s, pll_index* idx, uint64_t* used_arena) {
    DevAllocs M;
    M.s = s;
    HostCounters HC;
    PhaseProfiler P;
    P.on = (flags & PLL_FLAG_PROFILE) != 0;
    P.s = s;
    TRY_HIP(pll_pinned_alloc((void**)&HC.p, sizeof(DevCounters)));
    DevCounters* h = HC.p;
    const uint32_t W = (b + 63) / 64;

    DevCounters* ctr = M.get<DevCounters>(1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(ctr, 0, sizeof(DevCounters), s));
    hipEvent_t e_prep = P.mark();
    RankCsr RC;
    int rc = prepare_rank_csr(M, ctr, h, n, nnz, row_ptr, col, order, flags, true, s, &RC, w);
    if (rc) return rc;
    BuildArgs A{};
    uint64_t* spare_off = nullptr;
    rc = init_state(M, A, n, nnz, W, RC.rrow, RC.rcol, ctr, s, &spare_off);
    if (rc) return rc;
    A.rw = RC.rw;
    A.D = M.get<uint8_t>((size_t)n * A.bstride);
    for (int q = 0; q < 2; ++q) A.act_rng[q] = M.get<uint2>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(A.D, 0xFF, (size_t)n * A.bstride, s));
    const uint64_t region_cap = std::max<uint64_t>(4096, arena_hint / PLL_SHARDS);
    rc = relayout_arena(M, A, spare_off, RC.tmp32, RC.scan_scratch, true, region_cap, arena_fixed ? arena_hint : 0, s);
    if (rc) return rc;
    P.span(PLL_PHASE_PREP, e_prep, P.mark(), (flags & PLL_FLAG_VALIDATE) ? 16 : 15);

    uint32_t rstamp = 0, bstamp = 0;
    uint64_t rounds = 0, batches = 0;
    unsigned long long accepted_seen = 0;
    for (uint32_t ib = 0; ib < n; ib += b) {
        const uint32_t bs = std::min(b, n - ib);
        ++bstamp;
        ++batches;
        hipEvent_t e0 = P.mark();
        k_batch_prep<<<1, 64, 0, s>>>(ctr);
        k_batch_init<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs, bstamp);
        P.span(PLL_PHASE_INIT, e0, P.mark(), 2);
        uint32_t p = 0, nact = bs;
        uint64_t heavy_waves = 1024;
        for (;;) {
            ++rstamp;
            ++rounds;
            hipEvent_t r0 = P.mark();
            k_push_w<<<blocks_for_waves(nact + heavy_waves), kBlock, 0, s>>>(A, ib, p, nact, rstamp, bstamp);
            hipEvent_t r1 = P.mark();
            dispatch_check_w(blocks_for_waves(std::min<uint64_t>(n, 16ull * nact + 2048)), s, A, ib, bs, p);
            hipEvent_t r2 = P.mark();
            P.span(PLL_PHASE_PUSH, r0, r1, 1);
            P.span(PLL_PHASE_CHECK, r1, r2, 1);
            TRY_HIP(hipGetLastError());
            rc = read_counters(ctr, h, s);
            if (rc) return rc;
            P.resolve();
            if (h->error) return device_error_status(h->error);
            const unsigned long long acc_now = sum_stat(h, PLL_ST_ACC);
            if (acc_now == accepted_seen) break;
            accepted_seen = acc_now;
            nact = sum_recv(h, p);
            p ^= 1u;
            heavy_waves = sum_hq(h, p);
        }
        hipEvent_t e1 = P.mark();
        dispatch_batch_end_w(blocks_for_waves(sum_touched(h)), s, A, ib, bs);
        k_clear_table<<<blocks_for_waves(4ull * bs), kBlock, 0, s>>>(A, ib, bs, nullptr);
        P.span(PLL_PHASE_END, e1, P.mark(), 2);
        TRY_HIP(hipGetLastError());
        if (!arena_fixed && ib + b < n && max_top(h) * 2 > A.region_cap) {
            rc = relayout_arena(M, A, spare_off, RC.tmp32, RC.scan_scratch, false, A.region_cap * 2, 0, s);
            if (rc) return rc;
        }
    }

    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return device_error_status(h->error);
    P.resolve();
    hipEvent_t e_fin = P.mark();
    uint64_t* d_off = nullptr;
    uint32_t* d_ent = nullptr;
    uint2* d_lb = nullptr;
    uint64_t total = 0;
    rc = finalize_labels(M, A, RC.rank, RC.tmp32, RC.scan_scratch, s, &d_off, &d_ent, &d_lb, &total, n);
    if (rc) return rc;
    uint32_t* d_order = M.get_out<uint32_t>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemcpyAsync(d_order, order, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipGetLastError());
    P.span(PLL_PHASE_FINAL, e_fin, P.mark(), 5);
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    P.resolve();

    idx->n = n;
    idx->total = total;
    idx->d_off = d_off;
    idx->d_ent = d_ent;
    idx->d_lb = d_lb;
    idx->d_order = d_order;
    M.forget(d_off);
    M.forget(d_ent);
    M.forget(d_lb);
    M.forget(d_order);
    pll_index_info& I = idx->info;
    I.n = n;
    I.batch_size = b;
    I.weighted = 1;
    I.total_entries = total;
    I.in_entries = total;
    I.out_entries = total;
    I.label_bytes = total * sizeof(uint32_t) + ((uint64_t)n + 1) * sizeof(uint64_t) + (uint64_t)n * sizeof(uint2);
    I.max_dist = h->max_dist;
    I.max_label = h->max_label;
    I.batches = batches;
    I.rounds = rounds;
    I.candidates = sum_stat(h, PLL_ST_CAND);
    I.accepted = sum_stat(h, PLL_ST_ACC);
    I.edges_scanned = sum_stat(h, PLL_ST_EDGES);
    I.recheck_removed = sum_stat(h, PLL_ST_RECHECK);
    I.gang = 1;
    I.check_entries_read = sum_stat(h, PLL_ST_READ);
    I.check_table_reads = sum_stat(h, PLL_ST_TABLE);
    I.check_cost_pos = sum_stat(h, PLL_ST_COST_POS);
    I.check_cost_neg = sum_stat(h, PLL_ST_COST_NEG);
    for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
        I.phase_ms[ph] = P.ms[ph];
        I.phase_launches[ph] = P.launches[ph];
    }
    *used_arena = A.region_base + PLL_SHARDS * A.region_cap;
    return PLL_OK;
}

// Directed graphs (Section 5.1).  Two coupled builds run in lockstep:
// the forward side grows L_in along out-arcs and the backward side grows
// L_out along in-arcs, each with its own candidate bit-vectors, queues and
// distance table.  A side's table holds its own label of the batch roots
// (forward: L_in(u_k), filled at batch init and when a root accepts an
// entry); a side's pruning checks read the other side's table, so a forward
// check of u_k at v scans L_in(v) against L_out(u_k) and a backward check
// scans L_out(v) against L_in(u_k).  Round j of both sides runs after round
// j-1 of both: an entry that must prune a round-j candidate has distance
// below j on both of its sides, and an entry accepted in round j on either
// side cannot prune a round-j candidate of the other (its hub would have to
// be the candidate vertex itself, which the rank mask keeps out).
int build_attempt_directed(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col,
                           const uint32_t* order, uint32_t b, uint32_t flags, uint64_t arena_hint, bool arena_fixed,
                           hipStream_t s, pll_index* idx, uint64_t* used_arena) {
    DevAllocs M;
    M.s = s;
    HostCounters HC[2];
    PhaseProfiler P;
    P.on = (flags & PLL_FLAG_PROFILE) != 0;
    P.s = s;
    for (auto& hc : HC) TRY_HIP(pll_pinned_alloc((void**)&hc.p, sizeof(DevCounters)));
    DevCounters* h[2] = {HC[0].p, HC[1].p};
    const uint32_t W = (b + 63) / 64;

    DevCounters* ctr = M.get<DevCounters>(2);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(ctr, 0, 2 * sizeof(DevCounters), s));
    hipEvent_t e_prep = P.mark();
    RankCsr RC;
    int rc = prepare_rank_csr(M, ctr, h[0], n, nnz, row_ptr, col, order, flags, false, s, &RC);
    if (rc) return rc;
    uint32_t* tmp32 = RC.tmp32;
    uint64_t* scan_scratch = RC.scan_scratch;

    // in-arcs in rank space
    uint64_t* irow = M.get<uint64_t>((size_t)n + 1);
    uint32_t* icol = M.get<uint32_t>(nnz ? nnz : 1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(tmp32, 0, sizeof(uint32_t) * ((size_t)n + 1), s));
    if (nnz) k_count_heads<<<blocks_for_threads(nnz), kBlock, 0, s>>>(nnz, RC.rcol, tmp32);
    TRY_HIP(scan_u32_to_u64(tmp32, n, irow, scan_scratch, s));
    TRY_HIP(hipMemsetAsync(tmp32, 0, sizeof(uint32_t) * ((size_t)n + 1), s));
    k_fill_transpose<<<blocks_for_waves(n), kBlock, 0, s>>>(n, RC.rrow, RC.rcol, irow, tmp32, icol);
    TRY_HIP(hipGetLastError());

    // side 0: forward (L_in, out-arcs); side 1: backward (L_out, in-arcs)
    BuildArgs A[2];
    uint64_t* spare_off[2] = {nullptr, nullptr};
    rc = init_state(M, A[0], n, nnz, W, RC.rrow, RC.rcol, ctr, s, &spare_off[0]);
    if (rc) return rc;
    rc = init_state(M, A[1], n, nnz, W, irow, icol, ctr + 1, s, &spare_off[1]);
    if (rc) return rc;
    for (int d = 0; d < 2; ++d) {
        A[d].Tchk = A[d ^ 1].T;
        A[d].rmchk = A[d ^ 1].rowmask;
    }
    // second message buffer and receiver list of each side's fused rounds
    uint64_t* mbuf[2][2] = {{A[0].msgs, nullptr}, {A[1].msgs, nullptr}};
    uint32_t* rbuf[2][2] = {{A[0].recv, nullptr}, {A[1].recv, nullptr}};
    for (int d = 0; d < 2; ++d) {
        mbuf[d][1] = M.get<uint64_t>((size_t)n * W);
        rbuf[d][1] = M.get<uint32_t>((size_t)PLL_SHARDS * n);
        if (M.err != hipSuccess) return status_of(M.err);
        TRY_HIP(hipMemsetAsync(mbuf[d][1], 0, sizeof(uint64_t) * n * W, s));
    }
    const uint64_t region_cap = std::max<uint64_t>(4096, arena_hint / (2 * PLL_SHARDS));
    for (int d = 0; d < 2; ++d) {
        rc = relayout_arena(M, A[d], spare_off[d], tmp32, scan_scratch, true, region_cap,
                            arena_fixed ? arena_hint / 2 : 0, s);
        if (rc) return rc;
    }
    P.span(PLL_PHASE_PREP, e_prep, P.mark(), (flags & PLL_FLAG_VALIDATE) ? 20 : 19);

    auto read_both = [&]() -> int {
        TRY_HIP(hipMemcpyAsync(h[0], ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        TRY_HIP(hipMemcpyAsync(h[1], ctr + 1, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
        TRY_HIP(hipStreamSynchronize(s));
        return PLL_OK;
    };
    const uint32_t recheck = (flags & PLL_FLAG_RECHECK) ? 1u : 0u;
    uint32_t rstamp = 0, bstamp = 0;
    uint64_t rounds = 0, batches = 0;
    unsigned long long accepted_seen[2] = {0, 0};
    for (uint32_t ib = 0; ib < n; ib += b) {
        const uint32_t bs = std::min(b, n - ib);
        ++bstamp;
        ++batches;
        hipEvent_t e0 = P.mark();
        for (int d = 0; d < 2; ++d) {
            k_batch_prep<<<1, 64, 0, s>>>(A[d].ctr);
            k_batch_init<<<blocks_for_waves(bs), kBlock, 0, s>>>(A[d], ib, bs, bstamp);
        }
        P.span(PLL_PHASE_INIT, e0, P.mark(), 4);
        // fused rounds as in the undirected build, both sides in one launch
        ++rstamp;
        for (int d = 0; d < 2; ++d) {
            BuildArgs A1 = A[d];
            A1.msgs = mbuf[d][1];
            A1.recv = rbuf[d][1];
            hipEvent_t r0 = P.mark();
            k_push<<<blocks_for_waves((uint64_t)bs + 1024), kBlock, 0, s>>>(A1, ib, 0, bs, rstamp, bstamp);
            P.span(PLL_PHASE_PUSH, r0, P.mark(), 1);
        }
        uint64_t next_est[2] = {bs, bs};
        bool live[2] = {true, true};
        for (uint32_t j = 1; live[0] || live[1]; ++j) {
            ++rounds;
            pll::NextRound nr[2];
            BuildArgs Aj[2];
            uint32_t nb[2] = {0, 0};
            for (int d = 0; d < 2; ++d) {
                nr[d] = pll::NextRound{mbuf[d][(j + 1) & 1u], rbuf[d][(j + 1) & 1u], (j - 1) % 3, j % 3, (j + 1) % 3,
                                       j & 1u, rstamp + 1, bstamp};
                Aj[d] = A[d];
                Aj[d].msgs = mbuf[d][j & 1u];
                Aj[d].recv = rbuf[d][j & 1u];
                if (live[d]) nb[d] = blocks_for_waves(std::min<uint64_t>(n, next_est[d] + 2048));
            }
            ++rstamp;
            hipEvent_t r1 = P.mark();
            dispatch_check_push2(nb[0], nb[1], s, Aj[0], nr[0], Aj[1], nr[1], ib, bs, j);
            P.span(PLL_PHASE_CHECK, r1, P.mark(), 1);
            TRY_HIP(hipGetLastError());
            rc = read_both();
            if (rc) return rc;
            P.resolve();
            for (int d = 0; d < 2; ++d) {
                if (h[d]->error) return device_error_status(h[d]->error);
                if (!live[d]) continue;
                const unsigned long long acc_now = sum_stat(h[d], PLL_ST_ACC);
                if (acc_now == accepted_seen[d]) {  // this side accepted nothing: its search is done
                    live[d] = false;
                    continue;
                }
                accepted_seen[d] = acc_now;
                const uint32_t nh = sum_hq(h[d], nr[d].hout);
                if (nh) {
                    hipEvent_t r2 = P.mark();
                    k_push_heavy<<<blocks_for_waves(nh), kBlock, 0, s>>>(A[d], ib, nr[d].hout, nr[d].rout, nr[d].msgs,
                                                                         nr[d].recv, nr[d].rstamp, bstamp);
                    P.span(PLL_PHASE_PUSH, r2, P.mark(), 1);
                }
                next_est[d] = (uint64_t)sum_recv(h[d], nr[d].rout) + 1024ull * nh;
            }
        }
        // both sides' batch ends read the other side's table, so the tables
        // are cleared only after both
        hipEvent_t e1 = P.mark();
        for (int d = 0; d < 2; ++d) dispatch_batch_end(blocks_for_waves(sum_touched(h[d])), s, A[d], ib, bs, recheck);
        for (int d = 0; d < 2; ++d) k_clear_table<<<blocks_for_waves(4ull * bs), kBlock, 0, s>>>(A[d], ib, bs, nullptr);
        P.span(PLL_PHASE_END, e1, P.mark(), 4);
        TRY_HIP(hipGetLastError());
        for (int d = 0; d < 2; ++d) {
            if (!arena_fixed && ib + b < n && max_top(h[d]) * 2 > A[d].region_cap) {
                rc = relayout_arena(M, A[d], spare_off[d], tmp32, scan_scratch, false, A[d].region_cap * 2, 0, s);
                if (rc) return rc;
            }
        }
    }

    // --- finalize: L_in and L_out by vertex id
    rc = read_both();
    if (rc) return rc;
    for (int d = 0; d < 2; ++d)
        if (h[d]->error) return device_error_status(h[d]->error);
    P.resolve();
    hipEvent_t e_fin = P.mark();
    uint64_t* d_off[2] = {nullptr, nullptr};
    uint32_t* d_ent[2] = {nullptr, nullptr};
    uint2* d_lb[2] = {nullptr, nullptr};
    uint64_t total[2] = {0, 0};
    for (int d = 0; d < 2; ++d) {
        rc = finalize_labels(M, A[d], RC.rank, tmp32, scan_scratch, s, &d_off[d], &d_ent[d], &d_lb[d], &total[d], n);
        if (rc) return rc;
    }
    uint32_t* d_order = M.get_out<uint32_t>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemcpyAsync(d_order, order, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipGetLastError());
    P.span(PLL_PHASE_FINAL, e_fin, P.mark(), 9);
    rc = read_both();
    if (rc) return rc;
    P.resolve();

    idx->n = n;
    idx->directed = true;
    idx->total = total[0];
    idx->d_off = d_off[0];
    idx->d_ent = d_ent[0];
    idx->total_out = total[1];
    idx->d_off_out = d_off[1];
    idx->d_ent_out = d_ent[1];
    idx->d_lb = d_lb[0];
    idx->d_lb_out = d_lb[1];
    idx->d_order = d_order;
    for (int d = 0; d < 2; ++d) {
        M.forget(d_off[d]);
        M.forget(d_ent[d]);
        M.forget(d_lb[d]);
    }
    M.forget(d_order);
    pll_index_info& I = idx->info;
    I.n = n;
    I.batch_size = b;
    I.directed = 1;
    I.in_entries = total[0];
    I.out_entries = total[1];
    I.total_entries = total[0] + total[1];
    I.label_bytes = (total[0] + total[1]) * sizeof(uint32_t) + 2 * ((uint64_t)n + 1) * sizeof(uint64_t) +
                    2 * (uint64_t)n * sizeof(uint2);
    I.max_dist = std::max(h[0]->max_dist, h[1]->max_dist);
    I.max_label = std::max(h[0]->max_label, h[1]->max_label);
    I.batches = batches;
    I.rounds = rounds;
    auto both = [&](int k) { return sum_stat(h[0], k) + sum_stat(h[1], k); };
    I.candidates = both(PLL_ST_CAND);
    I.accepted = both(PLL_ST_ACC);
    I.edges_scanned = both(PLL_ST_EDGES);
    I.recheck_removed = both(PLL_ST_RECHECK);
    I.gang = 1;
    I.check_entries_read = both(PLL_ST_READ);
    I.check_table_reads = both(PLL_ST_TABLE);
    I.check_cost_pos = both(PLL_ST_COST_POS);
    I.check_cost_neg = both(PLL_ST_COST_NEG);
    I.check_push_edges = both(PLL_ST_FUSED_EDGES);
    for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
        I.phase_ms[ph] = P.ms[ph];
        I.phase_launches[ph] = P.launches[ph];
    }
    *used_arena = 0;
    for (int d = 0; d < 2; ++d) *used_arena += A[d].region_base + PLL_SHARDS * A[d].region_cap;
    return PLL_OK;
}

}  // namespace

namespace {

int build_index(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint8_t* d_w,
                bool weighted, const uint32_t* d_order, const pll_build_opts* opts, bool directed, hipStream_t stream,
                pll_index** out) {
    if (!out) return PLL_EINVAL;
    *out = nullptr;
    pll_build_opts o{};
    if (opts) o = *opts;
    for (uint32_t r : o.reserved)
        if (r) return PLL_EINVAL;
    const uint32_t b = o.batch_size ? o.batch_size : PLL_BMAX;
    if (b > PLL_BMAX || n >= PLL_MAX_N) return PLL_EINVAL;
    if ((o.flags & PLL_FLAG_RELAXED) && !(o.flags & PLL_FLAG_RECHECK)) return PLL_EINVAL;
    if (o.flags & ~(PLL_FLAG_VALIDATE | PLL_FLAG_RECHECK | PLL_FLAG_RELAXED | PLL_FLAG_PROFILE | PLL_FLAG_PERSISTENT |
                    PLL_FLAG_PACK4))
        return PLL_EINVAL;
    if ((directed || weighted) && (o.flags & (PLL_FLAG_RELAXED | PLL_FLAG_PERSISTENT))) return PLL_EINVAL;
    if (o.bp_roots > 64 || (o.bp_roots && (directed || weighted || (o.flags & PLL_FLAG_PERSISTENT))))
        return PLL_EINVAL;
    const uint32_t ql = o.query_lanes;
    if (!(ql == 0 || ql == 1 || ql == 4 || ql == 8 || ql == 16 || ql == 32 || ql == 64)) return PLL_EINVAL;
    if (n > 0 && (!d_row_ptr || !d_order || (nnz && !d_col))) return PLL_EINVAL;
    if (weighted && (directed || (nnz && !d_w))) return PLL_EINVAL;
    if (nnz > 0xFFFFFFFFull * 2) return PLL_EINVAL;

    auto t0 = std::chrono::steady_clock::now();
    pll_index* idx = new (std::nothrow) pll_index{};
    if (!idx) return PLL_ENOMEM;
    if (hipGetDevice(&idx->device) != hipSuccess) {
        delete idx;
        return PLL_EDEVICE;
    }
    idx->query_lanes = ql;
    int rc = PLL_OK;
    if (n == 0) {
        DevAllocs M;
        M.s = stream;
        idx->d_off = M.get_out<uint64_t>(1);
        idx->d_ent = M.get_out<uint32_t>(4);
        idx->d_lb = M.get_out<uint2>(1);
        idx->d_order = M.get_out<uint32_t>(1);
        if (directed) {
            idx->directed = true;
            idx->info.directed = 1;
            idx->d_off_out = M.get_out<uint64_t>(1);
            idx->d_ent_out = M.get_out<uint32_t>(4);
            idx->d_lb_out = M.get_out<uint2>(1);
        }
        if (M.err != hipSuccess) {
            rc = status_of(M.err);
        } else if (hipMemsetAsync(idx->d_off, 0, sizeof(uint64_t), stream) != hipSuccess ||
                   (directed && hipMemsetAsync(idx->d_off_out, 0, sizeof(uint64_t), stream) != hipSuccess) ||
                   hipStreamSynchronize(stream) != hipSuccess) {
            rc = PLL_EDEVICE;
        } else {
            M.forget(idx->d_off);
            M.forget(idx->d_ent);
            M.forget(idx->d_lb);
            M.forget(idx->d_order);
            M.forget(idx->d_off_out);
            M.forget(idx->d_ent_out);
            M.forget(idx->d_lb_out);
            idx->info.weighted = weighted ? 1u : 0u;
            idx->info.batch_size = b;
            idx->info.label_bytes = sizeof(uint64_t);
            idx->info.build_attempts = 1;
        }
    } else {
        const bool fixed = o.arena_entries != 0;
        uint64_t cap = fixed ? o.arena_entries : std::max<uint64_t>(1ull << 20, 4 * nnz + 16ull * n);
        for (uint32_t attempt = 1;; ++attempt) {
            uint64_t used = 0;
            if (directed)
                rc = build_attempt_directed(n, nnz, d_row_ptr, d_col, d_order, b, o.flags, cap, fixed, stream, idx,
                                            &used);
            else if (weighted)
                rc = build_attempt_weighted(n, nnz, d_row_ptr, d_col, d_w, d_order, b, o.flags, cap, fixed, stream,
                                            idx, &used);
            else
                rc = build_attempt(n, nnz, d_row_ptr, d_col, d_order, b, o.flags, cap, fixed, o.max_workgroups,
                                   o.bp_roots, stream, idx, &used);
            idx->info.build_attempts = attempt;
            idx->info.arena_entries = used;
            if (rc == PLL_ENOSPC && !fixed && attempt < 8) {
                cap *= 4;
                continue;
            }
            break;
        }
    }
    if (rc != PLL_OK) {
        delete idx;
        return rc;
    }
    idx->info.build_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = idx;
    return PLL_OK;
}

}  // namespace

int pll_build_one(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                  const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out) {
    return build_index(n, nnz, d_row_ptr, d_col, nullptr, false, d_order, opts, false, stream, out);
}

int pll_build_directed(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                       const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out) {
    return build_index(n, nnz, d_row_ptr, d_col, nullptr, false, d_order, opts, true, stream, out);
}

int pll_build_weighted(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint8_t* d_w,
                       const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out) {
    return build_index(n, nnz, d_row_ptr, d_col, d_w, true, d_order, opts, false, stream, out);
}

// ---- allocation-free build (pll_build_labels_noalloc) --------------------------------------------

namespace {

constexpr size_t kScratchBytes = 64ull << 20;
constexpr size_t kScratchSlack = 64u << 10;  // alignment padding and small blocks beyond the estimate
constexpr int kMaxDevices = 64;

// Every working buffer of the allocation-free builds, carved in order by a
// fixed-region DevAllocs.  Each device holds its own copy from the time this
// code object is loaded on it until the process ends.  Host code must use the
// address hipGetSymbolAddress gives for the current device, never this name.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu[kMaxDevices];       // one allocation-free build at a time per device
void* g_scratch_ptr[kMaxDevices];           // device address of `scratch`, set once per device under its mutex
DevCounters g_scratch_host[kMaxDevices];    // host copy of the build's counters

size_t blk(size_t bytes) { return (std::max<size_t>(bytes, 256) + 255) & ~size_t(255); }

// Bytes build_attempt carves before its label arena and final CSR for a
// graph of n vertices and nnz CSR entries at W words per candidate
// bit-vector, with neither bit-parallel roots nor the persistent loop (the
// blocks of prepare_rank_csr, init_state, the second message buffer and
// receiver list of the fused rounds, and the pulled rounds' items).
size_t noalloc_state_bytes(uint32_t n, uint64_t nnz, uint32_t W) {
    const size_t N = n, E = nnz ? nnz : 1;
    size_t b = blk(sizeof(DevCounters));
    b += blk(4 * N) + blk(4 * (N + 1)) + blk(8 * ((N + 1) / kScanTile + 2)) + blk(8 * (N + 1)) + blk(4 * E);
    b += 2 * blk(8 * (N + 1)) + 2 * blk(4 * N) + 2 * blk(8 * N * W) + blk(64 * W * N) + blk(8 * N);
    const size_t hq_seg = 2 * (nnz / pll::kHeavyItem) + 64;
    b += 2 * (blk(4 * N) + blk(8 * N * W) + blk(8 * PLL_SHARDS * hq_seg));
    b += 3 * blk(4 * PLL_SHARDS * N) + 2 * blk(4 * N);
    b += blk(8 * N * W) + blk(4 * PLL_SHARDS * N);
    if (n >= kPullMinN) b += blk(8 * (N + nnz / pll::kPullSeg + 1)) + blk(4) + blk(8 * N);
    return b;
}

}  // namespace

int pll_export_launch(uint64_t total, const uint32_t* ent, const uint32_t* order, uint32_t* hubs, uint8_t* dists,
                      hipStream_t s);

extern "C" int pll_build_labels_noalloc(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                                        const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream,
                                        uint64_t* d_offsets, uint32_t* d_hubs, uint8_t* d_dists, uint64_t capacity,
                                        uint64_t* total) {
    if (!total) return PLL_EINVAL;
    *total = 0;
    pll_build_opts o{};
    if (opts) o = *opts;
    for (uint32_t r : o.reserved)
        if (r) return PLL_EINVAL;
    const uint32_t b = o.batch_size ? o.batch_size : PLL_BMAX;
    if (b > PLL_BMAX || n >= PLL_MAX_N || nnz > 0xFFFFFFFFull * 2) return PLL_EINVAL;
    if (o.flags & ~(PLL_FLAG_VALIDATE | PLL_FLAG_RECHECK | PLL_FLAG_RELAXED)) return PLL_EINVAL;
    if ((o.flags & PLL_FLAG_RELAXED) && !(o.flags & PLL_FLAG_RECHECK)) return PLL_EINVAL;
    if (o.bp_roots || o.arena_entries) return PLL_EINVAL;
    if (!d_offsets || (n > 0 && (!d_row_ptr || !d_order || (nnz && !d_col))) || (capacity && (!d_hubs || !d_dists)))
        return PLL_EINVAL;
    const uint32_t W = (b + 63) / 64;
    // the label arena takes half of what the working state leaves, the final
    // entries (as many at most) the other half
    const size_t state = noalloc_state_bytes(n, nnz, W);
    const size_t fin = 2 * blk(8 * ((size_t)n + 1)) + blk(4 * (size_t)n) + blk(8 * (size_t)n);
    if (state + fin + kScratchSlack >= kScratchBytes) return PLL_ESCRATCH;
    const uint64_t arena = (kScratchBytes - state - fin - kScratchSlack) / 8;
    if (arena < 32ull * n + 4096) return PLL_ESCRATCH;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PLL_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PLL_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    if (n == 0) {
        if (hipMemsetAsync(d_offsets, 0, sizeof(uint64_t), stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return PLL_EDEVICE;
        return PLL_OK;
    }
    FixedWs fw;
    fw.base = g_scratch_ptr[dev];
    fw.bytes = kScratchBytes;
    fw.host_ctr = &g_scratch_host[dev];
    pll_index idx{};  // host record of this build; its device arrays lie in the scratch
    idx.device = dev;
    uint64_t used = 0;
    int rc = build_attempt(n, nnz, d_row_ptr, d_col, d_order, b, o.flags, arena, true, 0, 0, stream, &idx, &used,
                           &fw);
    // with a fixed region, running out of arena or of scratch both mean the
    // graph's labels do not fit
    if (rc == PLL_ENOSPC || rc == PLL_ENOMEM) return PLL_ESCRATCH;
    if (rc) return rc;
    *total = idx.total;
    if (idx.total > capacity) return PLL_ENOSPC;
    if (hipMemcpyAsync(d_offsets, idx.d_off, sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
        return PLL_EDEVICE;
    rc = pll_export_launch(idx.total, idx.d_ent, idx.d_order, d_hubs, d_dists, stream);
    if (rc) return rc;
    // the next call may reuse the scratch as soon as this one returns
    return hipStreamSynchronize(stream) == hipSuccess ? PLL_OK : PLL_EDEVICE;
}
