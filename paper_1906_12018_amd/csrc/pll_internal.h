// Internal declarations shared by the HIP sources of libpll (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "pll.h"

#define PLL_WAVE 64
#define PLL_BMAX 1024                 // largest batch size b
#define PLL_WMAX (PLL_BMAX / 64)      // 64-bit words in a b-bit candidate bit-vector
#define PLL_INF8 255u                 // "no entry" in the per-batch distance table
#define PLL_MAX_N (1u << 24)          // hub ranks are packed in 24 bits

// Label entry: (hub rank << 8) | dist, so entries sort by hub rank.
__host__ __device__ inline uint32_t pll_pack(uint32_t hub_rank, uint32_t d) { return (hub_rank << 8) | d; }

// Device error bits (DevCounters::error).
#define PLL_ERR_ARENA 0x1u
#define PLL_ERR_DIST 0x2u
#define PLL_ERR_BOUNDS 0x4u
#define PLL_ERR_CSR 0x8u
#define PLL_ERR_ORDER 0x10u
#define PLL_ERR_TIMEOUT 0x20u  // a persistent launch waited too long at a barrier
#define PLL_ERR_STOP 0x40u     // not an error: a persistent launch hands back to the host

// Device-scope atomics on one address serialise (about 12 ns each on
// MI355X), so every counter that many waves update is split into
// PLL_SHARDS copies, one per 128-byte line; a workgroup uses shard
// blockIdx.x % PLL_SHARDS.  Queues are split the same way: shard s owns its
// own segment of each queue array.
#define PLL_SHARDS 32

enum {
    PLL_ST_CAND = 0,     // distance checks (candidates surviving the C(v) filter)
    PLL_ST_ACC = 1,      // entries accepted by round checks
    PLL_ST_EDGES = 2,    // CSR entries read by push
    PLL_ST_READ = 3,     // label entries read by pruning scans
    PLL_ST_TABLE = 4,    // 16-byte table quarters read by pruning scans
    PLL_ST_GROW = 5,     // label lists moved to a larger block
    PLL_ST_RECHECK = 6,  // entries dropped by the recheck
    PLL_ST_COST_POS = 7, // sum of |L(v)| over checks that added an entry
    PLL_ST_COST_NEG = 8, // sum of |L(v)| over checks that pruned
    PLL_ST_BP = 9,       // candidates pruned by the bit-parallel bound
    PLL_ST_FUSED_EDGES = 10,  // CSR entries pushed inside the fused check-and-push launches
    PLL_NUM_ST = 12
};

struct alignas(128) Shard {
    uint32_t recv[3];     // receivers appended to this shard's segment, by round (parity; the
                          // fused check-and-push rounds rotate over three)
    uint32_t hq[2];       // heavy push items, by active-list parity
    uint32_t touched;     // vertices first touched in the batch
    unsigned long long arena_top;  // bump pointer of this shard's arena region (entries, region-relative)
    unsigned long long stat[PLL_NUM_ST];
};
static_assert(sizeof(Shard) == 128, "one shard per 128-byte line");

// Device-side control block of one build; zeroed at the start.
struct DevCounters {
    uint32_t error;  // PLL_ERR_* bits
    uint32_t max_dist;
    uint32_t max_label;
    uint32_t edge_end;  // 1 + the highest rank with an edge (0: the graph has no edges)
    uint32_t pad[28];
    Shard sh[PLL_SHARDS];
};

// Everything the batch kernels of one build touch.  Vertex ids inside the
// build are ranks (rank space), so batch i is the rank range [ib, ib + bs).
struct BuildArgs {
    uint32_t n;
    uint32_t W;        // words per candidate bit-vector (ceil(b / 64))
    uint32_t bstride;  // bytes per distance-table row (64 * W)
    uint32_t hot;      // rows h < hot keep every row-mask bit set for the whole build
    uint32_t nbr_hubs; // 1: round-2 checks read v's higher-ranked neighbours instead of L(v) (undirected,
                       // unweighted builds without bit-parallel roots; see prune_scan_nbrs)
    const uint64_t* rrow;   // rank-space CSR row pointers [n+1]
    const uint32_t* rcol;   // rank-space CSR columns [nnz]
    const uint8_t* rw;      // weighted graphs: weight of each rank-space CSR entry (null otherwise)
    // growing labels: list of rank r is arena[loff[r] .. loff[r] + llen[r])
    uint64_t* loff;
    uint32_t* llen;
    uint32_t* lcap;
    uint32_t* arena;
    uint64_t region_base;  // PLL_SHARDS bump regions follow the compacted lists
    uint64_t region_cap;   // entries per region
    // per-vertex bit-vectors (W words each)
    uint64_t* C;     // candidate bit-vector C(v) of the batch (Section 4.1)
    uint64_t* msgs;  // candidates received this round, already filtered by C (the fused
                     // check-and-push rounds alternate two buffers and filter in the check)
    // per-batch distance table: T[h * bstride + k] = d(u_k, h) for (h, d) in L(u_k)
    uint8_t* T;
    // bit q set when row h of T has an entry for a batch vertex u_k with k / 16 = q; the
    // check skips row segments whose bits are clear.  The top-ranked rows h < hot hold
    // entries for nearly every batch vertex, so their masks stay all ones instead of
    // taking one contended atomic per label entry (a set bit only costs a segment load)
    uint64_t* rowmask;
    // table the pruning checks read: T itself for an undirected graph; for a
    // directed one, the other side's table (a forward check of candidate u_k
    // at v scans L_in(v) against the table of L_out(u_k), and vice versa)
    const uint8_t* Tchk;
    const uint64_t* rmchk;
    // weighted graphs: D[v * bstride + k] = the smallest candidate distance
    // of u_k that reached v in this batch (255: none); it plays the part of
    // C(v), since a candidate may come back shorter in a later round
    uint8_t* D;
    // frontier queues (shard s owns [s * seg, (s + 1) * seg) of each)
    uint32_t* act_v[2];      // active list by parity (compact)
    uint64_t* act_delta[2];  // W words per active slot: delta L of that vertex
    uint2* act_rng[2];       // weighted graphs: (first, count) of the label entries the slot's vertex accepted
    uint64_t* act_at;        // pulled rounds: (round stamp << 32) | active slot of a vertex that accepted
    // bit-parallel labels (rank space; bp_t = 0: none): bp_used[r] marks the
    // BP roots and their neighbour sets; per (rank r, BP root i) at r * bp_t + i:
    // bp_dist = d_i(r), bp_sets = (S^-1, S^0)
    uint32_t bp_t;
    const uint8_t* bp_used;
    const uint8_t* bp_dist;
    const ulonglong2* bp_sets;
    // the same data of the current batch's vertices, transposed so that
    // lanes over batch vertices read consecutive addresses: root i, batch
    // vertex k at i * bstride + k
    uint8_t* bpb_dist;
    ulonglong2* bpb_sets;
    uint2* hq[2];            // (active slot, chunk) items for rows longer than the heavy threshold
    uint64_t hq_seg;
    uint32_t* recv;          // receivers of the current round, segment per shard (seg = n)
    uint32_t* recv_stamp;
    uint32_t* touched;       // first touches of the batch, segment per shard (seg = n)
    uint32_t* tstart;        // label length of touched[i] when first touched in the batch
    uint32_t* touch_stamp;
    DevCounters* ctr;
};

// ---- wavefront helpers (wave64) ----------------------------------------------------------------

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint64_t lanemask_lt() {
    const uint32_t l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }

__device__ inline uint32_t readlane32(uint32_t x, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}

__device__ inline uint64_t readlane64(uint64_t x, uint32_t l) {
    uint32_t lo = readlane32((uint32_t)x, l);
    uint32_t hi = readlane32((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_or64(uint64_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}

__device__ inline uint32_t wave_sum32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline unsigned long long wave_sum64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ inline uint32_t wave_min32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = min(x, (uint32_t)__shfl_xor(x, o, 64));
    return x;
}

__device__ inline uint32_t wave_max32(uint32_t x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = max(x, (uint32_t)__shfl_xor(x, o, 64));
    return x;
}

// OR over the 64 lanes by DPP moves (the whole wave must be active); the
// result is wave-uniform.  row_shr:1,2,4,8 leave each 16-lane row's OR in
// its lane 15; row_bcast:15 adds row 0 into row 1 and row 2 into row 3;
// row_bcast:31 adds rows 0-1 into rows 2-3, so lane 63 holds the total.
__device__ inline uint32_t wave_or32_dpp(uint32_t x) {
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); // row_bcast:15, rows 1, 3
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); // row_bcast:31, rows 2, 3
    return readlane32(x, 63);
}

// Exclusive prefix sum over the 64 lanes.
__device__ inline uint32_t wave_excl_scan32(uint32_t x) {
    const uint32_t l = lane_id();
    uint32_t s = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(s, o, 64);
        if (l >= (uint32_t)o) s += y;
    }
    return s - x;
}

// Orders this wave's LDS writes before its later LDS reads.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- host helpers --------------------------------------------------------------------------------

// Result of one persistent batch-loop launch (pll_rounds.hip).
struct BatchRun {
    uint32_t next_ib;  // first batch not run (n when every batch ran)
    uint32_t grid;     // workgroups of the launch
    unsigned long long batches, rounds;
    double ms[PLL_NUM_PHASES];                 // device wall-clock time per phase
    unsigned long long counts[PLL_NUM_PHASES];  // phase instances
};

// Run batches from ib0 on in one persistent launch (stamps continue from
// *bstamp / *rstamp and are updated); stops early after a batch whose arena
// region is half used when `compact` is set.  Synchronous on `s`.
// ev_begin / ev_end (may be null) are recorded on `s` right around the launch.
int pll_run_batches(const BuildArgs& A, uint32_t ib0, uint32_t b, uint32_t flags, uint32_t* bstamp,
                    uint32_t* rstamp, bool compact, uint32_t max_workgroups, hipStream_t s, hipEvent_t ev_begin,
                    hipEvent_t ev_end, BatchRun* out);

// Caching allocators (pll_alloc.hip).  A workspace block goes back with
// pll_ws_free only after the work using it has completed; index outputs are
// plain hipMalloc memory (indexes free them with hipFree).
hipError_t pll_ws_alloc(void** out, size_t bytes);
void pll_ws_free(void* p);
size_t pll_ws_cached(int device);  // bytes held in the cache of a device
hipError_t pll_pinned_alloc(void** out, size_t bytes);
void pll_pinned_free(void* p);

// Persistent launches of this process are serialised by this mutex.
#include <mutex>
std::mutex& pll_persistent_mutex();

int pll_build_one(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                  const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out);
int pll_query_launch(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v,
                     uint32_t* d_out, hipStream_t stream);
// Lanes per pair the next pll_query on idx uses (query_lanes, or the
// automatic choice from the mean label length).
uint32_t pll_query_lanes(const pll_index* idx);

int pll_build_directed(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                       const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out);

int pll_build_weighted(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col, const uint8_t* d_w,
                       const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out);

int pll_build_multi(uint32_t count, const pll_graph_desc* graphs, const pll_build_opts* opts, hipStream_t stream,
                    pll_index** outs);

// Label entries of several indexes built together live in one allocation,
// released when the last of those indexes is freed.
struct pll_shared_store {
    void* ptr;
    std::atomic<int> refs;  // indexes still using it (they may be freed from different threads)
    int device;
};

// Final label store (what pll_index owns).  An undirected index has one
// label per vertex (d_off / d_ent); a directed one keeps L_in there and L_out
// in d_off_out / d_ent_out.
struct pll_index {
    // references held on the index: 1 for the handle the build returned, plus
    // one per server that keeps it resident without owning it; the device
    // memory is released when the last one is dropped (pll_index_free)
    std::atomic<uint32_t> refs{1};
    int device;
    uint32_t n;
    uint64_t total;
    uint64_t* d_off;    // [n+1], by vertex id
    uint32_t* d_ent;    // [total], packed (hub rank << 8) | dist, ascending within each list
    bool directed;
    uint64_t total_out;
    uint64_t* d_off_out;  // directed only: L_out, laid out as d_off / d_ent
    uint32_t* d_ent_out;
    uint32_t* d_order;  // [n], rank -> vertex id
    // list bounds by vertex id: {hub rank of the first entry, hub rank of the
    // last entry} of L(v) ({0xFFFFFFFF, 0} for an empty list); the query tells
    // from them alone when two lists cannot share a hub.  A directed index
    // keeps L_in's in d_lb and L_out's in d_lb_out.  In the many-graph build
    // they lie in the shared block `meta`.
    uint2* d_lb;
    uint2* d_lb_out;
    uint32_t query_lanes;
    pll_shared_store* store;  // non-null when d_ent points into a shared allocation
    pll_shared_store* meta;   // non-null when d_off and d_order point into a shared allocation
    // bit-parallel labels (info.bp_roots roots; null when none), by vertex id
    uint32_t* d_bp_roots;      // [t] vertex ids
    uint32_t* d_bp_nbrs;       // [t * 64] vertex ids, PLL_DIST_INF padding
    uint8_t* d_bp_dist;        // [n * t]
    ulonglong2* d_bp_sets;     // [n * t] (S^-1, S^0)
    pll_index_info info;
};

// Take one more reference on an index (dropped again by pll_index_free).
inline void pll_index_retain(pll_index* idx) { idx->refs.fetch_add(1, std::memory_order_relaxed); }
