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
//                  (Algorithm 4, lines 6-10); collect the receivers
//     k_check      gather: cand(v) = msgs(v); C(v) |= cand(v); a candidate
//                  u_k survives iff no (h, d) in L(v) with d < j has
//                  T[h][k] + d <= j (lines 13-17); append survivors with
//                  distance j, write T for batch vertices (line 19), build the
//                  next active list (line 18)
//   k_batch_end    clear C(v) over the touched vertices (line 22, Section 5.2
//                  bitmap + queue), optional recheck (Section 5.1), sort each
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
#include <vector>

#include "pll_internal.h"

namespace {

constexpr int kBlock = 256;              // 4 waves
constexpr int kWavesPerBlock = kBlock / PLL_WAVE;
constexpr uint32_t kMaxBlocks = 4096;

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
// self-loop, and every edge present in both directions.  Runs only after the
// row pointers and column ids passed the bounds checks.
__global__ void __launch_bounds__(kBlock) k_check_csr(uint32_t n, const uint64_t* row_ptr, const uint32_t* col,
                                                      DevCounters* ctr) {
    const uint32_t lane = lane_id();
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint64_t beg = row_ptr[v], end = row_ptr[v + 1];
        bool bad = false;
        for (uint64_t e = beg + lane; e < end; e += 64) {
            uint32_t c = col[e];
            if (c == v) bad = true;
            if (e > beg && col[e - 1] >= c) bad = true;
            uint64_t lo = row_ptr[c], hi = row_ptr[c + 1];
            while (lo < hi) {
                uint64_t mid = (lo + hi) >> 1;
                if (col[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo >= row_ptr[c + 1] || col[lo] != v) bad = true;
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

// ---- batch kernels ---------------------------------------------------------------------------------

// Rows longer than this are pushed as several work items of kHeavy edges,
// spread over all waves of the push kernel.
constexpr uint32_t kHeavy = 1024;

// Per byte of x: 1 if byte <= t, where tt = t * 0x01010101 (t <= 254).  Bytes
// are compared without carries between them: s holds, in bit 7 of each
// byte, [low 7 bits of t >= low 7 bits of x]; the high bits decide the rest.
__device__ inline uint32_t le4(uint32_t x, uint32_t tt) {
    const uint32_t H = 0x80808080u;
    const uint32_t s = (tt | H) - (x & ~H);
    const uint32_t r = ((tt & ~x) | (~(tt ^ x) & s)) & H;
    return ((r >> 7) * 0x01020408u) >> 24;  // gather bits 7, 15, 23, 31 into bits 0..3
}

// Bit i of the result: T row byte p[i] <= t, for 64 consecutive bytes.
__device__ inline uint64_t le_mask64(const uint8_t* p, uint32_t tt) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 v = q[i];
        const uint32_t b = le4(v.x, tt) | (le4(v.y, tt) << 4) | (le4(v.z, tt) << 8) | (le4(v.w, tt) << 12);
        m |= (uint64_t)b << (16 * i);
    }
    return m;
}

// OR over the 64 lanes (DPP wave reduction); the result is wave-uniform.
__device__ inline uint64_t wave_or64_u(uint64_t x) {
    const unsigned lo = __reduce_or_sync(~0ull, (unsigned)x);
    const unsigned hi = __reduce_or_sync(~0ull, (unsigned)(x >> 32));
    return ((uint64_t)__builtin_amdgcn_readfirstlane(hi) << 32) | (uint32_t)__builtin_amdgcn_readfirstlane(lo);
}

// Scan the label list arena[off .. off+len) of one vertex v.  Lane w (< W)
// holds candidate word cw = bits k of batch vertices u_{64w+k} that arrived
// at distance j.  Returns, in lane w, the candidates of word w for which some
// entry (h, d) of the list with d < j has T[h][k] + d <= j, i.e. the distance
// j is already covered through a hub ranked above u_k (Algorithm 4, line 14).
// With `relaxed`, entries whose hub is in the current batch are skipped.
// The table loads of all candidate words of a chunk are independent; lanes
// are OR-reduced every 4 chunks (and at the end), which is also where the
// scan stops once every candidate is pruned.
template <int WM>
__device__ inline uint64_t prune_scan(const BuildArgs& A, uint64_t off, uint32_t len, uint32_t j, uint64_t cw,
                                      bool relaxed, uint32_t ib, unsigned long long& n_read,
                                      unsigned long long& n_table) {
    const uint32_t lane = lane_id();
    uint64_t pw = 0;
    uint64_t accm[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) accm[w] = 0;
    uint32_t chunk = 0;
    for (uint32_t base = 0; base < len; base += 64, ++chunk) {
        const uint32_t idx = base + lane;
        bool ok = idx < len;
        n_read += ok;
        const uint32_t ent = ok ? A.arena[off + idx] : 0u;
        const uint32_t h = ent >> 8, d = ent & 255u;
        ok = ok && d < j;
        if (relaxed) ok = ok && h < ib;
        const uint32_t rm = ok ? A.rowmask[h] : 0u;
        const uint32_t tt = ok ? (j - d) * 0x01010101u : 0u;
        const uint8_t* row = A.T + (size_t)h * A.bstride;
        const uint64_t live_lane = cw & ~pw;
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            const uint64_t live = readlane64(live_lane, w);
            if (live != 0 && ((rm >> w) & 1u)) {
                accm[w] |= le_mask64(row + 64u * w, tt) & live;
                ++n_table;
            }
        }
        if ((chunk & 3u) == 3u || base + 64 >= len) {
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                if (readlane64(live_lane, w)) {
                    const uint64_t red = wave_or64_u(accm[w]);
                    if (lane == (uint32_t)w) pw |= red;
                    accm[w] = 0;
                }
            }
            if (!ballot64((cw & ~pw) != 0)) break;
        }
    }
    return pw;
}

__device__ inline uint32_t my_shard() { return blockIdx.x % PLL_SHARDS; }

// Per-lane statistics summed over the workgroup, then one atomic per value
// into the workgroup's shard.  Every thread of the block must call this.
template <int N>
__device__ inline void block_add_stats(DevCounters* ctr, const unsigned long long (&v)[N], const int (&which)[N]) {
    static_assert(N <= 4, "at most 4 statistics per call");
    __shared__ unsigned long long s_part[kWavesPerBlock][4];
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

// Sharded queue enumeration: lane s (< PLL_SHARDS) holds the count of shard
// s; `pre` receives its exclusive prefix and the return value the total.
__device__ inline uint32_t shard_prefix(uint32_t cnt_lane, uint32_t& pre) {
    pre = wave_excl_scan32(cnt_lane);
    return readlane32(pre + cnt_lane, 63);
}

// Shard holding global queue position i (wave-uniform i < total).
__device__ inline uint32_t shard_of(uint32_t pre_lane, uint32_t i) {
    const uint64_t m = ballot64(lane_id() < PLL_SHARDS && pre_lane <= i);
    return 63u - (uint32_t)__builtin_clzll(m);
}

// Room for `need` more entries in the list of rank v (capacity doubling).
// New blocks come from the bump region of the workgroup's shard, or of the
// next shard with room.  Wave-uniform; returns the list's offset, or ~0
// when every region is exhausted.
__device__ inline uint64_t wave_reserve(const BuildArgs& A, uint32_t v, uint64_t off, uint32_t len, uint32_t need) {
    const uint32_t cap = A.lcap[v];
    if (len + need <= cap) return off;
    uint32_t newcap = max(cap * 2u, (len + need + 15u) & ~15u);
    newcap = max(newcap, 16u);
    unsigned long long nb = ~0ull;
    if (lane_id() == 0) {
        const uint32_t s0 = my_shard();
        for (uint32_t t = 0; t < PLL_SHARDS; ++t) {
            const uint32_t sh = (s0 + t) % PLL_SHARDS;
            unsigned long long* top = &A.ctr->sh[sh].arena_top;
            if (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + newcap > A.region_cap) continue;
            const unsigned long long at = atomicAdd(top, (unsigned long long)newcap);
            if (at + newcap <= A.region_cap) {
                nb = A.region_base + (unsigned long long)sh * A.region_cap + at;
                break;
            }
        }
        atomicAdd(&A.ctr->sh[s0].stat[PLL_ST_GROW], 1ull);
    }
    nb = readlane64(nb, 0);
    if (nb == ~0ull) {
        if (lane_id() == 0) atomicOr(&A.ctr->error, PLL_ERR_ARENA);
        return ~0ull;
    }
    for (uint32_t k = lane_id(); k < len; k += 64) A.arena[nb + k] = A.arena[off + k];
    if (lane_id() == 0) {
        A.loff[v] = nb;
        A.lcap[v] = newcap;
    }
    return nb;
}

// Queue the row of active slot `slot` (list q) as kHeavy-edge items when
// it is longer than kHeavy.
__device__ inline void enqueue_heavy(const BuildArgs& A, uint32_t q, uint32_t slot, uint64_t deg) {
    if (deg <= kHeavy) return;
    const uint32_t nch = (uint32_t)((deg + kHeavy - 1) / kHeavy);
    const uint32_t sh = my_shard();
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&A.ctr->sh[sh].hq[q], nch);
    base = readlane32(base, 0);
    for (uint32_t c = lane_id(); c < nch; c += 64) A.hq[q][sh * A.hq_seg + base + c] = make_uint2(slot, c);
}

// Wave-aggregated append of the lanes with `take` to the workgroup's shard
// of a queue; returns each taking lane's position in the queue array.
__device__ inline uint32_t shard_append(uint32_t* counter, bool take, uint64_t seg_base) {
    const uint64_t bal = ballot64(take);
    if (!bal) return 0;
    const uint32_t lane = lane_id();
    const uint32_t leader = (uint32_t)__builtin_ctzll(bal);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__builtin_popcountll(bal));
    base = readlane32(base, leader);
    return (uint32_t)(seg_base + base + __builtin_popcountll(bal & lanemask_lt()));
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
        sh.recv[0] = 0;
        sh.hq[0] = 0;
        sh.touched = 0;
    }
}

// Algorithm 4, line 4: delta L(u) = {(u,0)}, L(u) gets (u,0), L(u) -> H(u).
// The initial active list holds batch vertex u_k in slot k.
__global__ void __launch_bounds__(kBlock) k_batch_init(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t bstamp) {
    const uint32_t lane = lane_id();
    const uint32_t sh = my_shard();
    for (uint32_t k = global_wave(); k < bs; k += num_waves()) {
        const uint32_t u = ib + k;
        const uint32_t len = A.llen[u];
        const uint32_t tpos = shard_append(&A.ctr->sh[sh].touched, lane == 0, (uint64_t)sh * A.n);
        if (lane == 0) {
            A.touch_stamp[u] = bstamp;
            A.touched[tpos] = u;
            A.tstart[tpos] = len;
        }
        uint64_t off = wave_reserve(A, u, A.loff[u], len, 1);
        if (off == ~0ull) continue;
        const uint32_t kw = 1u << (k >> 6);
        if (lane == 0) {
            A.arena[off + len] = pll_pack(u, 0);
            A.llen[u] = len + 1;
            A.T[(size_t)u * A.bstride + k] = 0;
            atomicOr(&A.rowmask[u], kw);
        }
        for (uint32_t i = lane; i < len; i += 64) {
            const uint32_t e = A.arena[off + i];
            const uint32_t h = e >> 8;
            A.T[(size_t)h * A.bstride + k] = (uint8_t)(e & 255u);
            atomicOr(&A.rowmask[h], kw);
        }
        if (lane == 0) A.act_v[0][k] = u;
        if (lane < A.W) A.act_delta[0][(size_t)k * A.W + lane] = (lane == (k >> 6)) ? (1ull << (k & 63)) : 0ull;
        enqueue_heavy(A, 0, k, A.rrow[u + 1] - A.rrow[u]);
    }
}

__device__ inline uint64_t rank_mask(uint32_t rel, uint32_t w) {
    const uint32_t lo = w * 64u;
    if (rel >= lo + 64u) return ~0ull;
    if (rel <= lo) return 0ull;
    return (1ull << (rel - lo)) - 1ull;
}

// Push delta L(a) (lane w < W holds word w in dl; nz marks the nonzero
// words) along the CSR entries [beg, end) of the active vertex a.
__device__ inline void push_edges(const BuildArgs& A, uint32_t ib, uint32_t p, uint32_t rstamp, uint32_t bstamp,
                                  uint64_t dl, uint64_t nz, uint64_t beg, uint64_t end) {
    const uint32_t lane = lane_id();
    const uint32_t sh = my_shard();
    for (uint64_t e0 = beg; e0 < end; e0 += 64) {
        const uint64_t e = e0 + lane;
        const uint32_t r = e < end ? A.rcol[e] : 0u;
        bool any = false;
        if (e < end && r > ib) {
            const uint32_t rel = r - ib;
            uint64_t todo = nz;
            while (todo) {
                const uint32_t w = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1;
                uint64_t m = readlane64(dl, w) & rank_mask(rel, w);
                if (m) {
                    m &= ~A.C[(size_t)r * A.W + w];
                    if (m) {
                        atomicOr((unsigned long long*)&A.msgs[(size_t)r * A.W + w], (unsigned long long)m);
                        any = true;
                    }
                }
            }
        }
        // one receiver slot per vertex and round; the lane that wins the
        // slot also records the vertex's first touch in this batch
        bool enq = false;
        if (any && A.recv_stamp[r] != rstamp) enq = atomicExch(&A.recv_stamp[r], rstamp) != rstamp;
        bool first = false;
        if (enq && A.touch_stamp[r] != bstamp) {
            A.touch_stamp[r] = bstamp;
            first = true;
        }
        if (ballot64(enq)) {
            const uint32_t rp = shard_append(&A.ctr->sh[sh].recv[p], enq, (uint64_t)sh * A.n);
            if (enq) A.recv[rp] = r;
            const uint32_t tp = shard_append(&A.ctr->sh[sh].touched, first, (uint64_t)sh * A.n);
            if (first) {
                A.touched[tp] = r;
                A.tstart[tp] = A.llen[r];
            }
        }
    }
}

// Scatter phase (Algorithm 4, lines 6-10) over active list p (nact slots).
// Batch vertex u_k may be sent to v only when u_k outranks v (rank ib + k
// < v) and C(v) does not hold it yet.  Slots whose delta is empty are
// skipped; rows longer than kHeavy were queued as items and are spread over
// every wave after the per-slot pass.
__global__ void __launch_bounds__(kBlock) k_push(BuildArgs A, uint32_t ib, uint32_t p, uint32_t nact, uint32_t rstamp,
                                                 uint32_t bstamp) {
    const uint32_t lane = lane_id();
    if (blockIdx.x == 0 && threadIdx.x < PLL_SHARDS) A.ctr->sh[threadIdx.x].hq[p ^ 1u] = 0;
    const uint32_t* act_v = A.act_v[p];
    const uint64_t* act_d = A.act_delta[p];
    unsigned long long edges = 0;
    for (uint32_t i = global_wave(); i < nact; i += num_waves()) {
        const uint64_t dl = lane < A.W ? act_d[(size_t)i * A.W + lane] : 0ull;
        const uint64_t nz = ballot64(dl != 0);
        if (!nz) continue;
        const uint32_t a = act_v[i];
        const uint64_t beg = A.rrow[a], end = A.rrow[a + 1];
        if (end - beg > kHeavy) continue;
        if (lane == 0) edges += end - beg;
        push_edges(A, ib, p, rstamp, bstamp, dl, nz, beg, end);
    }
    uint32_t pre;
    const uint32_t nh = shard_prefix(lane < PLL_SHARDS ? A.ctr->sh[lane].hq[p] : 0u, pre);
    for (uint32_t t = global_wave(); t < nh; t += num_waves()) {
        const uint32_t s = shard_of(pre, t);
        const uint2 item = A.hq[p][s * A.hq_seg + (t - readlane32(pre, s))];
        const uint64_t dl = lane < A.W ? act_d[(size_t)item.x * A.W + lane] : 0ull;
        const uint64_t nz = ballot64(dl != 0);
        const uint32_t a = act_v[item.x];
        const uint64_t beg = A.rrow[a] + (uint64_t)item.y * kHeavy;
        const uint64_t end = min(A.rrow[a + 1], beg + kHeavy);
        if (lane == 0) edges += end - beg;
        push_edges(A, ib, p, rstamp, bstamp, dl, nz, beg, end);
    }
    const unsigned long long v[1] = {edges};
    const int which[1] = {PLL_ST_EDGES};
    block_add_stats<1>(A.ctr, v, which);
}

// Gather phase (Algorithm 4, lines 11-19) for round j: one wave per
// receiver.  Receiver i (in shard order) becomes slot i of the next active
// list (with an empty delta when nothing was accepted).
template <int WM>
__global__ void __launch_bounds__(kBlock) k_check(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t j, uint32_t p,
                                                  uint32_t relaxed) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t q = p ^ 1u;
    uint32_t pre;
    const uint32_t nrecv = shard_prefix(lane < PLL_SHARDS ? A.ctr->sh[lane].recv[p] : 0u, pre);
    // clear the other parity's receiver counts for the next round's push
    if (blockIdx.x == 0 && threadIdx.x < PLL_SHARDS) A.ctr->sh[threadIdx.x].recv[q] = 0;
    unsigned long long n_cand = 0, n_acc = 0, n_read = 0, n_table = 0;
    for (uint32_t i = global_wave(); i < nrecv; i += num_waves()) {
        const uint32_t s = shard_of(pre, i);
        const uint32_t v = A.recv[(size_t)s * A.n + (i - readlane32(pre, s))];
        uint64_t mine = 0;
        if (lane < W) {
            const size_t at = (size_t)v * W + lane;
            mine = A.msgs[at];
            A.msgs[at] = 0;
            A.C[at] |= mine;
        }
        const uint32_t len = A.llen[v];
        uint64_t off = A.loff[v];
        const uint64_t pw = prune_scan<WM>(A, off, len, j, mine, relaxed != 0, ib, n_read, n_table);
        const uint64_t acc = lane < W ? (mine & ~pw) : 0ull;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(acc);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t total = readlane32(pos + cnt, 63);
        n_cand += __builtin_popcountll(mine);
        if (lane == 0) A.act_v[q][i] = v;
        if (lane < W) A.act_delta[q][(size_t)i * W + lane] = acc;
        if (total == 0) continue;
        if (j >= PLL_INF8) {
            if (lane == 0) atomicOr(&A.ctr->error, PLL_ERR_DIST);
            continue;
        }
        off = wave_reserve(A, v, off, len, total);
        if (off == ~0ull) continue;
        if (lane == 0) n_acc += total;
        const bool in_batch = v - ib < bs;
        const uint64_t lt = lanemask_lt();
        uint64_t todo = ballot64(acc != 0);
        while (todo) {
            const uint32_t w = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t aw = readlane64(acc, w);
            const uint32_t pwos = readlane32(pos, w);
            if ((aw >> lane) & 1ull) {
                const uint32_t k = w * 64u + lane;
                A.arena[off + len + pwos + __builtin_popcountll(aw & lt)] = pll_pack(ib + k, j);
                if (in_batch) {
                    A.T[(size_t)(ib + k) * A.bstride + (v - ib)] = (uint8_t)j;
                    atomicOr(&A.rowmask[ib + k], 1u << ((v - ib) >> 6));
                }
            }
        }
        if (lane == 0) A.llen[v] = len + total;
        enqueue_heavy(A, q, i, A.rrow[v + 1] - A.rrow[v]);
    }
    const unsigned long long v[4] = {n_cand, n_acc, n_read, n_table};
    const int which[4] = {PLL_ST_CAND, PLL_ST_ACC, PLL_ST_READ, PLL_ST_TABLE};
    block_add_stats<4>(A.ctr, v, which);
}

// Batch end, one wave per touched vertex v: clear C(v) (line 22); sort the
// entries this batch appended to L(v) by hub rank; with `recheck`, first
// drop every such entry (u, d) that L(u) and L(v) already cover through
// another hub at distance <= d (Section 5.1's recheck with the batch's
// tables still in memory).
template <int WM>
__global__ void __launch_bounds__(kBlock) k_batch_end(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t recheck) {
    __shared__ uint64_t s_pres[kWavesPerBlock][PLL_WMAX];
    __shared__ uint8_t s_dist[kWavesPerBlock][PLL_BMAX];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    const uint32_t W = A.W;
    uint32_t pre;
    const uint32_t ntouched = shard_prefix(lane < PLL_SHARDS ? A.ctr->sh[lane].touched : 0u, pre);
    unsigned long long removed = 0, n_read = 0, n_table = 0;
    for (uint32_t i = global_wave(); i < ntouched; i += num_waves()) {
        const uint32_t sh = shard_of(pre, i);
        const size_t at = (size_t)sh * A.n + (i - readlane32(pre, sh));
        const uint32_t v = A.touched[at];
        const uint32_t ts = A.tstart[at];
        const uint32_t len = A.llen[v];
        const uint64_t off = A.loff[v];
        if (lane < W) A.C[(size_t)v * W + lane] = 0;
        const uint32_t tail = len - ts;
        if (tail < 2 && !(recheck && tail >= 1)) continue;
        if (lane < W) s_pres[wv][lane] = 0;
        wave_lds_sync();
        for (uint32_t x = ts + lane; x < len; x += 64) {
            const uint32_t e = A.arena[off + x];
            const uint32_t k = (e >> 8) - ib;
            s_dist[wv][k] = (uint8_t)(e & 255u);
            atomicOr((unsigned long long*)&s_pres[wv][k >> 6], 1ull << (k & 63));
        }
        wave_lds_sync();
        if (recheck) {
            const bool in_batch = v - ib < bs;
            uint32_t prev = 0;
            for (;;) {
                uint32_t mn = PLL_INF8;
                for (uint32_t k = lane; k < bs; k += 64) {
                    const uint32_t d = s_dist[wv][k];
                    if (((s_pres[wv][k >> 6] >> (k & 63)) & 1ull) && d > prev) mn = min(mn, d);
                }
                mn = wave_min32(mn);
                if (mn == PLL_INF8) break;
                uint64_t cw = 0;
                if (lane < W) {
                    const uint64_t pw = s_pres[wv][lane];
                    for (uint32_t bit = 0; bit < 64; ++bit) {
                        const uint32_t k = lane * 64u + bit;
                        if (((pw >> bit) & 1ull) && s_dist[wv][k] == mn) cw |= 1ull << bit;
                    }
                }
                const uint64_t pr = prune_scan<WM>(A, off, len, mn, cw, false, ib, n_read, n_table);
                if (lane < W && pr) s_pres[wv][lane] &= ~pr;
                removed += __builtin_popcountll(pr);
                if (in_batch) {
                    uint64_t todo = ballot64(pr != 0);
                    while (todo) {
                        const uint32_t w = (uint32_t)__builtin_ctzll(todo);
                        todo &= todo - 1;
                        if ((readlane64(pr, w) >> lane) & 1ull)
                            A.T[(size_t)(ib + w * 64u + lane) * A.bstride + (v - ib)] = (uint8_t)PLL_INF8;
                    }
                }
                wave_lds_sync();
                prev = mn;
            }
        }
        // emit the batch segment in ascending hub rank
        const uint64_t pw = lane < W ? s_pres[wv][lane] : 0ull;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(pw);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t total = readlane32(pos + cnt, 63);
        uint64_t todo = ballot64(pw != 0);
        while (todo) {
            const uint32_t w = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t aw = readlane64(pw, w);
            const uint32_t base = readlane32(pos, w);
            if ((aw >> lane) & 1ull) {
                const uint32_t k = w * 64u + lane;
                A.arena[off + ts + base + __builtin_popcountll(aw & lanemask_lt())] = pll_pack(ib + k, s_dist[wv][k]);
            }
        }
        if (lane == 0 && total != tail) A.llen[v] = ts + total;
        wave_lds_sync();
    }
    const unsigned long long v3[3] = {removed, n_read, n_table};
    const int which[3] = {PLL_ST_RECHECK, PLL_ST_READ, PLL_ST_TABLE};
    block_add_stats<3>(A.ctr, v3, which);
}

// Reset the distance table rows written during batch i.
__global__ void __launch_bounds__(kBlock) k_clear_table(BuildArgs A, uint32_t ib, uint32_t bs) {
    const uint32_t lane = lane_id();
    for (uint32_t k = global_wave(); k < bs; k += num_waves()) {
        const uint32_t u = ib + k;
        const uint32_t len = A.llen[u];
        const uint64_t off = A.loff[u];
        for (uint32_t i = lane; i < len; i += 64) {
            const uint32_t h = A.arena[off + i] >> 8;
            A.T[(size_t)h * A.bstride + k] = (uint8_t)PLL_INF8;
            A.rowmask[h] = 0;
        }
        if (lane == 0) A.rowmask[u] = 0;
    }
}

// ---- finalize -----------------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_final_lens(uint32_t n, const uint32_t* rank, const uint32_t* llen,
                                                       uint32_t* lens, DevCounters* ctr) {
    __shared__ uint32_t smax[kWavesPerBlock];
    uint32_t ml = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t l = llen[rank[v]];
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
                                                       const uint64_t* off, uint32_t* ent, DevCounters* ctr) {
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

struct DevAllocs {
    std::vector<void*> ptrs;
    hipError_t err = hipSuccess;
    template <class T>
    T* get(size_t count) {
        if (err != hipSuccess) return nullptr;
        void* p = nullptr;
        size_t bytes = count * sizeof(T);
        if (bytes < 256) bytes = 256;
        err = hipMalloc(&p, bytes);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
    void forget(void* p) {
        for (auto& q : ptrs)
            if (q == p) q = nullptr;
    }
    void drop(void* p) {
        for (auto& q : ptrs)
            if (q == p) {
                (void)hipFree(q);
                q = nullptr;
            }
    }
    ~DevAllocs() {
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
    }
};

inline int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? PLL_ENOMEM : PLL_EDEVICE; }

#define TRY_HIP(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return status_of(_e);    \
    } while (0)

struct HostCounters {
    DevCounters* p = nullptr;
    ~HostCounters() {
        if (p) (void)hipHostFree(p);
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
    if (err & (PLL_ERR_BOUNDS | PLL_ERR_CSR | PLL_ERR_ORDER)) return PLL_EINVAL;
    if (err & PLL_ERR_DIST) return PLL_EDIST;
    if (err & PLL_ERR_ARENA) return PLL_ENOSPC;
    return PLL_OK;
}

template <int WM>
void launch_check(uint32_t blocks, hipStream_t s, const BuildArgs& A, uint32_t ib, uint32_t bs, uint32_t j,
                  uint32_t p, uint32_t relaxed) {
    k_check<WM><<<blocks, kBlock, 0, s>>>(A, ib, bs, j, p, relaxed);
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

// One complete build attempt with a given initial arena size.
int build_attempt(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                  uint32_t b, uint32_t flags, uint64_t arena_hint, bool arena_fixed, hipStream_t s,
                  pll_index* idx, uint64_t* used_arena) {
    DevAllocs M;
    HostCounters HC;
    PhaseProfiler P;
    P.on = (flags & PLL_FLAG_PROFILE) != 0;
    P.s = s;
    TRY_HIP(hipHostMalloc((void**)&HC.p, sizeof(DevCounters), hipHostMallocDefault));
    DevCounters* h = HC.p;
    const uint32_t W = (b + 63) / 64;
    const uint32_t bstride = 64 * W;

    DevCounters* ctr = M.get<DevCounters>(1);
    uint32_t* rank = M.get<uint32_t>(n);
    uint32_t* tmp32 = M.get<uint32_t>((size_t)n + 1);
    uint64_t* scan_scratch = M.get<uint64_t>((n + 1) / kScanTile + 2);
    uint64_t* rrow = M.get<uint64_t>((size_t)n + 1);
    uint32_t* rcol = M.get<uint32_t>(nnz ? nnz : 1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(ctr, 0, sizeof(DevCounters), s));
    hipEvent_t e_prep = P.mark();

    // --- input checks (bounds always; full CSR structure on request)
    k_check_rowptr<<<blocks_for_threads((uint64_t)n + 1), kBlock, 0, s>>>(n, nnz, row_ptr, ctr);
    TRY_HIP(hipMemsetAsync(tmp32, 0, sizeof(uint32_t) * n, s));
    k_count_order<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, tmp32, ctr);
    k_check_order_counts<<<blocks_for_threads(n), kBlock, 0, s>>>(n, tmp32, ctr);
    TRY_HIP(hipGetLastError());
    int rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return PLL_EINVAL;
    if (nnz) k_check_cols<<<blocks_for_threads(nnz), kBlock, 0, s>>>(n, nnz, col, ctr);
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return PLL_EINVAL;
    if (flags & PLL_FLAG_VALIDATE) {
        k_check_csr<<<blocks_for_waves(n), kBlock, 0, s>>>(n, row_ptr, col, ctr);
        rc = read_counters(ctr, h, s);
        if (rc) return rc;
        if (h->error) return PLL_EINVAL;
    }

    // --- rank space (a0)
    k_make_rank<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, rank);
    k_rank_degrees<<<blocks_for_threads(n), kBlock, 0, s>>>(n, order, row_ptr, tmp32);
    TRY_HIP(scan_u32_to_u64(tmp32, n, rrow, scan_scratch, s));
    k_relabel_cols<<<blocks_for_waves(n), kBlock, 0, s>>>(n, order, row_ptr, col, rank, rrow, rcol);
    TRY_HIP(hipGetLastError());

    // --- build state
    BuildArgs A{};
    A.n = n;
    A.W = W;
    A.bstride = bstride;
    A.rrow = rrow;
    A.rcol = rcol;
    A.loff = M.get<uint64_t>((size_t)n + 1);
    uint64_t* spare_off = M.get<uint64_t>((size_t)n + 1);
    A.llen = M.get<uint32_t>(n);
    A.lcap = M.get<uint32_t>(n);
    A.C = M.get<uint64_t>((size_t)n * W);
    A.msgs = M.get<uint64_t>((size_t)n * W);
    A.T = M.get<uint8_t>((size_t)n * bstride);
    A.rowmask = M.get<uint32_t>(n);
    A.hq_seg = 2 * (nnz / kHeavy) + 64;
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
    TRY_HIP(hipMemsetAsync(A.T, 0xFF, (size_t)n * bstride, s));
    TRY_HIP(hipMemsetAsync(A.rowmask, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.recv_stamp, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.touch_stamp, 0, sizeof(uint32_t) * n, s));
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

    // --- batches (a1-a7)
    for (uint32_t ib = 0; ib < n; ib += b) {
        const uint32_t bs = std::min(b, n - ib);
        ++bstamp;
        ++batches;
        hipEvent_t e0 = P.mark();
        k_batch_prep<<<1, 64, 0, s>>>(ctr);
        k_batch_init<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs, bstamp);
        P.span(PLL_PHASE_INIT, e0, P.mark(), 2);
        uint32_t p = 0, nact = bs;
        uint64_t heavy_waves = 1024;  // heavy items of the first round are not known on the host
        for (uint32_t j = 1;; ++j) {
            ++rstamp;
            ++rounds;
            hipEvent_t r0 = P.mark();
            k_push<<<blocks_for_waves(nact + heavy_waves), kBlock, 0, s>>>(A, ib, p, nact, rstamp, bstamp);
            hipEvent_t r1 = P.mark();
            // receivers are unknown until the push has run; the grid-stride
            // loop covers any count, the grid only sets how many waves share it
            const uint32_t check_blocks = blocks_for_waves(std::min<uint64_t>(n, 16ull * nact + 2048));
            dispatch_check(check_blocks, s, A, ib, bs, j, p, relaxed);
            hipEvent_t r2 = P.mark();
            P.span(PLL_PHASE_PUSH, r0, r1, 1);
            P.span(PLL_PHASE_CHECK, r1, r2, 1);
            TRY_HIP(hipGetLastError());
            const double push_ms0 = P.ms[PLL_PHASE_PUSH], check_ms0 = P.ms[PLL_PHASE_CHECK];
            rc = read_counters(ctr, h, s);
            if (rc) return rc;
            P.resolve();
            const unsigned long long acc_now = sum_stat(h, PLL_ST_ACC);
            if (trace) {
                unsigned long long cur[PLL_NUM_ST];
                for (int k = 0; k < PLL_NUM_ST; ++k) cur[k] = sum_stat(h, k);
                std::fprintf(stderr,
                             "pll-trace batch=%u round=%u active=%u recv=%u cand=%llu acc=%llu read=%llu table=%llu "
                             "grow=%llu push_us=%.1f check_us=%.1f\n",
                             (unsigned)(ib / b), j, nact, sum_recv(h, p), cur[PLL_ST_CAND] - last[PLL_ST_CAND],
                             cur[PLL_ST_ACC] - last[PLL_ST_ACC], cur[PLL_ST_READ] - last[PLL_ST_READ],
                             cur[PLL_ST_TABLE] - last[PLL_ST_TABLE], cur[PLL_ST_GROW] - last[PLL_ST_GROW],
                             (P.ms[PLL_PHASE_PUSH] - push_ms0) * 1e3, (P.ms[PLL_PHASE_CHECK] - check_ms0) * 1e3);
                for (int k = 0; k < PLL_NUM_ST; ++k) last[k] = cur[k];
            }
            if (h->error) return device_error_status(h->error);
            if (acc_now == accepted_seen) break;  // nobody accepted anything: the batch is done
            accepted_seen = acc_now;
            nact = sum_recv(h, p);
            p ^= 1u;
            heavy_waves = sum_hq(h, p);
        }
        hipEvent_t e1 = P.mark();
        dispatch_batch_end(blocks_for_waves(sum_touched(h)), s, A, ib, bs, recheck);
        k_clear_table<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs);
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
    k_final_lens<<<blocks_for_threads(n), kBlock, 0, s>>>(n, rank, A.llen, tmp32, ctr);
    uint64_t* d_off = M.get<uint64_t>((size_t)n + 1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(scan_u32_to_u64(tmp32, n, d_off, scan_scratch, s));
    uint64_t total = 0;
    TRY_HIP(hipMemcpyAsync(&total, d_off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    uint32_t* d_ent = M.get<uint32_t>(total ? total : 1);
    uint32_t* d_order = M.get<uint32_t>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    k_final_copy<<<std::min<uint32_t>(blocks_for_waves(n), 1024), kBlock, 0, s>>>(n, rank, A.loff, A.llen, A.arena,
                                                                                   d_off, d_ent, ctr);
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
    idx->d_order = d_order;
    M.forget(d_off);
    M.forget(d_ent);
    M.forget(d_order);
    pll_index_info& I = idx->info;
    I.n = n;
    I.batch_size = b;
    I.total_entries = total;
    I.label_bytes = total * sizeof(uint32_t) + ((uint64_t)n + 1) * sizeof(uint64_t);
    I.max_dist = h->max_dist;
    I.max_label = h->max_label;
    I.batches = batches;
    I.rounds = rounds;
    I.candidates = sum_stat(h, PLL_ST_CAND);
    I.accepted = sum_stat(h, PLL_ST_ACC);
    I.edges_scanned = sum_stat(h, PLL_ST_EDGES);
    I.recheck_removed = sum_stat(h, PLL_ST_RECHECK);
    I.check_entries_read = sum_stat(h, PLL_ST_READ);
    I.check_table_reads = sum_stat(h, PLL_ST_TABLE);
    for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
        I.phase_ms[ph] = P.ms[ph];
        I.phase_launches[ph] = P.launches[ph];
    }
    *used_arena = A.region_base + PLL_SHARDS * A.region_cap;
    return PLL_OK;
}

}  // namespace

int pll_build_one(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                  const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out) {
    if (!out) return PLL_EINVAL;
    *out = nullptr;
    pll_build_opts o{};
    if (opts) o = *opts;
    for (uint32_t r : o.reserved)
        if (r) return PLL_EINVAL;
    const uint32_t b = o.batch_size ? o.batch_size : PLL_BMAX;
    if (b > PLL_BMAX || n >= PLL_MAX_N) return PLL_EINVAL;
    if ((o.flags & PLL_FLAG_RELAXED) && !(o.flags & PLL_FLAG_RECHECK)) return PLL_EINVAL;
    if (o.flags & ~(PLL_FLAG_VALIDATE | PLL_FLAG_RECHECK | PLL_FLAG_RELAXED | PLL_FLAG_PROFILE)) return PLL_EINVAL;
    const uint32_t ql = o.query_lanes;
    if (!(ql == 0 || ql == 1 || ql == 4 || ql == 8 || ql == 16 || ql == 32 || ql == 64)) return PLL_EINVAL;
    if (n > 0 && (!d_row_ptr || !d_order || (nnz && !d_col))) return PLL_EINVAL;
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
        idx->d_off = M.get<uint64_t>(1);
        idx->d_ent = M.get<uint32_t>(1);
        idx->d_order = M.get<uint32_t>(1);
        if (M.err != hipSuccess) {
            rc = status_of(M.err);
        } else if (hipMemsetAsync(idx->d_off, 0, sizeof(uint64_t), stream) != hipSuccess ||
                   hipStreamSynchronize(stream) != hipSuccess) {
            rc = PLL_EDEVICE;
        } else {
            M.forget(idx->d_off);
            M.forget(idx->d_ent);
            M.forget(idx->d_order);
            idx->info.batch_size = b;
            idx->info.label_bytes = sizeof(uint64_t);
            idx->info.build_attempts = 1;
        }
    } else {
        const bool fixed = o.arena_entries != 0;
        uint64_t cap = fixed ? o.arena_entries : std::max<uint64_t>(1ull << 20, 4 * nnz + 16ull * n);
        for (uint32_t attempt = 1;; ++attempt) {
            uint64_t used = 0;
            rc = build_attempt(n, nnz, d_row_ptr, d_col, d_order, b, o.flags, cap, fixed, stream, idx, &used);
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
