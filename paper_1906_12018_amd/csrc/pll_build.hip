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

// Scan the label list arena[off .. off+len) of one vertex v.  Lane w (< W)
// holds candidate word cw = bits k of batch vertices u_k to test at
// distance j.  Returns, in lane w, the bits of cw for which some entry
// (h, d) of the list with d < j has T[h][k] + d <= j, i.e. the distance j is
// already covered through a hub ranked above u_k (Algorithm 4, line 14).
// With `relaxed`, entries whose hub is in the current batch are skipped.
__device__ inline uint64_t prune_scan(const BuildArgs& A, uint64_t off, uint32_t len, uint32_t j, uint64_t cw,
                                      uint64_t nz, bool relaxed, uint32_t ib, unsigned long long& n_read,
                                      unsigned long long& n_table) {
    const uint32_t lane = lane_id();
    uint64_t pruned = 0;
    for (uint32_t base = 0; base < len; base += 64) {
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
        uint64_t todo = nz;
        while (todo) {
            const uint32_t w = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t live = readlane64(cw & ~pruned, w);
            if (!live) continue;
            uint64_t m = 0;
            if ((rm >> w) & 1u) {
                m = le_mask64(row + 64u * w, tt) & live;
                ++n_table;
            }
            m = wave_or64(m);
            if (lane == w) pruned |= m;
        }
        if (!ballot64(lane < A.W && (cw & ~pruned) != 0)) break;
    }
    return pruned;
}

// Room for `need` more entries in the list of rank v (capacity doubling from
// the arena's bump pointer).  Wave-uniform; returns the list's offset, or
// ~0 when the arena is exhausted.
__device__ inline uint64_t wave_reserve(const BuildArgs& A, uint32_t v, uint64_t off, uint32_t len, uint32_t need) {
    const uint32_t cap = A.lcap[v];
    if (len + need <= cap) return off;
    uint32_t newcap = max(cap * 2u, (len + need + 15u) & ~15u);
    newcap = max(newcap, 16u);
    unsigned long long nb = 0;
    if (lane_id() == 0) nb = atomicAdd(&A.ctr->arena_top, (unsigned long long)newcap);
    nb = readlane64(nb, 0);
    if (nb + newcap > A.arena_cap) {
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

__global__ void k_batch_prep(DevCounters* ctr, uint32_t bs) {
    if (threadIdx.x == 0) {
        ctr->touched_count = bs;
        ctr->act_count[0] = bs;
        ctr->act_count[1] = 0;
    }
}

__global__ void k_round_prep(DevCounters* ctr, uint32_t p) {
    if (threadIdx.x == 0) {
        ctr->recv_count = 0;
        ctr->act_count[p ^ 1u] = 0;
    }
}

// Algorithm 4, line 4: delta L(u) = {(u,0)}, L(u) gets (u,0), L(u) -> H(u).
__global__ void __launch_bounds__(kBlock) k_batch_init(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t bstamp) {
    const uint32_t lane = lane_id();
    for (uint32_t k = global_wave(); k < bs; k += num_waves()) {
        const uint32_t u = ib + k;
        const uint32_t len = A.llen[u];
        if (lane == 0) {
            A.touch_stamp[u] = bstamp;
            A.touched[k] = u;
            A.tstart[k] = len;
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
        A.act_v[0][k] = u;
        if (lane < A.W) A.act_delta[0][(size_t)k * A.W + lane] = (lane == (k >> 6)) ? (1ull << (k & 63)) : 0ull;
    }
}

__device__ inline uint64_t rank_mask(uint32_t rel, uint32_t w) {
    const uint32_t lo = w * 64u;
    if (rel >= lo + 64u) return ~0ull;
    if (rel <= lo) return 0ull;
    return (1ull << (rel - lo)) - 1ull;
}

// Scatter phase (Algorithm 4, lines 6-10).  One wave per active vertex a,
// lanes over its CSR row.  Batch vertex u_k may be sent to v only when
// u_k outranks v (rank ib + k < v) and C(v) does not hold it yet.
__global__ void __launch_bounds__(kBlock) k_push(BuildArgs A, uint32_t ib, uint32_t p, uint32_t rstamp) {
    const uint32_t lane = lane_id();
    const uint32_t nact = A.ctr->act_count[p];
    const uint32_t* act_v = A.act_v[p];
    const uint64_t* act_d = A.act_delta[p];
    unsigned long long edges = 0;
    for (uint32_t i = global_wave(); i < nact; i += num_waves()) {
        const uint32_t a = act_v[i];
        const uint64_t dl = lane < A.W ? act_d[(size_t)i * A.W + lane] : 0ull;
        const uint64_t nz = ballot64(dl != 0);
        const uint64_t beg = A.rrow[a], end = A.rrow[a + 1];
        edges += end - beg;
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
            bool enq = false;
            if (any && A.recv_stamp[r] != rstamp) enq = atomicExch(&A.recv_stamp[r], rstamp) != rstamp;
            const uint64_t bal = ballot64(enq);
            if (bal) {
                const uint32_t leader = (uint32_t)__builtin_ctzll(bal);
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(&A.ctr->recv_count, (uint32_t)__builtin_popcountll(bal));
                base = readlane32(base, leader);
                if (enq) A.recv[base + __builtin_popcountll(bal & lanemask_lt())] = r;
            }
        }
    }
    if (lane == 0 && edges) atomicAdd(&A.ctr->edges, edges);
}

// Gather phase (Algorithm 4, lines 11-19) for round j: one wave per receiver.
__global__ void __launch_bounds__(kBlock) k_check(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t j, uint32_t p,
                                                  uint32_t bstamp, uint32_t relaxed) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t nrecv = A.ctr->recv_count;
    const uint32_t q = p ^ 1u;
    unsigned long long n_cand = 0, n_acc = 0, n_read = 0, n_table = 0;
    for (uint32_t i = global_wave(); i < nrecv; i += num_waves()) {
        const uint32_t v = A.recv[i];
        uint64_t cw = 0;
        if (lane < W) {
            const size_t at = (size_t)v * W + lane;
            cw = A.msgs[at];
            A.msgs[at] = 0;
            A.C[at] |= cw;
        }
        const uint64_t nz = ballot64(cw != 0);
        uint32_t len = A.llen[v];
        uint64_t off = A.loff[v];
        if (lane == 0 && A.touch_stamp[v] != bstamp) {
            A.touch_stamp[v] = bstamp;
            const uint32_t s = atomicAdd(&A.ctr->touched_count, 1u);
            A.touched[s] = v;
            A.tstart[s] = len;
        }
        n_cand += __builtin_popcountll(cw);
        const uint64_t pruned = prune_scan(A, off, len, j, cw, nz, relaxed != 0, ib, n_read, n_table);
        const uint64_t acc = lane < W ? (cw & ~pruned) : 0ull;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(acc);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t total = readlane32(pos + cnt, 63);
        if (total == 0) continue;
        if (j >= PLL_INF8) {
            if (lane == 0) atomicOr(&A.ctr->error, PLL_ERR_DIST);
            continue;
        }
        off = wave_reserve(A, v, off, len, total);
        if (off == ~0ull) continue;
        n_acc += total;
        const bool in_batch = v - ib < bs;
        uint64_t todo = ballot64(acc != 0);
        while (todo) {
            const uint32_t w = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint64_t aw = readlane64(acc, w);
            const uint32_t pw = readlane32(pos, w);
            if ((aw >> lane) & 1ull) {
                const uint32_t k = w * 64u + lane;
                A.arena[off + len + pw + __builtin_popcountll(aw & lanemask_lt())] = pll_pack(ib + k, j);
                if (in_batch) {
                    A.T[(size_t)(ib + k) * A.bstride + (v - ib)] = (uint8_t)j;
                    atomicOr(&A.rowmask[ib + k], 1u << ((v - ib) >> 6));
                }
            }
        }
        uint32_t slot = 0;
        if (lane == 0) {
            A.llen[v] = len + total;
            slot = atomicAdd(&A.ctr->act_count[q], 1u);
            A.act_v[q][slot] = v;
        }
        slot = readlane32(slot, 0);
        if (lane < W) A.act_delta[q][(size_t)slot * W + lane] = acc;
    }
    n_cand = wave_sum64(n_cand);  // lane w counted the candidates of word w
    n_read = wave_sum64(n_read);
    n_table = wave_sum64(n_table);
    if (lane == 0) {
        if (n_cand) atomicAdd(&A.ctr->candidates, n_cand);
        if (n_acc) atomicAdd(&A.ctr->accepted, n_acc);
        if (n_read) atomicAdd(&A.ctr->check_entries, n_read);
        if (n_table) atomicAdd(&A.ctr->check_table_reads, n_table);
    }
}

// Batch end, one wave per touched vertex v: clear C(v) (line 22); sort the
// entries this batch appended to L(v) by hub rank; with `recheck`, first
// drop every such entry (u, d) that L(u) and L(v) already cover through
// another hub at distance <= d (Section 5.1's recheck with the batch's
// tables still in memory).
__global__ void __launch_bounds__(kBlock) k_batch_end(BuildArgs A, uint32_t ib, uint32_t bs, uint32_t recheck) {
    __shared__ uint64_t s_pres[kWavesPerBlock][PLL_WMAX];
    __shared__ uint8_t s_dist[kWavesPerBlock][PLL_BMAX];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    const uint32_t W = A.W;
    const uint32_t ntouched = A.ctr->touched_count;
    unsigned long long removed = 0, n_read = 0, n_table = 0;
    for (uint32_t i = global_wave(); i < ntouched; i += num_waves()) {
        const uint32_t v = A.touched[i];
        const uint32_t ts = A.tstart[i];
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
                const uint64_t nz = ballot64(cw != 0);
                const uint64_t pr = prune_scan(A, off, len, mn, cw, nz, false, ib, n_read, n_table);
                if (lane < W && pr) {
                    s_pres[wv][lane] &= ~pr;
                    removed += __builtin_popcountll(pr);
                }
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
    removed = wave_sum64(removed);  // lane w counted the removals of word w
    if (lane == 0 && removed) atomicAdd(&A.ctr->recheck_removed, removed);
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

__global__ void k_final_lens(uint32_t n, const uint32_t* rank, const uint32_t* llen, uint32_t* lens) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) lens[v] = llen[rank[v]];
}

__global__ void __launch_bounds__(kBlock) k_final_copy(uint32_t n, const uint32_t* rank, const uint64_t* loff,
                                                       const uint32_t* llen, const uint32_t* arena,
                                                       const uint64_t* off, uint32_t* ent, DevCounters* ctr) {
    const uint32_t lane = lane_id();
    uint32_t md = 0, ml = 0;
    for (uint32_t v = global_wave(); v < n; v += num_waves()) {
        const uint32_t r = rank[v];
        const uint64_t src = loff[r], dst = off[v];
        const uint32_t len = llen[r];
        ml = max(ml, len);
        for (uint32_t i = lane; i < len; i += 64) {
            const uint32_t e = arena[src + i];
            ent[dst + i] = e;
            md = max(md, e & 255u);
        }
    }
    md = wave_max32(md);
    if (lane == 0) {
        atomicMax(&ctr->max_dist, md);
        atomicMax(&ctr->max_label, ml);
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

// One complete build attempt with a given arena capacity.
int build_attempt(uint32_t n, uint64_t nnz, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                  uint32_t b, uint32_t flags, uint64_t arena_cap, bool arena_fixed, hipStream_t s,
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
    P.span(PLL_PHASE_PREP, e_prep, P.mark(), (flags & PLL_FLAG_VALIDATE) ? 10 : 9);

    // --- build state
    BuildArgs A{};
    A.n = n;
    A.W = W;
    A.bstride = bstride;
    A.rrow = rrow;
    A.rcol = rcol;
    A.loff = M.get<uint64_t>(n);
    A.llen = M.get<uint32_t>(n);
    A.lcap = M.get<uint32_t>(n);
    A.arena = M.get<uint32_t>(arena_cap);
    A.arena_cap = arena_cap;
    A.C = M.get<uint64_t>((size_t)n * W);
    A.msgs = M.get<uint64_t>((size_t)n * W);
    A.T = M.get<uint8_t>((size_t)n * bstride);
    A.rowmask = M.get<uint32_t>(n);
    for (int q = 0; q < 2; ++q) {
        A.act_v[q] = M.get<uint32_t>(n);
        A.act_delta[q] = M.get<uint64_t>((size_t)n * W);
    }
    A.recv = M.get<uint32_t>(n);
    A.recv_stamp = M.get<uint32_t>(n);
    A.touched = M.get<uint32_t>(n);
    A.tstart = M.get<uint32_t>(n);
    A.touch_stamp = M.get<uint32_t>(n);
    A.ctr = ctr;
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(hipMemsetAsync(A.loff, 0, sizeof(uint64_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.llen, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.lcap, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.C, 0, sizeof(uint64_t) * n * W, s));
    TRY_HIP(hipMemsetAsync(A.msgs, 0, sizeof(uint64_t) * n * W, s));
    TRY_HIP(hipMemsetAsync(A.T, 0xFF, (size_t)n * bstride, s));
    TRY_HIP(hipMemsetAsync(A.rowmask, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.recv_stamp, 0, sizeof(uint32_t) * n, s));
    TRY_HIP(hipMemsetAsync(A.touch_stamp, 0, sizeof(uint32_t) * n, s));

    const bool recheck = (flags & PLL_FLAG_RECHECK) != 0;
    const uint32_t relaxed = (flags & PLL_FLAG_RELAXED) ? 1u : 0u;
    uint32_t rstamp = 0, bstamp = 0;
    uint64_t rounds = 0, batches = 0;
    const uint32_t check_blocks = blocks_for_waves(n);

    // --- batches (a1-a7)
    for (uint32_t ib = 0; ib < n; ib += b) {
        const uint32_t bs = std::min(b, n - ib);
        ++bstamp;
        ++batches;
        hipEvent_t e0 = P.mark();
        k_batch_prep<<<1, 64, 0, s>>>(ctr, bs);
        k_batch_init<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs, bstamp);
        P.span(PLL_PHASE_INIT, e0, P.mark(), 2);
        uint32_t p = 0, nact = bs;
        for (uint32_t j = 1;; ++j) {
            ++rstamp;
            ++rounds;
            hipEvent_t r0 = P.mark();
            k_round_prep<<<1, 64, 0, s>>>(ctr, p);
            k_push<<<blocks_for_waves(nact), kBlock, 0, s>>>(A, ib, p, rstamp);
            hipEvent_t r1 = P.mark();
            k_check<<<check_blocks, kBlock, 0, s>>>(A, ib, bs, j, p, bstamp, relaxed);
            hipEvent_t r2 = P.mark();
            P.span(PLL_PHASE_PUSH, r0, r1, 2);
            P.span(PLL_PHASE_CHECK, r1, r2, 1);
            TRY_HIP(hipGetLastError());
            rc = read_counters(ctr, h, s);
            if (rc) return rc;
            P.resolve();
            if (h->error) return device_error_status(h->error);
            nact = h->act_count[p ^ 1u];
            if (nact == 0) break;
            p ^= 1u;
        }
        hipEvent_t e1 = P.mark();
        k_batch_end<<<blocks_for_waves(h->touched_count), kBlock, 0, s>>>(A, ib, bs, recheck ? 1u : 0u);
        k_clear_table<<<blocks_for_waves(bs), kBlock, 0, s>>>(A, ib, bs);
        P.span(PLL_PHASE_END, e1, P.mark(), 2);
        TRY_HIP(hipGetLastError());
        // grow the arena between batches when it is more than half used
        if (!arena_fixed && h->arena_top * 2 > A.arena_cap) {
            const uint64_t ncap = A.arena_cap * 2;
            uint32_t* na = M.get<uint32_t>(ncap);
            if (na) {
                TRY_HIP(hipMemcpyAsync(na, A.arena, sizeof(uint32_t) * h->arena_top, hipMemcpyDeviceToDevice, s));
                TRY_HIP(hipStreamSynchronize(s));
                M.drop(A.arena);
                A.arena = na;
                A.arena_cap = ncap;
            } else {
                M.err = hipSuccess;
                (void)hipGetLastError();
            }
        }
    }

    // --- finalize (a8): CSR by vertex id, hubs as ranks
    rc = read_counters(ctr, h, s);
    if (rc) return rc;
    if (h->error) return device_error_status(h->error);
    P.resolve();
    hipEvent_t e_fin = P.mark();
    k_final_lens<<<blocks_for_threads(n), kBlock, 0, s>>>(n, rank, A.llen, tmp32);
    uint64_t* d_off = M.get<uint64_t>((size_t)n + 1);
    if (M.err != hipSuccess) return status_of(M.err);
    TRY_HIP(scan_u32_to_u64(tmp32, n, d_off, scan_scratch, s));
    uint64_t total = 0;
    TRY_HIP(hipMemcpyAsync(&total, d_off + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    uint32_t* d_ent = M.get<uint32_t>(total ? total : 1);
    uint32_t* d_order = M.get<uint32_t>(n);
    if (M.err != hipSuccess) return status_of(M.err);
    k_final_copy<<<blocks_for_waves(n), kBlock, 0, s>>>(n, rank, A.loff, A.llen, A.arena, d_off, d_ent, ctr);
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
    I.candidates = h->candidates;
    I.accepted = h->accepted;
    I.edges_scanned = h->edges;
    I.recheck_removed = h->recheck_removed;
    I.check_entries_read = h->check_entries;
    I.check_table_reads = h->check_table_reads;
    for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
        I.phase_ms[ph] = P.ms[ph];
        I.phase_launches[ph] = P.launches[ph];
    }
    *used_arena = A.arena_cap;
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
        uint64_t cap = fixed ? o.arena_entries : std::max<uint64_t>(1ull << 20, 4 * nnz + 48ull * n);
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
