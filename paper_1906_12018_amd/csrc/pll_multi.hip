// Many independent graphs in one persistent-kernel launch (captured in a
// hipGraph).  Every graph is built by a gang of G workgroups (G = 1 for
// small graphs, more for large ones, in proportion to the graph's share of
// the estimated work).  Workgroups take (graph, member) slots from one list
// ordered by decreasing graph size, so a gang's members join in order and a
// gang always completes: the kernel is launched with no more workgroups than
// can be resident and no gang is larger than that.  Inside a gang the phases
// of pll_phases.h run over all G x 16 waves, with queue counters in per-graph
// global shards (one per member) and a gang barrier between phases; a gang of
// one only uses __syncthreads.  Member 0 also checks the input, relabels to
// rank space and lays out the final offsets; every member copies labels into
// one output buffer shared by all graphs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "pll_internal.h"
#include "pll_phases.h"

namespace {

using pll::Exec;
using pll::PhaseStats;

constexpr int kMultiBlock = 1024;  // 16 waves per workgroup
constexpr int kMultiWaves = kMultiBlock / PLL_WAVE;
constexpr uint32_t kMaxGang = 16;

// Per-graph gang control block (zero-filled before the launch).
struct alignas(128) GangCtl {
    uint32_t bar_count, bar_gen;
    uint32_t err[2];        // sticky error words, one per barrier parity
    uint32_t round_acc[2];  // entries accepted in the current round, by round parity
    uint32_t pad0[2];
    unsigned long long out_base;
    uint32_t pad1[22];
    Shard shards[kMaxGang];
};
static_assert(sizeof(GangCtl) == 128 * (kMaxGang + 1), "layout");

struct GraphJob {
    BuildArgs A;  // the graph's working buffers, filled in by the host
    uint64_t nnz;
    const uint64_t* row_ptr;
    const uint32_t* col;
    const uint32_t* order;
    uint32_t* rank;
    uint64_t* out_off;  // [n+1] label offsets by vertex id, relative to the graph's output base
    uint2* out_lb;      // [n] list bounds by vertex id (first and last hub rank; see pll_index)
    GangCtl* gc;
    uint32_t gang;      // workgroups building this graph
};

struct GraphResult {
    unsigned long long out_base, total;
    uint32_t error, max_dist, max_label, pad;
    unsigned long long batches, rounds, cand, acc, edges, read, table, removed, cost_pos, cost_neg;
};

struct MultiCtl {
    uint32_t next_slot;
    uint32_t spin_limit;
    uint32_t pad[30];
    unsigned long long out_top;
    unsigned long long out_cap;
};

// Exclusive prefix sums of in[0..n) into out[0..n] by one workgroup.
__device__ void wg_scan(const uint32_t* in, uint32_t n, uint64_t* out, uint64_t* s_wsum, uint64_t* s_carry) {
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    if (threadIdx.x == 0) *s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t x = i < n ? in[i] : 0u;
        uint64_t s = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(s, o, 64);
            if (lane >= (uint32_t)o) s += y;
        }
        if (lane == 63) s_wsum[wv] = s;
        __syncthreads();
        uint64_t pre = *s_carry, tot = 0;
        for (uint32_t w = 0; w < nwv; ++w) {
            if (w < wv) pre += s_wsum[w];
            tot += s_wsum[w];
        }
        if (i < n) out[i] = pre + s - x;
        __syncthreads();
        if (threadIdx.x == 0) *s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = *s_carry;
    __syncthreads();
}

__device__ inline uint32_t load_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier k of a gang.  Memory effects of every member before it are
// visible to every member after it.  Returns the gang's error word, the
// same in every member: errors seen before barrier k are published into
// err[k & 1] before arriving and read back after the barrier completes (a
// member cannot reach barrier k+2, which writes the same word again, before
// all members have left barrier k+1).  A member that waits longer than the
// spin limit records a timeout and gives up on the graph.
__device__ uint32_t gang_sync(GangCtl* gc, uint32_t G, uint32_t& k, DevCounters* ctr, uint32_t spin_limit,
                              uint32_t* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e = load_agent(&ctr->error);
        if (G > 1) {
            const uint32_t par = k & 1u;
            if (e) atomicOr(&gc->err[par], e);
            __threadfence();
            const uint32_t gen = load_agent(&gc->bar_gen);
            if (atomicAdd(&gc->bar_count, 1u) == G - 1) {
                __hip_atomic_store(&gc->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __threadfence();
                atomicAdd(&gc->bar_gen, 1u);
            } else {
                uint32_t spins = 0;
                while (load_agent(&gc->bar_gen) == gen) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > spin_limit) {
                        atomicOr(&gc->err[0], PLL_ERR_TIMEOUT);
                        atomicOr(&gc->err[1], PLL_ERR_TIMEOUT);
                        atomicOr(&ctr->error, PLL_ERR_TIMEOUT);
                        break;
                    }
                }
            }
            __threadfence();
            e = load_agent(&gc->err[par]);
        }
        *s_flag = e;
    }
    __syncthreads();
    ++k;
    return *s_flag;
}

template <int WM>
__global__ void __launch_bounds__(kMultiBlock) k_multi_build(const GraphJob* __restrict__ jobs,
                                                             const uint2* __restrict__ slots, uint32_t nslots,
                                                             GraphResult* results, MultiCtl* ctl, DevCounters* ctr,
                                                             uint32_t* out, uint32_t b, uint32_t flags) {
    __shared__ uint64_t s_pres[kMultiWaves][PLL_WMAX];
    __shared__ uint8_t s_dist[kMultiWaves][PLL_BMAX];
    __shared__ uint64_t s_wsum[kMultiWaves];
    __shared__ uint64_t s_carry;
    __shared__ uint32_t s_slot, s_err, s_flag;
    __shared__ unsigned long long s_tot[8];
    __shared__ uint32_t s_max[2];

    const uint32_t lane = lane_id();
    const uint32_t tid = threadIdx.x;
    const uint32_t wv = tid >> 6;
    const bool recheck = (flags & PLL_FLAG_RECHECK) != 0;
    const bool relaxed = (flags & PLL_FLAG_RELAXED) != 0;
    const uint32_t spin_limit = ctl->spin_limit;

    for (;;) {
        if (tid == 0) s_slot = atomicAdd(&ctl->next_slot, 1u);
        __syncthreads();
        const uint32_t si = s_slot;
        __syncthreads();
        if (si >= nslots) break;
        const uint2 sl = slots[si];
        const uint32_t g = sl.x, r = sl.y;
        const GraphJob& J = jobs[g];
        const BuildArgs& A = J.A;
        GangCtl* gc = J.gc;
        const uint32_t G = J.gang;
        const uint32_t n = A.n;
        const uint64_t nnz = J.nnz;
        uint32_t k = 0;  // gang barriers passed

        Exec X;
        X.w = r * (uint32_t)kMultiWaves + wv;
        X.nw = G * (uint32_t)kMultiWaves;
        X.qs = gc->shards;
        X.nq = G;
        X.my = r;
        X.seg = n;
        X.zero_i = r == 0 ? tid : ~0u;
        X.arena_sh = blockIdx.x % PLL_SHARDS;

        // ---- member 0: input checks and rank space (a0)
        if (r == 0) {
            if (tid == 0) s_err = 0;
            __syncthreads();
            if (n > 0) {
                for (uint32_t v = tid; v <= n; v += blockDim.x) {
                    const uint64_t a = J.row_ptr[v];
                    if ((v == 0 && a != 0) || (v == n && a != nnz) || (v < n && a > J.row_ptr[v + 1]) || a > nnz)
                        atomicOr(&s_err, PLL_ERR_BOUNDS);
                }
                for (uint32_t i = tid; i < n; i += blockDim.x) {
                    const uint32_t o = J.order[i];
                    if (o >= n) atomicOr(&s_err, PLL_ERR_ORDER);
                    else atomicAdd(&A.touch_stamp[o], 1u);  // zero-filled; reused as a count
                }
                __syncthreads();
                for (uint32_t v = tid; v < n; v += blockDim.x) {
                    if (A.touch_stamp[v] != 1u) atomicOr(&s_err, PLL_ERR_ORDER);
                    A.touch_stamp[v] = 0;
                }
                __syncthreads();
                if (!s_err)
                    for (uint64_t e = tid; e < nnz; e += blockDim.x)
                        if (J.col[e] >= n) atomicOr(&s_err, PLL_ERR_BOUNDS);
                __syncthreads();
                if (!s_err && (flags & PLL_FLAG_VALIDATE)) {
                    for (uint32_t v = wv; v < n; v += kMultiWaves) {
                        const uint64_t beg = J.row_ptr[v], end = J.row_ptr[v + 1];
                        bool bad = false;
                        for (uint64_t e = beg + lane; e < end; e += 64) {
                            const uint32_t c = J.col[e];
                            if (c == v || (e > beg && J.col[e - 1] >= c)) bad = true;
                            uint64_t lo = J.row_ptr[c], hi = J.row_ptr[c + 1];
                            while (lo < hi) {
                                const uint64_t mid = (lo + hi) >> 1;
                                if (J.col[mid] < v) lo = mid + 1; else hi = mid;
                            }
                            if (lo >= J.row_ptr[c + 1] || J.col[lo] != v) bad = true;
                        }
                        if (ballot64(bad) && lane == 0) atomicOr(&s_err, PLL_ERR_CSR);
                    }
                }
                __syncthreads();
                if (s_err) {
                    if (tid == 0) {
                        results[g].error = s_err;
                        atomicOr(&ctr->error, s_err);
                    }
                } else {
                    for (uint32_t i = tid; i < n; i += blockDim.x) {
                        const uint32_t v = J.order[i];
                        J.rank[v] = i;
                        A.llen[i] = (uint32_t)(J.row_ptr[v + 1] - J.row_ptr[v]);  // degrees, scanned below
                    }
                    __syncthreads();
                    wg_scan(A.llen, n, const_cast<uint64_t*>(A.rrow), s_wsum, &s_carry);
                    for (uint32_t i = wv; i < n; i += kMultiWaves) {
                        const uint32_t v = J.order[i];
                        const uint64_t src = J.row_ptr[v], dst = A.rrow[i];
                        const uint32_t deg = (uint32_t)(J.row_ptr[v + 1] - src);
                        for (uint32_t x = lane; x < deg; x += 64)
                            const_cast<uint32_t*>(A.rcol)[dst + x] = J.rank[J.col[src + x]];
                    }
                    for (uint32_t i = tid; i < n; i += blockDim.x) A.llen[i] = 0;
                }
            }
        }
        if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) continue;  // bad input here or elsewhere

        // ---- batches (a1-a7)
        PhaseStats st;
        uint32_t rstamp = 0, bstamp = 0;
        unsigned long long batches = 0, rounds = 0;
        bool failed = false;
        for (uint32_t ib = 0; ib < n && !failed; ib += b) {
            const uint32_t bs = min(b, n - ib);
            ++bstamp;
            ++batches;
            if (r == 0) {
                if (tid < G) {
                    Shard& q = gc->shards[tid];
                    q.recv[0] = q.recv[1] = 0;
                    q.hq[0] = q.hq[1] = 0;
                    q.touched = 0;
                }
                if (tid == 0) gc->round_acc[0] = gc->round_acc[1] = 0;
            }
            if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
            pll::phase_batch_init(A, X, ib, bs, bstamp);
            if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
            uint32_t p = 0, nact = bs;
            for (uint32_t j = 1;; ++j) {
                ++rstamp;
                ++rounds;
                pll::phase_push(A, X, ib, p, nact, rstamp, bstamp, st);
                if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
                // the counter of round j+1 was last read after round j-1
                if (r == 0 && tid == 0) gc->round_acc[(j + 1) & 1u] = 0;
                const unsigned long long acc0 = st.acc;
                pll::phase_check<WM, false, false, true>(A, X, ib, bs, j, p, relaxed, st);
                if (lane == 0 && st.acc != acc0) atomicAdd(&gc->round_acc[j & 1u], (uint32_t)(st.acc - acc0));
                if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
                if (load_agent(&gc->round_acc[j & 1u]) == 0) break;
                uint32_t cnt = 0;
                for (uint32_t s = 0; s < G; ++s) cnt += load_agent(&gc->shards[s].recv[p]);
                nact = cnt;
                p ^= 1u;
            }
            if (failed) break;
            pll::phase_batch_end<WM>(A, X, ib, bs, recheck, s_pres[wv], s_dist[wv], nullptr, st);
            if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
            pll::phase_clear_table(A, X, ib, bs);
            if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) { failed = true; break; }
        }
        if (failed) continue;

        // ---- finalize (a8): member 0 lays out offsets by vertex id, everyone copies
        if (r == 0) {
            for (uint32_t v = tid; v < n; v += blockDim.x) A.touch_stamp[v] = A.llen[J.rank[v]];
            __syncthreads();
            wg_scan(A.touch_stamp, n, J.out_off, s_wsum, &s_carry);
            if (tid == 0) {
                const unsigned long long total = J.out_off[n];
                // regions start on 16-byte boundaries and span whole 4-entry
                // chunks: the query kernel reads labels in aligned 16-byte loads
                const unsigned long long base = atomicAdd(&ctl->out_top, (total + 3) & ~3ull);
                gc->out_base = base;
                results[g].out_base = base;
                results[g].total = total;
                results[g].batches = batches;
                results[g].rounds = rounds;
                if (base + ((total + 3) & ~3ull) > ctl->out_cap) atomicOr(&ctr->error, PLL_ERR_ARENA);
            }
        }
        if (gang_sync(gc, G, k, ctr, spin_limit, &s_flag)) continue;
        const unsigned long long base = gc->out_base;
        if (tid == 0) {
            s_max[0] = s_max[1] = 0;
            for (int x = 0; x < 8; ++x) s_tot[x] = 0;
        }
        __syncthreads();
        uint32_t md = 0, ml = 0;
        for (uint32_t v = X.w; v < n; v += X.nw) {
            const uint32_t rv = J.rank[v];
            const uint64_t src = A.loff[rv], dst = base + J.out_off[v];
            const uint32_t len = A.llen[rv];
            ml = max(ml, len);
            for (uint32_t i = lane; i < len; i += 64) {
                const uint32_t e = A.arena[src + i];
                out[dst + i] = e;
                md = max(md, e & 255u);
            }
            if (lane == 0)
                J.out_lb[v] = len ? make_uint2(A.arena[src] >> 8, A.arena[src + len - 1] >> 8)
                                  : make_uint2(0xFFFFFFFFu, 0u);
        }
        md = wave_max32(md);
        const unsigned long long sums[8] = {wave_sum64(st.cand),  wave_sum64(st.acc),     wave_sum64(st.edges),
                                            wave_sum64(st.read),  wave_sum64(st.table),   wave_sum64(st.removed),
                                            wave_sum64(st.cost_pos), wave_sum64(st.cost_neg)};
        if (lane == 0) {
            atomicMax(&s_max[0], md);
            atomicMax(&s_max[1], ml);
            for (int x = 0; x < 8; ++x)
                if (sums[x]) atomicAdd(&s_tot[x], sums[x]);
        }
        __syncthreads();
        if (tid == 0) {
            GraphResult& R = results[g];
            atomicMax(&R.max_dist, s_max[0]);
            atomicMax(&R.max_label, s_max[1]);
            atomicAdd(&R.cand, s_tot[0]);
            atomicAdd(&R.acc, s_tot[1]);
            atomicAdd(&R.edges, s_tot[2]);
            atomicAdd(&R.read, s_tot[3]);
            atomicAdd(&R.table, s_tot[4]);
            atomicAdd(&R.removed, s_tot[5]);
            atomicAdd(&R.cost_pos, s_tot[6]);
            atomicAdd(&R.cost_neg, s_tot[7]);
        }
        __syncthreads();
    }
}

// Fill `words` 32-bit words with `value` (graph-capturable instead of a memset node).
__global__ void k_fill32(uint32_t* p, uint64_t words, uint32_t value) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Workspace block of one launch, returned to the cache once the launch's
// stream has drained.
struct Buf {
    void* p = nullptr;
    hipStream_t* s = nullptr;
    ~Buf() {
        if (!p) return;
        if (s && *s) (void)hipStreamSynchronize(*s);
        pll_ws_free(p);
    }
};

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline int words_class(uint32_t W) { return W <= 1 ? 1 : W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16; }

template <int WM>
hipError_t launch_multi(uint32_t grid, hipStream_t s, const GraphJob* jobs, const uint2* slots, uint32_t nslots,
                        GraphResult* results, MultiCtl* ctl, DevCounters* ctr, uint32_t* out, uint32_t b,
                        uint32_t flags) {
    k_multi_build<WM><<<grid, kMultiBlock, 0, s>>>(jobs, slots, nslots, results, ctl, ctr, out, b, flags);
    return hipGetLastError();
}

template <int WM>
int resident_blocks() {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_multi_build<WM>, kMultiBlock, 0) != hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

int resident_for(uint32_t W) {
    switch (words_class(W)) {
        case 1: return resident_blocks<1>();
        case 2: return resident_blocks<2>();
        case 4: return resident_blocks<4>();
        case 8: return resident_blocks<8>();
        default: return resident_blocks<16>();
    }
}

hipError_t dispatch_multi(uint32_t W, uint32_t grid, hipStream_t s, const GraphJob* jobs, const uint2* slots,
                          uint32_t nslots, GraphResult* results, MultiCtl* ctl, DevCounters* ctr, uint32_t* out,
                          uint32_t b, uint32_t flags) {
    switch (words_class(W)) {
        case 1: return launch_multi<1>(grid, s, jobs, slots, nslots, results, ctl, ctr, out, b, flags);
        case 2: return launch_multi<2>(grid, s, jobs, slots, nslots, results, ctl, ctr, out, b, flags);
        case 4: return launch_multi<4>(grid, s, jobs, slots, nslots, results, ctl, ctr, out, b, flags);
        case 8: return launch_multi<8>(grid, s, jobs, slots, nslots, results, ctl, ctr, out, b, flags);
        default: return launch_multi<16>(grid, s, jobs, slots, nslots, results, ctl, ctr, out, b, flags);
    }
}

double work_estimate(const pll_graph_desc& d) { return (double)d.nnz * std::log2(d.n + 2.0) + d.n; }

// Gang sizes: a graph's share of the estimated work (CSR entries times
// log n, plus n) times the resident workgroups, times gang_scale percent,
// clamped to [1, min(kMaxGang, resident, max_gang)].
std::vector<uint32_t> gang_sizes(uint32_t count, const pll_graph_desc* graphs, uint32_t resident, uint32_t scale_pct,
                                 uint32_t max_gang) {
    std::vector<double> w(count);
    double tot = 0;
    for (uint32_t g = 0; g < count; ++g) tot += (w[g] = work_estimate(graphs[g]));
    const uint32_t cap =
        std::max<uint32_t>(1, std::min<uint32_t>({kMaxGang, resident, max_gang ? max_gang : kMaxGang}));
    std::vector<uint32_t> G(count, 1);
    if (tot <= 0) return G;
    for (uint32_t g = 0; g < count; ++g) {
        const double want = w[g] / tot * resident * (scale_pct / 100.0);
        G[g] = std::max<uint32_t>(1, std::min<uint32_t>(cap, (uint32_t)std::lround(want)));
    }
    return G;
}

int multi_attempt(uint32_t count, const pll_graph_desc* graphs, uint32_t b, uint32_t flags, uint32_t scale_pct,
                  uint32_t max_gang, uint32_t query_lanes, uint32_t max_workgroups, uint64_t arena_total, uint64_t out_cap, hipStream_t caller, pll_index** outs,
                  bool* retry) {
    *retry = false;
    // the work is captured on the caller's stream, or, for the legacy
    // default stream (which cannot be captured), on a private stream ordered
    // after the caller's pending work.  No extra stream otherwise: streams
    // beyond the hardware queues share one, and work behind a long launch waits.
    struct StreamGuard {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        bool own = false;
        ~StreamGuard() {
            if (e) (void)hipEventDestroy(e);
            if (own && s) (void)hipStreamDestroy(s);
        }
    } SG;
    if (caller) {
        SG.s = caller;
    } else {
        SG.own = true;
        if (hipStreamCreateWithFlags(&SG.s, hipStreamNonBlocking) != hipSuccess) return PLL_EDEVICE;
        if (hipEventCreateWithFlags(&SG.e, hipEventDisableTiming) != hipSuccess) return PLL_EDEVICE;
        if (hipEventRecord(SG.e, caller) != hipSuccess || hipStreamWaitEvent(SG.s, SG.e, 0) != hipSuccess)
            return PLL_EDEVICE;
    }
    hipStream_t s = SG.s;

    const uint32_t W = (b + 63) / 64;
    const uint64_t bstride = 64ull * W;
    int resident = resident_for(W);
    if (resident <= 0) return PLL_EDEVICE;
    if (max_workgroups) resident = std::min<int>(resident, (int)max_workgroups);
    const std::vector<uint32_t> G = gang_sizes(count, graphs, (uint32_t)resident, scale_pct, max_gang);

    std::vector<GraphJob> jobs(count);
    uint64_t zb = 0, tb = 0, ob = 0;
    auto take = [](uint64_t& cur, uint64_t bytes) {
        const uint64_t at = cur;
        cur = align_up(cur + bytes, 256);
        return at;
    };
    struct Off {
        uint64_t gc, loff, llen, lcap, C, msgs, rowmask, recv_stamp, touch_stamp, T;
        uint64_t rank, rrow, rcol, act_v0, act_v1, ad0, ad1, hq0, hq1, recv, touched, tstart;
    };
    std::vector<Off> off(count);
    for (uint32_t g = 0; g < count; ++g) {
        const uint64_t n = graphs[g].n, nnz = graphs[g].nnz, gs = G[g];
        const uint64_t hq_seg = 2 * (nnz / pll::kHeavyItem) + 64;
        Off& o = off[g];
        o.gc = take(zb, sizeof(GangCtl));
        o.loff = take(zb, 8 * (n + 1));
        o.llen = take(zb, 4 * n);
        o.lcap = take(zb, 4 * n);
        o.C = take(zb, 8 * n * W);
        o.msgs = take(zb, 8 * n * W);
        o.rowmask = take(zb, 8 * n);
        o.recv_stamp = take(zb, 4 * n);
        o.touch_stamp = take(zb, 4 * (n + 1));
        o.T = take(tb, n * bstride);
        o.rank = take(ob, 4 * n);
        o.rrow = take(ob, 8 * (n + 1));
        o.rcol = take(ob, 4 * std::max<uint64_t>(nnz, 1));
        o.act_v0 = take(ob, 4 * n);
        o.act_v1 = take(ob, 4 * n);
        o.ad0 = take(ob, 8 * n * W);
        o.ad1 = take(ob, 8 * n * W);
        o.hq0 = take(ob, 8 * hq_seg * gs);
        o.hq1 = take(ob, 8 * hq_seg * gs);
        o.recv = take(ob, 4 * n * gs);
        o.touched = take(ob, 4 * n * gs);
        o.tstart = take(ob, 4 * n * gs);
        jobs[g] = GraphJob{};
        jobs[g].A.n = graphs[g].n;
        jobs[g].A.W = W;
        jobs[g].A.bstride = (uint32_t)bstride;
        jobs[g].A.hq_seg = hq_seg;
        jobs[g].nnz = graphs[g].nnz;
        jobs[g].row_ptr = graphs[g].d_row_ptr;
        jobs[g].col = graphs[g].d_col;
        jobs[g].order = graphs[g].d_order;
        jobs[g].gang = G[g];
    }
    // slots: graphs by decreasing estimated work, members of a gang in order
    std::vector<uint32_t> gorder(count);
    std::iota(gorder.begin(), gorder.end(), 0u);
    std::stable_sort(gorder.begin(), gorder.end(),
                     [&](uint32_t a, uint32_t c) { return work_estimate(graphs[a]) > work_estimate(graphs[c]); });
    std::vector<uint2> slots;
    for (uint32_t g : gorder)
        for (uint32_t m = 0; m < G[g]; ++m) slots.push_back(make_uint2(g, m));

    Buf Z, TT, O, JB, SL, RS, CT, DC, AR;
    for (Buf* bf : {&Z, &TT, &O, &JB, &SL, &RS, &CT, &DC, &AR}) bf->s = &SG.s;
    const uint64_t region_cap = std::max<uint64_t>(4096, arena_total / PLL_SHARDS);
    if (pll_ws_alloc(&Z.p, std::max<uint64_t>(zb, 256)) != hipSuccess ||
        pll_ws_alloc(&TT.p, std::max<uint64_t>(tb, 256)) != hipSuccess ||
        pll_ws_alloc(&O.p, std::max<uint64_t>(ob, 256)) != hipSuccess ||
        pll_ws_alloc(&AR.p, sizeof(uint32_t) * region_cap * PLL_SHARDS) != hipSuccess ||
        pll_ws_alloc(&JB.p, sizeof(GraphJob) * count) != hipSuccess ||
        pll_ws_alloc(&SL.p, sizeof(uint2) * slots.size()) != hipSuccess ||
        pll_ws_alloc(&RS.p, sizeof(GraphResult) * count) != hipSuccess ||
        pll_ws_alloc(&CT.p, sizeof(MultiCtl)) != hipSuccess || pll_ws_alloc(&DC.p, sizeof(DevCounters)) != hipSuccess)
        return PLL_ENOMEM;
    // outputs the indexes keep: the label store, and one block holding every
    // graph's offsets and order (both shared, reference-counted)
    struct OutMem {
        void* p = nullptr;
        hipStream_t* s = nullptr;
        ~OutMem() {
            if (!p) return;
            if (s && *s) (void)hipStreamSynchronize(*s);
            (void)hipFree(p);
        }
    } OUT, META;
    OUT.s = META.s = &SG.s;
    if (hipMalloc(&OUT.p, sizeof(uint32_t) * std::max<uint64_t>(out_cap, 64)) != hipSuccess) return PLL_ENOMEM;
    uint64_t meta_bytes = 0;
    for (uint32_t g = 0; g < count; ++g)
        meta_bytes += align_up(8 * ((uint64_t)graphs[g].n + 1), 256) + align_up(4 * std::max<uint64_t>(graphs[g].n, 1), 256) +
                      align_up(8 * std::max<uint64_t>(graphs[g].n, 1), 256);
    if (hipMalloc(&META.p, std::max<uint64_t>(meta_bytes, 256)) != hipSuccess) return PLL_ENOMEM;
    std::vector<uint64_t*> out_offs(count, nullptr);
    std::vector<uint32_t*> orders(count, nullptr);
    std::vector<uint2*> out_lbs(count, nullptr);
    {
        char* mp = (char*)META.p;
        for (uint32_t g = 0; g < count; ++g) {
            out_offs[g] = (uint64_t*)mp;
            mp += align_up(8 * ((uint64_t)graphs[g].n + 1), 256);
            orders[g] = (uint32_t*)mp;
            mp += align_up(4 * std::max<uint64_t>(graphs[g].n, 1), 256);
            out_lbs[g] = (uint2*)mp;
            mp += align_up(8 * std::max<uint64_t>(graphs[g].n, 1), 256);
        }
    }
    char* zp = (char*)Z.p;
    char* tp = (char*)TT.p;
    char* op = (char*)O.p;
    for (uint32_t g = 0; g < count; ++g) {
        const Off& o = off[g];
        GraphJob& J = jobs[g];
        BuildArgs& A = J.A;
        J.gc = (GangCtl*)(zp + o.gc);
        A.loff = (uint64_t*)(zp + o.loff);
        A.llen = (uint32_t*)(zp + o.llen);
        A.lcap = (uint32_t*)(zp + o.lcap);
        A.C = (uint64_t*)(zp + o.C);
        A.msgs = (uint64_t*)(zp + o.msgs);
        A.rowmask = (uint64_t*)(zp + o.rowmask);
        A.recv_stamp = (uint32_t*)(zp + o.recv_stamp);
        A.touch_stamp = (uint32_t*)(zp + o.touch_stamp);
        A.T = (uint8_t*)(tp + o.T);
        A.Tchk = A.T;
        A.rmchk = A.rowmask;
        A.rw = nullptr;  // unweighted, no bit-parallel labels
        A.D = nullptr;
        A.act_rng[0] = A.act_rng[1] = nullptr;
        A.bp_t = 0;
        A.hot = 0;  // small graphs leave rows sparse: every row mask is kept exact
        A.nbr_hubs = 1;  // undirected, unweighted, no bit-parallel roots
        J.rank = (uint32_t*)(op + o.rank);
        A.rrow = (uint64_t*)(op + o.rrow);
        A.rcol = (uint32_t*)(op + o.rcol);
        A.act_v[0] = (uint32_t*)(op + o.act_v0);
        A.act_v[1] = (uint32_t*)(op + o.act_v1);
        A.act_delta[0] = (uint64_t*)(op + o.ad0);
        A.act_delta[1] = (uint64_t*)(op + o.ad1);
        A.hq[0] = (uint2*)(op + o.hq0);
        A.hq[1] = (uint2*)(op + o.hq1);
        A.recv = (uint32_t*)(op + o.recv);
        A.touched = (uint32_t*)(op + o.touched);
        A.tstart = (uint32_t*)(op + o.tstart);
        A.arena = (uint32_t*)AR.p;
        A.region_base = 0;
        A.region_cap = region_cap;
        A.ctr = (DevCounters*)DC.p;
        J.out_off = out_offs[g];
        J.out_lb = out_lbs[g];
    }
    MultiCtl hctl{};
    hctl.out_cap = out_cap;
    hctl.spin_limit = 1u << 22;  // a few seconds at most per barrier
    int rc = PLL_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    do {
        if (hipMemcpyAsync(JB.p, jobs.data(), sizeof(GraphJob) * count, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(SL.p, slots.data(), sizeof(uint2) * slots.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(CT.p, &hctl, sizeof(MultiCtl), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = PLL_EDEVICE;
            break;
        }
        // every workgroup resident at once, so a partially joined gang is
        // always completed by workgroups that finish other graphs
        const uint32_t grid = std::min<uint32_t>((uint32_t)slots.size(), (uint32_t)resident);
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = PLL_EDEVICE;
            break;
        }
        k_fill32<<<2048, 256, 0, s>>>((uint32_t*)Z.p, zb / 4, 0u);
        k_fill32<<<2048, 256, 0, s>>>((uint32_t*)TT.p, tb / 4, 0xFFFFFFFFu);
        k_fill32<<<64, 256, 0, s>>>((uint32_t*)DC.p, sizeof(DevCounters) / 4, 0u);
        k_fill32<<<64, 256, 0, s>>>((uint32_t*)RS.p, sizeof(GraphResult) * count / 4, 0u);
        hipError_t le = dispatch_multi(W, grid, s, (const GraphJob*)JB.p, (const uint2*)SL.p, (uint32_t)slots.size(),
                                       (GraphResult*)RS.p, (MultiCtl*)CT.p, (DevCounters*)DC.p, (uint32_t*)OUT.p, b,
                                       flags);
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (le != hipSuccess || ce != hipSuccess || !graph) {
            rc = PLL_EDEVICE;
            break;
        }
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            rc = PLL_EDEVICE;
            break;
        }
        // persistent launches of this process run one at a time
        std::lock_guard<std::mutex> lock(pll_persistent_mutex());
        if (hipGraphLaunch(exec, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            rc = PLL_EDEVICE;
            break;
        }
    } while (false);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != PLL_OK) return rc;
    DevCounters hc;
    std::vector<GraphResult> res(count);
    if (hipMemcpy(&hc, DC.p, sizeof(DevCounters), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(res.data(), RS.p, sizeof(GraphResult) * count, hipMemcpyDeviceToHost) != hipSuccess)
        return PLL_EDEVICE;
    if (hc.error) {
        if (hc.error & (PLL_ERR_BOUNDS | PLL_ERR_CSR | PLL_ERR_ORDER)) return PLL_EINVAL;
        if (hc.error & PLL_ERR_DIST) return PLL_EDIST;
        if (hc.error & PLL_ERR_TIMEOUT) return PLL_EDEVICE;
        *retry = true;
        return PLL_ENOSPC;
    }
    for (uint32_t g = 0; g < count; ++g)
        if (graphs[g].n &&
            hipMemcpyAsync(orders[g], graphs[g].d_order, 4 * (uint64_t)graphs[g].n, hipMemcpyDeviceToDevice, s) !=
                hipSuccess)
            return PLL_EDEVICE;
    for (uint32_t g = 0; g < count; ++g)
        if (graphs[g].n == 0 && hipMemsetAsync(out_offs[g], 0, sizeof(uint64_t), s) != hipSuccess) return PLL_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return PLL_EDEVICE;
    // hand the shared output buffer to the indexes
    std::vector<pll_index*> made(count, nullptr);
    for (uint32_t g = 0; g < count; ++g) {
        made[g] = new (std::nothrow) pll_index{};
        if (!made[g]) {
            for (auto* p : made) delete p;
            return PLL_ENOMEM;
        }
    }
    pll_shared_store* store = new (std::nothrow) pll_shared_store{};
    pll_shared_store* meta = new (std::nothrow) pll_shared_store{};
    if (!store || !meta) {
        for (auto* p : made) delete p;
        delete store;
        delete meta;
        return PLL_ENOMEM;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    store->ptr = OUT.p;
    store->refs = (int)count;
    store->device = dev;
    OUT.p = nullptr;
    meta->ptr = META.p;
    meta->refs = (int)count;
    meta->device = dev;
    META.p = nullptr;
    for (uint32_t g = 0; g < count; ++g) {
        pll_index* idx = made[g];
        const GraphResult& R = res[g];
        idx->device = dev;
        idx->n = graphs[g].n;
        idx->total = R.total;
        idx->d_off = out_offs[g];
        idx->d_lb = out_lbs[g];
        idx->d_ent = (uint32_t*)store->ptr + R.out_base;
        idx->d_order = orders[g];
        idx->store = store;
        idx->meta = meta;
        idx->query_lanes = query_lanes;
        pll_index_info& I = idx->info;
        I.n = graphs[g].n;
        I.batch_size = b;
        I.total_entries = R.total;
        I.in_entries = R.total;
        I.out_entries = R.total;
        I.label_bytes = R.total * 4 + 8 * ((uint64_t)graphs[g].n + 1) + 8 * (uint64_t)graphs[g].n;
        I.max_dist = R.max_dist;
        I.max_label = R.max_label;
        I.batches = R.batches;
        I.rounds = R.rounds;
        I.candidates = R.cand;
        I.accepted = R.acc;
        I.edges_scanned = R.edges;
        I.recheck_removed = R.removed;
        I.check_entries_read = R.read;
        I.check_table_reads = R.table;
        I.check_cost_pos = R.cost_pos;
        I.check_cost_neg = R.cost_neg;
        I.arena_entries = region_cap * PLL_SHARDS;
        I.build_attempts = 1;
        I.gang = G[g];
        outs[g] = idx;
    }
    return PLL_OK;
}

}  // namespace

int pll_build_multi(uint32_t count, const pll_graph_desc* graphs, const pll_build_opts* opts, hipStream_t stream,
                    pll_index** outs) {
    if (!outs || (count && !graphs)) return PLL_EINVAL;
    for (uint32_t i = 0; i < count; ++i) outs[i] = nullptr;
    if (count == 0) return PLL_OK;
    pll_build_opts o{};
    if (opts) o = *opts;
    if (o.bp_roots) return PLL_EINVAL;  // bit-parallel labels: single-graph builds only
    for (uint32_t r : o.reserved)
        if (r) return PLL_EINVAL;
    const uint32_t b = o.batch_size ? o.batch_size : PLL_BMAX;
    if (b > PLL_BMAX) return PLL_EINVAL;
    if ((o.flags & PLL_FLAG_RELAXED) && !(o.flags & PLL_FLAG_RECHECK)) return PLL_EINVAL;
    if (o.flags & ~(PLL_FLAG_VALIDATE | PLL_FLAG_RECHECK | PLL_FLAG_RELAXED | PLL_FLAG_PROFILE)) return PLL_EINVAL;
    if (o.max_gang > kMaxGang) return PLL_EINVAL;
    const uint32_t ql = o.query_lanes;
    if (!(ql == 0 || ql == 1 || ql == 4 || ql == 8 || ql == 16 || ql == 32 || ql == 64)) return PLL_EINVAL;
    uint64_t sum_est = 0;
    for (uint32_t g = 0; g < count; ++g) {
        const pll_graph_desc& d = graphs[g];
        if (d.n >= PLL_MAX_N || (d.n && (!d.d_row_ptr || !d.d_order)) || (d.nnz && !d.d_col)) return PLL_EINVAL;
        // label-size guess: grows with the CSR and with log n (adjusted by retries)
        uint64_t lg = 1;
        while ((1ull << lg) < d.n) ++lg;
        sum_est += 16ull * d.n + 4ull * d.nnz * lg;
    }
    auto t0 = std::chrono::steady_clock::now();
    uint64_t arena = o.arena_entries ? o.arena_entries : std::max<uint64_t>(1ull << 20, sum_est);
    uint64_t out_cap = std::max<uint64_t>(1ull << 16, arena / 2);
    const uint32_t scale = o.gang_scale ? o.gang_scale : 100;
    int rc = PLL_OK;
    for (uint32_t attempt = 1; attempt <= 6; ++attempt) {
        bool retry = false;
        rc = multi_attempt(count, graphs, b, o.flags, scale, o.max_gang, o.query_lanes, o.max_workgroups, arena, out_cap, stream, outs, &retry);
        if (rc == PLL_OK) {
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            for (uint32_t g = 0; g < count; ++g) {
                outs[g]->info.build_attempts = attempt;
                outs[g]->info.build_ms = ms;
            }
            return PLL_OK;
        }
        if (!retry || o.arena_entries) break;
        arena *= 2;
        out_cap *= 2;
    }
    return rc;
}
