// Device-driven batch loop of the single-graph build (Algorithm 4, the
// batches and their vertex-centric rounds, rows a1-a7).
//
// One persistent launch of at most as many workgroups as fit on the device
// at once runs batch after batch: batch init, then rounds of push and check
// until a round accepts nothing, then batch end and table clear.  Phases are
// separated by a grid-wide barrier instead of a return to the host, so a
// round costs two barriers rather than two launches and a counter read-back.
// The barrier is two-level: workgroups arrive on one of PLL_SHARDS counters
// (each on its own cache line); the last arrival of a shard arrives on the
// top counter, and the last of those bumps the generation word that everyone
// waits on.  Every decision taken after a barrier (stop on an error, a batch
// that is done, a label arena that must be compacted) is read from words
// that were complete before the barrier ended, so all workgroups take it
// together.  Waits are bounded by the device wall clock: a workgroup that
// waits too long records PLL_ERR_TIMEOUT and leaves, and so does everyone
// after it, so the launch always drains.
//
// The phases are the same device functions the per-phase kernels and the
// many-graph kernel run (pll_phases.h); only their sequencing differs.
#include <mutex>

#include "pll_internal.h"
#include "pll_phases.h"

namespace {

using pll::Exec;
using pll::PhaseStats;

constexpr int kRoundBlock = 1024;
constexpr int kRoundWaves = kRoundBlock / PLL_WAVE;

struct alignas(128) CountLine {
    uint32_t count;
    uint32_t pad[31];
};

struct alignas(128) AccLine {
    uint32_t acc[2];  // entries accepted in the round, by round parity
    uint32_t pad[30];
};

// Control block of one launch (zero-filled before it).
struct GridCtl {
    uint32_t top, gen;
    uint32_t flag[2];  // error / stop bits, by barrier parity
    uint32_t pad0[28];
    CountLine arrive[PLL_SHARDS];
    AccLine acc[PLL_SHARDS];
    // written by workgroup 0 when the launch ends
    uint32_t next_ib, bstamp, rstamp, pad1;
    unsigned long long batches, rounds;
    unsigned long long ticks[PLL_NUM_PHASES];   // device wall-clock ticks per phase
    unsigned long long counts[PLL_NUM_PHASES];  // phase instances
};

__device__ inline uint32_t load_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long load_agent64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier k.  `extra` is ORed into the flag word of this barrier by the
// caller's workgroup; the return value (the same in every workgroup) is that
// word once every workgroup has arrived: device errors seen by any
// workgroup before arriving, plus every `extra`.  The word of parity k & 1 is
// written again only at barrier k + 2, which nobody can reach before all
// have left barrier k + 1.
__device__ uint32_t grid_sync(GridCtl* gc, uint32_t& k, DevCounters* ctr, uint64_t timeout_ticks, uint32_t extra,
                              uint32_t* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t par = k & 1u;
        const uint32_t e = load_agent(&ctr->error) | extra;
        if (e) atomicOr(&gc->flag[par], e);
        const uint32_t nsh = min(gridDim.x, (uint32_t)PLL_SHARDS);
        const uint32_t s = blockIdx.x % nsh;
        const uint32_t members = (gridDim.x - s + nsh - 1) / nsh;
        const uint32_t gen = load_agent(&gc->gen);
        __threadfence();
        bool last = false;
        if (atomicAdd(&gc->arrive[s].count, 1u) == members - 1) {
            store_agent(&gc->arrive[s].count, 0u);
            __threadfence();
            if (atomicAdd(&gc->top, 1u) == nsh - 1) {
                store_agent(&gc->top, 0u);
                __threadfence();
                atomicAdd(&gc->gen, 1u);
                last = true;
            }
        }
        if (!last) {
            const uint64_t t0 = wall_clock64();
            while (load_agent(&gc->gen) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (wall_clock64() - t0 > timeout_ticks) {
                    atomicOr(&gc->flag[0], PLL_ERR_TIMEOUT);
                    atomicOr(&gc->flag[1], PLL_ERR_TIMEOUT);
                    atomicOr(&ctr->error, PLL_ERR_TIMEOUT);
                    break;
                }
            }
        }
        __threadfence();
        *s_flag = load_agent(&gc->flag[par]);
    }
    __syncthreads();
    ++k;
    return *s_flag;
}

// Sum of v over the workgroup (every thread gets it).
__device__ unsigned long long block_sum(unsigned long long v, unsigned long long* s_part) {
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
    const unsigned long long t = wave_sum64(v);
    __syncthreads();
    if (lane == 0) s_part[wv] = t;
    __syncthreads();
    unsigned long long s = 0;
    for (int w = 0; w < kRoundWaves; ++w) s += s_part[w];
    return s;
}

// Workgroup 0, thread 0: charge the time since the last mark to `phase`.
struct PhaseClock {
    bool on;
    uint64_t last;
    unsigned long long ticks[PLL_NUM_PHASES];
    unsigned long long counts[PLL_NUM_PHASES];
    __device__ void mark(int phase) {
        if (!on) return;
        const uint64_t t = wall_clock64();
        ticks[phase] += t - last;
        counts[phase] += 1;
        last = t;
    }
};

template <int WM>
__global__ void __launch_bounds__(kRoundBlock) k_batches(BuildArgs A, GridCtl* gc, uint32_t ib0, uint32_t b,
                                                         uint32_t flags, uint32_t bstamp0, uint32_t rstamp0,
                                                         uint64_t timeout_ticks, uint32_t compact) {
    __shared__ uint64_t s_pres[kRoundWaves][PLL_WMAX];
    __shared__ uint8_t s_dist[kRoundWaves][PLL_BMAX];
    __shared__ unsigned long long s_part[kRoundWaves];
    __shared__ uint32_t s_flag, s_acc, s_nact;

    const uint32_t tid = threadIdx.x, wv = tid >> 6;
    const uint32_t n = A.n;
    DevCounters* ctr = A.ctr;
    const bool recheck = (flags & PLL_FLAG_RECHECK) != 0;
    const bool relaxed = (flags & PLL_FLAG_RELAXED) != 0;
    const uint32_t my = blockIdx.x % PLL_SHARDS;

    Exec X;
    X.w = blockIdx.x * (uint32_t)kRoundWaves + wv;
    X.nw = gridDim.x * (uint32_t)kRoundWaves;
    X.qs = ctr->sh;
    X.nq = PLL_SHARDS;
    X.my = my;
    X.seg = n;
    X.zero_i = blockIdx.x == 0 ? tid : ~0u;
    X.arena_sh = my;

    PhaseClock clk{};
    clk.on = blockIdx.x == 0 && tid == 0;
    if (clk.on) clk.last = wall_clock64();

    PhaseStats st;
    uint32_t k = 0, bstamp = bstamp0, rstamp = rstamp0;
    unsigned long long batches = 0, rounds = 0;
    uint32_t next_ib = n;
    for (uint32_t ib = ib0; ib < n; ib += b) {
        const uint32_t bs = min(b, n - ib);
        ++bstamp;
        ++batches;
        if (blockIdx.x == 0 && tid < PLL_SHARDS) {
            Shard& q = ctr->sh[tid];
            q.recv[0] = q.recv[1] = 0;
            q.hq[0] = q.hq[1] = 0;
            q.touched = 0;
            gc->acc[tid].acc[0] = gc->acc[tid].acc[1] = 0;
        }
        if (grid_sync(gc, k, ctr, timeout_ticks, 0u, &s_flag)) break;
        pll::phase_batch_init(A, X, ib, bs, bstamp);
        if (grid_sync(gc, k, ctr, timeout_ticks, 0u, &s_flag)) break;
        clk.mark(PLL_PHASE_INIT);
        uint32_t p = 0, nact = bs;
        bool failed = false;
        for (uint32_t j = 1;; ++j) {
            ++rstamp;
            ++rounds;
            pll::phase_push(A, X, ib, p, nact, rstamp, bstamp, st);
            if (grid_sync(gc, k, ctr, timeout_ticks, 0u, &s_flag)) {
                failed = true;
                break;
            }
            clk.mark(PLL_PHASE_PUSH);
            // the counter of round j+1 was last read after round j-1
            if (blockIdx.x == 0 && tid < PLL_SHARDS) gc->acc[tid].acc[(j + 1) & 1u] = 0;
            const unsigned long long acc0 = st.acc;
            pll::phase_check<WM>(A, X, ib, bs, j, p, relaxed, st);
            const unsigned long long got = block_sum(st.acc - acc0, s_part);
            if (tid == 0 && got) atomicAdd(&gc->acc[my].acc[j & 1u], (uint32_t)got);
            if (grid_sync(gc, k, ctr, timeout_ticks, 0u, &s_flag)) {
                failed = true;
                break;
            }
            clk.mark(PLL_PHASE_CHECK);
            if (tid == 0) {
                uint32_t a = 0, r = 0;
                for (int s = 0; s < PLL_SHARDS; ++s) {
                    a += load_agent(&gc->acc[s].acc[j & 1u]);
                    r += load_agent(&ctr->sh[s].recv[p]);
                }
                s_acc = a;
                s_nact = r;
            }
            __syncthreads();
            const uint32_t acc_round = s_acc, recv_round = s_nact;
            __syncthreads();
            if (acc_round == 0) break;  // nobody accepted anything: the batch is done
            nact = recv_round;
            p ^= 1u;
        }
        if (failed) break;
        pll::phase_batch_end<WM>(A, X, ib, bs, recheck, s_pres[wv], s_dist[wv], nullptr, st);
        if (grid_sync(gc, k, ctr, timeout_ticks, 0u, &s_flag)) break;
        pll::phase_clear_table(A, X, ib, bs);
        // hand back to the host for compaction once a bump region is half used
        uint32_t extra = 0;
        if (compact && blockIdx.x == 0 && tid == 0 && ib + b < n) {
            unsigned long long top = 0;
            for (int s = 0; s < PLL_SHARDS; ++s) top = max(top, load_agent64(&ctr->sh[s].arena_top));
            if (top * 2 > A.region_cap) extra = PLL_ERR_STOP;
        }
        const uint32_t f = grid_sync(gc, k, ctr, timeout_ticks, extra, &s_flag);
        clk.mark(PLL_PHASE_END);
        if (f) {
            if (f == PLL_ERR_STOP) next_ib = ib + b;
            break;
        }
    }

    // statistics of this workgroup, one sharded atomic each
    const unsigned long long v[8] = {st.cand, st.acc, st.edges, st.read, st.table, st.removed, st.cost_pos,
                                     st.cost_neg};
    const int which[8] = {PLL_ST_CAND,  PLL_ST_ACC,     PLL_ST_EDGES,    PLL_ST_READ,
                          PLL_ST_TABLE, PLL_ST_RECHECK, PLL_ST_COST_POS, PLL_ST_COST_NEG};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const unsigned long long t = block_sum(v[i], s_part);
        if (tid == 0 && t) atomicAdd(&ctr->sh[my].stat[which[i]], t);
    }
    if (blockIdx.x == 0 && tid == 0) {
        gc->next_ib = next_ib;
        gc->bstamp = bstamp;
        gc->rstamp = rstamp;
        gc->batches = batches;
        gc->rounds = rounds;
        for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
            gc->ticks[ph] = clk.ticks[ph];
            gc->counts[ph] = clk.counts[ph];
        }
    }
}

template <int WM>
int resident_rounds_blocks() {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batches<WM>, kRoundBlock, 0) != hipSuccess)
        return 0;
    return per_cu * cus;
}

template <int WM>
hipError_t launch_batches(uint32_t grid, hipStream_t s, const BuildArgs& A, GridCtl* gc, uint32_t ib0, uint32_t b,
                          uint32_t flags, uint32_t bstamp, uint32_t rstamp, uint64_t timeout_ticks, uint32_t compact) {
    k_batches<WM><<<grid, kRoundBlock, 0, s>>>(A, gc, ib0, b, flags, bstamp, rstamp, timeout_ticks, compact);
    return hipGetLastError();
}

int words_class(uint32_t W) { return W <= 1 ? 1 : W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16; }

}  // namespace

std::mutex& pll_persistent_mutex() {
    static std::mutex mu;
    return mu;
}

int pll_run_batches(const BuildArgs& A, uint32_t ib0, uint32_t b, uint32_t flags, uint32_t* bstamp,
                    uint32_t* rstamp, bool compact, uint32_t max_workgroups, hipStream_t s, hipEvent_t ev_begin,
                    hipEvent_t ev_end, BatchRun* out) {
    const int wc = words_class(A.W);
    int resident = 0;
    switch (wc) {
        case 1: resident = resident_rounds_blocks<1>(); break;
        case 2: resident = resident_rounds_blocks<2>(); break;
        case 4: resident = resident_rounds_blocks<4>(); break;
        case 8: resident = resident_rounds_blocks<8>(); break;
        default: resident = resident_rounds_blocks<16>(); break;
    }
    if (resident <= 0) return PLL_EDEVICE;
    uint32_t grid = (uint32_t)resident;
    if (max_workgroups) grid = std::min(grid, max_workgroups);
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        return PLL_EDEVICE;
    const uint64_t timeout_ticks = (uint64_t)khz * 1000ull * 30ull;  // 30 s of waiting at one barrier

    GridCtl* gc = nullptr;
    if (pll_ws_alloc((void**)&gc, sizeof(GridCtl)) != hipSuccess) return PLL_ENOMEM;
    GridCtl* h = nullptr;
    if (pll_pinned_alloc((void**)&h, sizeof(GridCtl)) != hipSuccess) {
        pll_ws_free(gc);
        return PLL_ENOMEM;
    }
    int rc = PLL_OK;
    {
        // persistent launches of this process run one at a time: two of them
        // sharing the device could each wait for workgroups the other holds
        std::lock_guard<std::mutex> lock(pll_persistent_mutex());
        hipError_t e = hipMemsetAsync(gc, 0, sizeof(GridCtl), s);
        if (e == hipSuccess && ev_begin) e = hipEventRecord(ev_begin, s);
        if (e == hipSuccess) {
            switch (wc) {
                case 1: e = launch_batches<1>(grid, s, A, gc, ib0, b, flags, *bstamp, *rstamp, timeout_ticks, compact); break;
                case 2: e = launch_batches<2>(grid, s, A, gc, ib0, b, flags, *bstamp, *rstamp, timeout_ticks, compact); break;
                case 4: e = launch_batches<4>(grid, s, A, gc, ib0, b, flags, *bstamp, *rstamp, timeout_ticks, compact); break;
                case 8: e = launch_batches<8>(grid, s, A, gc, ib0, b, flags, *bstamp, *rstamp, timeout_ticks, compact); break;
                default: e = launch_batches<16>(grid, s, A, gc, ib0, b, flags, *bstamp, *rstamp, timeout_ticks, compact); break;
            }
        }
        if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h, gc, sizeof(GridCtl), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = PLL_EDEVICE;
    }
    if (rc == PLL_OK) {
        out->next_ib = h->next_ib;
        out->batches = h->batches;
        out->rounds = h->rounds;
        out->grid = grid;
        for (int ph = 0; ph < PLL_NUM_PHASES; ++ph) {
            out->ms[ph] = (double)h->ticks[ph] / (double)khz;
            out->counts[ph] = h->counts[ph];
        }
        *bstamp = h->bstamp;
        *rstamp = h->rstamp;
    }
    (void)hipStreamSynchronize(s);
    pll_pinned_free(h);
    pll_ws_free(gc);
    return rc;
}
