// Device-side building blocks of one BVC-PLL batch (Algorithm 4), shared by
// the whole-grid kernels of a single large graph (pll_build.hip) and by the
// persistent kernel that builds many graphs, one workgroup per graph
// (pll_multi.hip).  A phase is run by an execution group described by Exec:
// wave w of nw waves; queue counters live in nq shards at qs (32 global
// shards for the whole-grid kernels, one LDS shard for a workgroup), and
// this wave appends to shard `my`, whose queue segments start at
// my * seg.
#pragma once

#include "pll_internal.h"

namespace pll {

// Rows longer than kHeavy are not pushed by the wave that owns them but
// queued as work items of kHeavyItem edges, spread over every wave.
constexpr uint32_t kHeavy = 1024;
constexpr uint32_t kHeavyItem = 256;

struct Exec {
    uint32_t w, nw;   // this wave's index in the group, waves in the group
    Shard* qs;        // queue / statistics shards
    uint32_t nq;      // number of shards
    uint32_t my;      // shard this wave appends to
    uint32_t seg;     // entries per shard segment of recv / touched / tstart
    uint32_t zero_i;  // shard this thread clears when a phase resets counters (>= nq: none)
    uint32_t arena_sh;  // first arena region to try
};

// Per-lane statistics a phase accumulates (summed over lanes by the caller).
struct PhaseStats {
    unsigned long long cand = 0, acc = 0, edges = 0, read = 0, table = 0, removed = 0, bp = 0;
    // cost of the positive / negative checks: |L(v)| at each check that
    // added / pruned a candidate (Section 4.3, Table 3)
    unsigned long long cost_pos = 0, cost_neg = 0;
    // CSR entries of the vertices whose next-round deliveries are pulled: the
    // edge accesses of Algorithm 4 (the gather itself reads more)
    unsigned long long pulled = 0;
};

// Bit 7 of each byte of the result: that byte of x is <= t, where
// tt = t * 0x01010101 (t <= 254).  Bytes are compared without carries
// between them: s holds, in bit 7 of each byte, [low 7 bits of t >= low 7
// bits of x]; the high bits decide the rest.
__device__ inline uint32_t le4_flags(uint32_t x, uint32_t tt) {
    const uint32_t H = 0x80808080u;
    const uint32_t s = (tt | H) - (x & ~H);
    return ((tt & ~x) | (~(tt ^ x) & s)) & H;
}

// The flags of two words (bits 7, 15, 23, 31 of a and of b) as 8 bits, a's
// in bits 0..3: one multiply gathers both, since with a's flags moved to
// bits 0, 8, 16, 24 and b's to 4, 12, 20, 28, every cross term of the
// product lands below bit 24 or above bit 31, each on a bit of its own.
__device__ inline uint32_t gather8(uint32_t a, uint32_t b) {
    return (((a >> 7) | (b >> 3)) * 0x01020408u) >> 24;
}

// The 16 flags of a 16-byte quarter, byte i in bit i.
__device__ inline uint32_t gather16(uint32_t fx, uint32_t fy, uint32_t fz, uint32_t fw) {
    return gather8(fx, fy) | (gather8(fz, fw) << 8);
}

// Bit i of the result: table byte p[i] <= t, for 64 consecutive bytes.
__device__ inline uint64_t le_mask64(const uint8_t* p, uint32_t tt) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 v = q[i];
        const uint32_t b = gather16(le4_flags(v.x, tt), le4_flags(v.y, tt), le4_flags(v.z, tt), le4_flags(v.w, tt));
        m |= (uint64_t)b << (16 * i);
    }
    return m;
}

// le_mask64 for thresholds t <= kSmallT, with tt1 = (t + 1) * 0x01010101:
// every byte of x | 0x80 is at least 128 > t + 1, so the subtraction
// borrows within no byte, and bit 7 of the difference is clear exactly when
// the byte's low 7 bits are <= t; a byte with bit 7 set (128..255) is above
// t.  Four instructions per word instead of le4_flags's seven.
constexpr uint32_t kSmallT = 126;

// bit 7 of each byte of the result: that byte of x is <= t
__device__ inline uint32_t le4s_flags(uint32_t x, uint32_t tt1) {
    const uint32_t H = 0x80808080u;
    return ~(((x | H) - tt1) | x) & H;
}

__device__ inline uint64_t le_mask64s(const uint8_t* p, uint32_t tt1) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint32_t half[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint4 v0 = q[2 * h], v1 = q[2 * h + 1];
        const uint32_t b0 = gather16(le4s_flags(v0.x, tt1), le4s_flags(v0.y, tt1), le4s_flags(v0.z, tt1),
                                     le4s_flags(v0.w, tt1));
        const uint32_t b1 = gather16(le4s_flags(v1.x, tt1), le4s_flags(v1.y, tt1), le4s_flags(v1.z, tt1),
                                     le4s_flags(v1.w, tt1));
        half[h] = b0 | (b1 << 16);
    }
    return ((uint64_t)half[1] << 32) | half[0];
}

// The segment compare of the scans: SMALLT (every threshold <= kSmallT) takes
// le_mask64s with tt = (t + 1) * 0x01010101, else le_mask64 with t * 0x01010101.
template <bool SMALLT>
__device__ inline uint32_t seg_tt(uint32_t t) {
    return (SMALLT ? t + 1u : t) * 0x01010101u;
}

template <bool SMALLT>
__device__ inline uint64_t seg_le(const uint8_t* p, uint32_t tt) {
    return SMALLT ? le_mask64s(p, tt) : le_mask64(p, tt);
}

// le_mask64 over the 16-byte quarters selected by `need` (bit i: bytes
// 16i .. 16i+15); the other quarters are neither loaded nor matched.
__device__ inline uint64_t le_mask64_q(const uint8_t* p, uint32_t tt, uint32_t need) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if ((need >> i) & 1u) {
            const uint4 v = q[i];
            const uint32_t b = gather16(le4_flags(v.x, tt), le4_flags(v.y, tt), le4_flags(v.z, tt), le4_flags(v.w, tt));
            m |= (uint64_t)b << (16 * i);
        }
    }
    return m;
}

// Bit i set when quarter i (candidates 16i .. 16i+15) of a word has a bit.
__device__ inline uint32_t quarters(uint64_t x) {
    return (uint32_t)((x & 0xFFFFull) != 0) | ((uint32_t)((x & 0xFFFF0000ull) != 0) << 1) |
           ((uint32_t)((x & 0xFFFF00000000ull) != 0) << 2) | ((uint32_t)((x >> 48) != 0) << 3);
}

// OR over the 64 lanes (DPP wave reduction, the whole wave active); the
// result is wave-uniform.
__device__ inline uint64_t wave_or64_u(uint64_t x) {
    const uint32_t lo = wave_or32_dpp((uint32_t)x);
    const uint32_t hi = wave_or32_dpp((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Scan the label list arena[off .. off+len) of one vertex v.  Lane w (< W)
// holds candidate word cw = bits k of batch vertices u_{64w+k} that arrived
// at distance j.  Returns, in lane w, the candidates of word w for which some
// entry (h, d) of the list with d < j has T[h][k] + d <= j, i.e. the distance
// j is already covered through a hub ranked above u_k (the pruning test of
// Algorithm 4).
// With `relaxed`, entries whose hub is in the current batch are skipped.
// Each chunk of 64 entries makes one pass per candidate word that still
// holds live candidates, and the wave OR-reduces that word's prunes in the
// pass, so the scan stops after the first chunk that leaves no candidate
// live (the top-ranked hubs of the first chunk prune most candidates of the
// late rounds).  The next chunk's entries are loaded while this chunk's
// segments are.  With QGATE only the 16-byte
// quarters of a table segment that both hold entries (row mask) and have
// live candidates are loaded; without it a segment is loaded whole when any
// of its quarters qualifies (fewer, wider loads: measured faster on the large
// single-graph builds, while the many-graph kernel, whose small graphs leave
// table rows sparse, gains from the gating).
template <int WM, bool QGATE = false, bool SMALLT = false>
__device__ inline uint64_t prune_scan(const BuildArgs& A, uint64_t off, uint32_t len, uint32_t j, uint64_t cw,
                                      bool relaxed, uint32_t ib, PhaseStats& st) {
    const uint32_t lane = lane_id();
    uint64_t pw = 0;
    // the next chunk's entry is loaded while this chunk's table segments are
    uint32_t next = lane < len ? A.arena[off + lane] : 0u;
    for (uint32_t base = 0; base < len; base += 64) {
        const uint32_t idx = base + lane;
        bool ok = idx < len;
        st.read += ok;
        const uint32_t ent = next;
        next = idx + 64 < len ? A.arena[off + idx + 64] : 0u;
        const uint32_t h = ent >> 8, d = ent & 255u;
        ok = ok && d < j;
        if (relaxed) ok = ok && h < ib;
        const uint64_t rm = ok ? A.rmchk[h] : 0ull;
        // threshold at most 254, the largest finite table byte: at round 255
        // (which only reports the overflow) an empty cell must not prune
        const uint32_t tt = ok ? seg_tt<SMALLT>(min(j - d, PLL_INF8 - 1u)) : 0u;
        const uint8_t* row = A.Tchk + (size_t)h * A.bstride;
        // One pass per word that still holds live candidates (a scalar loop
        // over their mask): every lane compares its entry's table segment,
        // and the wave OR-reduces the word's prunes at once.  So the
        // candidates pruned by this chunk (the top-ranked hubs of the first
        // chunk prune most) load no later segments, one copy of the compare
        // serves every word, and no per-word accumulators are kept.
        const uint64_t live_lane = cw & ~pw;
        uint64_t lw = ballot64(live_lane != 0) & (WM >= 64 ? ~0ull : ((1ull << WM) - 1ull));
        while (lw) {
            const uint32_t w = (uint32_t)__builtin_ctzll(lw);
            lw &= lw - 1;
            uint64_t m = 0;
            if (QGATE) {
                const uint64_t live = readlane64(live_lane, w);
                const uint32_t need = (uint32_t)(rm >> (4 * w)) & quarters(live);
                if (need & 15u) {
                    m = le_mask64_q(row + 64u * w, tt, need);
                    st.table += __builtin_popcount(need & 15u);
                }
            } else if ((rm >> (4 * w)) & 15u) {
                m = seg_le<SMALLT>(row + 64u * w, tt);
                st.table += 4;
            }
            // lane w masks the reduced prunes with its live candidates
            const uint64_t red = wave_or64_u(m);
            if (lane == w) pw |= red & live_lane;
        }
        if (!ballot64((cw & ~pw) != 0)) break;
    }
    return pw;
}

// The round-2 check of receiver v through its neighbours.  At distance 2
// only entries (h, 1) of L(v) can prune (the self entry cannot, as in round
// 1), and in an undirected unweighted graph those are exactly the
// neighbours h of v ranked above both v and the end of the current batch
// (lim): the edge is the only shortest h-v path, so h is its top-ranked
// vertex, and h's batch has run (or, inside the current batch, round 1
// accepted (h, 1) unconditionally).  So the rank-space CSR row of v can
// stand in for L(v): the caller takes it when it is the shorter of the two
// (a low-ranked vertex has a few dozen neighbours and hundreds of label
// entries).  Candidate u_k is pruned when T[h][k] <= 1; the table loads,
// which are the same as those of the label scan, and the lane reductions
// are those of prune_scan.
template <int WM, bool QGATE = false, bool SMALLT = false>
__device__ inline uint64_t prune_scan_nbrs(const BuildArgs& A, uint32_t v, uint32_t lim, uint64_t cw,
                                           PhaseStats& st) {
    const uint32_t lane = lane_id();
    uint64_t pw = 0;
    const uint64_t beg = A.rrow[v], end = A.rrow[v + 1];
    const uint32_t tt = seg_tt<SMALLT>(1u);  // T[h][k] <= 2 - 1
    for (uint64_t base = beg; base < end; base += 64) {
        const uint64_t idx = base + lane;
        const uint32_t h = idx < end ? A.rcol[idx] : ~0u;
        const bool ok = h < lim;
        st.read += idx < end;
        const uint64_t rm = ok ? A.rmchk[h] : 0ull;
        const uint8_t* row = A.Tchk + (size_t)(ok ? h : 0u) * A.bstride;
        // one pass per word with live candidates, as in prune_scan
        const uint64_t live_lane = cw & ~pw;
        uint64_t lw = ballot64(live_lane != 0) & (WM >= 64 ? ~0ull : ((1ull << WM) - 1ull));
        while (lw) {
            const uint32_t w = (uint32_t)__builtin_ctzll(lw);
            lw &= lw - 1;
            uint64_t m = 0;
            if (QGATE) {
                const uint64_t live = readlane64(live_lane, w);
                const uint32_t need = (uint32_t)(rm >> (4 * w)) & quarters(live);
                if (need & 15u) {
                    m = le_mask64_q(row + 64u * w, tt, need);
                    st.table += __builtin_popcount(need & 15u);
                }
            } else if ((rm >> (4 * w)) & 15u) {
                m = seg_le<SMALLT>(row + 64u * w, tt);
                st.table += 4;
            }
            // lane w masks the reduced prunes with its live candidates
            const uint64_t red = wave_or64_u(m);
            if (lane == w) pw |= red & live_lane;
        }
        if (!ballot64((cw & ~pw) != 0)) break;
    }
    return pw;
}

// Room for `need` more entries in the list of rank v (capacity doubling).
// New blocks come from the bump region X.arena_sh of the arena, or from the
// next region with room.  Wave-uniform; returns the list's offset, or ~0
// when every region is exhausted.
__device__ inline uint64_t wave_reserve(const BuildArgs& A, const Exec& X, uint32_t v, uint64_t off, uint32_t len,
                                        uint32_t need) {
    const uint32_t cap = A.lcap[v];
    if (len + need <= cap) return off;
    uint32_t newcap = max(cap * 2u, (len + need + 15u) & ~15u);
    newcap = max(newcap, 16u);
    unsigned long long nb = ~0ull;
    if (lane_id() == 0) {
        for (uint32_t t = 0; t < PLL_SHARDS; ++t) {
            const uint32_t sh = (X.arena_sh + t) % PLL_SHARDS;
            unsigned long long* top = &A.ctr->sh[sh].arena_top;
            if (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + newcap > A.region_cap) continue;
            const unsigned long long at = atomicAdd(top, (unsigned long long)newcap);
            if (at + newcap <= A.region_cap) {
                nb = A.region_base + (unsigned long long)sh * A.region_cap + at;
                break;
            }
        }
        atomicAdd(&A.ctr->sh[X.arena_sh % PLL_SHARDS].stat[PLL_ST_GROW], 1ull);
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

// Sharded queue enumeration: lane s (< nq) holds the count of shard s;
// `pre` receives its exclusive prefix and the return value the total.
__device__ inline uint32_t shard_prefix(uint32_t cnt_lane, uint32_t& pre) {
    pre = wave_excl_scan32(cnt_lane);
    return readlane32(pre + cnt_lane, 63);
}

// Shard holding global queue position i (wave-uniform i < total).
__device__ inline uint32_t shard_of(uint32_t nq, uint32_t pre_lane, uint32_t i) {
    const uint64_t m = ballot64(lane_id() < nq && pre_lane <= i);
    return 63u - (uint32_t)__builtin_clzll(m);
}

// Wave-aggregated append of the lanes with `take` to a queue counter;
// returns each taking lane's position (seg_base + index).
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

// Queue the row of active slot `slot` (list q) as kHeavyItem-edge items
// when it is longer than kHeavy.
__device__ inline void enqueue_heavy(const BuildArgs& A, const Exec& X, uint32_t q, uint32_t slot, uint64_t deg) {
    if (deg <= kHeavy) return;
    const uint32_t nch = (uint32_t)((deg + kHeavyItem - 1) / kHeavyItem);
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&X.qs[X.my].hq[q], nch);
    base = readlane32(base, 0);
    for (uint32_t c = lane_id(); c < nch; c += 64) A.hq[q][X.my * A.hq_seg + base + c] = make_uint2(slot, c);
}

__device__ inline uint64_t rank_mask(uint32_t rel, uint32_t w) {
    const uint32_t lo = w * 64u;
    if (rel >= lo + 64u) return ~0ull;
    if (rel <= lo) return 0ull;
    return (1ull << (rel - lo)) - 1ull;
}

// Batch initialisation of Algorithm 4: delta L(u) = {(u,0)}, L(u) gets
// (u,0), L(u) -> H(u).
// The initial active list holds batch vertex u_k in slot k.
__device__ inline void phase_batch_init(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs, uint32_t bstamp) {
    const uint32_t lane = lane_id();
    for (uint32_t k = X.w; k < bs; k += X.nw) {
        const uint32_t u = ib + k;
        const uint32_t len = A.llen[u];
        const uint64_t off0 = A.loff[u];
        // the first four chunks of L(u) and u's degree are loaded ahead of
        // the bookkeeping (a relocation by wave_reserve copies the same
        // entries, so they stay valid)
        uint32_t e[4];
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) {
            const uint32_t i = 64u * c + lane;
            e[c] = i < len ? A.arena[off0 + i] : 0u;
        }
        const uint64_t deg = A.rrow[u + 1] - A.rrow[u];
        const uint32_t tpos = shard_append(&X.qs[X.my].touched, lane == 0, (uint64_t)X.my * X.seg);
        if (lane == 0) {
            A.touch_stamp[u] = bstamp;
            A.touched[tpos] = u;
            A.tstart[tpos] = len;
        }
        if (A.bp_t && A.bp_used[u]) {  // a bit-parallel vertex is no root of the rounds
            if (lane == 0) A.act_v[0][k] = u;
            if (lane < A.W) A.act_delta[0][(size_t)k * A.W + lane] = 0ull;
            continue;
        }
        const uint64_t off = wave_reserve(A, X, u, off0, len, 1);
        if (off == ~0ull) continue;
        const unsigned long long kq = 1ull << (k >> 4);
        if (lane == 0) {
            A.arena[off + len] = pll_pack(u, 0);
            A.llen[u] = len + 1;
            A.T[(size_t)u * A.bstride + k] = 0;
            if (u >= A.hot) atomicOr((unsigned long long*)&A.rowmask[u], kq);
        }
        // four chunks at a time: loaded before any is written out
        for (uint32_t i0 = 0; i0 < len; i0 += 256) {
            if (i0) {
#pragma unroll
                for (uint32_t c = 0; c < 4; ++c) {
                    const uint32_t i = i0 + 64u * c + lane;
                    e[c] = i < len ? A.arena[off + i] : 0u;
                }
            }
#pragma unroll
            for (uint32_t c = 0; c < 4; ++c) {
                if (i0 + 64u * c + lane < len) {
                    const uint32_t h = e[c] >> 8;
                    A.T[(size_t)h * A.bstride + k] = (uint8_t)(e[c] & 255u);
                    if (h >= A.hot) atomicOr((unsigned long long*)&A.rowmask[h], kq);
                }
            }
        }
        if (lane == 0) A.act_v[0][k] = u;
        if (lane == 0 && A.act_rng[0]) A.act_rng[0][k] = make_uint2(len, 1u);  // the self entry
        if (lane < A.W) A.act_delta[0][(size_t)k * A.W + lane] = (lane == (k >> 6)) ? (1ull << (k & 63)) : 0ull;
        enqueue_heavy(A, X, 0, k, deg);
    }
}

// The lanes whose vertex r got a delivery (`any`) take r's receiver slot
// of the next round (one per vertex and round, via its round stamp) into
// queue rq stored in recv; the lane that wins the slot also records r's
// first touch in this batch.  The whole wave calls it.
__device__ inline void enqueue_receivers(const BuildArgs& A, const Exec& X, uint32_t* recv, uint32_t rq,
                                         uint32_t rstamp, uint32_t bstamp, uint32_t r, bool any) {
    bool enq = false;
    if (any && A.recv_stamp[r] != rstamp) enq = atomicExch(&A.recv_stamp[r], rstamp) != rstamp;
    bool first = false;
    if (enq && A.touch_stamp[r] != bstamp) {
        A.touch_stamp[r] = bstamp;
        first = true;
    }
    if (ballot64(enq)) {
        const uint32_t rp = shard_append(&X.qs[X.my].recv[rq], enq, (uint64_t)X.my * X.seg);
        if (enq) recv[rp] = r;
        const uint32_t tp = shard_append(&X.qs[X.my].touched, first, (uint64_t)X.my * X.seg);
        if (first) {
            A.touched[tp] = r;
            A.tstart[tp] = A.llen[r];
        }
    }
}

// Deliver to vertex r the words w[k] of a delta whose candidates ranked
// above r are m[k] (0 for unused slots): each is filtered by C(r) and ORed
// into msgs(r).  The four C loads are issued before any is used, so the
// words of one edge cost one round trip.  Returns whether anything was
// delivered.
__device__ inline bool deliver4(const BuildArgs& A, uint64_t* msgs, uint32_t r, const uint32_t (&w)[4],
                                const uint64_t (&m)[4]) {
    uint64_t c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = m[k] ? A.C[(size_t)r * A.W + w[k]] : 0ull;
    bool any = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t x = m[k] & ~c[k];
        if (x) {
            atomicOr((unsigned long long*)&msgs[(size_t)r * A.W + w[k]], (unsigned long long)x);
            any = true;
        }
    }
    return any;
}

// Push delta L(a) (lane w < W holds word w in dl; nz marks the nonzero
// words) along the CSR entries [beg, end) of the active vertex a, into the
// message buffer msgs and receiver queue rq (counters) stored in recv.
__device__ inline void push_edges(const BuildArgs& A, const Exec& X, uint64_t* msgs, uint32_t* recv, uint32_t ib,
                                  uint32_t rq, uint32_t rstamp, uint32_t bstamp, uint64_t dl, uint64_t nz,
                                  uint64_t beg, uint64_t end) {
    const uint32_t lane = lane_id();
    for (uint64_t e0 = beg; e0 < end; e0 += 64) {
        const uint64_t e = e0 + lane;
        const uint32_t r = e < end ? A.rcol[e] : 0u;
        const bool fwd = e < end && r > ib;
        const uint32_t rel = r - ib;
        bool any = false;
        uint64_t todo = nz;
        while (todo) {  // four words at a time
            uint32_t w[4];
            uint64_t m[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = todo ? (uint32_t)__builtin_ctzll(todo) : 0u;
                m[k] = todo && fwd ? readlane64(dl, w[k]) & rank_mask(rel, w[k]) : 0ull;
                todo &= todo - 1;
            }
            any |= deliver4(A, msgs, r, w, m);
        }
        enqueue_receivers(A, X, recv, rq, rstamp, bstamp, r, any);
    }
}

// The heavy-row items of active list p, spread over every wave: pushes
// into msgs and receiver queue rq stored in recv.
__device__ inline void phase_push_heavy(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t p, uint32_t rq,
                                        uint64_t* msgs, uint32_t* recv, uint32_t rstamp, uint32_t bstamp,
                                        PhaseStats& st) {
    const uint32_t lane = lane_id();
    const uint32_t* act_v = A.act_v[p];
    const uint64_t* act_d = A.act_delta[p];
    uint32_t pre;
    const uint32_t nh = shard_prefix(lane < X.nq ? X.qs[lane].hq[p] : 0u, pre);
    for (uint32_t t = X.w; t < nh; t += X.nw) {
        const uint32_t s = shard_of(X.nq, pre, t);
        const uint2 item = A.hq[p][s * A.hq_seg + (t - readlane32(pre, s))];
        const uint64_t dl = lane < A.W ? act_d[(size_t)item.x * A.W + lane] : 0ull;
        const uint64_t nz = ballot64(dl != 0);
        const uint32_t a = act_v[item.x];
        const uint64_t beg = A.rrow[a] + (uint64_t)item.y * kHeavyItem;
        const uint64_t end = min(A.rrow[a + 1], beg + kHeavyItem);
        if (lane == 0) st.edges += end - beg;
        push_edges(A, X, msgs, recv, ib, rq, rstamp, bstamp, dl, nz, beg, end);
    }
}

// Where a fused check delivers the next round: its message buffer, receiver
// queue and counters, the round stamps, and whether that round is pulled.
struct NextRound {
    uint64_t* msgs;
    uint32_t* recv;
    uint32_t rin, rout, rclr, hout;
    uint32_t rstamp, bstamp;
    uint32_t pull;  // the next round is pulled (phase_pull) instead of pushed
};

// A pulled round (the direction-optimizing alternative to push_edges, for
// rounds whose active vertices cover much of the graph): every vertex
// r > ib ORs the deltas of its active neighbours (act_at carries this
// round's stamp) and delivers the result exactly as the pushes from those
// neighbours would: masked to candidates ranked above r and not yet in
// C(r), into msgs(r), with one receiver slot and the first-touch record.
// Items are (vertex, segment of kPullSeg CSR entries); the segments of one
// vertex merge through atomicOr and the receiver stamp, like pushes do.
// Four active neighbours are gathered at a time, one per 16-lane group.
constexpr uint32_t kPullSeg = 256;

__device__ inline void phase_pull(const BuildArgs& A, const Exec& X, uint32_t ib, const uint2* items,
                                  const uint32_t* nitems, uint32_t q, const NextRound& nr) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t grp = lane >> 4, wd = lane & 15u;
    const uint64_t* act_d = A.act_delta[q];
    const uint32_t total = *nitems;
    for (uint32_t t = X.w; t < total; t += X.nw) {
        const uint2 it = items[t];
        const uint32_t r = it.x;
        if (r <= ib) continue;
        const uint64_t beg = A.rrow[r] + (uint64_t)it.y * kPullSeg;
        const uint64_t end = min(A.rrow[r + 1], beg + kPullSeg);
        uint64_t m = 0;
        for (uint64_t e0 = beg; e0 < end; e0 += 64) {
            const uint64_t e = e0 + lane;
            const uint64_t at = e < end ? A.act_at[A.rcol[e]] : 0ull;
            uint64_t act = ballot64((uint32_t)(at >> 32) == nr.rstamp);
            while (act) {
                uint32_t slot = 0;
                bool have = false;
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k) {
                    if (act) {
                        const uint32_t s = (uint32_t)__builtin_ctzll(act);
                        act &= act - 1;
                        const uint32_t sl = readlane32((uint32_t)at, s);
                        if (grp == k) {
                            slot = sl;
                            have = true;
                        }
                    }
                }
                if (have && wd < W) m |= act_d[(size_t)slot * W + wd];
            }
        }
        m |= __shfl_xor(m, 16, 64);
        m |= __shfl_xor(m, 32, 64);
        if (lane < W) {
            m &= rank_mask(r - ib, lane);
            if (m) m &= ~A.C[(size_t)r * W + lane];
        } else {
            m = 0;
        }
        if (m) atomicOr((unsigned long long*)&nr.msgs[(size_t)r * W + lane], (unsigned long long)m);
        if (!ballot64(m != 0)) continue;
        bool enq = false, first = false;
        if (lane == 0) {
            if (A.recv_stamp[r] != nr.rstamp) enq = atomicExch(&A.recv_stamp[r], nr.rstamp) != nr.rstamp;
            if (enq && A.touch_stamp[r] != nr.bstamp) {
                A.touch_stamp[r] = nr.bstamp;
                first = true;
            }
        }
        const uint32_t rp = shard_append(&X.qs[X.my].recv[nr.rout], enq, (uint64_t)X.my * X.seg);
        if (enq) nr.recv[rp] = r;
        const uint32_t tp = shard_append(&X.qs[X.my].touched, first, (uint64_t)X.my * X.seg);
        if (first) {
            A.touched[tp] = r;
            A.tstart[tp] = A.llen[r];
        }
    }
}

// phase_pull with four items per wave: the 16-lane group g = lane / 16
// gathers item i0 + g, 16 CSR entries at a time, and its lane 16g + w holds
// word w of the delta it collects.  Each step, every group ORs in the delta
// of one of its active neighbours (the groups' steps run side by side), so
// four items' chains of dependent loads (item, row, neighbour, stamp,
// delta) are in flight in one wave.  Deliveries are phase_pull's.
__device__ inline void phase_pull4(const BuildArgs& A, const Exec& X, uint32_t ib, const uint2* items,
                                   const uint32_t* nitems, uint32_t q, const NextRound& nr) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t wd = lane & 15u, gsh = lane & 48u;
    const uint64_t* act_d = A.act_delta[q];
    const uint32_t total = *nitems;
    for (uint32_t t0 = 4u * X.w; t0 < total; t0 += 4u * X.nw) {
        const uint32_t t = t0 + (lane >> 4);
        const uint2 it = t < total ? items[t] : make_uint2(0u, 0u);
        const uint32_t r = it.x;
        const bool valid = t < total && r > ib;
        uint64_t beg = 0, end = 0;
        if (valid) {
            beg = A.rrow[r] + (uint64_t)it.y * kPullSeg;
            end = min(A.rrow[r + 1], beg + kPullSeg);
        }
        uint64_t m = 0;
        for (uint64_t e0 = 0;; e0 += 16) {
            if (!ballot64(valid && beg + e0 < end)) break;
            const uint64_t e = beg + e0 + wd;
            const bool in = valid && e < end;
            const uint64_t at = in ? A.act_at[A.rcol[e]] : 0ull;
            const bool act = in && (uint32_t)(at >> 32) == nr.rstamp;
            uint64_t am = ballot64(act);
            while (am) {
                const uint32_t gm = (uint32_t)(am >> gsh) & 0xFFFFu;
                const uint32_t k = gm ? (uint32_t)__builtin_ctz(gm) : 0u;
                const uint32_t slot = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((gsh + k) * 4u), (int)(uint32_t)at);
                if (gm && wd < W) m |= act_d[(size_t)slot * W + wd];
                am &= ~ballot64(gm && wd == k);
            }
        }
        if (valid && wd < W) {
            m &= rank_mask(r - ib, wd);
            if (m) m &= ~A.C[(size_t)r * W + wd];
        } else {
            m = 0;
        }
        if (m) atomicOr((unsigned long long*)&nr.msgs[(size_t)r * W + wd], (unsigned long long)m);
        const uint64_t got = ballot64(m != 0);
        if (!got) continue;
        // one receiver slot per vertex and round, taken by lane 0 of the group
        bool enq = false, first = false;
        if (wd == 0 && ((got >> gsh) & 0xFFFFull)) {
            if (A.recv_stamp[r] != nr.rstamp) enq = atomicExch(&A.recv_stamp[r], nr.rstamp) != nr.rstamp;
            if (enq && A.touch_stamp[r] != nr.bstamp) {
                A.touch_stamp[r] = nr.bstamp;
                first = true;
            }
        }
        const uint32_t rp = shard_append(&X.qs[X.my].recv[nr.rout], enq, (uint64_t)X.my * X.seg);
        if (enq) nr.recv[rp] = r;
        const uint32_t tp = shard_append(&X.qs[X.my].touched, first, (uint64_t)X.my * X.seg);
        if (first) {
            A.touched[tp] = r;
            A.tstart[tp] = A.llen[r];
        }
    }
}

// The pull items of a rank-space CSR: (r, c) for every segment c of
// kPullSeg entries of every vertex r with neighbours, appended in any order.
__device__ inline void phase_pull_items(const BuildArgs& A, const Exec& X, uint2* items, uint32_t* nitems) {
    const uint32_t lane = lane_id();
    for (uint32_t r0 = X.w * 64u; r0 < A.n; r0 += X.nw * 64u) {
        const uint32_t r = r0 + lane;
        const uint64_t deg = r < A.n ? A.rrow[r + 1] - A.rrow[r] : 0ull;
        const uint32_t cnt = (uint32_t)((deg + kPullSeg - 1) / kPullSeg);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t tot = readlane32(pos + cnt, 63);
        uint32_t base = 0;
        if (lane == 0 && tot) base = atomicAdd(nitems, tot);
        base = readlane32(base, 0);
        for (uint32_t c = 0; c < cnt; ++c) items[base + pos + c] = make_uint2(r, c);
    }
}

// Scatter phase of Algorithm 4 over active list p (nact slots).
// Batch vertex u_k may be sent to v only when u_k outranks v (rank ib + k
// < v) and C(v) does not hold it yet.  Slots whose delta is empty are
// skipped; rows longer than kHeavy were queued as items and are spread over
// every wave after the per-slot pass.
__device__ inline void phase_push(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t p, uint32_t nact,
                                  uint32_t rstamp, uint32_t bstamp, PhaseStats& st) {
    const uint32_t lane = lane_id();
    if (X.zero_i < X.nq) X.qs[X.zero_i].hq[p ^ 1u] = 0;
    const uint32_t* act_v = A.act_v[p];
    const uint64_t* act_d = A.act_delta[p];
    for (uint32_t i = X.w; i < nact; i += X.nw) {
        const uint64_t dl = lane < A.W ? act_d[(size_t)i * A.W + lane] : 0ull;
        const uint64_t nz = ballot64(dl != 0);
        if (!nz) continue;
        const uint32_t a = act_v[i];
        const uint64_t beg = A.rrow[a], end = A.rrow[a + 1];
        if (end - beg > kHeavy) continue;
        if (lane == 0) st.edges += end - beg;
        push_edges(A, X, A.msgs, A.recv, ib, p, rstamp, bstamp, dl, nz, beg, end);
    }
    phase_push_heavy(A, X, ib, p, p, A.msgs, A.recv, rstamp, bstamp, st);
}

// Bit-parallel bound (Section 5.2) of every candidate in `mine` at v for
// distance j: candidate u_k is pruned when, for some BP root i,
// d_i(u_k) + d_i(v) - c <= j, with c = 2 when the S^-1 sets of u_k and v
// meet, else 1 when S^-1 of one meets S^0 of the other, else 0.  Lane i
// (< bp_t) holds v's data of root i; lanes run over the candidates of one
// word at a time, reading the batch vertices' data from the transposed
// per-batch copy.  Returns, in lane w, the pruned bits of word w.
template <int WM>
__device__ inline uint64_t bp_prune_words(const BuildArgs& A, uint32_t v, uint32_t ib, uint32_t j, uint64_t mine) {
    const uint32_t lane = lane_id();
    const uint32_t t = A.bp_t;
    uint32_t dv = PLL_INF8;
    ulonglong2 sv = make_ulonglong2(0ull, 0ull);
    if (lane < t) {
        dv = A.bp_dist[(size_t)v * t + lane];
        sv = A.bp_sets[(size_t)v * t + lane];
    }
    const uint64_t roots_v = ballot64(lane < t && dv != PLL_INF8);
    uint64_t out = 0;
    // few candidates: lanes over the BP roots, one candidate at a time (its
    // data of all roots is one coalesced load); otherwise lanes over the
    // candidates of a word, one root at a time
    const uint32_t ncand = wave_sum32(lane < WM ? (uint32_t)__builtin_popcountll(mine) : 0u);
    const uint32_t nwords = (uint32_t)__builtin_popcountll(ballot64(lane < WM && mine != 0));
    if (ncand < nwords * (uint32_t)__builtin_popcountll(roots_v)) {
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            uint64_t m = readlane64(mine, w);
            while (m) {
                const uint32_t bit = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                const size_t at = (size_t)(ib + 64u * w + bit) * t + lane;
                uint32_t td = 0xFFFFFFFFu;
                if (lane < t && dv != PLL_INF8) {
                    const uint32_t du = A.bp_dist[at];
                    if (du != PLL_INF8) {
                        const ulonglong2 su = A.bp_sets[at];
                        td = du + dv;
                        if (su.x & sv.x) td -= 2;
                        else if ((su.x & sv.y) | (su.y & sv.x)) td -= 1;
                    }
                }
                if (wave_min32(td) <= j && lane == (uint32_t)w) out |= 1ull << bit;
            }
        }
        return out;
    }
#pragma unroll
    for (int w = 0; w < WM; ++w) {
        const uint64_t m = readlane64(mine, w);
        if (!m) continue;
        const bool cand = (m >> lane) & 1ull;
        const uint32_t kk = 64u * w + lane;
        uint32_t bound = 0xFFFFFFFFu;
        uint64_t todo = roots_v;
        while (todo) {
            const uint32_t i = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t dvi = readlane32(dv, i);
            const uint64_t v1 = readlane64(sv.x, i), v0 = readlane64(sv.y, i);
            if (cand) {
                const uint32_t du = A.bpb_dist[(size_t)i * A.bstride + kk];
                if (du != PLL_INF8) {
                    const ulonglong2 su = A.bpb_sets[(size_t)i * A.bstride + kk];
                    uint32_t td = du + dvi;
                    if (su.x & v1) td -= 2;
                    else if ((su.x & v0) | (su.y & v1)) td -= 1;
                    bound = min(bound, td);
                }
            }
        }
        const uint64_t pr = ballot64(cand && bound <= j);
        if (lane == (uint32_t)w) out = pr;
    }
    return out;
}

// Gather phase of Algorithm 4 for round j: one wave per
// receiver.  Receiver i (in shard order) becomes slot i of the next active
// list (with an empty delta when nothing was accepted).
//
// BP (bit-parallel labels present) is a separate instantiation: the BP
// bound's registers would otherwise cost every build occupancy.
//
// FUSE: the wave of a receiver that accepted something also pushes its
// delta L for round j+1 right away (rows up to kHeavy; longer rows become
// heavy items for a separate launch), into the other message buffer nr->msgs
// and receiver queue nr->rout, whose entries go to nr->recv (this round's
// receivers are read from A.recv, so the two lists never share storage).
// C(r) of a neighbour may not hold this round's arrivals yet when the push
// reads it, so the check filters its messages by C(v) itself.  Receiver
// counters rotate over three (this round's nr->rin = p, the next round's,
// and nr->rclr, cleared here); active lists and heavy items use parity
// nr->hout.

template <int WM, bool BP = false, bool FUSE = false, bool QGATE = false, bool SMALLT = false>
__device__ inline void phase_check(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs, uint32_t j, uint32_t p,
                                   bool relaxed, PhaseStats& st, const NextRound* nr = nullptr) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t q = FUSE ? nr->hout : p ^ 1u;
    uint32_t pre;
    const uint32_t nrecv = shard_prefix(lane < X.nq ? X.qs[lane].recv[p] : 0u, pre);
    // clear the counts the next launch appends to
    if (X.zero_i < X.nq) {
        if (FUSE) {
            X.qs[X.zero_i].recv[nr->rclr] = 0;
            X.qs[X.zero_i].hq[q ^ 1u] = 0;
        } else {
            X.qs[X.zero_i].recv[q] = 0;
        }
    }
    for (uint32_t i = X.w; i < nrecv; i += X.nw) {
        const uint32_t s = shard_of(X.nq, pre, i);
        const uint32_t v = A.recv[(size_t)s * X.seg + (i - readlane32(pre, s))];
        uint64_t mine = 0;
        if (lane < W) {
            const size_t at = (size_t)v * W + lane;
            mine = A.msgs[at];
            A.msgs[at] = 0;
            if (FUSE) mine &= ~A.C[at];
            A.C[at] |= mine;
        }
        const uint32_t len = A.llen[v];
        uint64_t off = A.loff[v];
        uint64_t scan = mine;
        if (BP) {
            const uint64_t bpp = bp_prune_words<WM>(A, v, ib, j, mine);
            st.bp += __builtin_popcountll(lane < W ? bpp : 0ull);
            scan &= ~bpp;
        }
        // Round 1 never prunes: only an entry at distance 0, the self entry
        // (v, 0), could cover a candidate at distance 1, through T[v][k] <= 1,
        // i.e. with v a hub of u_k; but a candidate u_k only reaches vertices
        // ranked below it, and L(u_k) holds only hubs ranked above u_k.
        uint64_t pw = 0;
        if (j == 2 && A.nbr_hubs && A.rrow[v + 1] - A.rrow[v] < len)
            pw = prune_scan_nbrs<WM, QGATE, SMALLT>(A, v, min(v, relaxed ? ib : ib + bs), scan, st);
        else if (j > 1)
            pw = prune_scan<WM, QGATE, SMALLT>(A, off, len, j, scan, relaxed, ib, st);
        const uint64_t acc = lane < W ? (scan & ~pw) : 0ull;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(acc);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t total = readlane32(pos + cnt, 63);
        st.cand += __builtin_popcountll(mine);
        st.cost_pos += (unsigned long long)len * (uint32_t)__builtin_popcountll(acc);
        st.cost_neg += (unsigned long long)len * (uint32_t)__builtin_popcountll(mine & ~acc);
        // the active list: the fused rounds read a slot only for a vertex
        // that accepted (its heavy-row items and pulled rounds); the
        // unfused ones push from every slot
        if (!FUSE || total != 0) {
            if (lane == 0) A.act_v[q][i] = v;
            if (lane < W) A.act_delta[q][(size_t)i * W + lane] = acc;
        }
        if (total == 0) continue;
        if (j >= PLL_INF8) {
            if (lane == 0) atomicOr(&A.ctr->error, PLL_ERR_DIST);
            continue;
        }
        off = wave_reserve(A, X, v, off, len, total);
        if (off == ~0ull) continue;
        if (lane == 0) st.acc += total;
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
                    if (ib + k >= A.hot)
                        atomicOr((unsigned long long*)&A.rowmask[ib + k], 1ull << ((v - ib) >> 4));
                }
            }
        }
        if (lane == 0) A.llen[v] = len + total;
        if (FUSE && nr->pull) {  // the receivers gather: record where delta L(v) is
            if (lane == 0) {
                A.act_at[v] = ((uint64_t)nr->rstamp << 32) | i;
                st.pulled += A.rrow[v + 1] - A.rrow[v];
            }
            continue;
        }
        const uint64_t beg = A.rrow[v], end = A.rrow[v + 1];
        if (FUSE && end - beg <= kHeavy) {
            if (lane == 0) st.edges += end - beg;
            push_edges(A, X, nr->msgs, nr->recv, ib, nr->rout, nr->rstamp, nr->bstamp, acc, ballot64(acc != 0), beg,
                       end);
        } else {
            enqueue_heavy(A, X, q, i, end - beg);
        }
    }
}

// OR over each 16-lane row by DPP row rotations: every lane of a row gets
// its row's OR (the whole wave must be active).
__device__ inline uint32_t row_or32_dpp(uint32_t x) {
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x121, 0xf, 0xf, false);  // row_ror:1
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x122, 0xf, 0xf, false);  // row_ror:2
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xf, 0xf, false);  // row_ror:4
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xf, 0xf, false);  // row_ror:8
    return x;
}

__device__ inline uint64_t row_or64_dpp(uint64_t x) {
    return ((uint64_t)row_or32_dpp((uint32_t)(x >> 32)) << 32) | row_or32_dpp((uint32_t)x);
}

// Lane `src`'s x in every lane (the LDS crossbar; src may differ per lane).
__device__ inline uint64_t shfl64(uint64_t x, uint32_t src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src * 4u), (int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src * 4u), (int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The pruning scans of four receivers at once: group g = lane / 16 scans
// the list of its own receiver 16 entries at a time, and lane 16g + w holds
// word w (< W <= 16) of that receiver's candidates in cw.  The test is the
// one of prune_scan and prune_scan_nbrs, per group: the source is either
// L(v) (entries arena[off .. off+len)) or, with `nbr`, v's neighbour row
// (rcol[off .. off+len), hubs ranked below lim at distance 1).  Each chunk
// makes one pass per live candidate word of each group (the groups'
// passes run side by side), and each group OR-reduces its word's prunes
// within its 16-lane row.  A group stops after the chunk that leaves none
// of its candidates live, or at its list's end.  Returns, in lane 16g + w,
// the pruned candidates of word w of receiver g.
template <int WM, bool SMALLT>
__device__ inline uint64_t prune_scan4(const BuildArgs& A, uint64_t off, uint32_t len, bool nbr, uint32_t lim,
                                       uint32_t j, uint64_t cw, bool relaxed, uint32_t ib, PhaseStats& st) {
    const uint32_t lane = lane_id();
    const uint32_t sub = lane & 15u;
    const uint32_t gsh = lane & 48u;  // 16 * group
    const uint32_t* src = (nbr ? A.rcol : A.arena) + off;
    uint64_t pw = 0;
    uint32_t next = sub < len ? src[sub] : 0u;
    for (uint32_t base = 0;; base += 16) {
        const uint64_t live_lane = cw & ~pw;
        const uint64_t lb = ballot64(live_lane != 0);
        // this group still scans: candidates live and entries left
        const bool gon = ((lb >> gsh) & 0xFFFFull) != 0 && base < len;
        const uint64_t todo0 = ballot64(gon && live_lane != 0);
        if (!todo0) break;
        const uint32_t idx = base + sub;
        bool ok = gon && idx < len;
        st.read += ok;
        const uint32_t ent = next;
        next = gon && idx + 16 < len ? src[idx + 16] : 0u;
        uint32_t h, tt;
        if (nbr) {
            h = ent;
            ok = ok && h < lim;
            tt = seg_tt<SMALLT>(1u);  // T[h][k] <= 2 - 1
        } else {
            h = ent >> 8;
            const uint32_t d = ent & 255u;
            ok = ok && d < j;
            if (relaxed) ok = ok && h < ib;
            // at most 254, the largest finite table byte (see prune_scan)
            tt = ok ? seg_tt<SMALLT>(min(j - d, PLL_INF8 - 1u)) : 0u;
        }
        const uint64_t rm = ok ? A.rmchk[h] : 0ull;
        const uint8_t* row = A.Tchk + (size_t)(ok ? h : 0u) * A.bstride;
        uint64_t todo = todo0;
        while (todo) {
            const uint32_t gm = (uint32_t)(todo >> gsh) & 0xFFFFu;
            const bool act = gm != 0;
            const uint32_t w = act ? (uint32_t)__builtin_ctz(gm) : 0u;
            uint64_t m = 0;
            if (act && ((rm >> (4 * w)) & 15u)) {
                m = seg_le<SMALLT>(row + 64u * w, tt);
                st.table += 4;
            }
            // the lane that holds word w masks the group's OR with its live
            // candidates (the OR of masked words is the masked OR)
            const uint64_t red = row_or64_dpp(m);
            const bool here = act && sub == w;
            if (here) pw |= red & live_lane;
            todo &= ~ballot64(here);
        }
    }
    return pw;
}

// Inclusive prefix sum within each 16-lane row (DPP row shifts; lanes
// shifted in from outside the row add 0; the whole wave must be active).
__device__ inline uint32_t row_incl_scan32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
    return x;
}

// push_edges for up to four receivers of one wave at once: group g's delta
// words are in lanes 16g + w of acc4, and its row is rcol[beg .. beg + deg)
// (beg and deg held by the group's lanes; deg = 0 for a group that pushes
// nothing here).  The rows are walked as one concatenated range, 64 edges
// per step, each lane taking the delta of its edge's receiver; deliveries
// and receiver slots are those of push_edges.
__device__ inline void push_edges4(const BuildArgs& A, const Exec& X, const NextRound& nr, uint32_t ib, uint64_t acc4,
                                   uint64_t beg, uint32_t deg) {
    const uint32_t lane = lane_id();
    // starts of groups 1..3 in the concatenation, and its length
    const uint32_t s1 = readlane32(deg, 0);
    const uint32_t s2 = s1 + readlane32(deg, 16);
    const uint32_t s3 = s2 + readlane32(deg, 32);
    const uint32_t D = s3 + readlane32(deg, 48);
    const uint64_t b0 = readlane64(beg, 0), b1 = readlane64(beg, 16), b2 = readlane64(beg, 32),
                   b3 = readlane64(beg, 48);
    // bit 16g + w: group g has a delta in word w
    const uint64_t nzl = ballot64(acc4 != 0);
    for (uint32_t t0 = 0; t0 < D; t0 += 64) {
        const uint32_t t = t0 + lane;
        // the last group whose start is <= t (empty groups share the next one's start)
        const uint32_t gl = (uint32_t)(t >= s1) + (uint32_t)(t >= s2) + (uint32_t)(t >= s3);
        const uint64_t bg = gl == 0 ? b0 : gl == 1 ? b1 : gl == 2 ? b2 : b3;
        const uint32_t sg = gl == 0 ? 0u : gl == 1 ? s1 : gl == 2 ? s2 : s3;
        const bool in = t < D;
        const uint32_t r = in ? A.rcol[bg + (t - sg)] : 0u;
        const bool fwd = in && r > ib;
        const uint32_t rel = r - ib;
        bool any = false;
        // the nonzero words of this edge's receiver, four at a time
        uint32_t todo = fwd ? (uint32_t)(nzl >> (16u * gl)) & 0xFFFFu : 0u;
        while (ballot64(todo != 0)) {
            uint32_t w[4];
            uint64_t m[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = todo ? (uint32_t)__builtin_ctz(todo) : 0u;
                const uint64_t x = shfl64(acc4, 16u * gl + w[k]);
                m[k] = todo ? x & rank_mask(rel, w[k]) : 0ull;
                todo &= todo - 1;
            }
            any |= deliver4(A, nr.msgs, r, w, m);
        }
        enqueue_receivers(A, X, nr.recv, nr.rout, nr.rstamp, nr.bstamp, r, any);
    }
}

// The fused check (FUSE of phase_check, without bit-parallel labels) with
// four receivers per wave: receivers i0 .. i0+3 are read and scanned side by
// side by the four 16-lane groups (prune_scan4), so four receivers' chains
// of dependent loads (receiver, list, label chunk, row mask, table segment)
// are in flight in one wave.  The accepted entries are then appended one
// receiver after another, and the next round's deliveries of all four go
// out in one pass over their concatenated rows (push_edges4).  Active-list
// slots, heavy rows, pulled rounds and statistics are phase_check's.
template <int WM, bool SMALLT>
__device__ inline void phase_check4(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs, uint32_t j,
                                    bool relaxed, PhaseStats& st, const NextRound& nr) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t sub = lane & 15u, g = lane >> 4;
    const uint32_t q = nr.hout;
    uint32_t pre;
    const uint32_t nrecv = shard_prefix(lane < X.nq ? X.qs[lane].recv[nr.rin] : 0u, pre);
    // clear the counts the next launch appends to
    if (X.zero_i < X.nq) {
        X.qs[X.zero_i].recv[nr.rclr] = 0;
        X.qs[X.zero_i].hq[q ^ 1u] = 0;
    }
    for (uint32_t i0 = 4u * X.w; i0 < nrecv; i0 += 4u * X.nw) {
        const uint32_t ng = min(4u, nrecv - i0);
        uint32_t slot = 0;
        for (uint32_t gg = 0; gg < ng; ++gg) {
            const uint32_t s = shard_of(X.nq, pre, i0 + gg);
            const uint32_t at = s * X.seg + (i0 + gg - readlane32(pre, s));
            if (g == gg) slot = at;
        }
        const bool has = g < ng;
        const uint32_t i = i0 + g;
        const uint32_t v = has ? A.recv[slot] : 0u;
        uint64_t mine = 0;
        if (has && sub < W) {
            const size_t at = (size_t)v * W + sub;
            mine = A.msgs[at];
            A.msgs[at] = 0;
            mine &= ~A.C[at];
            A.C[at] |= mine;
        }
        const uint32_t len = has ? A.llen[v] : 0u;
        const uint64_t off = has ? A.loff[v] : 0ull;
        // round 1 never prunes (see phase_check); round 2 reads the
        // neighbour row when it is the shorter source
        uint64_t pw = 0;
        if (j > 1) {
            bool nbr = false;
            uint64_t soff = off;
            uint32_t slen = len, lim = 0;
            if (j == 2 && A.nbr_hubs && has) {
                const uint64_t rb = A.rrow[v], re = A.rrow[v + 1];
                if (re - rb < len) {
                    nbr = true;
                    soff = rb;
                    slen = (uint32_t)(re - rb);
                    lim = min(v, relaxed ? ib : ib + bs);
                }
            }
            pw = prune_scan4<WM, SMALLT>(A, soff, slen, nbr, lim, j, mine, relaxed, ib, st);
        }
        const uint64_t acc4 = mine & ~pw;
        st.cand += __builtin_popcountll(mine);
        st.cost_pos += (unsigned long long)len * (uint32_t)__builtin_popcountll(acc4);
        st.cost_neg += (unsigned long long)len * (uint32_t)__builtin_popcountll(mine & ~acc4);
        const uint64_t accl = ballot64(acc4 != 0);
        if (!accl) continue;  // nothing accepted: no slots, no pushes
        const bool gacc = ((accl >> (lane & 48u)) & 0xFFFFull) != 0;
        if (gacc) {  // the active-list slot of a receiver that accepted
            if (sub == 0) A.act_v[q][i] = v;
            if (sub < W) A.act_delta[q][(size_t)i * W + sub] = acc4;
        }
        if (j >= PLL_INF8) {
            if (lane == 0) atomicOr(&A.ctr->error, PLL_ERR_DIST);
            continue;
        }
        // entries of each word before it, within each receiver's candidates
        const uint32_t incl = row_incl_scan32((uint32_t)__builtin_popcountll(acc4));
        uint32_t appended = 0;  // bit gg: receiver gg's entries are in its list
        for (uint32_t gg = 0; gg < ng; ++gg) {
            uint64_t todo = (accl >> (16u * gg)) & 0xFFFFull;
            if (!todo) continue;
            const uint32_t vg = readlane32(v, 16u * gg);
            const uint32_t lg = readlane32(len, 16u * gg);
            const uint32_t total = readlane32(incl, 16u * gg + 15u);
            const uint64_t og = wave_reserve(A, X, vg, readlane64(off, 16u * gg), lg, total);
            if (og == ~0ull) continue;
            if (lane == 0) st.acc += total;
            const bool in_batch = vg - ib < bs;
            const uint64_t lt = lanemask_lt();
            while (todo) {
                const uint32_t w = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1;
                const uint64_t aw = readlane64(acc4, 16u * gg + w);
                const uint32_t pwos = readlane32(incl, 16u * gg + w) - (uint32_t)__builtin_popcountll(aw);
                if ((aw >> lane) & 1ull) {
                    const uint32_t k = w * 64u + lane;
                    A.arena[og + lg + pwos + __builtin_popcountll(aw & lt)] = pll_pack(ib + k, j);
                    if (in_batch) {
                        A.T[(size_t)(ib + k) * A.bstride + (vg - ib)] = (uint8_t)j;
                        if (ib + k >= A.hot)
                            atomicOr((unsigned long long*)&A.rowmask[ib + k], 1ull << ((vg - ib) >> 4));
                    }
                }
            }
            if (lane == 0) A.llen[vg] = lg + total;
            appended |= 1u << gg;
        }
        // round j+1: pulled (record where delta L(v) is) or pushed along the
        // rows, those longer than kHeavy as heavy items of a separate launch
        const bool out = (appended >> g) & 1u;
        uint64_t rb = 0;
        uint32_t deg = 0;
        if (out) {
            rb = A.rrow[v];
            deg = (uint32_t)(A.rrow[v + 1] - rb);
        }
        if (nr.pull) {
            if (out && sub == 0) {
                A.act_at[v] = ((uint64_t)nr.rstamp << 32) | i;
                st.pulled += deg;
            }
            continue;
        }
        const bool heavy = deg > kHeavy;
        if (out && !heavy && sub == 0) st.edges += deg;
        uint64_t hv = ballot64(out && heavy && sub == 0);
        while (hv) {
            const uint32_t l = (uint32_t)__builtin_ctzll(hv);
            hv &= hv - 1;
            enqueue_heavy(A, X, q, i0 + l / 16u, readlane32(deg, l));
        }
        push_edges4(A, X, nr, ib, acc4, rb, out && !heavy ? deg : 0u);
    }
}

// Batch end, one wave per touched vertex v: clear C(v); sort the
// entries this batch appended to L(v) by hub rank; with `recheck`, first
// drop every such entry (u, d) that L(u) and L(v) already cover through
// another hub at distance <= d (Section 5.1's recheck with the batch's
// tables still in memory).  s_pres (W words) and s_dist (b bytes) are this
// wave's LDS scratch.
//
// Weighted graphs (WEIGHTED): the recheck always runs (it is what makes the
// labels canonical there), D(v) is reset instead of C(v), and a hub may
// appear several times in the batch segment, each later entry shorter than
// the one before; only the last one is kept (s_pos, b words of LDS, holds
// the position of each hub's last entry).
template <int WM, bool WEIGHTED = false>
__device__ inline void phase_batch_end(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs, bool recheck,
                                       uint64_t* s_pres, uint8_t* s_dist, uint32_t* s_pos, PhaseStats& st) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    if (WEIGHTED) recheck = true;
    uint32_t pre;
    const uint32_t ntouched = shard_prefix(lane < X.nq ? X.qs[lane].touched : 0u, pre);
    for (uint32_t i = X.w; i < ntouched; i += X.nw) {
        const uint32_t sh = shard_of(X.nq, pre, i);
        const size_t at = (size_t)sh * X.seg + (i - readlane32(pre, sh));
        const uint32_t v = A.touched[at];
        const uint32_t ts = A.tstart[at];
        const uint32_t len = A.llen[v];
        const uint64_t off = A.loff[v];
        if (WEIGHTED) {
            uint4* drow = reinterpret_cast<uint4*>(A.D + (size_t)v * A.bstride);
            for (uint32_t c = lane; c < 4 * W; c += 64) drow[c] = make_uint4(~0u, ~0u, ~0u, ~0u);
        } else if (lane < W) {
            A.C[(size_t)v * W + lane] = 0;
        }
        const uint32_t tail = len - ts;
        if (tail < 2 && !(recheck && tail >= 1)) continue;
        // A segment appended in one round is already in ascending hub rank
        // (each acceptance appends its candidates in ascending order): without
        // the recheck, a segment of up to 64 entries that is sorted stays.
        if (!recheck && tail <= 64) {
            const uint32_t e = lane < tail ? A.arena[off + ts + lane] : ~0u;
            const uint32_t nx = (uint32_t)__shfl_down((int)e, 1, 64);
            if (!ballot64(lane + 1 < tail && e >= nx)) continue;
        }
        if (lane < W) s_pres[lane] = 0;
        if (WEIGHTED) {
            for (uint32_t k = lane; k < bs; k += 64) s_pos[k] = 0;
            wave_lds_sync();
            for (uint32_t x = ts + lane; x < len; x += 64) atomicMax(&s_pos[(A.arena[off + x] >> 8) - ib], x - ts + 1);
        }
        wave_lds_sync();
        for (uint32_t x = ts + lane; x < len; x += 64) {
            const uint32_t e = A.arena[off + x];
            const uint32_t k = (e >> 8) - ib;
            if (WEIGHTED && s_pos[k] != x - ts + 1) continue;
            s_dist[k] = (uint8_t)(e & 255u);
            atomicOr((unsigned long long*)&s_pres[k >> 6], 1ull << (k & 63));
        }
        wave_lds_sync();
        if (recheck) {
            const bool in_batch = v - ib < bs;
            uint32_t prev = 0;
            for (;;) {
                uint32_t mn = PLL_INF8;
                for (uint32_t k = lane; k < bs; k += 64) {
                    const uint32_t d = s_dist[k];
                    if (((s_pres[k >> 6] >> (k & 63)) & 1ull) && d > prev) mn = min(mn, d);
                }
                mn = wave_min32(mn);
                if (mn == PLL_INF8) break;
                uint64_t cw = 0;
                if (lane < W) {
                    const uint64_t pw = s_pres[lane];
                    for (uint32_t bit = 0; bit < 64; ++bit) {
                        const uint32_t k = lane * 64u + bit;
                        if (((pw >> bit) & 1ull) && s_dist[k] == mn) cw |= 1ull << bit;
                    }
                }
                const uint64_t pr = prune_scan<WM>(A, off, len, mn, cw, false, ib, st);
                if (lane < W && pr) s_pres[lane] &= ~pr;
                st.removed += __builtin_popcountll(pr);
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
        const uint64_t pw = lane < W ? s_pres[lane] : 0ull;
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
                A.arena[off + ts + base + __builtin_popcountll(aw & lanemask_lt())] = pll_pack(ib + k, s_dist[k]);
            }
        }
        if (lane == 0 && total != tail) A.llen[v] = ts + total;
        wave_lds_sync();
    }
}

// ---- weighted graphs (Section 5.1) ----------------------------------------------------------------
//
// A candidate now carries its own distance d + w_e, and a round no longer
// equals a distance: a candidate can come back shorter in a later round.
// D(v) replaces C(v) as the filter (a candidate passes only if it lowers
// D(v)[k]); the pruning check compares each candidate with its own
// distance; a vertex that accepts pushes the entries it accepted (its
// delta L) rather than a bit-vector.  Entries accepted on the way may be
// non-canonical; the batch-end recheck removes them.

// Per byte: min(x + d, 255) with dd = d * 0x01010101.  The low 7 bits of
// each byte are added without carries leaving the byte; the carry out of
// bit 7 marks the bytes that saturate.
__device__ inline uint32_t add_sat4(uint32_t x, uint32_t dd) {
    const uint32_t H = 0x80808080u;
    const uint32_t low = (x & ~H) + (dd & ~H);
    const uint32_t sum = low ^ ((x ^ dd) & H);
    const uint32_t ovf = ((x & dd) | ((x | dd) & ~sum)) & H;
    return sum | ((ovf >> 7) * 0xFFu);
}

// Bit i: min(p[i] + d, 255) <= thr[i], for 64 consecutive table bytes p and
// thresholds thr (le4_flags compares bytes against any per-byte threshold).
__device__ inline uint64_t sum_le_mask64(const uint8_t* p, uint32_t dd, const uint4* thr) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint4 v = q[i];
        const uint4 t = thr[i];
        const uint32_t b = gather16(le4_flags(add_sat4(v.x, dd), t.x), le4_flags(add_sat4(v.y, dd), t.y),
                                    le4_flags(add_sat4(v.z, dd), t.z), le4_flags(add_sat4(v.w, dd), t.w));
        m |= (uint64_t)b << (16 * i);
    }
    return m;
}

// prune_scan with a distance per candidate: s_thr (LDS, 64 * W bytes) holds
// D(v); candidate u_k is pruned when some entry (h, d) of the list has
// T[h][k] + d <= D(v)[k].  Lanes beyond the live candidates are masked off,
// so bytes of 255 (no candidate) never count.
template <int WM>
__device__ inline uint64_t prune_scan_w(const BuildArgs& A, uint64_t off, uint32_t len, uint64_t cw,
                                        const uint4* s_thr, PhaseStats& st) {
    const uint32_t lane = lane_id();
    uint64_t pw = 0;
    uint64_t accm[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) accm[w] = 0;
    uint32_t chunk = 0;
    for (uint32_t base = 0; base < len; base += 64, ++chunk) {
        const uint32_t idx = base + lane;
        const bool ok = idx < len;
        st.read += ok;
        const uint32_t ent = ok ? A.arena[off + idx] : 0u;
        const uint32_t h = ent >> 8;
        const uint64_t rm = ok ? A.rmchk[h] : 0ull;
        const uint32_t dd = (ent & 255u) * 0x01010101u;
        const uint8_t* row = A.Tchk + (size_t)h * A.bstride;
        const uint64_t live_lane = cw & ~pw;
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            const uint64_t live = readlane64(live_lane, w);
            if (live != 0 && ((rm >> (4 * w)) & 15u)) {
                accm[w] |= sum_le_mask64(row + 64u * w, dd, s_thr + 4 * w) & live;
                st.table += 4;
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

// D[p] = min(D[p], nd) on one byte (a compare-and-swap on its aligned word);
// true when this call lowered it.
__device__ inline bool byte_atomic_min(uint8_t* p, uint32_t nd) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    uint32_t* wp = reinterpret_cast<uint32_t*>(a & ~uintptr_t(3));
    const uint32_t sh = (uint32_t)(a & 3u) * 8u;
    uint32_t old = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (nd >= ((old >> sh) & 255u)) return false;
        const uint32_t nw = (old & ~(255u << sh)) | (nd << sh);
        const uint32_t prev = atomicCAS(wp, old, nw);
        if (prev == old) return true;
        old = prev;
    }
}

// Push the cnt entries at arena[eoff ..] (what the active vertex accepted
// last round) along its weighted CSR entries [beg, end).
__device__ inline void push_edges_w(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t p, uint32_t rstamp,
                                    uint32_t bstamp, uint64_t eoff, uint32_t cnt, uint64_t beg, uint64_t end) {
    const uint32_t lane = lane_id();
    for (uint64_t e0 = beg; e0 < end; e0 += 64) {
        const uint64_t e = e0 + lane;
        const bool in = e < end;
        const uint32_t r = in ? A.rcol[e] : 0u;
        const uint32_t wt = in ? A.rw[e] : 0u;
        const bool cand = in && r > ib;
        bool any = false, over = false;
        if (ballot64(cand)) {
            for (uint32_t t = 0; t < cnt; ++t) {
                const uint32_t ent = A.arena[eoff + t];
                const uint32_t k = (ent >> 8) - ib;
                const uint32_t nd = (ent & 255u) + wt;
                if (cand && r - ib > k) {  // only to vertices ranked below u_k
                    uint8_t* pd = A.D + (size_t)r * A.bstride + k;
                    if (nd >= PLL_INF8) {
                        // too long for the labels; harmless when a shorter
                        // candidate already reached r, else the build fails
                        over = over || *pd == PLL_INF8;
                    } else {
                        if (nd < *pd && byte_atomic_min(pd, nd)) {
                            atomicOr((unsigned long long*)&A.msgs[(size_t)r * A.W + (k >> 6)],
                                     (unsigned long long)(1ull << (k & 63)));
                            any = true;
                        }
                    }
                }
            }
        }
        if (ballot64(over) && lane == 0) atomicOr(&A.ctr->error, PLL_ERR_DIST);
        bool enq = false;
        if (any && A.recv_stamp[r] != rstamp) enq = atomicExch(&A.recv_stamp[r], rstamp) != rstamp;
        bool first = false;
        if (enq && A.touch_stamp[r] != bstamp) {
            A.touch_stamp[r] = bstamp;
            first = true;
        }
        if (ballot64(enq)) {
            const uint32_t rp = shard_append(&X.qs[X.my].recv[p], enq, (uint64_t)X.my * X.seg);
            if (enq) A.recv[rp] = r;
            const uint32_t tp = shard_append(&X.qs[X.my].touched, first, (uint64_t)X.my * X.seg);
            if (first) {
                A.touched[tp] = r;
                A.tstart[tp] = A.llen[r];
            }
        }
    }
}

// Scatter phase for weighted graphs over active list p.
__device__ inline void phase_push_w(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t p, uint32_t nact,
                                    uint32_t rstamp, uint32_t bstamp, PhaseStats& st) {
    const uint32_t lane = lane_id();
    if (X.zero_i < X.nq) X.qs[X.zero_i].hq[p ^ 1u] = 0;
    for (uint32_t i = X.w; i < nact; i += X.nw) {
        const uint2 rg = A.act_rng[p][i];
        if (rg.y == 0) continue;
        const uint32_t a = A.act_v[p][i];
        const uint64_t beg = A.rrow[a], end = A.rrow[a + 1];
        if (end - beg > kHeavy) continue;
        if (lane == 0) st.edges += end - beg;
        push_edges_w(A, X, ib, p, rstamp, bstamp, A.loff[a] + rg.x, rg.y, beg, end);
    }
    uint32_t pre;
    const uint32_t nh = shard_prefix(lane < X.nq ? X.qs[lane].hq[p] : 0u, pre);
    for (uint32_t t = X.w; t < nh; t += X.nw) {
        const uint32_t s = shard_of(X.nq, pre, t);
        const uint2 item = A.hq[p][s * A.hq_seg + (t - readlane32(pre, s))];
        const uint2 rg = A.act_rng[p][item.x];
        const uint32_t a = A.act_v[p][item.x];
        const uint64_t beg = A.rrow[a] + (uint64_t)item.y * kHeavyItem;
        const uint64_t end = min(A.rrow[a + 1], beg + kHeavyItem);
        if (lane == 0) st.edges += end - beg;
        push_edges_w(A, X, ib, p, rstamp, bstamp, A.loff[a] + rg.x, rg.y, beg, end);
    }
}

// Gather phase for weighted graphs: the candidates of receiver v are the
// bits of msgs(v); candidate u_k has distance D(v)[k], staged in this
// wave's LDS s_thr (64 * W bytes).  Survivors are appended with that
// distance (a hub may already hold a longer entry from an earlier round;
// the batch end keeps the last one); the slot records where they start.
template <int WM>
__device__ inline void phase_check_w(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs, uint32_t p,
                                     uint4* s_thr, PhaseStats& st) {
    const uint32_t lane = lane_id();
    const uint32_t W = A.W;
    const uint32_t q = p ^ 1u;
    uint32_t pre;
    const uint32_t nrecv = shard_prefix(lane < X.nq ? X.qs[lane].recv[p] : 0u, pre);
    if (X.zero_i < X.nq) X.qs[X.zero_i].recv[q] = 0;
    const uint8_t* thr_bytes = reinterpret_cast<const uint8_t*>(s_thr);
    for (uint32_t i = X.w; i < nrecv; i += X.nw) {
        const uint32_t s = shard_of(X.nq, pre, i);
        const uint32_t v = A.recv[(size_t)s * X.seg + (i - readlane32(pre, s))];
        uint64_t mine = 0;
        if (lane < W) {
            const size_t at = (size_t)v * W + lane;
            mine = A.msgs[at];
            A.msgs[at] = 0;
        }
        const uint4* drow = reinterpret_cast<const uint4*>(A.D + (size_t)v * A.bstride);
        for (uint32_t c = lane; c < 4 * W; c += 64) s_thr[c] = drow[c];
        wave_lds_sync();
        const uint32_t len = A.llen[v];
        uint64_t off = A.loff[v];
        const uint64_t pw = prune_scan_w<WM>(A, off, len, mine, s_thr, st);
        const uint64_t acc = lane < W ? (mine & ~pw) : 0ull;
        const uint32_t cnt = (uint32_t)__builtin_popcountll(acc);
        const uint32_t pos = wave_excl_scan32(cnt);
        const uint32_t total = readlane32(pos + cnt, 63);
        st.cand += __builtin_popcountll(mine);
        st.cost_pos += (unsigned long long)len * (uint32_t)__builtin_popcountll(acc);
        st.cost_neg += (unsigned long long)len * (uint32_t)__builtin_popcountll(mine & ~acc);
        if (lane == 0) {
            A.act_v[q][i] = v;
            A.act_rng[q][i] = make_uint2(len, total);
        }
        if (total != 0) {
            off = wave_reserve(A, X, v, off, len, total);
            if (off != ~0ull) {
                if (lane == 0) st.acc += total;
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
                        const uint32_t dk = thr_bytes[k];
                        A.arena[off + len + pwos + __builtin_popcountll(aw & lt)] = pll_pack(ib + k, dk);
                        if (in_batch) {
                            A.T[(size_t)(ib + k) * A.bstride + (v - ib)] = (uint8_t)dk;
                            atomicOr((unsigned long long*)&A.rowmask[ib + k], 1ull << ((v - ib) >> 4));
                        }
                    }
                }
                if (lane == 0) A.llen[v] = len + total;
                enqueue_heavy(A, X, q, i, A.rrow[v + 1] - A.rrow[v]);
            } else if (lane == 0) {
                A.act_rng[q][i] = make_uint2(len, 0u);
            }
        }
        wave_lds_sync();
    }
}

// Reset the distance table rows written during the batch.
__device__ inline void phase_clear_table(const BuildArgs& A, const Exec& X, uint32_t ib, uint32_t bs) {
    const uint32_t lane = lane_id();
    // four waves per root: task t clears the 64-entry chunks c, c + 4, ...
    // of root k (t = 4k + c)
    for (uint32_t t = X.w; t < 4u * bs; t += X.nw) {
        const uint32_t k = t >> 2, c = t & 3u;
        const uint32_t u = ib + k;
        const uint32_t len = A.llen[u];
        const uint64_t off = A.loff[u];
        for (uint32_t i = 64u * c + lane; i < len; i += 256u) {
            const uint32_t h = A.arena[off + i] >> 8;
            A.T[(size_t)h * A.bstride + k] = (uint8_t)PLL_INF8;
            if (h >= A.hot) A.rowmask[h] = 0;
        }
        if (c == 0 && lane == 0 && u >= A.hot) A.rowmask[u] = 0;
    }
}

}  // namespace pll
