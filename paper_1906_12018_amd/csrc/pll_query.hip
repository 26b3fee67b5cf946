// Batched exact distance queries (the 2-hop query of Section 2.1):
// Dis(u,v) = min over common hubs h of d(u,h) + d(h,v), found by merging the
// two hub-rank-sorted label lists.  Labels are packed (hub rank << 8) | dist.
//
// Three kernels:
//  * k_query_lane: one lane per pair, a scalar two-pointer merge.  Kept for
//    tiny labels and as the simplest form of the operation.
//  * k_query_wave (64 lanes per pair): one pair per wave, the lists merged in
//    merge-path tiles staged in LDS (described below, before the kernel).
//  * k_query_group<G> (G = 4..32): G lanes per pair merge the lists window
//    by window.  A
//    u-window is 2G consecutive entries of L(u) and a v-window 4G entries of
//    L(v), read as one aligned 8- or 16-byte load per lane (label arrays are
//    padded to whole 4-entry chunks).  The v-window is published in LDS;
//    every valid u-entry binary-searches it for its hub, and the window whose
//    last list entry has the smaller hub moves on (both when equal).  Every
//    common hub lies in a pair of windows that meet: a window only moves on
//    once every entry of the other list that could match it has been seen,
//    and once the window holding a list's end moves on the pair is done, so
//    neither list is read past the point where the sequential merge stops.
//    The pair's minimum is reduced across the group at the end.
// For a directed index (Section 5.1) the distance from u to v merges
// L_out(u) with L_in(v); the kernels take the two lists' arrays apart.
// With bit-parallel labels (Section 5.2) the answer is the smaller of the
// merge and the BP bound; the group's lanes split the BP roots.
#include <atomic>

#include "pll_internal.h"

namespace {

constexpr int kBlock = 256;

// Bit-parallel bound of (u, v) over BP roots i = first, first + step, ...
// (Section 5.2): d_i(u) + d_i(v), minus 2 when the S^-1 sets meet, else
// minus 1 when S^-1 of one meets S^0 of the other.
__device__ inline uint32_t bp_bound(const uint8_t* __restrict__ bpd, const ulonglong2* __restrict__ bps, uint32_t t,
                                    uint32_t u, uint32_t v, uint32_t first, uint32_t step) {
    uint32_t best = PLL_DIST_INF;
    for (uint32_t i = first; i < t; i += step) {
        const uint32_t du = bpd[(size_t)u * t + i], dv = bpd[(size_t)v * t + i];
        if (du == PLL_INF8 || dv == PLL_INF8) continue;
        const ulonglong2 su = bps[(size_t)u * t + i], sv = bps[(size_t)v * t + i];
        uint32_t td = du + dv;
        if (su.x & sv.x) td -= 2;
        else if ((su.x & sv.y) | (su.y & sv.x)) td -= 1;
        best = min(best, td);
    }
    return best;
}
constexpr uint32_t kAfter = 0xFFFFFFFFu;  // sorts after every key

template <bool BP>
__global__ void __launch_bounds__(kBlock) k_query_lane(const uint64_t* __restrict__ offu,
                                                       const uint32_t* __restrict__ entu,
                                                       const uint64_t* __restrict__ offv,
                                                       const uint32_t* __restrict__ entv, uint32_t n, uint64_t count,
                                                       const uint32_t* __restrict__ qu,
                                                       const uint32_t* __restrict__ qv, uint32_t* __restrict__ out,
                                                       const uint8_t* __restrict__ bpd,
                                                       const ulonglong2* __restrict__ bps, uint32_t bpt) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = qu[i], v = qv[i];
        uint32_t best = PLL_DIST_INF;
        uint64_t a = 0, ae = 0, b = 0, be = 0;
        if (u < n && v < n) {  // an id out of range has no label: no common hub
            a = offu[u];
            ae = offu[u + 1];
            b = offv[v];
            be = offv[v + 1];
        }
        if (a < ae && b < be) {
            uint32_t ea = entu[a], eb = entv[b];
            for (;;) {
                const uint32_t ha = ea >> 8, hb = eb >> 8;
                if (ha == hb) {
                    best = min(best, (ea & 255u) + (eb & 255u));
                    if (++a == ae || ++b == be) break;
                    ea = entu[a];
                    eb = entv[b];
                } else if (ha < hb) {
                    if (++a == ae) break;
                    ea = entu[a];
                } else {
                    if (++b == be) break;
                    eb = entv[b];
                }
            }
        }
        if (BP && u < n && v < n) best = min(best, bp_bound(bpd, bps, bpt, u, v, 0, 1));
        out[i] = best;
    }
}

// Lane gl's E entries of a window of E*G entries starting at w (w aligned to
// E entries, so the load is one aligned 4E-byte load), as sortable keys: an
// entry becomes ((hub rank + 1) << 8) | dist, window positions before lo
// become 0 and positions at or after hi become kAfter, so the window stays
// sorted.  Positions are relative to the window start.
template <int E>
__device__ __forceinline__ void load_window(const uint32_t* __restrict__ w, int32_t lo, int32_t hi, uint32_t gl,
                                            uint32_t k[E]) {
    static_assert(E == 2 || E == 4, "entries per lane");
    const int32_t c = E * (int32_t)gl;
    uint32_t raw[E];
#pragma unroll
    for (int j = 0; j < E; ++j) raw[j] = kAfter;
    if (c < hi) {
        if constexpr (E == 4) {
            const uint4 x = *reinterpret_cast<const uint4*>(w + c);
            raw[0] = x.x;
            raw[1] = x.y;
            raw[2] = x.z;
            raw[3] = x.w;
        } else {
            const uint2 x = *reinterpret_cast<const uint2*>(w + c);
            raw[0] = x.x;
            raw[1] = x.y;
        }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int32_t q = c + j;
        k[j] = q < lo ? 0u : (q >= hi ? kAfter : raw[j] + 256u);
    }
}

// k[j] for a group-uniform j.
template <int E>
__device__ __forceinline__ uint32_t pick(const uint32_t k[E], int32_t j) {
    uint32_t t = k[0];
#pragma unroll
    for (int i = 1; i < E; ++i) t = j == i ? k[i] : t;
    return t;
}

// Values shared by a group; with one pair per wave they are wave-uniform and
// kept in scalar registers.
template <int G>
__device__ __forceinline__ uint32_t group_uniform(uint32_t x) {
    if constexpr (G == 64)
        return __builtin_amdgcn_readfirstlane(x);
    else
        return x;
}

template <int G>
__device__ __forceinline__ uint64_t group_uniform(uint64_t x) {
    if constexpr (G == 64)
        return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)x);
    else
        return x;
}

// u-windows hold 2 entries per lane and v-windows 4: each lane binary-searches
// two u-keys in the 4G-entry v-window per step (fewer keys per step cost less
// VALU work than four; measured best on both R-MAT scales).
constexpr int kEntriesU = 2;
constexpr int kEntriesV = 4;

template <int G, bool BP>
__global__ void __launch_bounds__(kBlock) k_query_group(const uint64_t* __restrict__ offu,
                                                        const uint32_t* __restrict__ entu,
                                                        const uint64_t* __restrict__ offv,
                                                        const uint32_t* __restrict__ entv, uint32_t n, uint64_t count,
                                                        const uint32_t* __restrict__ qu,
                                                        const uint32_t* __restrict__ qv, uint32_t* __restrict__ out,
                                                        const uint8_t* __restrict__ bpd,
                                                        const ulonglong2* __restrict__ bps, uint32_t bpt) {
    static_assert(G >= 4 && G <= 64 && (G & (G - 1)) == 0, "group size");
    constexpr int32_t kWinU = kEntriesU * G, kWinV = kEntriesV * G;
    __shared__ uint4 s_win[kBlock];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gl = lane & (G - 1);
    const uint32_t gfirst = lane & ~(uint32_t)(G - 1);
    const uint32_t* win = reinterpret_cast<const uint32_t*>(s_win + (threadIdx.x & ~(uint32_t)(G - 1)));
    const uint64_t stride = (uint64_t)gridDim.x * (kBlock / G);
    for (uint64_t p = group_uniform<G>(blockIdx.x * (uint64_t)(kBlock / G) + threadIdx.x / G); p < count;
         p += stride) {
        const uint32_t u = qu[p], v = qv[p];
        uint64_t a = 0, ae = 0, b = 0, be = 0;
        if (u < n && v < n) {  // an id out of range has no label: no common hub
            a = offu[u];
            ae = offu[u + 1];
            b = offv[v];
            be = offv[v + 1];
        }
        uint32_t best = PLL_DIST_INF;
        // windows: base pointers aligned to the entries per lane; list bounds
        // relative to the window start (lists are shorter than 2^31 entries)
        constexpr uint64_t kAlignU = kEntriesU - 1, kAlignV = kEntriesV - 1;
        const uint32_t* wa = entu + (a & ~kAlignU);
        const uint32_t* wb = entv + (b & ~kAlignV);
        int32_t a_lo = (int32_t)(a & kAlignU), a_hi = (int32_t)(ae - (a & ~kAlignU));
        int32_t b_lo = (int32_t)(b & kAlignV), b_hi = (int32_t)(be - (b & ~kAlignV));
        if (!(a < ae && b < be)) a_hi = 0;  // an empty list: no common hub
        uint32_t ka[kEntriesU], kb[kEntriesV];
        if (a_hi > 0) {
            load_window<kEntriesU>(wa, a_lo, a_hi, gl, ka);
            load_window<kEntriesV>(wb, b_lo, b_hi, gl, kb);
        }
        while (a_hi > 0 && b_hi > 0) {  // uniform over the group
            a_lo = (int32_t)group_uniform<G>((uint32_t)a_lo);
            a_hi = (int32_t)group_uniform<G>((uint32_t)a_hi);
            b_lo = (int32_t)group_uniform<G>((uint32_t)b_lo);
            b_hi = (int32_t)group_uniform<G>((uint32_t)b_hi);
            s_win[threadIdx.x] = make_uint4(kb[0], kb[1], kb[2], kb[3]);
            // hub of the last list entry inside each window
            const int32_t la = min(a_hi, kWinU) - 1, lb = min(b_hi, kWinV) - 1;
            const uint32_t ta = pick<kEntriesU>(ka, la % kEntriesU), tb = pick<kEntriesV>(kb, lb % kEntriesV);
            const uint32_t last_a = (uint32_t)__shfl((int)ta, (int)(gfirst + la / kEntriesU)) >> 8;
            const uint32_t last_b = (uint32_t)__shfl((int)tb, (int)(gfirst + lb / kEntriesV)) >> 8;
            wave_lds_sync();
            // lower bound of each u-key in the v-window; the searches advance
            // together so their LDS reads overlap
            uint32_t key[kEntriesU], pos[kEntriesU];
#pragma unroll
            for (int j = 0; j < kEntriesU; ++j) {
                key[j] = ka[j] & ~255u;
                pos[j] = 0;
            }
#pragma unroll
            for (int32_t step = kWinV / 2; step >= 1; step >>= 1) {
                uint32_t probe[kEntriesU];
#pragma unroll
                for (int j = 0; j < kEntriesU; ++j) probe[j] = win[pos[j] + step - 1];
#pragma unroll
                for (int j = 0; j < kEntriesU; ++j) pos[j] += probe[j] < key[j] ? step : 0;
            }
            // a hit needs a valid u-key (not a 0 or kAfter filler), the same
            // hub, and a position inside the v list
#pragma unroll
            for (int j = 0; j < kEntriesU; ++j) {
                const uint32_t w = win[pos[j]];
                const int32_t q = kEntriesU * (int32_t)gl + j;
                const bool hit = q >= a_lo && q < a_hi && (int32_t)pos[j] < b_hi && (w >> 8) == (key[j] >> 8);
                best = hit ? min(best, (ka[j] & 255u) + (w & 255u)) : best;
            }
            wave_lds_sync();
            // a window moves on once the other list has been seen up to its
            // last hub; the list whose window held its end is then exhausted
            if (last_a <= last_b) {
                wa += kWinU;
                a_lo -= kWinU;
                a_hi -= kWinU;
                if (a_hi > 0) load_window<kEntriesU>(wa, a_lo, a_hi, gl, ka);
            }
            if (last_b <= last_a) {
                wb += kWinV;
                b_lo -= kWinV;
                b_hi -= kWinV;
                if (b_hi > 0) load_window<kEntriesV>(wb, b_lo, b_hi, gl, kb);
            }
        }
        if (BP && u < n && v < n) best = min(best, bp_bound(bpd, bps, bpt, u, v, gl, G));
#pragma unroll
        for (int s = G / 2; s >= 1; s >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, s, G));
        if (gl == 0) out[p] = best;
    }
}

// ---- one pair per wave: merge-path tiles ----------------------------------------------------------
//
// The wave merges the two lists in tiles of up to kTile merged entries.  Each
// tile stages a window of each list in LDS: up to kWin entries from the first
// unmerged one rounded down to a 4-entry boundary, read as 16-byte chunks
// through a buffer resource that ends at the list's end, so chunks past it
// read as zero and are not fetched.  Entries past the smaller of the two
// lists' last hubs can match nothing (the list with that last hub ends there
// and the merge of Section 2.1 stops), so a window counts only its entries up
// to that hub, and the kPad positions after the counted ones are overwritten
// with a sentinel that sorts after every entry.  Lane l finds where diagonal
// S*l of the tile crosses the merge path by binary search (the number of A
// entries among the first S*l merged ones; on equal hubs the A entry goes
// first), then walks its S merged entries.  S is 8 in a full tile and 4, 2 or
// 1 when the last tile is short.  Because the A entry of a common hub
// immediately precedes the B entry in merged order, the lane that takes an A
// entry sees its partner as its current B entry, so every common hub is
// found, also across lane and tile boundaries.  A lane past both counted ends
// meets two sentinels, which look like one hub; their sum (kNoHub) exceeds
// every real sum (distances are below 255) and is read as no common hub.
constexpr int kTile = 512;
constexpr int kWinChunks = kTile / 4 + 2;   // 16-byte chunks staged per list: a tile plus the alignment
                                            // offset plus lookahead
constexpr int kWin = 4 * kWinChunks;        // entries
constexpr int kRows = (kWinChunks + 63) / 64;  // chunk rows a lane loads
constexpr int kPad = 16;                    // sentinel positions after the counted entries
constexpr uint32_t kSent = 0xFFFFFFFFu;     // sorts after every entry (hub ranks < 2^24 - 1)
constexpr uint32_t kNoHub = 2u * 255u;      // the sum of two sentinels' distance bytes
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kRawBufferWord3 = 0x00020000; // buffer resource word 3: 32-bit data, unswizzled (gfx9)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Minimum over the 64 lanes by DPP moves (the whole wave active); the result
// is wave-uniform.
__device__ __forceinline__ uint32_t wave_min32_dpp(uint32_t x) {
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)kSent, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// A window's chunks lane + 64 r, r < kRows (the window has kWinChunks of
// them).  Entries [base, base + hi) of `ent` are in range, hi rounded up to a
// whole chunk (label arrays are padded to whole 4-entry chunks and `base` is
// a multiple of 4); chunks past that read as zero without a memory access.
// All loads are in flight before any is used.
struct Window {
    u32x4 c[kRows];
};

__device__ __forceinline__ Window load_window(const uint32_t* __restrict__ ent, uint64_t base, uint32_t hi,
                                              uint32_t lane) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(ent + base), 0, (int)(((hi + 3u) & ~3u) * 4u), kRawBufferWord3);
    const int off = (int)(16u * lane);
    Window w;
#pragma unroll
    for (int r = 0; r < kRows; ++r) w.c[r] = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 1024 * r, 0, 0);
    return w;
}

// Publish a window in LDS and return how many of its positions from `lo` on
// count: list entries not above `limraw` (wave-uniform).  The list is sorted,
// so those form a prefix of it.  The first chunk whose last entry is above
// limraw is found by ballots, its leading entries not above limraw are
// counted from lane registers (positions before `lo` precede the first
// unmerged entry; they count and are subtracted), and the count is cut at the
// list's end `hi`.  After `hi` the window holds the next list's entries up to
// the chunk end, then zeros.  Those can only make the cut at `hi` decide, in
// which case list entries above limraw may count: that lengthens the merge
// but cannot change its result, since a hub common to both lists is a real
// common hub wherever it lies.
__device__ __forceinline__ uint32_t stage_window(const Window& w, uint32_t hi, uint32_t lo, uint32_t limraw,
                                                 uint32_t* __restrict__ win, uint32_t lane) {
    const uint32_t q0 = 4u * lane;
#pragma unroll
    for (int r = 0; r < kRows; ++r)
        if (r + 1 < kRows || lane < (uint32_t)(kWinChunks - 64 * (kRows - 1)))
            *reinterpret_cast<u32x4*>(win + q0 + 256u * r) = w.c[r];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint64_t bad = ballot64(w.c[r].w > limraw);
        if (bad) {
            const uint32_t l = (uint32_t)__builtin_ctzll(bad);
            const uint32_t x = readlane32(w.c[r].x, l), y = readlane32(w.c[r].y, l), z = readlane32(w.c[r].z, l);
            const uint32_t q = 4u * (l + 64u * r);
            const bool v0 = q < lo || x <= limraw;
            const bool v1 = v0 && (q + 1 < lo || y <= limraw);
            const bool v2 = v1 && (q + 2 < lo || z <= limraw);
            const uint32_t cnt = min(q + (uint32_t)v0 + (uint32_t)v1 + (uint32_t)v2, hi);
            return cnt > lo ? cnt - lo : 0u;
        }
    }
    return hi > lo ? hi - lo : 0u;
}

// Lane l's share of a tile of T merged entries (T <= 64 S): the S merged
// entries from diagonal S*l (none past T).  `lds` is the block's window
// array; the wave's A window starts at word wa of it and its counted entries
// are [loA, loA + nA) of that window, B likewise from word wb, both followed
// by sentinels.  Returns the lane's smallest sum over common hubs so far;
// pa_end is the A window position after its last step.
template <int S>
__device__ __forceinline__ uint32_t merge_tile(const uint32_t* __restrict__ lds, uint32_t wa, uint32_t wb,
                                               uint32_t loA, uint32_t loB, uint32_t nA, uint32_t nB, uint32_t T,
                                               uint32_t lane, uint32_t best, uint32_t& pa_end) {
    const uint32_t d = min((uint32_t)S * lane, T);
    uint32_t lo = d > nB ? d - nB : 0u, hi = min(d, nA);
    const uint32_t* sa = lds + wa + loA;
    const uint32_t* sb = lds + wb + loB + d - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sa[mid] <= (sb[-(int)mid] | 255u))
            lo = mid + 1;
        else
            hi = mid;
    }
    // The walk keeps the A head as a byte offset oa into `lds`; at step t
    // the B head is at byte offset kb + 4t - oa.  The A entry goes first
    // when its hub is not above the B entry's: x <= y, or the same hub.
    const char* base = reinterpret_cast<const char*>(lds);
    uint32_t oa = 4u * (wa + loA + lo);
    const uint32_t kb = 4u * (wa + wb + loA + loB + d);
    uint32_t x = *reinterpret_cast<const uint32_t*>(base + oa);
    uint32_t y = *reinterpret_cast<const uint32_t*>(base + (kb - oa));
#pragma unroll
    for (int t = 0; t < S; ++t) {
        const bool same = (x ^ y) < 256u;
        const uint32_t sum = (x & 255u) + (y & 255u);
        best = same ? min(best, sum) : best;
        oa += (x <= y || same) ? 4u : 0u;
        if (t + 1 < S) {
            x = *reinterpret_cast<const uint32_t*>(base + oa);
            y = *reinterpret_cast<const uint32_t*>(base + (kb + 4u * (uint32_t)(t + 1) - oa));
        }
    }
    pa_end = oa / 4u - wa;
    return best;
}

template <bool BP>
__global__ void __launch_bounds__(kBlock) k_query_wave(const uint64_t* __restrict__ offu,
                                                       const uint32_t* __restrict__ entu,
                                                       const uint2* __restrict__ lbu,
                                                       const uint64_t* __restrict__ offv,
                                                       const uint32_t* __restrict__ entv,
                                                       const uint2* __restrict__ lbv, uint32_t n, uint64_t count,
                                                       const uint32_t* __restrict__ qu,
                                                       const uint32_t* __restrict__ qv, uint32_t* __restrict__ out,
                                                       const uint8_t* __restrict__ bpd,
                                                       const ulonglong2* __restrict__ bps, uint32_t bpt) {
    constexpr uint32_t kWinWords = kWin + kPad;  // one list's window, a multiple of 4 words
    __shared__ __align__(16) uint32_t s_win[kWavesPerBlock * 2 * kWinWords];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t oA = wv * 2 * kWinWords, oB = oA + kWinWords;  // the wave's windows, in words
    uint32_t* sa = s_win + oA;
    uint32_t* sb = s_win + oB;
    // A wave takes groups of 64 consecutive pairs.  Lane l first gathers pair
    // l's ids, list bounds and list offsets, so these dependent loads are in
    // flight for all 64 pairs at once; the wave then merges the pairs one by
    // one, reading their bounds from lane registers, and stores the 64
    // answers together.
    const uint64_t groups = (count + 63) / 64;
    const uint64_t gstride = (uint64_t)gridDim.x * kWavesPerBlock;
    for (uint64_t g = blockIdx.x * kWavesPerBlock + wv; g < groups; g += gstride) {
        const uint64_t p0 = g * 64;
        const uint32_t np = (uint32_t)min<uint64_t>(64, count - p0);
        const uint64_t pl = p0 + lane;
        uint32_t ul = 0, vl = 0;
        if (lane < np) {
            ul = qu[pl];
            vl = qv[pl];
        }
        // an id out of range has no label: no common hub
        const bool has = lane < np && ul < n && vl < n;
        // Entries above the smaller of the two lists' last hubs cannot match
        // (the list ending there has nothing beyond it); when either list's
        // first hub is already above it, the lists share no hub and the pair
        // is answered without reading them (a vertex with no edges, or one
        // whose label holds no hub ranked above the other vertex).  The list
        // bounds tell that; only pairs that merge read offsets and entries.
        uint32_t liml = 0;
        bool mergel = false;
        if (has) {
            const uint2 bu = lbu[ul], bv = lbv[vl];
            const uint32_t lim = min(bu.y, bv.y);
            mergel = bu.x <= lim && bv.x <= lim;
            liml = (lim << 8) | 255u;  // compared with raw entries (hub << 8) | dist
        }
        uint64_t al = 0, ael = 0, bl = 0, bel = 0;
        if (mergel) {
            al = offu[ul];
            ael = offu[ul + 1];
            bl = offv[vl];
            bel = offv[vl + 1];
        }
        const uint64_t merge_mask = ballot64(mergel);
        // pairs to visit: those that merge (with bit-parallel labels every
        // pair with ids in range, for the BP bound)
        uint64_t todo = BP ? ballot64(has) : merge_mask;
        uint32_t res = PLL_DIST_INF;
        while (todo) {
            const uint32_t k = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            uint32_t best = PLL_DIST_INF;
            if ((merge_mask >> k) & 1ull) {
                uint64_t a = readlane64(al, k), b = readlane64(bl, k);
                const uint64_t ae = readlane64(ael, k), be = readlane64(bel, k);
                const uint32_t limraw = readlane32(liml, k);
                for (;;) {
                    const uint64_t baseA = a & ~3ull, baseB = b & ~3ull;
                    const uint32_t loA = (uint32_t)(a - baseA), loB = (uint32_t)(b - baseB);
                    const uint32_t hiA = (uint32_t)min<uint64_t>(ae - baseA, (uint64_t)kWin);
                    const uint32_t hiB = (uint32_t)min<uint64_t>(be - baseB, (uint64_t)kWin);
                    // both windows' loads are in flight before either is used
                    const Window wa = load_window(entu, baseA, hiA, lane);
                    const Window wb = load_window(entv, baseB, hiB, lane);
                    const uint32_t nA = stage_window(wa, hiA, loA, limraw, sa, lane);
                    const uint32_t nB = stage_window(wb, hiB, loB, limraw, sb, lane);
                    if (nA == 0 || nB == 0) break;
                    if (lane < (uint32_t)kPad) {
                        sa[loA + nA + lane] = kSent;
                        sb[loB + nB + lane] = kSent;
                    }
                    wave_lds_sync();
                    const uint32_t tot = nA + nB;
                    uint32_t pa;
                    if (tot <= (uint32_t)kTile) {
                        // the last tile: both counted parts end in it
                        if (tot <= 64)
                            best = merge_tile<1>(s_win, oA, oB, loA, loB, nA, nB, tot, lane, best, pa);
                        else if (tot <= 128)
                            best = merge_tile<2>(s_win, oA, oB, loA, loB, nA, nB, tot, lane, best, pa);
                        else if (tot <= 256)
                            best = merge_tile<4>(s_win, oA, oB, loA, loB, nA, nB, tot, lane, best, pa);
                        else if (kTile == 512 || tot <= 512)
                            best = merge_tile<8>(s_win, oA, oB, loA, loB, nA, nB, tot, lane, best, pa);
                        else
                            best = merge_tile<kTile / 64>(s_win, oA, oB, loA, loB, nA, nB, tot, lane, best, pa);
                        break;
                    }
                    best = merge_tile<kTile / 64>(s_win, oA, oB, loA, loB, nA, nB, (uint32_t)kTile, lane, best, pa);
                    // lane 63 ended exactly where the tile ends on the merge path
                    const uint32_t iT = readlane32(pa - loA, 63);
                    const uint32_t jT = (uint32_t)kTile - iT;
                    // a list whose counted entries are all merged ends the
                    // merge (a full window holds more than a tile)
                    if (iT == nA || jT == nB) break;
                    a += iT;
                    b += jT;
                    wave_lds_sync();
                }
                wave_lds_sync();
                best = best >= kNoHub ? PLL_DIST_INF : best;
            }
            if (BP) {
                const uint32_t u = readlane32(ul, k), v = readlane32(vl, k);
                best = min(best, bp_bound(bpd, bps, bpt, u, v, lane, 64));
            }
            best = wave_min32_dpp(best);
            res = lane == k ? best : res;
        }
        if (lane < np) out[pl] = res;
    }
}

// One pair at a time per wave, in groups of 64 pairs; waves loop over
// groups.  Grid: 8x the workgroups that fit on the device at once (measured
// on a 2^20-vertex R-MAT index with 10^7 pairs: 8x 4.18 ms, 32x 4.22 ms,
// 128x 4.28 ms).
void launch_wave(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v, uint32_t* d_out,
                 hipStream_t stream) {
    static std::atomic<uint64_t> cap_cache[64];
    uint64_t blocks = ((count + 63) / 64 + kWavesPerBlock - 1) / kWavesPerBlock;
    const int dev = idx->device;
    uint64_t cap = dev >= 0 && dev < 64 ? cap_cache[dev].load(std::memory_order_relaxed) : 0;
    if (cap == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query_wave<false>, kBlock, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
            cus < 1) {
            per_cu = 8;
            cus = 256;
        }
        cap = (uint64_t)per_cu * cus * 8;
        if (dev >= 0 && dev < 64) cap_cache[dev].store(cap, std::memory_order_relaxed);
    }
    if (blocks > cap) blocks = cap;
    const uint64_t* offu = idx->directed ? idx->d_off_out : idx->d_off;
    const uint32_t* entu = idx->directed ? idx->d_ent_out : idx->d_ent;
    const uint2* lbu = idx->directed ? idx->d_lb_out : idx->d_lb;
    if (idx->info.bp_roots)
        k_query_wave<true><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, lbu, idx->d_off, idx->d_ent, idx->d_lb,
                                                                    idx->n, count, d_u, d_v, d_out, idx->d_bp_dist,
                                                                    idx->d_bp_sets, idx->info.bp_roots);
    else
        k_query_wave<false><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, lbu, idx->d_off, idx->d_ent,
                                                                     idx->d_lb, idx->n, count, d_u, d_v, d_out,
                                                                     nullptr, nullptr, 0);
}

// Grid: a multiple of the workgroups that fit on the device at once (every
// group loops over pairs).  Short lists leave waves idle sooner, so more
// workgroups than fit at once balance better; measured: 32x for one pair per
// wave, 8x for smaller groups.
template <int G>
void launch_group(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v, uint32_t* d_out,
                  hipStream_t stream) {
    static std::atomic<uint64_t> cap_cache[64];
    constexpr uint64_t per_block = kBlock / G;
    uint64_t blocks = (count + per_block - 1) / per_block;
    const int dev = idx->device;
    uint64_t cap = dev >= 0 && dev < 64 ? cap_cache[dev].load(std::memory_order_relaxed) : 0;
    if (cap == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_query_group<G, false>, kBlock, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
            cus < 1) {
            per_cu = 8;
            cus = 256;
        }
        cap = (uint64_t)per_cu * cus * (G == 64 ? 32 : 8);
        if (dev >= 0 && dev < 64) cap_cache[dev].store(cap, std::memory_order_relaxed);
    }
    if (blocks > cap) blocks = cap;
    // the source's list comes from L_out and the target's from L_in (one
    // label serves both for an undirected index)
    const uint64_t* offu = idx->directed ? idx->d_off_out : idx->d_off;
    const uint32_t* entu = idx->directed ? idx->d_ent_out : idx->d_ent;
    if (idx->info.bp_roots)
        k_query_group<G, true><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, idx->d_off, idx->d_ent, idx->n,
                                                                         count, d_u, d_v, d_out, idx->d_bp_dist,
                                                                         idx->d_bp_sets, idx->info.bp_roots);
    else
        k_query_group<G, false><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, idx->d_off, idx->d_ent, idx->n,
                                                                          count, d_u, d_v, d_out, nullptr, nullptr, 0);
}

// Lanes per pair when the index leaves it open: the window (4 entries per
// lane) should hold about one average label.
uint32_t query_lanes_auto(const pll_index* idx) {
    const uint64_t mean = idx->n ? (idx->total + (idx->directed ? idx->total_out : idx->total)) / (2ull * idx->n) : 0;
    // a whole wave per pair from a mean label of 32 entries on (measured on
    // R-MAT indexes of 2^14..2^20 vertices, mean labels of 44..241 entries:
    // the wave kernel was fastest at every size); smaller groups below
    if (mean >= 32) return 64;
    uint32_t g = 4;
    while (g < 32 && 4ull * g < mean) g *= 2;
    return g;
}

}  // namespace

uint32_t pll_query_lanes(const pll_index* idx) {
    return idx->query_lanes ? idx->query_lanes : query_lanes_auto(idx);
}

int pll_query_launch(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v,
                     uint32_t* d_out, hipStream_t stream) {
    if (count == 0) return PLL_OK;
    const uint32_t g = pll_query_lanes(idx);
    switch (g) {
        case 1: {
            uint64_t blocks = (count + kBlock - 1) / kBlock;
            if (blocks > 65536) blocks = 65536;
            const uint64_t* offu = idx->directed ? idx->d_off_out : idx->d_off;
            const uint32_t* entu = idx->directed ? idx->d_ent_out : idx->d_ent;
            if (idx->info.bp_roots)
                k_query_lane<true><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, idx->d_off, idx->d_ent, idx->n,
                                                                            count, d_u, d_v, d_out, idx->d_bp_dist,
                                                                            idx->d_bp_sets, idx->info.bp_roots);
            else
                k_query_lane<false><<<(uint32_t)blocks, kBlock, 0, stream>>>(offu, entu, idx->d_off, idx->d_ent, idx->n,
                                                                             count, d_u, d_v, d_out, nullptr, nullptr,
                                                                             0);
            break;
        }
        case 4: launch_group<4>(idx, count, d_u, d_v, d_out, stream); break;
        case 8: launch_group<8>(idx, count, d_u, d_v, d_out, stream); break;
        case 16: launch_group<16>(idx, count, d_u, d_v, d_out, stream); break;
        case 32: launch_group<32>(idx, count, d_u, d_v, d_out, stream); break;
        case 64: launch_wave(idx, count, d_u, d_v, d_out, stream); break;
        default: return PLL_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? PLL_OK : PLL_EDEVICE;
}
