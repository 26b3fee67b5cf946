/*
 * Seeded synthetic inputs shared by the oracle side and the GPU side.
 *
 * This file holds only input generation: a counter-based PRNG and the two
 * random-graph edge samplers (Barabasi-Albert preferential attachment and
 * R-MAT recursive quadrant sampling).  It holds none of the labeling or query
 * arithmetic.  CSR assembly (symmetrise, dedup, drop self-loops) and the
 * degree order are done in numpy by synth/__init__.py.
 *
 * PRNG: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  Draw k (k = 0, 1, ...) of stream `seed` is
 * mix(seed + (k + 1) * 0x9E3779B97F4A7C15), so any draw can be computed
 * independently of the others.
 *   uniform double in [0,1): (x >> 11) * 2^-53
 *   bounded int in [0,r), r < 2^32: ((x >> 32) * r) >> 32  (Lemire's
 *   multiply-shift, without the rejection step)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_splitmix64_draw(uint64_t seed, uint64_t k) {
    return mix64(seed + (k + 1) * GOLDEN);
}

void synth_splitmix64_fill(uint64_t seed, uint64_t k0, uint64_t count, uint64_t* out) {
    for (uint64_t i = 0; i < count; ++i) out[i] = mix64(seed + (k0 + i + 1) * GOLDEN);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
static inline uint32_t bounded(uint64_t x, uint32_t r) { return (uint32_t)(((x >> 32) * (uint64_t)r) >> 32); }

/*
 * Barabasi-Albert graph, n vertices, m edges per new vertex.
 * Start from the star centred at 0 over {0..m}.  R lists both endpoints of
 * every edge so far.  Each new vertex t = m+1..n-1 draws m distinct targets
 * uniformly from R (a duplicate target is redrawn), then adds its m edges and
 * appends their endpoints to R.  Total edges m*(n-m), written as (src,dst)
 * pairs with src = t (or 0 for the star) into edges[2*i], edges[2*i+1].
 * Returns the number of edges, or -1 on bad arguments.
 */
int64_t synth_ba_edges(uint32_t n, uint32_t m, uint64_t seed, uint32_t* edges) {
    if (m < 1 || n < m + 1) return -1;
    uint64_t ne = (uint64_t)m * (uint64_t)(n - m);
    uint32_t* R = (uint32_t*)malloc(sizeof(uint32_t) * 2 * ne);
    uint32_t* tgt = (uint32_t*)malloc(sizeof(uint32_t) * m);
    if (!R || !tgt) { free(R); free(tgt); return -1; }
    uint64_t nr = 0, e = 0, k = 0;
    for (uint32_t i = 1; i <= m; ++i) {
        edges[2 * e] = 0; edges[2 * e + 1] = i; ++e;
        R[nr++] = 0; R[nr++] = i;
    }
    for (uint32_t t = m + 1; t < n; ++t) {
        uint32_t got = 0;
        while (got < m) {
            uint32_t c = R[bounded(synth_splitmix64_draw(seed, k++), (uint32_t)nr)];
            int dup = 0;
            for (uint32_t q = 0; q < got; ++q) if (tgt[q] == c) { dup = 1; break; }
            if (!dup) tgt[got++] = c;
        }
        for (uint32_t q = 0; q < m; ++q) {
            edges[2 * e] = t; edges[2 * e + 1] = tgt[q]; ++e;
            R[nr++] = t; R[nr++] = tgt[q];
        }
    }
    free(R); free(tgt);
    return (int64_t)e;
}

/*
 * R-MAT edge samples: ef * 2^scale samples over 2^scale vertices.  Sample s
 * uses draws s*scale .. s*scale+scale-1, one per level, most significant bit
 * first.  A draw below a keeps the quadrant (0,0); below a+b sets the column
 * bit; below a+b+c sets the row bit; otherwise both.  No noise, no vertex
 * permutation.  Self-loops and duplicates are kept here and removed by the
 * CSR assembly.
 */
void synth_rmat_edges(uint32_t scale, uint64_t nsamples, double a, double b, double c,
                      uint64_t seed, uint32_t* edges) {
    const double ab = a + b, abc = a + b + c;
    for (uint64_t s = 0; s < nsamples; ++s) {
        uint32_t r = 0, col = 0;
        for (uint32_t lv = 0; lv < scale; ++lv) {
            double x = u01(synth_splitmix64_draw(seed, s * scale + lv));
            uint32_t bit = 1u << (scale - 1 - lv);
            if (x < a) {
            } else if (x < ab) {
                col |= bit;
            } else if (x < abc) {
                r |= bit;
            } else {
                r |= bit; col |= bit;
            }
        }
        edges[2 * s] = r; edges[2 * s + 1] = col;
    }
}
