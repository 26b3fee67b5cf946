/*
 * pll.h -- C ABI of the MI355X (gfx950) pruned landmark labeling library.
 *
 * The library builds the canonical 2-hop distance labeling of a graph
 * (undirected; directed with in- and out-labels; or undirected with positive
 * integer edge weights) for a given vertex order, and answers exact distance
 * queries from it.  Paper: Jin et al., "Pruned Landmark Labeling Meets Vertex
 * Centric Computation" (arXiv 1906.12018).
 *
 *   Problem statement (Section 2.1, Definitions 1-2): given G = (V, E) and a
 *   total order pi on V, every vertex v gets a label L(v) of (hub, distance)
 *   pairs; u is a hub of v iff u has the highest rank among all vertices on
 *   shortest u-v paths (the canonical hierarchical hub labeling, which PLL,
 *   Algorithm 1, computes).
 *   Construction (Section 4.2, Algorithm 4, BVC-PLL): vertices are labeled in
 *   rank-ordered batches of b vertices; inside a batch, vertex-centric rounds
 *   push newly accepted entries to neighbours, filter duplicates with the
 *   per-vertex candidate bit-vector C(v), and keep a candidate (u, d) at v
 *   only if d < min over common hubs h of d(u,h) + d(h,v).
 *   Query (Section 2.1): Dis(u,v) = min over h in L(u) and L(v) of
 *   d(u,h) + d(h,v), computed by merging the two hub-sorted lists.
 *
 * Conventions
 *   - Vertex ids are uint32 in [0, n).  n < 2^24 (16,777,216).
 *   - order[k] is the vertex of rank k; rank 0 is the highest.  (The paper's
 *     pi is 1-based with 1 the highest.)
 *   - Every label list holds its hubs in ascending rank and includes (v, 0).
 *   - Distances are uint8; a distance of 255 or more fails with PLL_EDIST.
 *   - Unreachable pairs have no common hub; the query returns PLL_DIST_INF.
 *
 * Memory and ownership
 *   - Every pointer argument named d_* is a device pointer (HIP global memory
 *     on the current device); every other pointer is a host pointer.
 *   - The caller owns every input and output buffer; the library copies what
 *     it keeps.  A pll_index owns its device label store until
 *     pll_index_free.  No other allocation crosses the ABI.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *     return results in host memory synchronise with it; pll_query and
 *     pll_export_labels only enqueue work on it.
 *
 * Errors
 *   - Every call returns a status code (PLL_OK on success).  Nothing throws
 *     across the ABI.  On error, *out stays NULL and no existing index is
 *     modified.  pll_status_string gives a static description.
 */
#ifndef PLL_H_
#define PLL_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLL_OK 0
#define PLL_EINVAL 1  /* bad argument: malformed CSR, order not a permutation, NULL pointer */
#define PLL_ENOMEM 2  /* device or host allocation failed */
#define PLL_ENOSPC 3  /* the label arena given in pll_build_opts is too small; retry larger */
#define PLL_EDIST 4   /* some shortest distance is 255 or more (uint8 labels) */
#define PLL_EDEVICE 5 /* a HIP runtime error */
#define PLL_ESCRATCH 6 /* pll_build_labels_noalloc: the graph does not fit its fixed scratch */

#define PLL_DIST_INF 0xFFFFFFFFu

/* Build flags (pll_build_opts.flags). */
#define PLL_FLAG_VALIDATE 0x1u /* check the CSR (sorted, symmetric, no loops or duplicates) and the order on the device */
#define PLL_FLAG_RECHECK 0x2u  /* run the batch-end label-cleaning recheck (Section 5.1) and count what it removes */
#define PLL_FLAG_RELAXED 0x4u  /* testing: the round check ignores hubs of the current batch; needs PLL_FLAG_RECHECK
                                  to restore the canonical labels */
#define PLL_FLAG_PERSISTENT 0x10u /* run the batches in one persistent launch with grid-wide barriers between
                                    phases, instead of one launch per phase and a host read-back per round */
#define PLL_FLAG_PROFILE 0x8u  /* time each build phase with HIP events on `stream` (pll_index_info.phase_ms) */
#define PLL_FLAG_PACK4 0x20u   /* testing: every fused round of an undirected unweighted build without bit-parallel
                                  roots checks four receivers per wave; otherwise only rounds expected to have at
                                  least 16,384 receivers do.  The labels are the same either way; directed,
                                  weighted and bit-parallel builds ignore it */

/* Build phases timed under PLL_FLAG_PROFILE (indexes into pll_index_info.phase_ms / phase_launches). */
#define PLL_PHASE_PREP 0     /* input checks and relabelling to rank space */
#define PLL_PHASE_INIT 1     /* batch init: self entries, distance table fill */
#define PLL_PHASE_PUSH 2     /* scatter: candidate bit-vectors to neighbours */
#define PLL_PHASE_CHECK 3    /* gather: pruning checks, appends, next frontier */
#define PLL_PHASE_END 4      /* batch end: clear C, recheck, sort, clear the table */
#define PLL_PHASE_FINAL 5    /* finalize: label CSR by vertex id */
#define PLL_PHASE_LOOP 6     /* PLL_FLAG_PERSISTENT: the batch-loop launches as a whole (INIT..END run inside them
                                and are then timed with the device wall clock, barrier waits included) */
#define PLL_NUM_PHASES 7

typedef struct pll_index pll_index;

typedef struct {
    uint32_t batch_size;    /* b, 1..1024; 0 selects 1024 (Section 6, batch size of BVC-PLL) */
    uint32_t flags;         /* PLL_FLAG_* */
    uint64_t arena_entries; /* label arena capacity in 4-byte entries during the build; 0 = automatic
                               (grows and retries on its own; a nonzero value fails with PLL_ENOSPC) */
    uint32_t query_lanes;   /* lanes cooperating on one query pair: 0 = automatic, else 1, 4, 8, 16, 32 or 64 */
    uint32_t gang_scale;    /* batched build: percent applied to each graph's work-proportional number of
                               workgroups (0 = 100) */
    uint32_t max_gang;      /* batched build: most workgroups on one graph, 1..16 (0 = 16) */
    uint32_t max_workgroups; /* batched build: most workgroups in the persistent launch (0 = as many as fit
                                on the device at once); a smaller launch leaves room for concurrent work */
    uint32_t bp_roots;      /* bit-parallel roots, 0..64 (Section 5.2); 0 = none.  Single-graph undirected
                               unweighted builds only (PLL_EINVAL elsewhere, and with PLL_FLAG_PERSISTENT) */
    uint32_t reserved[3];   /* must be zero */
} pll_build_opts;

typedef struct {
    uint32_t n;               /* vertices */
    uint32_t batch_size;      /* b used by the build */
    uint64_t total_entries;   /* sum over v of |L(v)|, self entries included */
    uint64_t label_bytes;     /* device bytes of the final label store (entries + offsets) */
    uint32_t max_dist;        /* largest distance stored */
    uint32_t max_label;       /* largest |L(v)| */
    uint64_t batches;         /* batches run */
    uint64_t rounds;          /* vertex-centric rounds run, summed over batches */
    uint64_t candidates;      /* distance checks made (candidates surviving the C(v) filter) */
    uint64_t accepted;        /* entries accepted by the round checks */
    uint64_t edges_scanned;   /* edge accesses of Algorithm 4: CSR entries of every vertex that sends new entries
                                 on (counted the same whether a round pushes them or its receivers gather them) */
    uint64_t recheck_removed; /* entries dropped by the label-cleaning recheck (0 for exact rounds) */
    uint64_t arena_entries;   /* arena capacity the successful build used */
    uint32_t build_attempts;  /* 1 + automatic arena retries */
    uint32_t gang;            /* batched build: workgroups that built this graph (1 otherwise) */
    double build_ms;          /* host wall time of pll_build_labels */
    uint64_t check_entries_read;  /* label entries the pruning checks read */
    uint64_t check_table_reads;   /* 16-byte distance-table quarters the pruning checks read */
    uint64_t check_cost_pos;      /* sum over distance checks that added an entry of |L(v)| at the check */
    uint64_t check_cost_neg;      /* the same over checks that pruned (Section 4.3, the quantities of Table 3) */
    double phase_ms[PLL_NUM_PHASES];         /* device time per phase (PLL_FLAG_PROFILE, else 0) */
    uint64_t phase_launches[PLL_NUM_PHASES]; /* kernel launches per phase (PLL_FLAG_PROFILE, else 0) */
    uint32_t directed;        /* 1 for an index of pll_build_labels_directed */
    uint32_t weighted;        /* 1 for an index of pll_build_labels_weighted */
    uint64_t in_entries;      /* directed: sum of |L_in(v)|; undirected: total_entries (one label serves both) */
    uint64_t out_entries;     /* directed: sum of |L_out(v)|; undirected: total_entries */
    uint32_t bp_roots;        /* bit-parallel roots the build chose (<= pll_build_opts.bp_roots) */
    uint32_t bp_vertices;     /* vertices they use (roots plus their neighbour sets) */
    uint64_t bp_pruned;       /* candidates the bit-parallel bound pruned */
    uint64_t check_push_edges; /* CSR entries pushed by the check launches themselves (the rounds fuse the
                                  check of round j with the push of round j+1); the rest of edges_scanned is
                                  the first push of each batch, rows longer than 1,024 entries and the senders
                                  of gathered rounds (rounds with at least n/2 receivers, graphs of 16,384
                                  vertices or more) */
    uint32_t query_lanes;     /* lanes per pair pll_query uses on this index now (the automatic choice resolved):
                                 1, 4, 8, 16, 32 or 64 */
} pll_index_info;

/* One graph of a batched build (all pointers are device pointers). */
typedef struct {
    uint32_t n;
    uint64_t nnz;
    const uint64_t* d_row_ptr;
    const uint32_t* d_col;
    const uint32_t* d_order;
} pll_graph_desc;

/*
 * Build the canonical labeling of one graph (Algorithm 4).
 *   n, nnz      vertices and CSR entries (nnz = 2 |E|)
 *   d_row_ptr   uint64[n+1], d_row_ptr[0] = 0, d_row_ptr[n] = nnz
 *   d_col       uint32[nnz]; row v lists the neighbours of v in ascending id,
 *               with no self-loop and no duplicate; the graph is symmetric
 *   d_order     uint32[n], a permutation; d_order[k] = vertex of rank k
 *   opts        NULL for defaults
 *   out         receives the new index (host pointer to the handle)
 * The call returns once the labels are resident.  Row pointers, column
 * bounds and the order permutation are always checked (PLL_EINVAL);
 * sortedness, symmetry, self-loops and duplicates only under
 * PLL_FLAG_VALIDATE -- without it such a graph yields unspecified labels.
 */
int pll_build_labels(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                     const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream, pll_index** out);

/*
 * Allocation-free build, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the labels pll_build_labels would build, written straight into
 * the caller's buffers in the form pll_export_labels gives, with no device
 * or pinned-host allocation and no free.
 *   n, nnz, d_row_ptr, d_col, d_order, opts
 *               as for pll_build_labels; opts->batch_size and the flags
 *               PLL_FLAG_VALIDATE, PLL_FLAG_RECHECK and PLL_FLAG_RELAXED
 *               apply; other flags, bp_roots or arena_entries give
 *               PLL_EINVAL; the other fields are ignored
 *   d_offsets   uint64[n+1]: list offsets by vertex id
 *   d_hubs      uint32[capacity]: hub vertex ids, ascending hub rank per list
 *   d_dists     uint8[capacity]
 *   capacity    entries d_hubs and d_dists hold
 *   total       host pointer; receives the number of label entries, also
 *               when it exceeds capacity (then PLL_ENOSPC and nothing is
 *               written; call again with capacity >= *total)
 * Every working buffer comes from a fixed 64 MiB device array that each GPU
 * the library runs on holds until the process ends.  A graph whose working
 * set or labels do not fit it fails with PLL_ESCRATCH before anything is
 * written: about 16,000 vertices fit at b = 1024 and about 40,000 at
 * b = 256 (the working set is about 580 + 1.6 b bytes per vertex plus 4
 * bytes per CSR entry; the rest holds the labels twice).  All
 * calls on one GPU share that array, and the array keeps the last call's
 * contents: the library runs one such call at a time per device (calls from
 * several host threads wait for each other), and everything a call needs
 * zeroed it clears itself.  The call returns once the outputs are written
 * (it synchronises `stream`).
 */
int pll_build_labels_noalloc(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                             const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream,
                             uint64_t* d_offsets, uint32_t* d_hubs, uint8_t* d_dists, uint64_t capacity,
                             uint64_t* total);

/*
 * Build the labels of a directed graph (Section 5.1): every vertex v gets
 * L_in(v), the hubs u with (u, d(u,v)) such that u has the highest rank on
 * every shortest path from u to v, and L_out(v), the hubs u with (u, d(v,u))
 * such that u has the highest rank on every shortest path from v to u.  The
 * batches run a forward search (out-arcs, growing L_in) and a backward search
 * (in-arcs, growing L_out) in lockstep rounds; a forward check of root u at v
 * compares L_in(v) with L_out(u), a backward check L_out(v) with L_in(u).
 *   n, nnz      vertices and arcs
 *   d_row_ptr   uint64[n+1], d_row_ptr[0] = 0, d_row_ptr[n] = nnz
 *   d_col       uint32[nnz]; row v lists the heads w of the arcs v -> w, in
 *               ascending id, with no self-loop and no duplicate arc (the
 *               graph need not be symmetric; a symmetric one gives
 *               L_in = L_out = the undirected labels)
 *   d_order     uint32[n], a permutation; d_order[k] = vertex of rank k
 *   opts        NULL for defaults; PLL_FLAG_RELAXED and PLL_FLAG_PERSISTENT
 *               are rejected (PLL_EINVAL), the other fields act as for
 *               pll_build_labels
 *   out         receives the new index
 * The in-arc CSR is formed on the device.  pll_query on the index returns
 * d(u, v), the length of a shortest path from u to v (PLL_DIST_INF when there
 * is none), by merging L_out(u) with L_in(v).  pll_index_info reports both
 * labels summed (total_entries) and apart (in_entries, out_entries).  Checks
 * and errors as for pll_build_labels, except that PLL_FLAG_VALIDATE does not
 * ask for symmetry.
 */
int pll_build_labels_directed(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                              const uint32_t* d_order, const pll_build_opts* opts, hipStream_t stream,
                              pll_index** out);

/*
 * Build the labels of an undirected graph with positive integer edge weights
 * (Section 5.1, weighted graphs): Definition 2 with weighted distances, the
 * labels PLL with Dijkstra computes.  The batch rounds become Bellman-Ford
 * iterations: a candidate travels with its own distance d + w_e, passes only
 * if it is shorter than every earlier arrival of its root at that vertex in
 * the batch, and is checked at that distance.  Such rounds can accept
 * non-canonical entries, so every batch ends with the recheck (the one
 * PLL_FLAG_RECHECK asks for in unweighted builds), which here is always on
 * and removes them; recheck_removed counts them.
 *   d_w         uint8[nnz], the weight of each CSR entry, 1..254; both arcs
 *               of an edge carry the same weight (checked under
 *               PLL_FLAG_VALIDATE; a zero weight is always PLL_EINVAL)
 *   other arguments as for pll_build_labels; PLL_FLAG_RELAXED and
 *   PLL_FLAG_PERSISTENT are PLL_EINVAL
 * Distances stay uint8: PLL_EDIST when a candidate path of 255 or more
 * reaches a vertex that no shorter candidate of the same root has reached
 * yet (so a graph whose shortest distances all fit can still fail when a
 * long detour arrives first).  The index answers pll_query with weighted
 * distances.
 */
int pll_build_labels_weighted(uint32_t n, uint64_t nnz, const uint64_t* d_row_ptr, const uint32_t* d_col,
                              const uint8_t* d_w, const uint32_t* d_order, const pll_build_opts* opts,
                              hipStream_t stream, pll_index** out);

/*
 * Bit-parallel labels (Section 5.2, adopted from the original PLL).  With
 * opts->bp_roots = t > 0, pll_build_labels first picks up to t BP roots: each
 * is the highest-ranked vertex not used yet, with S_r = its first (up to) 64
 * unused neighbours in ascending rank, which all become used.  Every vertex v
 * gets, per BP root r: d_r(v) = d(r, v) (255: unreachable), S^-1_r(v) = the
 * members s of S_r with d(s, v) = d_r(v) - 1 and S^0_r(v) = those with
 * d(s, v) = d_r(v), as 64-bit sets (bit j = the j-th member).  The BP bound
 * of a pair is the minimum over BP roots of d_r(u) + d_r(v), minus 2 when
 * S^-1_r(u) and S^-1_r(v) meet, else minus 1 when S^-1 of one meets S^0 of
 * the other.  The batches then run over the unused vertices only, and a
 * candidate (u, d) at v is pruned first when its BP bound is <= d.  So the
 * stored labels are: (u, d(u,v)) with u unused, no used vertex on any
 * shortest u-v path, and u the highest-ranked vertex on every such path.
 * pll_query returns the smaller of the BP bound and the 2-hop merge.
 *
 * pll_export_bp copies the BP part out (vertex ids):
 *   d_roots     uint32[t]          BP root i
 *   d_nbrs      uint32[t * 64]     member j of S_{r_i}; PLL_DIST_INF past |S|
 *   d_dist      uint8[n * t]       d_dist[v * t + i] = d_{r_i}(v)
 *   d_sm1, d_s0 uint64[n * t]      S^-1 and S^0 of (v, root i)
 * t is pll_index_info.bp_roots; with t = 0 nothing is copied.  Asynchronous
 * on `stream`.
 */
int pll_export_bp(const pll_index* idx, uint32_t* d_roots, uint32_t* d_nbrs, uint8_t* d_dist, uint64_t* d_sm1,
                  uint64_t* d_s0, hipStream_t stream);

/*
 * Exact distances for `count` pairs (Section 2.1, the 2-hop query).
 *   d_u, d_v    uint32[count] vertex ids; an id >= n has no label, so its
 *               pairs answer PLL_DIST_INF
 *   d_out       uint32[count]; PLL_DIST_INF when v is unreachable from u
 * Asynchronous on `stream`; the index must outlive the enqueued work.
 * Lanes per pair follow opts->query_lanes of the build: 1 runs a scalar
 * two-pointer merge per lane; G in {4..32} lets G lanes merge the two lists
 * in windows of 4G entries; 64 gives each pair a whole wave, which merges
 * the lists in merge-path tiles of 512 entries staged in LDS; 0 picks 64
 * when the mean label holds 32 entries or more, else the smallest G in
 * {4..32} with 4G >= the mean.  pll_index_info.query_lanes reports the
 * value in use.
 */
int pll_query(const pll_index* idx, uint64_t count, const uint32_t* d_u, const uint32_t* d_v, uint32_t* d_out,
              hipStream_t stream);

/*
 * Change the lanes per pair of later pll_query calls on `idx` (the value
 * opts->query_lanes set at build time: 0 = automatic, else 1, 4, 8, 16, 32 or
 * 64; the window of a pair is 4 * lanes entries of each label).  Answers do
 * not depend on it.  Another value is PLL_EINVAL.  Not synchronised with
 * pll_query calls other threads make on the same index.  Used by the query
 * autotuner (paper_1906_12018_amd.autotune.tune_query).
 */
int pll_index_set_query_lanes(pll_index* idx, uint32_t lanes);

/* Summary and counters of an index (host struct, filled synchronously). */
int pll_index_info_get(const pll_index* idx, pll_index_info* out);

/*
 * Copy the labels out in CSR form, indexed by vertex id.
 *   d_offsets   uint64[n+1]
 *   d_hubs      uint32[total_entries]: hub vertex ids, in ascending hub rank
 *   d_dists     uint8[total_entries]
 * Asynchronous on `stream`.
 */
int pll_export_labels(const pll_index* idx, uint64_t* d_offsets, uint32_t* d_hubs, uint8_t* d_dists,
                      hipStream_t stream);

/*
 * Copy one side of the labels out, as pll_export_labels does: `side` is
 * PLL_LABELS_IN (L_in, what pll_export_labels copies) or PLL_LABELS_OUT
 * (L_out); d_hubs and d_dists hold in_entries or out_entries entries.  For an
 * undirected index both sides are its one label.  Another side value is
 * PLL_EINVAL.
 */
#define PLL_LABELS_IN 0u
#define PLL_LABELS_OUT 1u
int pll_export_labels_side(const pll_index* idx, uint32_t side, uint64_t* d_offsets, uint32_t* d_hubs,
                           uint8_t* d_dists, hipStream_t stream);

/*
 * Build `count` independent graphs in one persistent-kernel launch, captured
 * in a hipGraph (the same labels as pll_build_labels on each graph).  Each
 * graph is built by a gang of workgroups sized by its share of the estimated
 * work (opts->gang_scale, opts->max_gang); all graphs use opts->batch_size.
 * outs[i] receives the index of graphs[i]; the label entries of all of them
 * share one device allocation, released with the last of these indexes.
 * On error no index is returned.
 */
int pll_build_labels_batched(uint32_t count, const pll_graph_desc* graphs, const pll_build_opts* opts,
                             hipStream_t stream, pll_index** outs);

/* Drop the caller's reference to an index.  Its device memory is released once no server keeps it
   resident (pll_server_add_index without take_ownership holds a reference of its own). */
void pll_index_free(pll_index* idx);

const char* pll_status_string(int status);

/*
 * Serving loop (continuous batching over resident indexes).
 *
 * A server keeps label indexes resident and answers query requests as they
 * arrive: whenever one of its `slots` (a stream with staging buffers) is
 * free, it packs the queued requests of one index, oldest first, into one
 * device batch of at most max_batch_pairs pairs (a larger request spans
 * several batches), so batches of different requests overlap on the device.
 * Labeling requests (a graph in host memory) are built on their own stream
 * once hipMemGetInfo reports room for the job's estimated working set plus
 * mem_reserve; the new index becomes resident under a fresh index id.
 * Times are seconds on the server's clock; latency = t_done - t_arrival.
 * Host arrays of a request must stay valid until its result is polled.
 * Calls from several host threads are safe.
 */
#define PLL_REQ_QUERY 0u
#define PLL_REQ_BUILD 1u

typedef struct pll_server pll_server;

typedef struct {
    uint32_t slots;            /* query batches in flight, 1..16 (0 = 4) */
    uint32_t build_batch_size; /* b of builds run by the server (0 = 1024) */
    uint64_t max_batch_pairs;  /* pairs per device batch (0 = 1,048,576) */
    uint64_t mem_reserve;      /* device bytes left free when admitting a build (0 = 1 GiB) */
    uint32_t build_workgroups; /* max_workgroups of the server's many-graph builds (0 = 128): the rest of the
                                  device stays free for query batches */
    uint32_t reserved[3];      /* must be zero */
} pll_server_opts;

typedef struct {
    double at;                 /* pll_server_replay: arrival, seconds after the replay starts */
    uint32_t kind;             /* PLL_REQ_QUERY or PLL_REQ_BUILD */
    uint32_t index_id;         /* query: resident index to ask */
    uint64_t count;            /* query: pairs */
    const uint32_t* h_u;       /* query: host arrays of `count` vertex ids */
    const uint32_t* h_v;
    uint32_t* h_out;           /* query: host array receiving the distances */
    uint32_t n;                /* build: vertices */
    uint32_t reserved0;
    uint64_t nnz;              /* build: CSR entries */
    const uint64_t* h_row_ptr; /* build: host CSR and order, as for pll_build_labels */
    const uint32_t* h_col;
    const uint32_t* h_order;
} pll_request;

typedef struct {
    uint64_t id;
    int32_t status;            /* PLL_OK or an error of the request */
    uint32_t kind;
    uint32_t index_id;         /* query: the index asked; build: the new resident index */
    uint32_t batch_requests;   /* query: requests packed in the batch that carried its first pairs */
    double t_arrival, t_admit, t_done;
    double t_dev_start, t_dev_end; /* device time, seconds after the server was created: query, from the start of
                                      the first to the end of the last query kernel that carried its pairs; build,
                                      the launch that labeled it (its upload included); -1 when not known.
                                      Intervals of different requests that overlap ran on the device together */
} pll_result;

int pll_server_create(const pll_server_opts* opts, pll_server** out);
/* Make `idx` resident.  With take_ownership the caller hands its reference to the server (and must not
   use or free the handle afterwards); without it the server takes a reference of its own, so the caller
   may pll_index_free its handle at any time: the labels stay resident until pll_server_destroy drops the
   server's reference. */
int pll_server_add_index(pll_server* server, pll_index* idx, int take_ownership, uint32_t* index_id);
/* The resident index with this id (owned by the server if the server built it). */
int pll_server_index(pll_server* server, uint32_t index_id, pll_index** idx);
/* Queue one request (arrival = now); *id identifies its result. */
int pll_server_submit(pll_server* server, const pll_request* req, uint64_t* id);
/* Up to `max` finished results; with `wait`, block until at least one is ready or nothing is outstanding. */
int pll_server_poll(pll_server* server, pll_result* out, uint32_t max, uint32_t* got, int wait);
/* Open-loop replay: submit reqs[i] at reqs[i].at seconds after the call, wait for all, results in request order.
   Requests go in array order (sorted by `at` is the intended use); every request already due when the
   replay thread wakes is submitted under one lock with one wake-up of the scheduler. */
int pll_server_replay(pll_server* server, uint64_t count, const pll_request* reqs, pll_result* results);
/* Finish in-flight work, free the server and the indexes it owns. */
void pll_server_destroy(pll_server* server);

#ifdef __cplusplus
}
#endif

#endif /* PLL_H_ */
