/*
 * ORACLE — test infrastructure only.  Nothing in the product library links,
 * loads or calls this file; only the tests, the smoke check and the bench's
 * CPU-baseline leg do.
 *
 * Plain, slow, sequential C written from the paper (Jin et al., "Pruned
 * Landmark Labeling Meets Vertex Centric Computation", arXiv 1906.12018):
 *
 *   oracle_canonical  Definition 2 (canonical hierarchical hub labeling),
 *                     written out per vertex: u is a hub of v iff u has the
 *                     highest rank among all vertices on shortest u-v paths.
 *   oracle_pll        Algorithm 1 (PLL) with the "small revision" of
 *                     Section 2.1.1 (only push to lower-ranked neighbours) and
 *                     the dense array for L(u) from Section 3.3.
 *   oracle_pll_budget the same PLL stopped once a host-time budget is spent
 *                     (the first roots in rank order; a timing sample).
 *   oracle_bvc        Algorithm 4 (BVC-PLL), sequential, batch size b, with
 *                     the candidate bit-vector C(v) and the per-batch H(u)
 *                     arrays of Section 4.1.
 *   oracle_query      the 2-hop distance formula of Section 2.1, by a
 *                     two-pointer merge over hub-sorted lists.
 *   oracle_pll_directed / oracle_query_directed
 *                     the directed variant of Section 5.1: L_in and L_out
 *                     labels from a forward and a backward pruned BFS per
 *                     root; the query merges L_out(s) with L_in(t).
 *   oracle_pll_bp / oracle_query_bp
 *                     bit-parallel labels (Section 5.2) for the first BP
 *                     roots, then PLL over the other vertices pruning by
 *                     the BP bound first; the query takes the smaller of
 *                     the BP bound and the 2-hop merge.
 *   oracle_pll_weighted
 *                     PLL with Dijkstra for positive integer edge weights
 *                     (Section 5.1's weighted graphs); labels follow
 *                     Definition 2 with weighted distances.
 *   oracle_bfs        textbook breadth-first search distances.
 *
 * Conventions (readings of points the paper leaves open):
 *   - order[k] is the vertex of rank k; rank 0 is the highest (the paper's
 *     pi is 1-based with 1 highest).
 *   - every label list holds its hubs in ascending rank and includes (v,0).
 *   - distances are uint8; 255 is reserved for "absent", so a distance of
 *     255 or more is an error (ORACLE_EDIST).
 *   - the pruning test is strict: keep (u,d) iff d < min over common hubs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

#define ORACLE_OK 0
#define ORACLE_ENOMEM 2
#define ORACLE_EDIST 4
#define ORACLE_EINVAL 1
#define INF8 255u
#define DIST_INF 0xFFFFFFFFu

typedef struct {
    uint32_t n;          /* number of lists */
    uint64_t total;      /* total entries */
    uint64_t* offsets;   /* n+1 */
    uint32_t* hub_rank;  /* total; ascending within each list */
    uint8_t* dist;       /* total */
    /* counters: [0] distance checks (BFS pops / candidate messages),
     *           [1] entries added, [2] edge accesses, [3] rounds (BVC),
     *           [4] batches (BVC), [5] entries scanned by checks,
     *           [6] / [7] cost of the positive / negative checks: the sum of
     *           |L(v)| at the time of each check that added / pruned
     *           (Section 4.3, the quantities of Table 3) */
    uint64_t counters[8];
} oracle_labels;

/* ---- growable per-vertex label lists ------------------------------------ */
typedef struct {
    uint32_t* hub;  /* hub rank */
    uint8_t* d;
    uint32_t len, cap;
} vlist;

static int vlist_push(vlist* L, uint32_t hub, uint32_t d) {
    if (L->len == L->cap) {
        uint32_t nc = L->cap ? 2 * L->cap : 4;
        uint32_t* nh = (uint32_t*)realloc(L->hub, sizeof(uint32_t) * nc);
        if (!nh) return ORACLE_ENOMEM;
        L->hub = nh;
        uint8_t* nd = (uint8_t*)realloc(L->d, nc);
        if (!nd) return ORACLE_ENOMEM;
        L->d = nd;
        L->cap = nc;
    }
    L->hub[L->len] = hub;
    L->d[L->len] = (uint8_t)d;
    L->len++;
    return ORACLE_OK;
}

static void vlists_free(vlist* Ls, uint32_t n) {
    if (!Ls) return;
    for (uint32_t i = 0; i < n; ++i) { free(Ls[i].hub); free(Ls[i].d); }
    free(Ls);
}

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y);
}

/* Copy lists into CSR; each list sorted by hub rank (lists are only sorted
 * here when `sort_lists` is set; PLL produces them sorted already). */
static int vlists_to_csr(vlist* Ls, uint32_t n, int sort_lists, oracle_labels* out) {
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += Ls[i].len;
    out->n = n;
    out->total = total;
    out->offsets = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    out->hub_rank = (uint32_t*)malloc(sizeof(uint32_t) * (total ? total : 1));
    out->dist = (uint8_t*)malloc(total ? total : 1);
    if (!out->offsets || !out->hub_rank || !out->dist) return ORACLE_ENOMEM;
    uint64_t pos = 0;
    uint64_t* tmp = NULL;
    uint32_t tmpcap = 0;
    for (uint32_t i = 0; i < n; ++i) {
        out->offsets[i] = pos;
        vlist* L = &Ls[i];
        if (sort_lists && L->len > 1) {
            if (L->len > tmpcap) {
                free(tmp);
                tmpcap = L->len;
                tmp = (uint64_t*)malloc(sizeof(uint64_t) * tmpcap);
                if (!tmp) return ORACLE_ENOMEM;
            }
            for (uint32_t k = 0; k < L->len; ++k) tmp[k] = ((uint64_t)L->hub[k] << 8) | L->d[k];
            qsort(tmp, L->len, sizeof(uint64_t), cmp_u64);
            for (uint32_t k = 0; k < L->len; ++k) {
                out->hub_rank[pos + k] = (uint32_t)(tmp[k] >> 8);
                out->dist[pos + k] = (uint8_t)(tmp[k] & 255u);
            }
        } else {
            if (L->len) {
                memcpy(out->hub_rank + pos, L->hub, sizeof(uint32_t) * L->len);
                memcpy(out->dist + pos, L->d, L->len);
            }
        }
        pos += L->len;
    }
    out->offsets[n] = pos;
    free(tmp);
    return ORACLE_OK;
}

void oracle_labels_free(oracle_labels* L) {
    if (!L) return;
    free(L->offsets); free(L->hub_rank); free(L->dist);
    L->offsets = NULL; L->hub_rank = NULL; L->dist = NULL;
}

static uint32_t* make_rank(uint32_t n, const uint32_t* order) {
    uint32_t* rank = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!rank) return NULL;
    for (uint32_t i = 0; i < n; ++i) rank[i] = DIST_INF;
    for (uint32_t k = 0; k < n; ++k) {
        if (order[k] >= n || rank[order[k]] != DIST_INF) { free(rank); return NULL; }
        rank[order[k]] = k;
    }
    return rank;
}

/* ---- textbook BFS --------------------------------------------------------- */
void oracle_bfs(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, uint32_t src, uint32_t* dist) {
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    for (uint32_t i = 0; i < n; ++i) dist[i] = DIST_INF;
    uint32_t head = 0, tail = 0;
    dist[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        uint32_t x = q[head++];
        for (uint64_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
            uint32_t y = col[e];
            if (dist[y] == DIST_INF) { dist[y] = dist[x] + 1; q[tail++] = y; }
        }
    }
    free(q);
}

/* ---- Definition 2, one vertex at a time ------------------------------------
 * P_uv is the set of vertices on shortest u-v paths (u and v included).  u is
 * a hub of v iff no vertex of P_uv ranks above u.  One BFS from v gives every
 * hub of v: with best(w) = the highest rank (smallest rank number) over all
 * vertices of all shortest v-w paths, best(v) = rank(v) and, for w at
 * distance t >= 1, best(w) = min(rank(w), min over neighbours p of w at
 * distance t-1 of best(p)), since every shortest v-w path ends with such a
 * p followed by w.  Then u is a hub of v iff best(u) == rank(u).
 */
typedef struct {
    uint32_t n;
    const uint64_t* row_ptr;
    const uint32_t* col;
    const uint32_t* rank;
    const uint32_t* verts;
    uint32_t nverts;
    vlist* out;
    uint32_t next;  /* shared work counter */
    pthread_mutex_t mu;
    int err;
} canon_job;

static int canonical_one(canon_job* J, uint32_t v, uint32_t* dist, uint32_t* best, uint32_t* q, vlist* L) {
    const uint32_t n = J->n;
    for (uint32_t i = 0; i < n; ++i) dist[i] = DIST_INF;
    uint32_t head = 0, tail = 0;
    dist[v] = 0;
    best[v] = J->rank[v];
    q[tail++] = v;
    while (head < tail) {
        uint32_t x = q[head++];
        for (uint64_t e = J->row_ptr[x]; e < J->row_ptr[x + 1]; ++e) {
            uint32_t y = J->col[e];
            if (dist[y] == DIST_INF) {
                dist[y] = dist[x] + 1;
                best[y] = J->rank[y];
                q[tail++] = y;
            }
            if (dist[y] == dist[x] + 1 && best[x] < best[y]) best[y] = best[x];
        }
    }
    /* The BFS above processes x in nondecreasing distance; when x is popped,
     * best(x) is final because all its predecessors were popped before it. */
    for (uint32_t i = 0; i < tail; ++i) {
        uint32_t u = q[i];
        if (best[u] == J->rank[u]) {
            if (dist[u] >= INF8) return ORACLE_EDIST;
            int rc = vlist_push(L, J->rank[u], dist[u]);
            if (rc) return rc;
        }
    }
    return ORACLE_OK;
}

static void* canon_worker(void* arg) {
    canon_job* J = (canon_job*)arg;
    uint32_t n = J->n;
    uint32_t* dist = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* best = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!dist || !best || !q) {
        pthread_mutex_lock(&J->mu); J->err = ORACLE_ENOMEM; pthread_mutex_unlock(&J->mu);
    } else {
        for (;;) {
            pthread_mutex_lock(&J->mu);
            uint32_t i = J->next++;
            int stop = J->err != 0;
            pthread_mutex_unlock(&J->mu);
            if (stop || i >= J->nverts) break;
            int rc = canonical_one(J, J->verts[i], dist, best, q, &J->out[i]);
            if (rc) { pthread_mutex_lock(&J->mu); J->err = rc; pthread_mutex_unlock(&J->mu); }
        }
    }
    free(dist); free(best); free(q);
    return NULL;
}

/* Labels of the listed vertices (list i of the result belongs to verts[i]). */
int oracle_canonical(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                     uint32_t nverts, const uint32_t* verts, uint32_t nthreads, oracle_labels* out) {
    memset(out, 0, sizeof(*out));
    for (uint32_t i = 0; i < nverts; ++i) if (verts[i] >= n) return ORACLE_EINVAL;
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    canon_job J;
    J.n = n; J.row_ptr = row_ptr; J.col = col; J.rank = rank; J.verts = verts; J.nverts = nverts;
    J.out = (vlist*)calloc(nverts ? nverts : 1, sizeof(vlist));
    J.next = 0; J.err = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    uint32_t started = 0;
    for (uint32_t t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, canon_worker, &J) == 0) started++;
    if (started == 0) canon_worker(&J);
    for (uint32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    int rc = J.err;
    if (!rc) rc = vlists_to_csr(J.out, nverts, 1, out);
    vlists_free(J.out, nverts);
    free(rank);
    return rc;
}

/* ---- Algorithm 1: PLL ------------------------------------------------------
 * Vertices are taken in rank order.  For root u, L(u) is first spread into a
 * dense array T indexed by hub rank (Section 3.3), so a distance check at v
 * costs one pass over L(v).  The BFS from u pops (v, delta); if delta is
 * strictly below min over h in L(u) and L(v) of d(u,h) + d(h,v), (u, delta)
 * joins L(v) and the unvisited neighbours of v ranked below u are queued
 * with delta + 1 (the small revision); otherwise v is pruned.
 */
static double mono_seconds(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* PLL over the roots of rank 0 .. n-1, or, with budget_s > 0, over the roots
 * taken before budget_s seconds have passed (the root running when the budget
 * runs out is finished); *roots_done receives the number of roots run. */
static int pll_run(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                   double budget_s, uint32_t* roots_done, oracle_labels* out) {
    memset(out, 0, sizeof(*out));
    const double t_start = budget_s > 0 ? mono_seconds() : 0.0;
    uint32_t roots = 0;
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    vlist* L = (vlist*)calloc(n ? n : 1, sizeof(vlist));
    uint8_t* T = (uint8_t*)malloc(n ? n : 1);
    uint32_t* visited = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* qv = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* qd = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    int rc = ORACLE_OK;
    if (!L || !T || !visited || !qv || !qd) { rc = ORACLE_ENOMEM; goto done; }
    memset(T, INF8, n);
    for (uint32_t i = 0; i < n; ++i) visited[i] = DIST_INF;
    uint64_t checks = 0, added = 0, edges = 0, scanned = 0, cost_pos = 0, cost_neg = 0;
    for (uint32_t k = 0; k < n && !rc; ++k) {
        if (budget_s > 0 && mono_seconds() - t_start >= budget_s) break;
        roots = k + 1;
        uint32_t u = order[k];
        vlist* Lu = &L[u];
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = Lu->d[i];
        uint32_t head = 0, tail = 0;
        qv[tail] = u; qd[tail] = 0; tail++;
        visited[u] = k;
        while (head < tail) {
            uint32_t v = qv[head], delta = qd[head];
            head++;
            checks++;
            vlist* Lv = &L[v];
            uint32_t m = DIST_INF;
            for (uint32_t i = 0; i < Lv->len; ++i) {
                uint32_t th = T[Lv->hub[i]];
                if (th != INF8 && th + Lv->d[i] < m) m = th + Lv->d[i];
            }
            scanned += Lv->len;
            if (delta < m) {
                cost_pos += Lv->len;
                if (delta >= INF8) { rc = ORACLE_EDIST; break; }
                rc = vlist_push(Lv, k, delta);
                if (rc) break;
                added++;
                for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                    uint32_t w = col[e];
                    edges++;
                    if (visited[w] != k && rank[w] > k) {
                        visited[w] = k;
                        qv[tail] = w; qd[tail] = delta + 1; tail++;
                    }
                }
            } else {
                cost_neg += Lv->len;
            }
        }
        /* L(u) may have grown by (u,0) during this BFS; clear every hub it holds. */
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = INF8;
    }
    if (!rc) {
        /* lists are indexed by vertex id; PLL appends hubs in rank order */
        rc = vlists_to_csr(L, n, 0, out);
        out->counters[0] = checks;
        out->counters[1] = added;
        out->counters[2] = edges;
        out->counters[5] = scanned;
        out->counters[6] = cost_pos;
        out->counters[7] = cost_neg;
    }
done:
    if (L) vlists_free(L, n);
    free(T); free(visited); free(qv); free(qd); free(rank);
    if (roots_done) *roots_done = roots;
    return rc;
}

int oracle_pll(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
               oracle_labels* out) {
    return pll_run(n, row_ptr, col, order, 0.0, NULL, out);
}

/* The same PLL stopped after the first roots that fit in budget_s seconds of
 * host time (a timing sample of a build too long to run whole): the lists
 * hold the entries of hubs ranked below *roots_done only. */
int oracle_pll_budget(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                      double budget_s, uint32_t* roots_done, oracle_labels* out) {
    return pll_run(n, row_ptr, col, order, budget_s > 0 ? budget_s : 1e-9, roots_done, out);
}

/* ---- Algorithm 4: BVC-PLL (sequential) -------------------------------------
 * Batches B_i are consecutive rank ranges of size b (the last one partial).
 * Per batch: every u in B_i starts with delta L(u) = {(u,0)}, which also joins
 * L(u), and L(u) is mapped into the dense array H(u) (indexed by hub rank).
 * Rounds alternate a scatter phase and a gather phase until no vertex is
 * active.  Scatter: each active a sends every (u, d) of delta L(a) to each
 * neighbour v ranked below u whose candidate bit-vector C(v) does not yet
 * hold u; the bit is set and (u, d+1) is queued at v.  Gather: each v that
 * received messages keeps the (u, d) with d < min over h in L(u) and L(v) of
 * H(u)[h] + d(h,v), adds them to L(v) (and to H(v) when v is in the batch)
 * and becomes active.  C is cleared at the end of the batch.
 */
typedef struct { uint32_t* u; uint32_t len, cap; } ulist;

static int ulist_push(ulist* l, uint32_t x) {
    if (l->len == l->cap) {
        uint32_t nc = l->cap ? 2 * l->cap : 4;
        uint32_t* p = (uint32_t*)realloc(l->u, sizeof(uint32_t) * nc);
        if (!p) return ORACLE_ENOMEM;
        l->u = p; l->cap = nc;
    }
    l->u[l->len++] = x;
    return ORACLE_OK;
}

int oracle_bvc(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order, uint32_t b,
               oracle_labels* out) {
    memset(out, 0, sizeof(*out));
    if (b < 1) return ORACLE_EINVAL;
    if (b > n && n > 0) b = n;
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    int rc = ORACLE_OK;
    const uint32_t W = (b + 63) / 64;  /* words per bit-vector */
    vlist* L = (vlist*)calloc(n ? n : 1, sizeof(vlist));              /* by rank */
    uint64_t* C = (uint64_t*)calloc((size_t)(n ? n : 1) * W, sizeof(uint64_t));  /* by rank */
    uint8_t* H = (uint8_t*)malloc((size_t)b * (n ? n : 1));           /* H[k*n + hub] */
    ulist* delta = (ulist*)calloc(n ? n : 1, sizeof(ulist));          /* delta L: batch offsets */
    ulist* msgs = (ulist*)calloc(n ? n : 1, sizeof(ulist));
    uint32_t* active = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* next_active = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* recv = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t* is_recv = (uint8_t*)calloc(n ? n : 1, 1);
    uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t* is_touched = (uint8_t*)calloc(n ? n : 1, 1);
    if (!L || !C || !H || !delta || !msgs || !active || !next_active || !recv || !is_recv || !touched || !is_touched) {
        rc = ORACLE_ENOMEM;
        goto done;
    }
    memset(H, INF8, (size_t)b * n);
    uint64_t checks = 0, added = 0, edges = 0, rounds = 0, batches = 0, scanned = 0, cost_pos = 0, cost_neg = 0;
    for (uint32_t ib = 0; ib < n && !rc; ib += b) {
        uint32_t bs = (n - ib < b) ? n - ib : b;
        batches++;
        uint32_t nact = 0, ntouched = 0;
        /* batch initialisation of Algorithm 4, in rank space */
        for (uint32_t k = 0; k < bs; ++k) {
            uint32_t u = ib + k;
            if ((rc = vlist_push(&L[u], u, 0))) break;
            added++;
            delta[u].len = 0;
            if ((rc = ulist_push(&delta[u], k))) break;
            for (uint32_t i = 0; i < L[u].len; ++i) H[(size_t)k * n + L[u].hub[i]] = L[u].d[i];
            active[nact++] = u;
        }
        uint32_t j = 0;  /* distance carried by this round's messages */
        while (nact > 0 && !rc) {
            j++;
            rounds++;
            if (j >= INF8) { rc = ORACLE_EDIST; break; }
            /* scatter step */
            uint32_t nrecv = 0;
            for (uint32_t ai = 0; ai < nact && !rc; ++ai) {
                uint32_t a = active[ai];
                uint32_t va = order[a];
                for (uint64_t e = row_ptr[va]; e < row_ptr[va + 1] && !rc; ++e) {
                    uint32_t v = rank[col[e]];
                    edges++;
                    for (uint32_t di = 0; di < delta[a].len; ++di) {
                        uint32_t k = delta[a].u[di];
                        uint32_t u = ib + k;
                        if (!(u < v)) continue;  /* pi(u) < pi(v) */
                        uint64_t bit = 1ull << (k & 63);
                        if (C[(size_t)v * W + k / 64] & bit) continue;
                        C[(size_t)v * W + k / 64] |= bit;
                        if ((rc = ulist_push(&msgs[v], k))) break;
                        if (!is_recv[v]) { is_recv[v] = 1; recv[nrecv++] = v; }
                        if (!is_touched[v]) { is_touched[v] = 1; touched[ntouched++] = v; }
                    }
                }
            }
            if (rc) break;
            /* every active vertex has now sent its delta L: the active set is
             * emptied before the gather phase builds the next one */
            for (uint32_t ai = 0; ai < nact; ++ai) delta[active[ai]].len = 0;
            /* gather step: distance check, append, next active list */
            uint32_t nnext = 0;
            for (uint32_t ri = 0; ri < nrecv && !rc; ++ri) {
                uint32_t v = recv[ri];
                is_recv[v] = 0;
                delta[v].len = 0;
                uint32_t len_before = L[v].len;
                for (uint32_t mi = 0; mi < msgs[v].len; ++mi) {
                    uint32_t k = msgs[v].u[mi];
                    checks++;
                    const uint8_t* Hu = H + (size_t)k * n;
                    uint32_t m = DIST_INF;
                    for (uint32_t i = 0; i < len_before; ++i) {
                        uint32_t t = Hu[L[v].hub[i]];
                        if (t != INF8 && t + L[v].d[i] < m) m = t + L[v].d[i];
                    }
                    scanned += len_before;
                    if (j < m) {
                        cost_pos += len_before;
                        if ((rc = ulist_push(&delta[v], k))) break;
                    } else {
                        cost_neg += len_before;
                    }
                }
                msgs[v].len = 0;
                if (rc) break;
                if (delta[v].len > 0) {
                    for (uint32_t di = 0; di < delta[v].len; ++di) {
                        uint32_t k = delta[v].u[di];
                        if ((rc = vlist_push(&L[v], ib + k, j))) break;
                        added++;
                        if (v >= ib && v < ib + bs) H[(size_t)(v - ib) * n + ib + k] = (uint8_t)j;
                    }
                    next_active[nnext++] = v;
                }
            }
            memcpy(active, next_active, sizeof(uint32_t) * nnext);
            nact = nnext;
        }
        /* clear C over the touched vertices and H for this batch (the batch's last step) */
        for (uint32_t t = 0; t < ntouched; ++t) {
            uint32_t v = touched[t];
            memset(&C[(size_t)v * W], 0, sizeof(uint64_t) * W);
            is_touched[v] = 0;
        }
        for (uint32_t k = 0; k < bs; ++k) {
            uint32_t u = ib + k;
            for (uint32_t i = 0; i < L[u].len; ++i) H[(size_t)k * n + L[u].hub[i]] = INF8;
            delta[u].len = 0;
        }
    }
    if (!rc) {
        /* lists are in rank space; reorder to vertex ids, sorting each list */
        vlist* byid = (vlist*)calloc(n ? n : 1, sizeof(vlist));
        if (!byid) { rc = ORACLE_ENOMEM; goto done; }
        for (uint32_t r = 0; r < n; ++r) byid[order[r]] = L[r];
        rc = vlists_to_csr(byid, n, 1, out);
        free(byid);  /* the lists themselves are freed through L */
        out->counters[0] = checks;
        out->counters[1] = added;
        out->counters[2] = edges;
        out->counters[3] = rounds;
        out->counters[4] = batches;
        out->counters[5] = scanned;
        out->counters[6] = cost_pos;
        out->counters[7] = cost_neg;
    }
done:
    if (L) vlists_free(L, n);
    if (delta) { for (uint32_t i = 0; i < n; ++i) free(delta[i].u); free(delta); }
    if (msgs) { for (uint32_t i = 0; i < n; ++i) free(msgs[i].u); free(msgs); }
    free(C); free(H); free(active); free(next_active); free(recv); free(is_recv); free(touched); free(is_touched);
    free(rank);
    return rc;
}

/* ---- 2-hop distance query (Section 2.1) -------------------------------------
 * Dis(u,v) = min over common hubs h of d(u,h) + d(h,v), found by a two-pointer
 * merge over the two rank-sorted lists; DIST_INF when there is no common hub.
 * `consumed` (optional) receives, per pair, how many entries of both lists
 * have hub rank at most the smaller of the two lists' largest hub ranks:
 * the entries any merge has to read before one list is exhausted.
 */
void oracle_query(const uint64_t* offsets, const uint32_t* hub_rank, const uint8_t* dist, uint64_t count,
                  const uint32_t* qu, const uint32_t* qv, uint32_t* out, uint64_t* consumed) {
    for (uint64_t q = 0; q < count; ++q) {
        uint64_t a = offsets[qu[q]], ae = offsets[qu[q] + 1];
        uint64_t b = offsets[qv[q]], be = offsets[qv[q] + 1];
        uint32_t best = DIST_INF;
        uint64_t a0 = a, b0 = b;
        while (a < ae && b < be) {
            uint32_t ha = hub_rank[a], hb = hub_rank[b];
            if (ha == hb) {
                uint32_t s = (uint32_t)dist[a] + dist[b];
                if (s < best) best = s;
                a++; b++;
            } else if (ha < hb) {
                a++;
            } else {
                b++;
            }
        }
        out[q] = best;
        if (consumed) {
            uint64_t c = 0;
            if (ae > a0 && be > b0) {
                uint32_t lim = hub_rank[ae - 1] < hub_rank[be - 1] ? hub_rank[ae - 1] : hub_rank[be - 1];
                for (uint64_t i = a0; i < ae && hub_rank[i] <= lim; ++i) c++;
                for (uint64_t i = b0; i < be && hub_rank[i] <= lim; ++i) c++;
            }
            consumed[q] = c;
        }
    }
}

/* ---- directed graphs (Section 5.1) -----------------------------------------
 * Each vertex carries two labels: L_in(v) with entries (u, d(u,v)) and
 * L_out(v) with entries (u, d(v,u)); the distance from s to t is the minimum
 * of d(s,h) + d(h,t) over hubs h of both L_out(s) and L_in(t).  PLL becomes
 * two pruned BFSs per root u taken in rank order:
 *   forward, along out-arcs: a vertex v reached at delta = d(u,v) gets
 *     (u, delta) in L_in(v) unless some hub h of L_out(u) and L_in(v) has
 *     d(u,h) + d(h,v) <= delta; only then are its out-neighbours ranked below
 *     u queued;
 *   backward, along in-arcs: v reached at delta = d(v,u) gets (u, delta) in
 *     L_out(v) unless some hub h of L_out(v) and L_in(u) has
 *     d(v,h) + d(h,u) <= delta.
 * The result is the directed form of Definition 2: u is in L_in(v) iff u
 * has the highest rank on every shortest path from u to v (and L_out
 * likewise for paths from v to u).  The in-arc CSR is the transpose of the
 * given out-arc CSR, formed here by counting.
 */
static int transpose_csr(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, uint64_t** t_row,
                         uint32_t** t_col) {
    uint64_t nnz = row_ptr[n];
    uint64_t* tr = (uint64_t*)calloc((size_t)n + 1, sizeof(uint64_t));
    uint32_t* tc = (uint32_t*)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!tr || !tc || !fill) { free(tr); free(tc); free(fill); return ORACLE_ENOMEM; }
    for (uint64_t e = 0; e < nnz; ++e) {
        if (col[e] >= n) { free(tr); free(tc); free(fill); return ORACLE_EINVAL; }
        tr[col[e] + 1]++;
    }
    for (uint32_t i = 0; i < n; ++i) tr[i + 1] += tr[i];
    memcpy(fill, tr, sizeof(uint64_t) * ((size_t)n + 1));
    /* sources are visited in ascending id, so every in-row is sorted */
    for (uint32_t x = 0; x < n; ++x)
        for (uint64_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) tc[fill[col[e]]++] = x;
    free(fill);
    *t_row = tr;
    *t_col = tc;
    return ORACLE_OK;
}

/* One pruned BFS from the root u = order[k] along the arcs of (row_ptr, col):
 * T holds the root's other-side label spread by hub rank; a reached vertex v
 * is checked against its label Lx[v] and, if kept, gets (k, delta) appended. */
typedef struct {
    uint64_t checks, added, edges, scanned, cost_pos, cost_neg;
} dir_counts;

static int pruned_bfs(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* rank, uint32_t k,
                      uint32_t u, const uint8_t* T, vlist* Lx, uint32_t* visited, uint32_t stamp, uint32_t* qv,
                      uint32_t* qd, dir_counts* c) {
    uint32_t head = 0, tail = 0;
    qv[tail] = u; qd[tail] = 0; tail++;
    visited[u] = stamp;
    while (head < tail) {
        uint32_t v = qv[head], delta = qd[head];
        head++;
        c->checks++;
        vlist* Lv = &Lx[v];
        uint32_t m = DIST_INF;
        for (uint32_t i = 0; i < Lv->len; ++i) {
            uint32_t th = T[Lv->hub[i]];
            if (th != INF8 && th + Lv->d[i] < m) m = th + Lv->d[i];
        }
        c->scanned += Lv->len;
        if (!(delta < m)) {
            c->cost_neg += Lv->len;
            continue;
        }
        c->cost_pos += Lv->len;
        if (delta >= INF8) return ORACLE_EDIST;
        int rc = vlist_push(Lv, k, delta);
        if (rc) return rc;
        c->added++;
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            uint32_t w = col[e];
            c->edges++;
            if (visited[w] != stamp && rank[w] > k) {
                visited[w] = stamp;
                qv[tail] = w; qd[tail] = delta + 1; tail++;
            }
        }
    }
    (void)n;
    return ORACLE_OK;
}

int oracle_pll_directed(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order,
                        oracle_labels* lin, oracle_labels* lout) {
    memset(lin, 0, sizeof(*lin));
    memset(lout, 0, sizeof(*lout));
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    uint64_t* in_row = NULL;
    uint32_t* in_col = NULL;
    int rc = transpose_csr(n, row_ptr, col, &in_row, &in_col);
    if (rc) { free(rank); return rc; }
    vlist* Lin = (vlist*)calloc(n ? n : 1, sizeof(vlist));
    vlist* Lout = (vlist*)calloc(n ? n : 1, sizeof(vlist));
    uint8_t* T = (uint8_t*)malloc(n ? n : 1);
    uint32_t* visited = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* qv = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* qd = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    dir_counts fw = {0}, bw = {0};
    if (!Lin || !Lout || !T || !visited || !qv || !qd) { rc = ORACLE_ENOMEM; goto done; }
    memset(T, INF8, n);
    for (uint32_t i = 0; i < n; ++i) visited[i] = DIST_INF;
    for (uint32_t k = 0; k < n && !rc; ++k) {
        uint32_t u = order[k];
        /* forward: check through L_out(u), grow L_in */
        vlist* Lu = &Lout[u];
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = Lu->d[i];
        rc = pruned_bfs(n, row_ptr, col, rank, k, u, T, Lin, visited, 2 * k, qv, qd, &fw);
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = INF8;
        if (rc) break;
        /* backward: check through L_in(u), grow L_out */
        Lu = &Lin[u];
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = Lu->d[i];
        rc = pruned_bfs(n, in_row, in_col, rank, k, u, T, Lout, visited, 2 * k + 1, qv, qd, &bw);
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = INF8;
    }
    if (!rc) rc = vlists_to_csr(Lin, n, 0, lin);
    if (!rc) rc = vlists_to_csr(Lout, n, 0, lout);
    if (!rc) {
        const dir_counts* cs[2] = {&fw, &bw};
        oracle_labels* ls[2] = {lin, lout};
        for (int s = 0; s < 2; ++s) {
            ls[s]->counters[0] = cs[s]->checks;
            ls[s]->counters[1] = cs[s]->added;
            ls[s]->counters[2] = cs[s]->edges;
            ls[s]->counters[5] = cs[s]->scanned;
            ls[s]->counters[6] = cs[s]->cost_pos;
            ls[s]->counters[7] = cs[s]->cost_neg;
        }
    } else {
        oracle_labels_free(lin);
        oracle_labels_free(lout);
    }
done:
    if (Lin) vlists_free(Lin, n);
    if (Lout) vlists_free(Lout, n);
    free(T); free(visited); free(qv); free(qd); free(rank); free(in_row); free(in_col);
    return rc;
}

/* Directed 2-hop query: merge L_out(s) (lists offs/hubs/dists_s) with L_in(t)
 * (lists offt/hubt/distt) as in oracle_query. */
void oracle_query_directed(const uint64_t* offs, const uint32_t* hubs, const uint8_t* dists, const uint64_t* offt,
                           const uint32_t* hubt, const uint8_t* distt, uint64_t count, const uint32_t* qs,
                           const uint32_t* qt, uint32_t* out) {
    for (uint64_t q = 0; q < count; ++q) {
        uint64_t a = offs[qs[q]], ae = offs[qs[q] + 1];
        uint64_t b = offt[qt[q]], be = offt[qt[q] + 1];
        uint32_t best = DIST_INF;
        while (a < ae && b < be) {
            if (hubs[a] == hubt[b]) {
                uint32_t s = (uint32_t)dists[a] + distt[b];
                if (s < best) best = s;
                a++; b++;
            } else if (hubs[a] < hubt[b]) {
                a++;
            } else {
                b++;
            }
        }
        out[q] = best;
    }
}

/* ---- weighted graphs: PLL with Dijkstra (Section 5.1; the weighted
 * baseline of Section 6) -----------------------------------------------------
 * Edge e carries a positive integer weight w[e] (the CSR is symmetric and
 * both arcs of an edge carry the same weight).  Roots are taken in rank
 * order; from root u = order[k] a Dijkstra search settles vertices in
 * increasing tentative distance.  A settled v at delta gets (u, delta) in
 * L(v) unless some hub h of L(u) and L(v) has d(u,h) + d(h,v) <= delta; only
 * a kept v relaxes its edges, and only towards vertices ranked below u.  The
 * result is Definition 2 with weighted distances.  Distances are stored in
 * uint8 as in the unweighted oracle: a kept distance of 255 or more is
 * ORACLE_EDIST.  The priority queue is a binary heap of (distance, vertex)
 * with lazy deletion (stale items are skipped when popped).
 */
typedef struct { uint64_t* a; uint32_t len, cap; } heap64;

static int heap_push(heap64* H, uint64_t x) {
    if (H->len == H->cap) {
        uint32_t nc = H->cap ? 2 * H->cap : 64;
        uint64_t* na = (uint64_t*)realloc(H->a, sizeof(uint64_t) * nc);
        if (!na) return ORACLE_ENOMEM;
        H->a = na;
        H->cap = nc;
    }
    uint32_t i = H->len++;
    while (i > 0) {
        uint32_t p = (i - 1) / 2;
        if (H->a[p] <= x) break;
        H->a[i] = H->a[p];
        i = p;
    }
    H->a[i] = x;
    return ORACLE_OK;
}

static uint64_t heap_pop(heap64* H) {
    uint64_t top = H->a[0], x = H->a[--H->len];
    uint32_t i = 0;
    for (;;) {
        uint32_t c = 2 * i + 1;
        if (c >= H->len) break;
        if (c + 1 < H->len && H->a[c + 1] < H->a[c]) c++;
        if (H->a[c] >= x) break;
        H->a[i] = H->a[c];
        i = c;
    }
    if (H->len) H->a[i] = x;
    return top;
}

int oracle_pll_weighted(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint8_t* w,
                        const uint32_t* order, oracle_labels* out) {
    memset(out, 0, sizeof(*out));
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    for (uint64_t e = 0; e < row_ptr[n]; ++e)
        if (w[e] == 0) { free(rank); return ORACLE_EINVAL; }
    vlist* L = (vlist*)calloc(n ? n : 1, sizeof(vlist));
    uint8_t* T = (uint8_t*)malloc(n ? n : 1);
    uint32_t* tent = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* stamp = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t* settled = (uint8_t*)malloc(n ? n : 1);
    heap64 H = {0};
    int rc = ORACLE_OK;
    uint64_t checks = 0, added = 0, edges = 0, scanned = 0, cost_pos = 0, cost_neg = 0;
    if (!L || !T || !tent || !stamp || !settled) { rc = ORACLE_ENOMEM; goto done; }
    memset(T, INF8, n);
    for (uint32_t i = 0; i < n; ++i) stamp[i] = DIST_INF;
    for (uint32_t k = 0; k < n && !rc; ++k) {
        uint32_t u = order[k];
        vlist* Lu = &L[u];
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = Lu->d[i];
        /* stamp[v] == k: tent[v] and settled[v] belong to this search */
        stamp[u] = k; tent[u] = 0; settled[u] = 0;
        H.len = 0;
        rc = heap_push(&H, (uint64_t)u);
        while (!rc && H.len) {
            uint64_t top = heap_pop(&H);
            uint32_t v = (uint32_t)(top & 0xFFFFFFFFu), delta = (uint32_t)(top >> 32);
            if (settled[v] || delta != tent[v]) continue;  /* stale item */
            settled[v] = 1;
            checks++;
            vlist* Lv = &L[v];
            uint32_t m = DIST_INF;
            for (uint32_t i = 0; i < Lv->len; ++i) {
                uint32_t th = T[Lv->hub[i]];
                if (th != INF8 && th + Lv->d[i] < m) m = th + Lv->d[i];
            }
            scanned += Lv->len;
            if (!(delta < m)) { cost_neg += Lv->len; continue; }
            cost_pos += Lv->len;
            if (delta >= INF8) { rc = ORACLE_EDIST; break; }
            rc = vlist_push(Lv, k, delta);
            if (rc) break;
            added++;
            for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1] && !rc; ++e) {
                uint32_t x = col[e];
                edges++;
                if (rank[x] <= k) continue;
                uint32_t nd = delta + w[e];
                if (stamp[x] != k) { stamp[x] = k; tent[x] = DIST_INF; settled[x] = 0; }
                if (!settled[x] && nd < tent[x]) {
                    tent[x] = nd;
                    rc = heap_push(&H, ((uint64_t)nd << 32) | x);
                }
            }
        }
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = INF8;
    }
    if (!rc) {
        rc = vlists_to_csr(L, n, 0, out);
        out->counters[0] = checks;
        out->counters[1] = added;
        out->counters[2] = edges;
        out->counters[5] = scanned;
        out->counters[6] = cost_pos;
        out->counters[7] = cost_neg;
    }
done:
    if (L) vlists_free(L, n);
    free(T); free(tent); free(stamp); free(settled); free(rank); free(H.a);
    return rc;
}

/* ---- bit-parallel labels (Section 5.2, adopted from the original PLL) ----
 * Before the pruned searches, t bit-parallel (BP) roots are chosen and every
 * vertex v gets, per BP root r with neighbour set S_r (|S_r| <= 64):
 *   d_r(v)      = d(r, v)                      (255: unreachable)
 *   S^-1_r(v)   = { s in S_r : d(s, v) = d(r, v) - 1 }   (bit j: s_j)
 *   S^0_r(v)    = { s in S_r : d(s, v) = d(r, v) }
 * Selection: the BP root is the highest-ranked vertex not used yet; its S_r
 * is its first (up to) 64 unused neighbours in ascending rank; all of them
 * become used.  Here the three quantities are computed from their
 * definitions, with one BFS from r and one from every s in S_r.
 * The BP bound of a pair is min over BP roots of d_r(u) + d_r(v) minus 2 if
 * S^-1_r(u) and S^-1_r(v) meet, else minus 1 if S^-1 of one meets S^0 of
 * the other: the length of the best path through r or some s in S_r.
 * PLL then runs over the unused vertices in rank order; a reached (v, delta)
 * is pruned when the BP bound is <= delta or the labels cover it.  The pair
 * query is the smaller of the BP bound and the 2-hop merge.
 */
typedef struct {
    uint32_t t;          /* BP roots chosen (<= requested) */
    uint32_t* root;      /* t, vertex ids */
    uint32_t* nbr;       /* t * 64 vertex ids of S_r in bit order, DIST_INF past |S_r| */
    uint8_t* dist;       /* n * t: dist[v * t + i] = d_{r_i}(v) */
    uint64_t* sm1;       /* n * t: S^-1 */
    uint64_t* s0;        /* n * t: S^0 */
} oracle_bp;

void oracle_bp_free(oracle_bp* B) {
    if (!B) return;
    free(B->root); free(B->nbr); free(B->dist); free(B->sm1); free(B->s0);
    memset(B, 0, sizeof(*B));
}

static uint32_t bp_bound(const oracle_bp* B, uint32_t u, uint32_t v) {
    uint32_t best = DIST_INF;
    for (uint32_t i = 0; i < B->t; ++i) {
        uint32_t du = B->dist[(size_t)u * B->t + i], dv = B->dist[(size_t)v * B->t + i];
        if (du == INF8 || dv == INF8) continue;
        uint32_t td = du + dv;
        uint64_t mu = B->sm1[(size_t)u * B->t + i], mv = B->sm1[(size_t)v * B->t + i];
        uint64_t zu = B->s0[(size_t)u * B->t + i], zv = B->s0[(size_t)v * B->t + i];
        if (mu & mv) td -= 2;
        else if ((mu & zv) | (zu & mv)) td -= 1;
        if (td < best) best = td;
    }
    return best;
}

static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y);
}

int oracle_pll_bp(uint32_t n, const uint64_t* row_ptr, const uint32_t* col, const uint32_t* order, uint32_t t_req,
                  oracle_labels* out, oracle_bp* B) {
    memset(out, 0, sizeof(*out));
    memset(B, 0, sizeof(*B));
    if (t_req > 64) return ORACLE_EINVAL;
    uint32_t* rank = make_rank(n, order);
    if (!rank) return ORACLE_EINVAL;
    int rc = ORACLE_OK;
    uint8_t* used = (uint8_t*)calloc(n ? n : 1, 1);
    uint32_t* dr = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* ds = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t* nb = NULL;
    B->root = (uint32_t*)malloc(sizeof(uint32_t) * (t_req ? t_req : 1));
    B->nbr = (uint32_t*)malloc(sizeof(uint32_t) * 64 * (t_req ? t_req : 1));
    B->dist = (uint8_t*)malloc((size_t)n * (t_req ? t_req : 1) + 1);
    B->sm1 = (uint64_t*)calloc((size_t)n * (t_req ? t_req : 1) + 1, sizeof(uint64_t));
    B->s0 = (uint64_t*)calloc((size_t)n * (t_req ? t_req : 1) + 1, sizeof(uint64_t));
    vlist* L = NULL;
    uint8_t* T = NULL;
    uint32_t *visited = NULL, *qv = NULL, *qd = NULL;
    if (!used || !dr || !ds || !B->root || !B->nbr || !B->dist || !B->sm1 || !B->s0) { rc = ORACLE_ENOMEM; goto done; }

    /* selection, then the BP quantities of each root from their definitions */
    uint32_t next = 0, t = 0;
    for (; t < t_req; ++t) {
        while (next < n && used[order[next]]) next++;
        if (next == n) break;
        uint32_t r = order[next];
        used[r] = 1;
        uint32_t deg = (uint32_t)(row_ptr[r + 1] - row_ptr[r]);
        free(nb);
        nb = (uint32_t*)malloc(sizeof(uint32_t) * (deg ? deg : 1));
        if (!nb) { rc = ORACLE_ENOMEM; goto done; }
        uint32_t m = 0;
        for (uint64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
            if (!used[col[e]]) nb[m++] = rank[col[e]];
        qsort(nb, m, sizeof(uint32_t), cmp_u32);
        if (m > 64) m = 64;
        B->root[t] = r;
        for (uint32_t j = 0; j < 64; ++j) B->nbr[t * 64 + j] = j < m ? order[nb[j]] : DIST_INF;
        for (uint32_t j = 0; j < m; ++j) used[order[nb[j]]] = 1;
        oracle_bfs(n, row_ptr, col, r, dr);
        for (uint32_t v = 0; v < n; ++v) {
            if (dr[v] != DIST_INF && dr[v] >= INF8) { rc = ORACLE_EDIST; goto done; }
            B->dist[(size_t)v * t_req + t] = dr[v] == DIST_INF ? (uint8_t)INF8 : (uint8_t)dr[v];
        }
        for (uint32_t j = 0; j < m; ++j) {
            oracle_bfs(n, row_ptr, col, order[nb[j]], ds);
            for (uint32_t v = 0; v < n; ++v) {
                if (dr[v] == DIST_INF) continue;
                if (ds[v] + 1 == dr[v]) B->sm1[(size_t)v * t_req + t] |= 1ull << j;
                else if (ds[v] == dr[v]) B->s0[(size_t)v * t_req + t] |= 1ull << j;
            }
        }
    }
    /* compact the per-vertex stride from t_req to t */
    if (t < t_req) {
        for (uint32_t v = 0; v < n; ++v)
            for (uint32_t i = 0; i < t; ++i) {
                B->dist[(size_t)v * t + i] = B->dist[(size_t)v * t_req + i];
                B->sm1[(size_t)v * t + i] = B->sm1[(size_t)v * t_req + i];
                B->s0[(size_t)v * t + i] = B->s0[(size_t)v * t_req + i];
            }
    }
    B->t = t;

    /* PLL over the unused vertices, pruning by the BP bound first */
    L = (vlist*)calloc(n ? n : 1, sizeof(vlist));
    T = (uint8_t*)malloc(n ? n : 1);
    visited = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    qv = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    qd = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!L || !T || !visited || !qv || !qd) { rc = ORACLE_ENOMEM; goto done; }
    memset(T, INF8, n);
    for (uint32_t i = 0; i < n; ++i) visited[i] = DIST_INF;
    uint64_t checks = 0, added = 0, edges = 0, scanned = 0, bp_pruned = 0;
    for (uint32_t k = 0; k < n && !rc; ++k) {
        uint32_t u = order[k];
        if (used[u]) continue;
        vlist* Lu = &L[u];
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = Lu->d[i];
        uint32_t head = 0, tail = 0;
        qv[tail] = u; qd[tail] = 0; tail++;
        visited[u] = k;
        while (head < tail) {
            uint32_t v = qv[head], delta = qd[head];
            head++;
            checks++;
            if (bp_bound(B, u, v) <= delta) { bp_pruned++; continue; }
            vlist* Lv = &L[v];
            uint32_t mm = DIST_INF;
            for (uint32_t i = 0; i < Lv->len; ++i) {
                uint32_t th = T[Lv->hub[i]];
                if (th != INF8 && th + Lv->d[i] < mm) mm = th + Lv->d[i];
            }
            scanned += Lv->len;
            if (!(delta < mm)) continue;
            if (delta >= INF8) { rc = ORACLE_EDIST; break; }
            rc = vlist_push(Lv, k, delta);
            if (rc) break;
            added++;
            for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                uint32_t w = col[e];
                edges++;
                if (visited[w] != k && rank[w] > k) {
                    visited[w] = k;
                    qv[tail] = w; qd[tail] = delta + 1; tail++;
                }
            }
        }
        for (uint32_t i = 0; i < Lu->len; ++i) T[Lu->hub[i]] = INF8;
    }
    if (!rc) {
        rc = vlists_to_csr(L, n, 0, out);
        out->counters[0] = checks;
        out->counters[1] = added;
        out->counters[2] = edges;
        out->counters[5] = scanned;
        out->counters[6] = bp_pruned;  /* here: checks the BP bound pruned */
    }
done:
    if (rc) { oracle_labels_free(out); oracle_bp_free(B); }
    if (L) vlists_free(L, n);
    free(T); free(visited); free(qv); free(qd); free(rank); free(used); free(dr); free(ds); free(nb);
    return rc;
}

/* Pair query with BP labels: min of the BP bound and the 2-hop merge. */
void oracle_query_bp(const uint64_t* offsets, const uint32_t* hub_rank, const uint8_t* dist, const oracle_bp* B,
                     uint64_t count, const uint32_t* qu, const uint32_t* qv, uint32_t* out) {
    oracle_query(offsets, hub_rank, dist, count, qu, qv, out, NULL);
    for (uint64_t q = 0; q < count; ++q) {
        uint32_t b = bp_bound(B, qu[q], qv[q]);
        if (b < out[q]) out[q] = b;
    }
}
