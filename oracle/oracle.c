/*
 * oracle.c -- plain, slow CPU reference for hash-sampled Monte-Carlo
 * influence maximisation on undirected graphs, written from the paper
 * (Goktürk & Kaya, "Boosting Parallel Influence-Maximization Kernels for
 * Undirected Networks with Fusing and Vectorization", arXiv 2008.03095).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; both sides see
 * only the graph arrays produced by the input generators.
 *
 * What it computes, by plain definition (no fusing, no batching, no memo):
 *   - edge hash (Section III-A, Eq. 1): h(u,v) is a 32-bit Murmur3-style hash
 *     of the ordered pair (min, max), realised as fmix32(seed ^ key32(u,v));
 *   - per-simulation value X_r = fmix32(seed + r) and the liveness rule of
 *     Eq. 2: edge e is in sample r iff (h_e xor X_r) < floor(p_e * 2^32);
 *   - per-sample connected components by breadth-first search, labelled with
 *     the smallest vertex id of each component (the fixed point of the label
 *     propagation of Algorithm 5, which starts from l_v = v and keeps minima);
 *   - initial gains mg_v = sum_r |component of v in sample r| (Algorithm 5);
 *   - CELF lazy greedy (Algorithm 3 / Algorithm 7) where a stale vertex is
 *     re-evaluated RandCas-style (Algorithm 4) on the same R samples, with
 *     ties broken by the smaller vertex id;
 *   - sigma(S) counts: sum over samples of the number of vertices reachable
 *     from S (Algorithm 4 without the division by R);
 *   - the same count on a digraph, where an arc is hashed from the ordered
 *     pair and reachability follows the arcs (orc_sigma_count_arcs), and lazy
 *     greedy on it with gains over uncovered reachable vertices
 *     (orc_celf_arcs).
 *
 * Every count is an exact integer (int64).  sigma = count / R is formed only
 * by callers.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MODE_HASH 0  /* liveness from the edge hash and X_r (Eq. 2) */
#define ORC_MODE_ENUM 1  /* sample r = world whose live edges are the set bits of r */
#define ORC_MODE_TABLE 2 /* explicit liveness table [R][m] given by the caller */

/* ---------------------------------------------------------------------- */
/* Hash and sampling rule (Section III-A)                                  */
/* ---------------------------------------------------------------------- */

/* MurmurHash3's 32-bit finaliser (Appleby, public domain): three xor-shifts
 * separated by two multiplications by odd constants. */
uint32_t orc_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* Key of the unordered pair {u,v} (Eq. 1 hashes min||max): the 64-bit value
 * min*n + max folded to 32 bits as lo32 ^ fmix32(hi32).  For keys below 2^32
 * this is the key itself, because fmix32(0) = 0. */
uint32_t orc_edge_key(uint32_t u, uint32_t v, uint32_t n) {
    uint64_t lo = u < v ? u : v;
    uint64_t hi = u < v ? v : u;
    uint64_t key = lo * (uint64_t)n + hi;
    return (uint32_t)key ^ orc_fmix32((uint32_t)(key >> 32));
}

uint32_t orc_edge_hash(uint32_t seed, uint32_t u, uint32_t v, uint32_t n) {
    return orc_fmix32(seed ^ orc_edge_key(u, v, n));
}

/* X_r of Eq. 2: one 32-bit value per simulation r = 0..R-1. */
uint32_t orc_sample_value(uint32_t seed, uint32_t r) { return orc_fmix32(seed + r); }

/* Directed graphs (the paper leaves them to future work): an arc u -> v is
 * its own edge, hashed from the ordered pair, i.e. the 64-bit key u*n + v
 * folded the same way.  For u < v it equals the undirected key. */
uint32_t orc_arc_key(uint32_t u, uint32_t v, uint32_t n) {
    uint64_t key = (uint64_t)u * (uint64_t)n + (uint64_t)v;
    return (uint32_t)key ^ orc_fmix32((uint32_t)(key >> 32));
}
uint32_t orc_arc_hash(uint32_t seed, uint32_t u, uint32_t v, uint32_t n) {
    return orc_fmix32(seed ^ orc_arc_key(u, v, n));
}

/* Threshold floor(p * 2^32) held in 64 bits so that p = 1 keeps every edge.
 * Scaling a double by 2^32 is exact, so the floor is exactly determined. */
uint64_t orc_threshold(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

int orc_is_live(uint32_t h, uint32_t x, uint64_t threshold) {
    return (uint64_t)(h ^ x) < threshold;
}

/* ---------------------------------------------------------------------- */
/* Graph and sampler                                                        */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint32_t n;
    const uint64_t *row_ptr; /* [n+1] */
    const uint32_t *col;     /* [nnz], symmetric */
    int mode;
    uint32_t R;
    uint32_t seed;
    /* hash mode: per-slot hash and threshold, computed once (the paper
     * precomputes the m edge hashes, Section III-A) */
    uint32_t *h_slot;
    uint64_t *t_slot;
    uint32_t *x; /* X_r, r < R */
    /* enum / table modes: undirected edge id of every slot */
    uint32_t *eid;
    uint64_t m_und;
    const uint8_t *table; /* [R][m_und] */
} orc_graph;

static int slot_live(const orc_graph *g, uint64_t j, uint32_t r) {
    switch (g->mode) {
    case ORC_MODE_HASH:
        return orc_is_live(g->h_slot[j], g->x[r], g->t_slot[j]);
    case ORC_MODE_ENUM:
        return (int)((r >> g->eid[j]) & 1u);
    default:
        return g->table[(uint64_t)r * g->m_und + g->eid[j]] != 0;
    }
}

/* Builds the sampler.  p_slot (per slot) overrides p when non-NULL. */
static int graph_init(orc_graph *g, uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                      int mode, double p, const double *p_slot, uint32_t R, uint32_t seed,
                      const uint8_t *table) {
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->row_ptr = row_ptr;
    g->col = col;
    g->mode = mode;
    g->R = R;
    g->seed = seed;
    g->table = table;
    uint64_t nnz = row_ptr[n];
    if (mode == ORC_MODE_HASH) {
        g->h_slot = (uint32_t *)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
        g->t_slot = (uint64_t *)malloc(sizeof(uint64_t) * (nnz ? nnz : 1));
        g->x = (uint32_t *)malloc(sizeof(uint32_t) * (R ? R : 1));
        if (!g->h_slot || !g->t_slot || !g->x) return -1;
        uint64_t t_uniform = orc_threshold(p);
        for (uint32_t u = 0; u < n; ++u)
            for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                g->h_slot[j] = orc_edge_hash(seed, u, col[j], n);
                g->t_slot[j] = p_slot ? orc_threshold(p_slot[j]) : t_uniform;
            }
        for (uint32_t r = 0; r < R; ++r) g->x[r] = orc_sample_value(seed, r);
    } else {
        /* number the undirected edges {u<v} in CSR order of u; both slots of
         * an edge get the same id */
        g->eid = (uint32_t *)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
        if (!g->eid) return -1;
        uint64_t next = 0;
        for (uint32_t u = 0; u < n; ++u)
            for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
                if (u < col[j]) g->eid[j] = (uint32_t)next++;
        for (uint32_t u = 0; u < n; ++u)
            for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
                if (u > col[j]) {
                    uint32_t v = col[j]; /* find slot of (v,u) */
                    for (uint64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
                        if (col[k] == u) { g->eid[j] = g->eid[k]; break; }
                }
        g->m_und = next;
    }
    return 0;
}

static void graph_free(orc_graph *g) {
    free(g->h_slot);
    free(g->t_slot);
    free(g->x);
    free(g->eid);
}

/* ---------------------------------------------------------------------- */
/* One sample: components by BFS                                            */
/* ---------------------------------------------------------------------- */

/* Labels every vertex of sample r with the smallest id of its component and
 * stores the component size of every vertex.  Vertices are scanned in
 * increasing id order, so the vertex that starts a BFS is its component's
 * minimum. */
static void label_sample(const orc_graph *g, uint32_t r, int32_t *label, uint32_t *csize,
                         uint32_t *queue) {
    uint32_t n = g->n;
    for (uint32_t v = 0; v < n; ++v) label[v] = -1;
    for (uint32_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        uint32_t head = 0, tail = 0;
        label[s] = (int32_t)s;
        queue[tail++] = s;
        while (head < tail) {
            uint32_t u = queue[head++];
            for (uint64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j) {
                uint32_t w = g->col[j];
                if (label[w] < 0 && slot_live(g, j, r)) {
                    label[w] = (int32_t)s;
                    queue[tail++] = w;
                }
            }
        }
        for (uint32_t i = 0; i < tail; ++i) csize[queue[i]] = tail;
    }
}

/* Size of the component of `src` in sample r, or 0 if that component holds a
 * vertex with is_seed[] set.  `stamp`/`mark` implement a visited set that is
 * never cleared. */
static uint64_t component_if_free(const orc_graph *g, uint32_t r, uint32_t src,
                                  const uint8_t *is_seed, uint32_t *queue, uint32_t *mark,
                                  uint32_t stamp) {
    uint32_t head = 0, tail = 0;
    if (is_seed && is_seed[src]) return 0;
    mark[src] = stamp;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j) {
            uint32_t w = g->col[j];
            if (mark[w] != stamp && slot_live(g, j, r)) {
                if (is_seed && is_seed[w]) return 0;
                mark[w] = stamp;
                queue[tail++] = w;
            }
        }
    }
    return tail;
}

/* Number of vertices reachable from the set S in sample r (multi-source
 * BFS).  Duplicate entries of S are harmless. */
static uint64_t reach_count(const orc_graph *g, uint32_t r, const uint32_t *S, uint32_t s_len,
                            uint32_t *queue, uint32_t *mark, uint32_t stamp) {
    uint32_t head = 0, tail = 0;
    for (uint32_t i = 0; i < s_len; ++i)
        if (mark[S[i]] != stamp) {
            mark[S[i]] = stamp;
            queue[tail++] = S[i];
        }
    while (head < tail) {
        uint32_t u = queue[head++];
        for (uint64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j) {
            uint32_t w = g->col[j];
            if (mark[w] != stamp && slot_live(g, j, r)) {
                mark[w] = stamp;
                queue[tail++] = w;
            }
        }
    }
    return tail;
}

/* ---------------------------------------------------------------------- */
/* Threads over samples (each thread owns a contiguous range of r and its  */
/* own scratch; partial integer sums are added in thread order).           */
/* ---------------------------------------------------------------------- */

typedef struct {
    const orc_graph *g;
    uint32_t r0, r1;
    int task;                  /* 0 = label/g0, 1 = gain of one vertex, 2 = reach count */
    /* task 0 */
    int64_t *g0_part;          /* [n] */
    int32_t *labels_out;       /* [n][R] or NULL */
    uint32_t *sizes_out;       /* [n][R] or NULL: |C_r(v)| */
    uint64_t *digest_out;      /* [R] or NULL */
    const uint64_t *digest_w;  /* [n] */
    /* task 1 / 2 */
    uint32_t src;
    const uint8_t *is_seed;
    const uint32_t *S;
    uint32_t s_len;
    uint64_t acc;
} orc_job;

static void *job_run(void *arg) {
    orc_job *jb = (orc_job *)arg;
    const orc_graph *g = jb->g;
    uint32_t n = g->n;
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (jb->task == 0) {
        int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
        uint32_t *csize = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
        for (uint32_t r = jb->r0; r < jb->r1; ++r) {
            label_sample(g, r, label, csize, queue);
            for (uint32_t v = 0; v < n; ++v) jb->g0_part[v] += csize[v];
            if (jb->labels_out)
                for (uint32_t v = 0; v < n; ++v) jb->labels_out[(uint64_t)v * g->R + r] = label[v];
            if (jb->sizes_out)
                for (uint32_t v = 0; v < n; ++v) jb->sizes_out[(uint64_t)v * g->R + r] = csize[v];
            if (jb->digest_out) {
                uint64_t d = 0;
                for (uint32_t v = 0; v < n; ++v) d += (uint64_t)(uint32_t)(label[v] + 1) * jb->digest_w[v];
                jb->digest_out[r] = d;
            }
        }
        free(label);
        free(csize);
    } else {
        uint32_t *mark = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
        uint64_t acc = 0;
        uint32_t stamp = 0;
        for (uint32_t r = jb->r0; r < jb->r1; ++r) {
            ++stamp;
            if (jb->task == 1)
                acc += component_if_free(g, r, jb->src, jb->is_seed, queue, mark, stamp);
            else
                acc += reach_count(g, r, jb->S, jb->s_len, queue, mark, stamp);
        }
        jb->acc = acc;
        free(mark);
    }
    free(queue);
    return NULL;
}

static int run_jobs(orc_job *tmpl, int threads) {
    uint32_t R = tmpl->g->R;
    if (threads < 1) threads = 1;
    if ((uint32_t)threads > R && R > 0) threads = (int)R;
    orc_job *jobs = (orc_job *)calloc((size_t)threads, sizeof(orc_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    int64_t **parts = (int64_t **)calloc((size_t)threads, sizeof(int64_t *));
    uint32_t n = tmpl->g->n;
    for (int t = 0; t < threads; ++t) {
        jobs[t] = *tmpl;
        jobs[t].r0 = (uint32_t)((uint64_t)R * t / threads);
        jobs[t].r1 = (uint32_t)((uint64_t)R * (t + 1) / threads);
        if (tmpl->task == 0) {
            parts[t] = (int64_t *)calloc(n ? n : 1, sizeof(int64_t));
            jobs[t].g0_part = parts[t];
        }
    }
    for (int t = 1; t < threads; ++t) pthread_create(&tid[t], NULL, job_run, &jobs[t]);
    job_run(&jobs[0]);
    for (int t = 1; t < threads; ++t) pthread_join(tid[t], NULL);
    tmpl->acc = 0;
    for (int t = 0; t < threads; ++t) {
        tmpl->acc += jobs[t].acc;
        if (tmpl->task == 0) {
            for (uint32_t v = 0; v < n; ++v) tmpl->g0_part[v] += parts[t][v];
            free(parts[t]);
        }
    }
    free(parts);
    free(jobs);
    free(tid);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Public entry points                                                      */
/* ---------------------------------------------------------------------- */

/* Labels all R samples; accumulates g0[v] = sum_r |C_r(v)| (int64, must be
 * zeroed by the caller).  labels_out and sizes_out ([n][R], vertex-major, the
 * two arrays of Section III-C with sizes stored per vertex) and digest_out
 * ([R]) are optional. */
int orc_label_all(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
                  const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
                  int64_t *g0, int32_t *labels_out, uint32_t *sizes_out, uint64_t *digest_out,
                  const uint64_t *digest_w, int threads) {
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, mode, p, p_slot, R, seed, table)) return -1;
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = &g;
    jb.task = 0;
    jb.g0_part = g0;
    jb.labels_out = labels_out;
    jb.sizes_out = sizes_out;
    jb.digest_out = digest_out;
    jb.digest_w = digest_w;
    run_jobs(&jb, threads);
    graph_free(&g);
    return 0;
}

/* Labels only samples r0..r0+cnt-1 into out[n][cnt]. */
int orc_label_range(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
                    const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
                    uint32_t r0, uint32_t cnt, int32_t *out) {
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, mode, p, p_slot, R, seed, table)) return -1;
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    uint32_t *csize = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    for (uint32_t i = 0; i < cnt; ++i) {
        label_sample(&g, r0 + i, label, csize, queue);
        for (uint32_t v = 0; v < n; ++v) out[(uint64_t)v * cnt + i] = label[v];
    }
    free(label);
    free(csize);
    free(queue);
    graph_free(&g);
    return 0;
}

/* sigma count of S: sum_r |R_{G'_r}(S)| (Algorithm 4 before dividing by R). */
int64_t orc_sigma_count(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode,
                        double p, const double *p_slot, uint32_t R, uint32_t seed,
                        const uint8_t *table, const uint32_t *S, uint32_t s_len, int threads) {
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, mode, p, p_slot, R, seed, table)) return -1;
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = &g;
    jb.task = 2;
    jb.S = S;
    jb.s_len = s_len;
    run_jobs(&jb, threads);
    graph_free(&g);
    return (int64_t)jb.acc;
}

/* sigma count of S on a digraph (out-arc CSR): sum_r |vertices reachable
 * from S over the live arcs of sample r|, the independent-cascade spread of
 * Algorithm 4 with directed reachability.  Arc liveness follows Eq. 2 with
 * the arc hash above (hash sampling only). */
int64_t orc_sigma_count_arcs(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, double p,
                             const double *p_slot, uint32_t R, uint32_t seed, const uint32_t *S,
                             uint32_t s_len, int threads) {
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, ORC_MODE_HASH, p, p_slot, R, seed, NULL)) return -1;
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) g.h_slot[j] = orc_arc_hash(seed, u, col[j], n);
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = &g;
    jb.task = 2;
    jb.S = S;
    jb.s_len = s_len;
    run_jobs(&jb, threads);
    graph_free(&g);
    return (int64_t)jb.acc;
}

/* Greedy seed selection on a digraph by lazy evaluation (Algorithm 3 with the
 * spread of orc_sigma_count_arcs): gain(u | S) = sum_r |R_r(u) \ R_r(S)|,
 * the vertices reachable from u over live arcs of sample r and not from S.
 * Lazy queue as orc_celf: the largest stale gain is re-evaluated unless it
 * was computed for the current |S|, ties to the smaller id; every gain starts
 * unevaluated (+infinity).  R_r(S) is kept as one bit per (sample, vertex). */
int orc_celf_arcs(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, double p, const double *p_slot,
                  uint32_t R, uint32_t seed, uint32_t K, uint32_t *seeds, int64_t *marginal,
                  int64_t *cover_count, uint64_t *n_evals) {
    if (K > n) return -2;
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, ORC_MODE_HASH, p, p_slot, R, seed, NULL)) return -1;
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) g.h_slot[j] = orc_arc_hash(seed, u, col[j], n);
    const uint64_t words = ((uint64_t)n + 63) / 64;
    const uint64_t cov_words = words * R;
    uint64_t *cov = (uint64_t *)calloc((size_t)(cov_words ? cov_words : 1), sizeof(uint64_t));
    int64_t *mg = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t *iter = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    uint8_t *is_seed = (uint8_t *)calloc(n ? n : 1, 1);
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t *mark = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    if (!cov || !mg || !iter || !is_seed || !queue || !mark) return -1;
    for (uint32_t v = 0; v < n; ++v) {
        mg[v] = INT64_MAX;
        iter[v] = -1;
    }
    uint32_t stamp = 0, s_size = 0;
    int64_t cover = 0;
    uint64_t evals = 0;
    while (s_size < K) {
        int64_t best = -1;
        uint32_t top = 0;
        for (uint32_t v = 0; v < n; ++v)
            if (!is_seed[v] && mg[v] > best) {
                best = mg[v];
                top = v;
            }
        if (iter[top] == (int64_t)s_size) {
            /* commit: add R_r(top) to the covered sets */
            for (uint32_t r = 0; r < R; ++r) {
                uint64_t *cr = cov + (uint64_t)r * words;
                if ((cr[top >> 6] >> (top & 63)) & 1u) continue;
                uint32_t head = 0, tail = 0;
                cr[top >> 6] |= 1ull << (top & 63);
                queue[tail++] = top;
                while (head < tail) {
                    uint32_t u = queue[head++];
                    for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                        uint32_t w = col[j];
                        if (!((cr[w >> 6] >> (w & 63)) & 1u) && slot_live(&g, j, r)) {
                            cr[w >> 6] |= 1ull << (w & 63);
                            queue[tail++] = w;
                        }
                    }
                }
            }
            seeds[s_size] = top;
            marginal[s_size] = mg[top];
            cover += mg[top];
            is_seed[top] = 1;
            ++s_size;
        } else {
            /* gain: vertices reachable from top and not covered, per sample */
            int64_t gsum = 0;
            for (uint32_t r = 0; r < R; ++r) {
                const uint64_t *cr = cov + (uint64_t)r * words;
                if ((cr[top >> 6] >> (top & 63)) & 1u) continue;
                ++stamp;
                uint32_t head = 0, tail = 0;
                mark[top] = stamp;
                queue[tail++] = top;
                while (head < tail) {
                    uint32_t u = queue[head++];
                    for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
                        uint32_t w = col[j];
                        if (mark[w] != stamp && !((cr[w >> 6] >> (w & 63)) & 1u) && slot_live(&g, j, r)) {
                            mark[w] = stamp;
                            queue[tail++] = w;
                        }
                    }
                }
                gsum += tail;
            }
            mg[top] = gsum;
            iter[top] = s_size;
            ++evals;
        }
    }
    *cover_count = cover;
    if (n_evals) *n_evals = evals;
    free(cov);
    free(mg);
    free(iter);
    free(is_seed);
    free(queue);
    free(mark);
    graph_free(&g);
    return 0;
}

/* Marginal gain of u given the seed set marked in is_seed (may be NULL for
 * the empty set): sum over samples of |C_r(u)| when C_r(u) holds no seed.
 * In an undirected sample the set reachable from S u {u} is the union of the
 * components of its members, so this equals
 * RandCas(S u {u}) - RandCas(S) on the same samples (Algorithm 3). */
static int64_t gain_of(const orc_graph *g, uint32_t u, const uint8_t *is_seed, int threads) {
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = g;
    jb.task = 1;
    jb.src = u;
    jb.is_seed = is_seed;
    run_jobs(&jb, threads);
    return (int64_t)jb.acc;
}

int64_t orc_gain(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
                 const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
                 uint32_t u, const uint8_t *is_seed, int threads) {
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, mode, p, p_slot, R, seed, table)) return -1;
    int64_t r = gain_of(&g, u, is_seed, threads);
    graph_free(&g);
    return r;
}

/* CELF lazy greedy (Algorithm 7's queue discipline, Algorithm 3's RandCas
 * re-evaluation).  g0 holds the initial gains (fresh for S = {}).  The queue
 * is an array scanned for the largest (gain, -id): a vertex at the top whose
 * gain was computed for the current |S| is committed, otherwise its gain is
 * recomputed for the current S and it is put back.  Outputs the K seeds in
 * selection order, their marginal counts and the number of evaluations. */
int orc_celf(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
             const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
             const int64_t *g0, uint32_t K, uint32_t *seeds, int64_t *marginal,
             int64_t *cover_count, uint64_t *n_evals, int threads) {
    if (K > n) return -2;
    orc_graph g;
    if (graph_init(&g, n, row_ptr, col, mode, p, p_slot, R, seed, table)) return -1;
    int64_t *mg = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    uint32_t *iter = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    uint8_t *is_seed = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint32_t v = 0; v < n; ++v) mg[v] = g0[v];
    uint32_t s_size = 0;
    int64_t cover = 0;
    uint64_t evals = 0;
    while (s_size < K) {
        int64_t best = -1;
        uint32_t top = 0;
        for (uint32_t v = 0; v < n; ++v) {
            if (is_seed[v]) continue;
            if (mg[v] > best) { /* strict: the lowest id wins ties */
                best = mg[v];
                top = v;
            }
        }
        if (iter[top] == s_size) {
            seeds[s_size] = top;
            marginal[s_size] = mg[top];
            cover += mg[top];
            is_seed[top] = 1;
            ++s_size;
        } else {
            mg[top] = gain_of(&g, top, is_seed, threads);
            iter[top] = s_size;
            ++evals;
        }
    }
    *cover_count = cover;
    if (n_evals) *n_evals = evals;
    free(mg);
    free(iter);
    free(is_seed);
    graph_free(&g);
    return 0;
}

/* CELF whose re-evaluation uses the stored labels and sizes (the memo of
 * Section III-C, Algorithm 7): gain(u | S) = sum_r |C_r(u)| over the samples
 * where u's component holds no seed.  Same selection rule as orc_celf (the
 * largest (gain, -id) at the top is committed when its gain is current for
 * |S|, else re-evaluated and put back), with the queue of Algorithm 7 kept as
 * a binary heap and the seeds' components of every sample as a bitmap over
 * (label, sample), so that graphs of 10^6 vertices finish in minutes.
 * labels/sizes are [n][R] vertex-major. */
typedef struct {
    int64_t gain;
    uint32_t id;
} heap_item;

/* a ranks above b: larger gain, then smaller id */
static int heap_above(heap_item a, heap_item b) {
    return a.gain > b.gain || (a.gain == b.gain && a.id < b.id);
}

static void heap_sift_down(heap_item *h, uint32_t len, uint32_t i) {
    for (;;) {
        uint32_t l = 2 * i + 1, r = l + 1, top = i;
        if (l < len && heap_above(h[l], h[top])) top = l;
        if (r < len && heap_above(h[r], h[top])) top = r;
        if (top == i) return;
        heap_item t = h[i];
        h[i] = h[top];
        h[top] = t;
        i = top;
    }
}

int orc_celf_memo(uint32_t n, uint32_t R, const int32_t *labels, const uint32_t *sizes,
                  const int64_t *g0, uint32_t K, uint32_t *seeds, int64_t *marginal,
                  int64_t *cover_count, uint64_t *n_evals) {
    if (K > n) return -2;
    heap_item *heap = (heap_item *)malloc(sizeof(heap_item) * (n ? n : 1));
    uint32_t *iter = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    const uint64_t cbits = (uint64_t)n * R;
    uint64_t *covered = (uint64_t *)calloc(cbits / 64 + 1, sizeof(uint64_t));
    if (!heap || !iter || !covered) {
        free(heap);
        free(iter);
        free(covered);
        return -1;
    }
    uint32_t len = n;
    for (uint32_t v = 0; v < n; ++v) {
        heap[v].gain = g0[v];
        heap[v].id = v;
    }
    for (uint32_t i = n / 2; i-- > 0;) heap_sift_down(heap, len, i);
    uint32_t s_size = 0;
    int64_t cover = 0;
    uint64_t evals = 0;
    while (s_size < K) {
        const uint32_t top = heap[0].id;
        if (iter[top] == s_size) {
            seeds[s_size] = top;
            marginal[s_size] = heap[0].gain;
            cover += heap[0].gain;
            for (uint32_t r = 0; r < R; ++r) {
                const uint64_t b = (uint64_t)(uint32_t)labels[(uint64_t)top * R + r] * R + r;
                covered[b >> 6] |= 1ull << (b & 63);
            }
            ++s_size;
            heap[0] = heap[--len];
            heap_sift_down(heap, len, 0);
        } else {
            const int32_t *lu = labels + (uint64_t)top * R;
            const uint32_t *su = sizes + (uint64_t)top * R;
            int64_t gain = 0;
            for (uint32_t r = 0; r < R; ++r) {
                const uint64_t b = (uint64_t)(uint32_t)lu[r] * R + r;
                if (!((covered[b >> 6] >> (b & 63)) & 1)) gain += su[r];
            }
            heap[0].gain = gain;
            iter[top] = s_size;
            ++evals;
            heap_sift_down(heap, len, 0);
        }
    }
    *cover_count = cover;
    if (n_evals) *n_evals = evals;
    free(heap);
    free(iter);
    free(covered);
    return 0;
}
