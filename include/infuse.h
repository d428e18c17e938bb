/*
 * infuse.h -- C ABI of the MI355X (gfx950) library for hash-sampled
 * Monte-Carlo influence maximisation on undirected graphs under the
 * Independent Cascade model (Goktürk & Kaya, arXiv 2008.03095).
 *
 * The calls follow the paper's problem statement (Section II): given an
 * undirected graph G = (V, E) with edge probabilities w_{u,v}, a number of
 * Monte-Carlo simulations R and a seed-set size K, select S (|S| = K) that
 * greedily maximises the influence score sigma(S), and estimate sigma(S) for a
 * given S.
 *
 * Sampling rule (Section III-A, Eq. 1-2).  For edge {u,v} with u < v and
 * hash seed s:
 *     key  = u * n + v                               (64-bit)
 *     k32  = lo32(key) ^ fmix32(hi32(key))            (= key when key < 2^32)
 *     h_e  = fmix32(s ^ k32)                          (MurmurHash3 finaliser)
 *     X_r  = fmix32(s + r)       for r = 0 .. R-1     (mod 2^32)
 *     T_e  = floor(p_e * 2^32)   (IEEE double, held in 64 bits; p >= 1 -> 2^32)
 *     edge e is live in simulation r  iff  (h_e ^ X_r) < T_e   (unsigned)
 * Components are labelled with the smallest vertex id they contain
 * (Algorithm 5 starts from l_v = v and propagates minima).  All counts are
 * exact int64 integers; sigma = count / R is formed only at this boundary.
 *
 * Conventions
 *   - Every pointer argument is a HOST pointer unless the name ends in _dev.
 *     Host inputs are only read during the call (they are copied); host
 *     outputs are written only when the call returns IM_OK.
 *   - Objects (im_ctx, im_graph, im_server) are owned by the caller and must
 *     be released with the matching destroy/free call.  A graph must be freed
 *     before its context.
 *   - No exception crosses the ABI.  On failure a call returns a non-zero
 *     im_status and im_last_error() describes it (thread-local text).
 *   - All device work of a context runs on the stream given at
 *     im_ctx_create (or a stream the context creates when NULL is given).
 *     Calls that return host results synchronise that stream.
 *   - A context is not thread-safe; use one context per host thread, or the
 *     server API, which serialises access internally.
 */
#ifndef INFUSE_H
#define INFUSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IM_OK = 0,
    IM_ERR_INVALID_ARG = 1,   /* bad parameter (K > n, R = 0, id >= n, ...) */
    IM_ERR_INVALID_GRAPH = 2, /* CSR not symmetric/sorted/unique, loop, id >= n, bad p */
    IM_ERR_OUT_OF_MEMORY = 3, /* device allocation failed */
    IM_ERR_DEVICE = 4,        /* a HIP runtime call or kernel failed */
    IM_ERR_BUDGET = 5,        /* request larger than the context's HBM budget */
    IM_ERR_NOT_READY = 6,     /* server ticket still running */
    IM_ERR_CANCELLED = 7,     /* server ticket was cancelled */
    IM_ERR_NOT_FOUND = 8      /* unknown server ticket */
} im_status;

typedef struct im_ctx im_ctx;
typedef struct im_graph im_graph;
typedef struct im_server im_server;

/* Device allocator callbacks (for example PyTorch's caching allocator).
 * alloc returns a device pointer of at least `bytes` bytes usable on
 * `stream`, or NULL on failure; free releases it.  When the allocator
 * pointer given to im_ctx_create is NULL the library uses hipMalloc/hipFree. */
typedef void *(*im_alloc_fn)(void *user, size_t bytes, void *stream);
typedef void (*im_free_fn)(void *user, void *ptr, void *stream);
typedef struct {
    im_alloc_fn alloc;
    im_free_fn free;
    void *user;
} im_allocator;

/* Returns the text of the last error raised on the calling thread. */
const char *im_last_error(void);

/* Library version string. */
const char *im_version(void);

/* Binds a device, a HIP stream (hipStream_t passed as void*, NULL = the
 * context creates its own non-blocking stream) and an allocator.
 * hbm_budget bounds the bytes the context may hold in device memory
 * (0 = no bound).  Returns IM_ERR_DEVICE for a bad device ordinal. */
im_status im_ctx_create(int device, void *stream, const im_allocator *alloc, uint64_t hbm_budget,
                        im_ctx **out);
void im_ctx_destroy(im_ctx *ctx);

/* Bytes currently held in device memory by the context. */
uint64_t im_ctx_bytes_in_use(const im_ctx *ctx);

/* Uploads an undirected graph (Section III-D: CSR xadj/adj) holding both
 * orientations of every edge: row_ptr[n+1] (row_ptr[0] = 0,
 * row_ptr[n] = nnz), col_idx[nnz].  Each row must be strictly increasing,
 * without self-loops, with ids < n, and (u,v) present iff (v,u) present.
 * p_slot (nullable) gives a probability per slot; both slots of an edge must
 * hold the same value in [0,1] (not NaN).  When p_slot is given, the p passed
 * to im_set_params is ignored.  Requires n < 2^31 and nnz < 2^32.
 * Errors: IM_ERR_INVALID_GRAPH for malformed input, IM_ERR_OUT_OF_MEMORY. */
im_status im_graph_load_csr(im_ctx *ctx, uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                            const uint32_t *col_idx, const double *p_slot, im_graph **out);
/* Loads a directed graph (not a method of the paper, which leaves directed
 * graphs to future work; the spread follows its Algorithm 4 with directed
 * reachability).  row_ptr/col_idx give the out-arcs of every vertex in the
 * layout of im_graph_load_csr, without the symmetry requirement: arc u -> v
 * is an edge of its own, hashed from the ordered pair (key u*n + v, folded
 * like the undirected key) and live in sample r when (h ^ X_r) < T.
 * p_slot (nullable) gives a probability per arc, e.g. the weighted cascade
 * p(u -> v) = 1 / in-degree(v).  Only im_set_params and
 * im_estimate_sigma_direct (reachability from S over the live arcs) apply:
 * every memo call returns IM_ERR_INVALID_ARG.  Errors as im_graph_load_csr. */
im_status im_graph_load_arcs(im_ctx *ctx, uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                             const uint32_t *col_idx, const double *p_slot, im_graph **out);
void im_graph_free(im_graph *g);

/* Sets the uniform edge probability p (Section IV-B weight settings), the
 * number of simulations R >= 1 and the hash seed s.  A memo built for other
 * parameters is kept (it is keyed by (p, R, s)) until evicted.
 * Errors: IM_ERR_INVALID_ARG for R = 0, p outside [0,1] or NaN, or when
 * n*R*2^ceil(log2(n+1)) reaches 2^64. */
im_status im_set_params(im_graph *g, double p, uint32_t R, uint32_t hash_seed);

/* Runs the sampler and the fused multi-simulation connected-components
 * kernels for the current parameters and builds the memo: per (vertex,
 * simulation) the component label and the component size (Section III-C),
 * plus the initial gains mg_v = sum_r |C_r(v)| (Algorithm 5).  Called
 * implicitly by the calls below when no memo exists for the parameters. */
im_status im_build_memo(im_graph *g);

/* Drops every memo of the graph (frees its device memory). */
im_status im_drop_memo(im_graph *g);

/* Greedy CELF selection of K seeds on the memo (Algorithm 7).  Among
 * unselected vertices the one with the largest exact marginal count wins,
 * ties going to the smallest id.  Outputs (caller-allocated, host):
 * seeds[K] in selection order, marginal[K] the marginal coverage count of
 * each seed, and *cover_count = sum of marginal = sum_r |R_{G'_r}(S)|.
 * K = 0 is valid and returns an empty selection.  Errors: IM_ERR_INVALID_ARG
 * for K > n. */
im_status im_select_seeds(im_graph *g, uint32_t K, uint32_t *seeds, int64_t *marginal,
                          int64_t *cover_count);

/* Influence of a seed set (Algorithm 4 on the memo's R samples):
 * *count = sum_r |union_{s in S} C_r(s)| and *sigma = count / R.  S is a
 * set: duplicates count once; s_len = 0 gives 0.  Either output may be NULL.
 * Errors: IM_ERR_INVALID_ARG for an id >= n. */
im_status im_estimate_sigma(im_graph *g, const uint32_t *S, uint32_t s_len, int64_t *count,
                            double *sigma);

/* sigma(S) without a memo: the same count as im_estimate_sigma (RandCas,
 * Algorithm 4, on the same R hash samples), computed by a breadth-first
 * search from S over the live edges of every sample at once, for parameter
 * sets whose memo would not fit or is not wanted.  Needs 3 n R / 8 bytes of
 * device memory plus the sampler state (the memo needs 4 n R); builds
 * nothing that persists.  *levels (may be NULL) receives the number of
 * search levels.  Same semantics and errors as im_estimate_sigma. */
im_status im_estimate_sigma_direct(im_graph *g, const uint32_t *S, uint32_t s_len, int64_t *count,
                                   double *sigma, uint32_t *levels);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the count
 * of im_estimate_sigma, with the same semantics and outputs, computed on the
 * memo already resident for the graph's current parameters without any
 * device allocation.  The scratch (count, seed list and, for more than 128
 * distinct seeds, a bitmap of n * R / 8 bytes rounded up) lives in a 16 MiB
 * device array that the library holds on each GPU until the process ends.
 * Calls on one GPU share that array: calls that overlap on one GPU (other
 * host threads or unordered streams) race on it.  Synchronises the context's
 * stream.  Errors: IM_ERR_INVALID_ARG for an id >= n, when no memo is
 * resident for the current parameters (this call builds none: call
 * im_build_memo first) or when the query needs more than 16 MiB of scratch;
 * IM_ERR_DEVICE when the array is unavailable. */
im_status im_estimate_sigma_noalloc(im_graph *g, const uint32_t *S, uint32_t s_len, int64_t *count,
                                    double *sigma);

/* Greedy selection of K seeds without a memo, for graphs whose memo would
 * not fit and for directed graphs (whose spread is reachability, not
 * connectivity; the paper leaves them to future work): the marginal gain of
 * u is sum_r |R_r(u) \ R_r(S)|, the vertices reachable from u over the live
 * edges (arcs) of sample r and not from the seeds, computed by searches of
 * all samples at once, many candidates side by side.  Same queue and
 * tie-breaking as im_select_seeds (on an undirected graph the result is the
 * same), same outputs and errors.  Needs about 3 n R / 8 bytes per
 * candidate searched side by side (up to 1,024, within 8 GiB) plus the
 * sampler state; meant for graphs of up to about 10^5 vertices. */
im_status im_select_seeds_direct(im_graph *g, uint32_t K, uint32_t *seeds, int64_t *marginal,
                                 int64_t *cover_count);

/* Copies component labels of simulations first_sample .. first_sample +
 * n_samples - 1 for every vertex into host[n][n_samples] (vertex-major).
 * Errors: IM_ERR_INVALID_ARG when the range exceeds R. */
im_status im_copy_labels(im_graph *g, int32_t *host, uint64_t first_sample, uint32_t n_samples);

/* Copies the component size of every (vertex, simulation) pair for the same
 * range, host[n][n_samples]. */
im_status im_copy_sizes(im_graph *g, int32_t *host, uint64_t first_sample, uint32_t n_samples);

/* Copies the initial gains mg_v (int64[n], Algorithm 5) to the host. */
im_status im_copy_gains0(im_graph *g, int64_t *host);

/* Graph shape. */
uint32_t im_graph_n(const im_graph *g);
uint64_t im_graph_nnz(const im_graph *g);

/* ---- tuning and measurement ------------------------------------------- */

/* Kernel-launch shape knobs (0 keeps the current value).
 *   cc_chunk    simulations handled by one wavefront of a vertex with more
 *               than 64 neighbours when its parent pointers are set (256 *
 *               2^k, at most 8192; default 256); lighter vertices take
 *               their whole row in one wavefront
 *   celf_width  per-step mode: candidates re-evaluated together per round
 *   use_graphs  per-step mode: 1 = the K steps' launches are captured into
 *               one hipGraph (kernel nodes only) and launched once, 2 = direct
 *               launches (default)
 *   celf_mode   1 = all greedy steps in one persistent kernel whose grid
 *               is resident at once (default), 2 = one launch per step and
 *               phase
 *   celf_round0 persistent kernel: candidates re-evaluated in the first round
 *               of a step (doubling in later rounds); 0 = automatic (16,
 *               fewer when that exceeds one tile per wavefront)
 *   list_blocks workgroups of the kernels that walk the work lists (unions
 *               of light vertices, flatten, initial gains), 256 to 65536
 *               (default 8192); in a batched construction each graph takes
 *               at most this many                                          */
typedef struct {
    uint32_t cc_chunk;
    uint32_t celf_width;
    uint32_t use_graphs;
    uint32_t celf_mode;
    uint32_t celf_round0;
    uint32_t list_blocks;
    uint32_t reserved[2];
} im_tuning;
im_status im_set_tuning(im_ctx *ctx, const im_tuning *t);
im_status im_get_tuning(const im_ctx *ctx, im_tuning *t);

/* Autotuner (not part of the paper's method: it picks launch shapes).  Times
 * `reps` cold K-seed selections of g (memo dropped before each) for every
 * candidate cc_chunk in {256, 512, 1024}, list_blocks in {2048, 8192,
 * 32768} and, with the persistent CELF kernel, celf_round0 in {8, 16, 32};
 * checks that all of them select the same seeds (IM_ERR_DEVICE otherwise),
 * applies the fastest to g's context and writes it to *best.  g's memo is rebuilt each time (the resident memo is
 * dropped).  Errors: NULL arguments, parameters not set, K outside 1..n. */
im_status im_autotune(im_graph *g, uint32_t K, uint32_t reps, im_tuning *best);

/* Per-kernel device timing with HIP events recorded on the launching
 * stream around launches (off by default).  level 0: off; 1: the long
 * launches only, whose events cost nothing measurable: the persistent CELF
 * kernel (celf) and the memo-free search's levels (bfs_level, with the
 * search's work counts, im_last_search_stats); 2: also the kernels that run
 * once per memo construction or query (edge_hash, x_sort, hook, hook_hubs,
 * lists, link, link_hubs, flatten, count, gain0, sigma, sigma_direct, the
 * batched construction's phases), whose events add a few microseconds
 * each; 3: also every CELF round launch (celf_topw, celf_eval, celf_bulk)
 * and the persistent CELF kernel's phase clock; 4: also the work counts of
 * memo constructions (im_memo_work) and of the persistent CELF kernel.
 * im_kernel_stats returns the number of launches and the summed
 * milliseconds of the named kernel since the last reset. */
im_status im_set_profiling(im_ctx *ctx, int level);
im_status im_reset_kernel_stats(im_ctx *ctx);
im_status im_kernel_stats(im_ctx *ctx, const char *kernel, uint64_t *launches, double *total_ms);

/* Phase times (ms, device events) of the last im_build_memo /
 * im_select_seeds on this graph: [0] sampler prep, [1] connected components
 * (hook+link+compress), [2] initial gains, [3] CELF. */
im_status im_last_phase_ms(const im_graph *g, double *ms4);

/* Number of CELF evaluations (vertex re-evaluations) of the last selection. */
uint64_t im_last_celf_evals(const im_graph *g);

/* Work counts of the last memo-free call on g (im_estimate_sigma_direct,
 * or every search of im_select_seeds_direct summed): out4[0] non-empty
 * levels, out4[1] frontier items (vertex, 256-column tile) visited, out4[2]
 * arcs scanned in those items, out4[3] (arc, item) pairs live in at least
 * one frontier column.  The counts are kept only while profiling is on
 * (im_set_profiling level 1 or more; they cost atomics in every level),
 * else they read zero.  Errors: NULL arguments. */
im_status im_last_search_stats(const im_graph *g, uint64_t *out4);

/* Work counts of the construction of the memo resident for the current
 * parameters, kept when it was built while profiling was at level 4 (they
 * cost atomics in every labelling kernel).  Writes out[0 .. n_out-1] (zero
 * past the last count): out[0] live (edge, simulation) pairs, out[1] union
 * attempts of the link kernels, out[2] member entries the flatten pass
 * re-pointed at their root (those that pointed at a non-root),
 * out[3] component-size decrements made in device memory by the count pass,
 * out[4] and out[5] (vertex, 256-column tile) rows written by the hook of
 * light vertices and of vertices with more than 64 neighbours, out[6]
 * component-size gathers of the initial gains, out[7] union wavefronts of
 * the latter vertices.  Errors: IM_ERR_INVALID_ARG when no memo is resident or it was
 * built without counting. */
im_status im_memo_work(im_graph *g, uint64_t *out, uint32_t n_out);

/* Work counts of the resident memo for the current parameters (built if
 * needed; waits for it): out[0] (vertex, 256-column tile) pairs that may
 * hold a non-singleton component, out[1] pairs with a column of two or more
 * live smaller neighbours (union work), out[2] vertices with more than 64
 * neighbours, out[3] memo bytes. */
im_status im_memo_stats(im_graph *g, uint64_t *out4);

/* ---- batching: many graphs in one launch per phase --------------------- */

/* K[i]-seed selections on n_graphs graphs (each with its own parameters set
 * by im_set_params; the paper's CPU code gives each batch of simulations a
 * thread of its own, Section III).  The memos of the graphs that have none
 * resident are built together: one launch per labelling phase (set-up,
 * hooks, work lists, unions, flatten, count, initial gains) over all of
 * them, each launch's workgroups divided among the graphs by prefix sums of
 * per-graph shapes.  Then all selections are set up by one launch and run
 * in one launch of the persistent CELF kernel, each graph on a group of
 * workgroups sized by its memo; their results come back in one download.
 * seeds[i] / marginal[i] point to caller arrays of K[i] entries;
 * cover[i] receives the cover count.  All graphs must share the context and
 * appear once.  Results are identical to calling im_select_seeds per
 * graph.  Errors: IM_ERR_INVALID_ARG for a graph of another context, a
 * repeated or directed graph, missing parameters or K[i] > n. */
im_status im_batch_select(im_ctx *ctx, uint32_t n_graphs, im_graph *const *graphs,
                          const uint32_t *K, uint32_t *const *seeds, int64_t *const *marginal,
                          int64_t *cover);

/* ---- serving loop ------------------------------------------------------ */

/* A server owns worker threads that admit queries as device memory (the
 * context budget) and execution slots free up, keeps graphs and memos
 * resident (memos keyed by (graph, p, R, s), least-recently-used eviction)
 * and overlaps queries on per-slot streams.  Results equal those of the
 * direct calls.  Graphs passed to submit must outlive the server. */
typedef struct {
    uint32_t slots;        /* concurrent queries on the device (>= 1) */
    /* selections whose memo has fewer (vertex, simulation) words than this,
     * in units of 2^20, run the per-step CELF kernels on their slot, beside
     * the other slots' work; the others run the persistent CELF kernel,
     * which holds the whole device while it runs (the other slots wait).
     * 0 (default): every selection persistent; 0xFFFFFFFF: none. */
    uint32_t persistent_min_mwords;
    uint32_t reserved[6];
} im_server_config;

typedef struct {
    int32_t kind;          /* 0 = sigma(S), 1 = select K seeds */
    uint32_t K;            /* kind 1 */
    double p;
    uint32_t R;
    uint32_t hash_seed;
    const uint32_t *S;     /* kind 0: copied at submit */
    uint32_t s_len;
} im_query;

typedef struct {
    im_status status;
    int64_t count;         /* sigma count or cover count */
    double sigma;          /* count / R */
    double latency_ms;     /* submit -> completion */
    double queue_ms;       /* submit -> admission */
    uint32_t memo_hit;     /* 1 when the memo was resident at admission */
    uint32_t reserved;
} im_result;

im_status im_server_create(im_ctx *ctx, const im_server_config *cfg, im_server **out);
/* Queues a query for graph g; returns a ticket. */
im_status im_server_submit(im_server *srv, im_graph *g, const im_query *q, uint64_t *ticket);
/* Non-blocking (wait_ms = 0) or bounded wait for a ticket.  seeds/marginal
 * (nullable, K entries) receive a selection's output.  Returns
 * IM_ERR_NOT_READY while the query runs.  A completed ticket is released by
 * the poll that returns its result. */
im_status im_server_poll(im_server *srv, uint64_t ticket, uint32_t wait_ms, im_result *res,
                         uint32_t *seeds, int64_t *marginal);
im_status im_server_cancel(im_server *srv, uint64_t ticket);
/* Blocks until every submitted query completed. */
im_status im_server_drain(im_server *srv);
/* Counters: [0] admitted, [1] completed, [2] rejected, [3] memo hits,
 * [4] memo builds, [5] evictions, [6] peak concurrent queries. */
im_status im_server_stats(im_server *srv, uint64_t *out7);
void im_server_destroy(im_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* INFUSE_H */
