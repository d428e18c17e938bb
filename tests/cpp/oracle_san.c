/* Exercises the oracle's entry points on small random graphs in a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (the test compiles this
 * file together with oracle/oracle.c): every buffer access and integer
 * operation of labelling, gains, both CELF variants, sigma counts and the
 * directed functions runs under the sanitizers, and the results are checked
 * against each other (memo CELF = RandCas CELF; component sizes sum to n in
 * every sample; cover = sum of marginals; sigma of the seeds = cover). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_label_all(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
                  const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
                  int64_t *g0, int32_t *labels_out, uint32_t *sizes_out, uint64_t *digest_out,
                  const uint64_t *digest_w, int threads);
int64_t orc_sigma_count(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
                        const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table,
                        const uint32_t *S, uint32_t s_len, int threads);
int orc_celf(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, int mode, double p,
             const double *p_slot, uint32_t R, uint32_t seed, const uint8_t *table, const int64_t *g0,
             uint32_t K, uint32_t *seeds, int64_t *marginal, int64_t *cover_count, uint64_t *n_evals,
             int threads);
int orc_celf_memo(uint32_t n, uint32_t R, const int32_t *labels, const uint32_t *sizes, const int64_t *g0,
                  uint32_t K, uint32_t *seeds, int64_t *marginal, int64_t *cover_count, uint64_t *n_evals);
int64_t orc_sigma_count_arcs(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, double p,
                             const double *p_slot, uint32_t R, uint32_t seed, const uint32_t *S,
                             uint32_t s_len, int threads);
int orc_celf_arcs(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, double p, const double *p_slot,
                  uint32_t R, uint32_t seed, uint32_t K, uint32_t *seeds, int64_t *marginal,
                  int64_t *cover_count, uint64_t *n_evals);

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                   \
        }                                                               \
    } while (0)

static uint64_t rng_state = 0x1234567ull;
static uint32_t rnd(uint32_t bound) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)((rng_state >> 33) % bound);
}

/* random simple undirected graph as a symmetric sorted CSR (both slots) */
static void make_graph(uint32_t n, uint32_t m, uint64_t **rp_out, uint32_t **col_out) {
    uint8_t *adj = (uint8_t *)calloc((size_t)n * n, 1);
    uint32_t made = 0;
    while (made < m) {
        uint32_t u = rnd(n), v = rnd(n);
        if (u == v || adj[(size_t)u * n + v]) continue;
        adj[(size_t)u * n + v] = adj[(size_t)v * n + u] = 1;
        ++made;
    }
    uint64_t *rp = (uint64_t *)malloc(sizeof(uint64_t) * (n + 1));
    uint32_t *col = (uint32_t *)malloc(sizeof(uint32_t) * 2 * m);
    rp[0] = 0;
    for (uint32_t u = 0; u < n; ++u) {
        rp[u + 1] = rp[u];
        for (uint32_t v = 0; v < n; ++v)
            if (adj[(size_t)u * n + v]) col[rp[u + 1]++] = v;
    }
    free(adj);
    *rp_out = rp;
    *col_out = col;
}

static int run_case(uint32_t n, uint32_t m, double p, uint32_t R, uint32_t seed, uint32_t K) {
    uint64_t *rp;
    uint32_t *col;
    make_graph(n, m, &rp, &col);
    int64_t *g0 = (int64_t *)calloc(n, sizeof(int64_t));
    int32_t *labels = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * R);
    uint32_t *sizes = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * R);
    CHECK(orc_label_all(n, rp, col, 0, p, NULL, R, seed, NULL, g0, labels, sizes, NULL, NULL, 3) == 0);
    for (uint32_t r = 0; r < R; ++r) {
        uint64_t tot = 0;
        for (uint32_t v = 0; v < n; ++v) {
            const int32_t l = labels[(size_t)v * R + r];
            CHECK(l >= 0 && (uint32_t)l <= v);
            if ((uint32_t)l == v) tot += sizes[(size_t)v * R + r];
        }
        CHECK(tot == n);
    }
    uint32_t *s1 = (uint32_t *)calloc(K ? K : 1, 4), *s2 = (uint32_t *)calloc(K ? K : 1, 4);
    int64_t *m1 = (int64_t *)calloc(K ? K : 1, 8), *m2 = (int64_t *)calloc(K ? K : 1, 8);
    int64_t c1 = 0, c2 = 0;
    uint64_t e1 = 0, e2 = 0;
    CHECK(orc_celf(n, rp, col, 0, p, NULL, R, seed, NULL, g0, K, s1, m1, &c1, &e1, 2) == 0);
    CHECK(orc_celf_memo(n, R, labels, sizes, g0, K, s2, m2, &c2, &e2) == 0);
    CHECK(c1 == c2);
    int64_t tot = 0;
    for (uint32_t k = 0; k < K; ++k) {
        CHECK(s1[k] == s2[k] && m1[k] == m2[k]);
        tot += m1[k];
    }
    CHECK(tot == c1);
    CHECK(orc_sigma_count(n, rp, col, 0, p, NULL, R, seed, NULL, s1, K, 2) == c1);
    /* the same CSR read as a digraph with arcs both ways: reachability equals connectivity
     * only when each arc pair shares liveness, which it does not; check consistency instead */
    uint32_t *s3 = (uint32_t *)calloc(K ? K : 1, 4);
    int64_t *m3 = (int64_t *)calloc(K ? K : 1, 8);
    int64_t c3 = 0;
    uint64_t e3 = 0;
    CHECK(orc_celf_arcs(n, rp, col, p, NULL, R, seed, K, s3, m3, &c3, &e3) == 0);
    CHECK(orc_sigma_count_arcs(n, rp, col, p, NULL, R, seed, s3, K, 2) == c3);
    free(s1);
    free(s2);
    free(s3);
    free(m1);
    free(m2);
    free(m3);
    free(g0);
    free(labels);
    free(sizes);
    free(rp);
    free(col);
    return 0;
}

int main(void) {
    CHECK(run_case(60, 150, 0.2, 64, 3, 8) == 0);
    CHECK(run_case(200, 600, 0.05, 96, 7, 20) == 0);
    CHECK(run_case(40, 100, 1.0, 16, 9, 40) == 0);  /* K = n, zero-gain rounds */
    CHECK(run_case(30, 60, 0.0, 8, 1, 5) == 0);
    printf("oracle sanitizer run ok\n");
    return 0;
}
