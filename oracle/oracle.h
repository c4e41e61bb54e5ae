/*
 * ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately unoptimised CPU implementation of what
 * the Stop-and-Stare method computes (Nguyen, Thai, Dinh, "Stop-and-Stare:
 * Optimal Sampling Algorithms for Viral Marketing in Billion-scale
 * Networks", SIGMOD 2016, arXiv 1605.07990). It exists to check the HIP
 * library: only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code with the library.
 *
 * Paper anchors:
 *   graph and weights ............ Section 2 (G = (V, E, w), w in [0,1])
 *   IC / LT diffusion ............ Section 2.1
 *   RR set ........................ Section 3.1.1, Definition 2
 *   coverage, estimator .......... Section 3.1.1, Eq. 1 and Lemma 1
 *   Upsilon ....................... Table 1 and Corollary 1
 *   SSA ........................... Section 4, Algorithm 1, Eq. 15 defaults
 *   Max-Coverage .................. Algorithm 2
 *   Estimate-Inf .................. Algorithm 3
 *   D-SSA ......................... Section 6, Algorithm 4
 *
 * Randomness: the paper does not fix a generator. Every coin is a
 * Philox4x32-10 word (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers:
 * As Easy as 1, 2, 3", SC 2011) at a counter that names (sample, edge) or
 * (sample, node), so an RR set is a pure function of (key, sample index).
 * Counter layout (key = (lo32 K, hi32 K)):
 *   source of sample s ..... ctr (lo s, hi s, 0, 0); r = w0 | w1<<32;
 *                            source = floor(r * n / 2^64)
 *   IC coin of edge e ...... ctr (lo s, hi s, lo(e>>2), 1 | hi(e>>2)<<8); word e&3
 *   LT coin at node v ...... ctr (lo s, hi s, v, 2); word 0
 *   weighted source of s ... ctr (lo s, hi s, 0, 4); r = w0 | w1<<32;
 *                            target = floor(r * W / 2^64) for total weight W;
 *                            source = the v with cum(v) <= target < cum(v+1)
 *   derived key K_i ........ ctr (lo i, hi i, 0, 3) under key K; w0 | w1<<32
 *
 * Parity status of each function is stated at its definition in oracle.c.
 */
#ifndef IM_ORACLE_H
#define IM_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_IC = 0, ORA_LT = 1 };

enum {
    ORA_OK = 0,
    ORA_E_ARG = -1,
    ORA_E_OOM = -2,
    ORA_E_LT_WEIGHTS = -3,
};

/* Reverse adjacency: the in-edges of v are [off[v], off[v+1]); edge e runs
 * src[e] -> v and carries the 32-bit threshold thr[e]. */
typedef struct {
    uint32_t n;
    uint64_t m;
    int model;
    uint64_t *off;
    uint32_t *src;
    uint32_t *thr;
    /* optional integer source weights for weighted RR sampling: src_cum[v]
     * is the sum of the weights of nodes 0..v-1 (n+1 entries), else NULL */
    uint64_t *src_cum;
} ora_graph;

/* Collection of RR sets in sample order: set j is nodes[off[j] .. off[j+1]). */
typedef struct {
    uint64_t key;
    uint64_t count;
    uint64_t cap_sets;
    uint64_t cap_nodes;
    uint64_t *off;
    uint32_t *nodes;
    uint64_t edges; /* edges traversed, summed over the sets */
} ora_pool;

#define ORA_MAX_ITERS 64

typedef struct {
    uint32_t iterations;
    uint32_t stopped_by_cap;
    uint64_t n_sets;    /* SSA: |R| at stop; D-SSA: |R_t| + |R^c_t| at stop */
    uint64_t n_verify;  /* SSA: RR sets drawn by Estimate-Inf, all iterations */
    uint64_t cov;       /* Cov_R(S_k) at stop */
    uint64_t cov_c;     /* D-SSA: Cov on R^c_t; SSA: Estimate-Inf T at stop */
    double i_hat;       /* n * Cov / |R| at stop */
    double i_c;         /* verification estimate at stop (-1 if none) */
    double eps1, eps2, eps3, eps_t;
    uint64_t edges;     /* edges traversed by every RR set drawn */
    /* per-iteration log */
    uint64_t it_sets[ORA_MAX_ITERS];
    uint64_t it_cov[ORA_MAX_ITERS];
    uint64_t it_cov_c[ORA_MAX_ITERS]; /* D-SSA Cov_c; SSA Estimate-Inf T (0 = not run) */
    double it_eps_t[ORA_MAX_ITERS];   /* D-SSA eps_t; SSA I_c */
} ora_stats;

/* ---- graph ---- */
int ora_graph_init(ora_graph *g, int model, uint32_t n, uint64_t m, const uint32_t *src,
                   const uint32_t *dst, const float *w);
int ora_graph_set_source_weights(ora_graph *g, const uint32_t *node_w);
void ora_graph_free(ora_graph *g);

/* ---- randomness ---- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t ora_source(const ora_graph *g, uint64_t key, uint64_t s);
uint64_t ora_derived_key(uint64_t key, uint64_t i);

/* ---- RR sets ---- */
/* One RR set, sorted ascending, into out (capacity n). Returns |R|.
 * *edges receives the edges traversed (IC: sum of in-degrees of the set's
 * nodes; LT: number of in-lists consulted, i.e. |R|). */
uint32_t ora_rr_set(const ora_graph *g, uint64_t key, uint64_t s, uint32_t *out, uint64_t *edges);

int ora_pool_init(ora_pool *p, uint64_t key);
int ora_pool_extend(ora_pool *p, const ora_graph *g, uint64_t new_count);
/* the same sets drawn by `threads` host threads over contiguous blocks */
int ora_pool_extend_threads(ora_pool *p, const ora_graph *g, uint64_t new_count, int threads);
int ora_pool_load(ora_pool *p, uint64_t count, const uint64_t *off, const uint32_t *nodes);
void ora_pool_free(ora_pool *p);

/* ---- Max-Coverage (Algorithm 2) over sets [begin, end) ---- */
int ora_max_coverage(const ora_pool *p, uint64_t begin, uint64_t end, uint32_t n, uint32_t k,
                     uint32_t *seeds, uint64_t *cov);
uint64_t ora_coverage(const ora_pool *p, uint64_t begin, uint64_t end, uint32_t n,
                      const uint32_t *seeds, uint32_t k);

/* ---- constants ---- */
double ora_upsilon(double eps, double delta);
double ora_ln_choose(uint32_t n, uint32_t k);
/* out[]: eps1, eps2, eps3, n_max, i_max, lambda, lambda1, delta2p */
int ora_ssa_constants(uint32_t n, uint32_t k, double eps, double delta, double out[8]);
int ora_ssa_constants_eps(uint32_t n, uint32_t k, double eps, double eps1, double eps2, double eps3,
                          double delta, double out[8]);
/* 1 when (eps1, eps2, eps3) meets Eq. 14 for eps */
int ora_eps_admissible(double eps, double eps1, double eps2, double eps3);
/* fixed RIS threshold (simplified bound with OPT_k >= k) */
double ora_ris_theta(uint32_t n, uint32_t k, double eps, double delta);
/* out[]: n_max, t_max, lambda, lambda1 */
int ora_dssa_constants(uint32_t n, uint32_t k, double eps, double delta, double out[4]);

/* ---- Estimate-Inf (Algorithm 3) ---- */
double ora_estimate_inf(const ora_graph *g, const uint32_t *seeds, uint32_t k, double eps_p,
                        double delta_p, double t_max, uint64_t key, uint64_t *t_out,
                        uint64_t *edges);

/* ---- SSA (Algorithm 1) and D-SSA (Algorithm 4) ---- */
int ora_ssa(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key,
            uint32_t *seeds, ora_stats *st);
int ora_dssa(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key,
             uint32_t *seeds, ora_stats *st);
int ora_ssa_eps(const ora_graph *g, uint32_t k, double eps, double eps1, double eps2, double eps3,
                double delta, uint64_t key, uint32_t *seeds, ora_stats *st);
int ora_ris(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key, uint32_t *seeds,
            ora_stats *st);

#ifdef __cplusplus
}
#endif
#endif
