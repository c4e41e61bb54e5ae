/*
 * ORACLE — TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain sequential C, written for a reader who checks it against the paper
 * by eye: no blocking, no caching of random words, no fusion. Each function
 * names the passage it follows and how it is pinned by the CPU tests.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC 2011, Section 4: the Philox-4x32 round,  */
/* multipliers 0xD2511F53 and 0xCD9E8D57, Weyl key increments 0x9E3779B9 and */
/* 0xBB67AE85, ten rounds).                                                  */
/* Pinned against rocRAND's independent philox4x32_10 (test_oracle_philox).  */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static void philox_at(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    ora_philox4x32_10(ctr, k, out);
}

/* Derived stream key K_i: the fresh, independent verification stream of
 * SSA iteration i (Algorithm 1 draws R' independently of R). */
uint64_t ora_derived_key(uint64_t key, uint64_t i) {
    uint32_t w[4];
    philox_at(key, (uint32_t)i, (uint32_t)(i >> 32), 0u, 3u, w);
    return (uint64_t)w[0] | ((uint64_t)w[1] << 32);
}

/* Source of sample s: a node chosen uniformly at random (Definition 2, step
 * 1), or in proportion to integer node weights (weighted RIS for targeted
 * viral marketing, Section 7.3). Pinned by the Lemma 1 brute-force tests. */
uint32_t ora_source(const ora_graph *g, uint64_t key, uint64_t s) {
    uint32_t w[4];
    if (g->src_cum == NULL) {
        philox_at(key, (uint32_t)s, (uint32_t)(s >> 32), 0u, 0u, w);
        uint64_t r = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        return (uint32_t)(((unsigned __int128)r * g->n) >> 64);
    }
    philox_at(key, (uint32_t)s, (uint32_t)(s >> 32), 0u, 4u, w);
    uint64_t r = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    uint64_t total = g->src_cum[g->n];
    uint64_t target = (uint64_t)(((unsigned __int128)r * total) >> 64);
    /* plain linear search for the v with cum[v] <= target < cum[v+1] */
    uint32_t v = 0;
    while (!(g->src_cum[v] <= target && target < g->src_cum[v + 1])) ++v;
    return v;
}

/* IC coin of canonical edge e in sample s: one 32-bit word. */
static uint32_t coin_ic(uint64_t key, uint64_t s, uint64_t e) {
    uint32_t w[4];
    uint64_t grp = e >> 2;
    philox_at(key, (uint32_t)s, (uint32_t)(s >> 32), (uint32_t)grp, 1u | ((uint32_t)(grp >> 32) << 8), w);
    return w[e & 3];
}

/* LT coin of node v in sample s: the uniform draw that picks v's live in-edge. */
static uint32_t coin_lt(uint64_t key, uint64_t s, uint32_t v) {
    uint32_t w[4];
    philox_at(key, (uint32_t)s, (uint32_t)(s >> 32), v, 2u, w);
    return w[0];
}

/* ------------------------------------------------------------------------ */
/* Graph (Section 2). Edges arrive sorted by (dst, src) with weight w(u,v).  */
/* IC: edge (u,v) is live with probability w(u,v) (Section 2.1); stored as   */
/*     thr = floor(w * 2^32) clamped to 2^32-1; live iff coin < thr, and an  */
/*     edge with thr = 2^32-1 (w = 1) is always live.                        */
/* LT: v keeps at most one in-edge, edge i with probability w_i (the live-   */
/*     edge form of the threshold model that Kempe et al. prove equivalent); */
/*     stored as thr_i = floor(2^32 * (w_1 + ... + w_i)) clamped, the sum    */
/*     taken left to right in FP64; edge i is kept iff thr_{i-1} <= coin <   */
/*     thr_i.                                                                */
/* Pinned by the special-case and Lemma 1 tests.                             */
/* ------------------------------------------------------------------------ */
static uint32_t to_thr(double x) {
    double t = floor(x * 4294967296.0);
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    if (t <= 0.0) return 0u;
    return (uint32_t)t;
}

int ora_graph_init(ora_graph *g, int model, uint32_t n, uint64_t m, const uint32_t *src,
                   const uint32_t *dst, const float *w) {
    memset(g, 0, sizeof(*g));
    if (n == 0 || (model != ORA_IC && model != ORA_LT)) return ORA_E_ARG;
    for (uint64_t e = 0; e < m; ++e) {
        if (src[e] >= n || dst[e] >= n) return ORA_E_ARG;
        if (!(w[e] >= 0.0f && w[e] <= 1.0f)) return ORA_E_ARG;
        if (e > 0) {
            int ordered = dst[e - 1] < dst[e] || (dst[e - 1] == dst[e] && src[e - 1] < src[e]);
            if (!ordered) return ORA_E_ARG;
        }
    }
    g->n = n;
    g->m = m;
    g->model = model;
    g->off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->src = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    g->thr = (uint32_t *)malloc(sizeof(uint32_t) * (m ? m : 1));
    if (!g->off || !g->src || !g->thr) {
        ora_graph_free(g);
        return ORA_E_OOM;
    }
    for (uint64_t e = 0; e < m; ++e) g->off[dst[e] + 1]++;
    for (uint32_t v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
    for (uint64_t e = 0; e < m; ++e) g->src[e] = src[e];
    if (model == ORA_IC) {
        for (uint64_t e = 0; e < m; ++e) g->thr[e] = to_thr((double)w[e]);
    } else {
        for (uint32_t v = 0; v < n; ++v) {
            double sum = 0.0;
            for (uint64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
                sum = sum + (double)w[e];
                g->thr[e] = to_thr(sum);
            }
            if (sum > 1.0 + 1e-6) {
                ora_graph_free(g);
                return ORA_E_LT_WEIGHTS;
            }
        }
    }
    return ORA_OK;
}

int ora_graph_set_source_weights(ora_graph *g, const uint32_t *node_w) {
    free(g->src_cum);
    g->src_cum = NULL;
    if (node_w == NULL) return ORA_OK;
    uint64_t *cum = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)g->n + 1));
    if (!cum) return ORA_E_OOM;
    cum[0] = 0;
    for (uint32_t v = 0; v < g->n; ++v) cum[v + 1] = cum[v] + node_w[v];
    if (cum[g->n] == 0) {
        free(cum);
        return ORA_E_ARG;
    }
    g->src_cum = cum;
    return ORA_OK;
}

void ora_graph_free(ora_graph *g) {
    free(g->off);
    free(g->src);
    free(g->thr);
    free(g->src_cum);
    memset(g, 0, sizeof(*g));
}

/* ------------------------------------------------------------------------ */
/* RR set (Definition 2): pick the source v, draw a sample graph, return the */
/* nodes that reach v in it. The sample graph is drawn lazily: only the      */
/* in-edges of nodes already found are decided, each once.                   */
/* Pinned by Lemma 1 (exact spread by live-edge enumeration), the IC p=1     */
/* ancestor set and the p=0 / w=0 singleton cases.                           */
/* ------------------------------------------------------------------------ */
static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

uint32_t ora_rr_set(const ora_graph *g, uint64_t key, uint64_t s, uint32_t *out, uint64_t *edges) {
    /* out doubles as the BFS queue; `seen` marks members (one buffer per
     * host thread, so that independent runs may proceed on several threads) */
    static _Thread_local unsigned char *seen = NULL;
    static _Thread_local uint32_t seen_n = 0;
    if (seen_n < g->n) {
        free(seen);
        seen = (unsigned char *)calloc(g->n, 1);
        seen_n = g->n;
    }
    uint64_t examined = 0;
    uint32_t size = 0;
    uint32_t v0 = ora_source(g, key, s);
    out[size++] = v0;
    seen[v0] = 1;
    if (g->model == ORA_IC) {
        /* reverse breadth-first search over live in-edges */
        uint32_t head = 0;
        while (head < size) {
            uint32_t v = out[head++];
            for (uint64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
                examined++;
                uint32_t c = coin_ic(key, s, e);
                int live = (g->thr[e] == 0xFFFFFFFFu) || (c < g->thr[e]);
                uint32_t u = g->src[e];
                if (live && !seen[u]) {
                    seen[u] = 1;
                    out[size++] = u;
                }
            }
        }
    } else {
        /* reverse walk: each node keeps at most one in-edge */
        uint32_t v = v0;
        for (;;) {
            examined++;
            if (g->off[v] == g->off[v + 1]) break;
            uint32_t c = coin_lt(key, s, v);
            uint64_t pick = g->off[v + 1];
            for (uint64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
                if (c < g->thr[e]) {
                    pick = e;
                    break;
                }
            }
            if (pick == g->off[v + 1]) break; /* no in-edge kept */
            uint32_t u = g->src[pick];
            if (seen[u]) break; /* the walk closed a cycle */
            seen[u] = 1;
            out[size++] = u;
            v = u;
        }
    }
    for (uint32_t i = 0; i < size; ++i) seen[out[i]] = 0;
    qsort(out, size, sizeof(uint32_t), cmp_u32);
    if (edges) *edges = examined;
    return size;
}

/* ------------------------------------------------------------------------ */
/* Pool of RR sets in sample order (the collection R of Section 3.1.1).      */
/* ------------------------------------------------------------------------ */
int ora_pool_init(ora_pool *p, uint64_t key) {
    memset(p, 0, sizeof(*p));
    p->key = key;
    p->cap_sets = 1024;
    p->cap_nodes = 1 << 16;
    p->off = (uint64_t *)malloc(sizeof(uint64_t) * (p->cap_sets + 1));
    p->nodes = (uint32_t *)malloc(sizeof(uint32_t) * p->cap_nodes);
    if (!p->off || !p->nodes) return ORA_E_OOM;
    p->off[0] = 0;
    return ORA_OK;
}

/* Replace the pool's contents with given sets (used to test Max-Coverage on
 * hand-made collections). */
int ora_pool_load(ora_pool *p, uint64_t count, const uint64_t *off, const uint32_t *nodes) {
    uint64_t total = off[count];
    uint64_t *o = (uint64_t *)malloc(sizeof(uint64_t) * (count + 1));
    uint32_t *nd = (uint32_t *)malloc(sizeof(uint32_t) * (total ? total : 1));
    if (!o || !nd) return ORA_E_OOM;
    memcpy(o, off, sizeof(uint64_t) * (count + 1));
    memcpy(nd, nodes, sizeof(uint32_t) * total);
    free(p->off);
    free(p->nodes);
    p->off = o;
    p->nodes = nd;
    p->count = count;
    p->cap_sets = count;
    p->cap_nodes = total ? total : 1;
    return ORA_OK;
}

void ora_pool_free(ora_pool *p) {
    free(p->off);
    free(p->nodes);
    memset(p, 0, sizeof(*p));
}

int ora_pool_extend(ora_pool *p, const ora_graph *g, uint64_t new_count) {
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    if (!buf) return ORA_E_OOM;
    while (p->count < new_count) {
        uint64_t ex = 0;
        uint32_t size = ora_rr_set(g, p->key, p->count, buf, &ex);
        if (p->count + 1 > p->cap_sets) {
            p->cap_sets *= 2;
            p->off = (uint64_t *)realloc(p->off, sizeof(uint64_t) * (p->cap_sets + 1));
        }
        uint64_t base = p->off[p->count];
        while (base + size > p->cap_nodes) {
            p->cap_nodes *= 2;
            p->nodes = (uint32_t *)realloc(p->nodes, sizeof(uint32_t) * p->cap_nodes);
        }
        if (!p->off || !p->nodes) {
            free(buf);
            return ORA_E_OOM;
        }
        memcpy(p->nodes + base, buf, sizeof(uint32_t) * size);
        p->off[p->count + 1] = base + size;
        p->count++;
        p->edges += ex;
    }
    free(buf);
    return ORA_OK;
}

/* The same extension with the sample range split into `threads` contiguous */
/* blocks, one per host thread. Each set is a pure function of (key, s), so  */
/* the pool equals the sequential one; this exists only to time the oracle   */
/* on several host cores.                                                    */
typedef struct {
    const ora_graph *g;
    uint64_t key, s0, s1;
    uint32_t *nodes;
    uint64_t *sizes;
    uint64_t cap, used, edges;
    int failed;
} ora_block;

static void *draw_block(void *arg) {
    ora_block *b = (ora_block *)arg;
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * b->g->n);
    b->cap = 1 << 16;
    b->nodes = (uint32_t *)malloc(sizeof(uint32_t) * b->cap);
    b->sizes = (uint64_t *)malloc(sizeof(uint64_t) * (b->s1 - b->s0 + 1));
    if (!buf || !b->nodes || !b->sizes) {
        b->failed = 1;
        free(buf);
        return NULL;
    }
    for (uint64_t s = b->s0; s < b->s1; ++s) {
        uint64_t ex = 0;
        uint32_t size = ora_rr_set(b->g, b->key, s, buf, &ex);
        while (b->used + size > b->cap) {
            b->cap *= 2;
            b->nodes = (uint32_t *)realloc(b->nodes, sizeof(uint32_t) * b->cap);
            if (!b->nodes) {
                b->failed = 1;
                free(buf);
                return NULL;
            }
        }
        memcpy(b->nodes + b->used, buf, sizeof(uint32_t) * size);
        b->used += size;
        b->sizes[s - b->s0] = size;
        b->edges += ex;
    }
    free(buf);
    return NULL;
}

int ora_pool_extend_threads(ora_pool *p, const ora_graph *g, uint64_t new_count, int threads) {
    if (new_count <= p->count) return ORA_OK;
    if (threads < 1) threads = 1;
    uint64_t todo = new_count - p->count;
    if ((uint64_t)threads > todo) threads = (int)todo;
    ora_block *blocks = (ora_block *)calloc((size_t)threads, sizeof(ora_block));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!blocks || !tid) return ORA_E_OOM;
    for (int i = 0; i < threads; ++i) {
        blocks[i].g = g;
        blocks[i].key = p->key;
        blocks[i].s0 = p->count + todo * (uint64_t)i / (uint64_t)threads;
        blocks[i].s1 = p->count + todo * (uint64_t)(i + 1) / (uint64_t)threads;
        pthread_create(&tid[i], NULL, draw_block, &blocks[i]);
    }
    int rc = ORA_OK;
    for (int i = 0; i < threads; ++i) {
        pthread_join(tid[i], NULL);
        if (blocks[i].failed) rc = ORA_E_OOM;
    }
    for (int i = 0; i < threads && rc == ORA_OK; ++i) {
        ora_block *b = &blocks[i];
        uint64_t nsets = b->s1 - b->s0;
        while (p->count + nsets > p->cap_sets) {
            p->cap_sets *= 2;
            p->off = (uint64_t *)realloc(p->off, sizeof(uint64_t) * (p->cap_sets + 1));
        }
        uint64_t base = p->off[p->count];
        while (base + b->used > p->cap_nodes) {
            p->cap_nodes *= 2;
            p->nodes = (uint32_t *)realloc(p->nodes, sizeof(uint32_t) * p->cap_nodes);
        }
        if (!p->off || !p->nodes) {
            rc = ORA_E_OOM;
            break;
        }
        memcpy(p->nodes + base, b->nodes, sizeof(uint32_t) * b->used);
        for (uint64_t j = 0; j < nsets; ++j) {
            p->off[p->count + 1] = p->off[p->count] + b->sizes[j];
            p->count++;
        }
        p->edges += b->edges;
    }
    for (int i = 0; i < threads; ++i) {
        free(blocks[i].nodes);
        free(blocks[i].sizes);
    }
    free(blocks);
    free(tid);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Max-Coverage (Algorithm 2) on the sets with index in [begin, end):        */
/* k rounds; each adds the node whose addition covers the most sets not yet  */
/* covered. Readings: a node already chosen is never chosen again, ties go   */
/* to the lowest node id, and when every remaining gain is zero the lowest   */
/* unchosen id is taken, so exactly k distinct seeds are returned.           */
/* *cov = Cov_R(S_k) (Eq. 1). The estimate n*Cov/|R| is left to the caller.  */
/* Pinned by exhaustive max-coverage ((1-1/e) bound, Nemhauser et al.), by   */
/* the first-pick = most frequent node property, and by lazy evaluation.     */
/* ------------------------------------------------------------------------ */
int ora_max_coverage(const ora_pool *p, uint64_t begin, uint64_t end, uint32_t n, uint32_t k,
                     uint32_t *seeds, uint64_t *cov) {
    if (k == 0 || k > n || begin > end || end > p->count) return ORA_E_ARG;
    uint64_t nsets = end - begin;
    /* incidence lists: for each node, the sets (in [begin,end)) holding it */
    uint64_t *start = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    int64_t *cnt = (int64_t *)calloc(n, sizeof(int64_t));
    unsigned char *chosen = (unsigned char *)calloc(n, 1);
    unsigned char *covered = (unsigned char *)calloc(nsets ? nsets : 1, 1);
    if (!start || !cnt || !chosen || !covered) return ORA_E_OOM;
    for (uint64_t i = p->off[begin]; i < p->off[end]; ++i) start[p->nodes[i] + 1]++;
    for (uint32_t v = 0; v < n; ++v) start[v + 1] += start[v];
    uint64_t total = start[n];
    uint64_t *sets_of = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
    uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!sets_of || !fill) return ORA_E_OOM;
    memcpy(fill, start, sizeof(uint64_t) * ((size_t)n + 1));
    for (uint64_t j = begin; j < end; ++j)
        for (uint64_t i = p->off[j]; i < p->off[j + 1]; ++i) sets_of[fill[p->nodes[i]]++] = j - begin;
    /* marginal gain of every node = number of uncovered sets holding it */
    for (uint32_t v = 0; v < n; ++v) cnt[v] = (int64_t)(start[v + 1] - start[v]);

    uint64_t covered_count = 0;
    for (uint32_t round = 0; round < k; ++round) {
        uint32_t best = 0;
        int have = 0;
        for (uint32_t v = 0; v < n; ++v) {
            if (chosen[v]) continue;
            if (!have || cnt[v] > cnt[best]) {
                best = v;
                have = 1;
            }
        }
        chosen[best] = 1;
        seeds[round] = best;
        for (uint64_t i = start[best]; i < start[best + 1]; ++i) {
            uint64_t j = sets_of[i];
            if (covered[j]) continue;
            covered[j] = 1;
            covered_count++;
            for (uint64_t q = p->off[begin + j]; q < p->off[begin + j + 1]; ++q) cnt[p->nodes[q]]--;
        }
    }
    *cov = covered_count;
    free(start);
    free(cnt);
    free(chosen);
    free(covered);
    free(sets_of);
    free(fill);
    return ORA_OK;
}

/* Scale of an influence estimate. Lemma 1: I(S) = n Pr[S meets an RR set].
 * With sources drawn in proportion to node weights (WRIS for targeted viral
 * marketing, Section 7.3) the spread is the expected total weight of the
 * reached nodes, Pr[S meets R] = I_w(S) / W for the total weight W, and W
 * takes the place of n. Pinned by the weighted brute-force tests. */
static double estimate_scale(const ora_graph *g) {
    return g->src_cum ? (double)g->src_cum[g->n] : (double)g->n;
}

/* Cov_R(S) over the sets [begin, end) (Eq. 1). Pinned by direct set
 * intersection in the tests. */
uint64_t ora_coverage(const ora_pool *p, uint64_t begin, uint64_t end, uint32_t n,
                      const uint32_t *seeds, uint32_t k) {
    unsigned char *in_s = (unsigned char *)calloc(n, 1);
    for (uint32_t i = 0; i < k; ++i) in_s[seeds[i]] = 1;
    uint64_t c = 0;
    for (uint64_t j = begin; j < end; ++j) {
        int hit = 0;
        for (uint64_t i = p->off[j]; i < p->off[j + 1]; ++i)
            if (in_s[p->nodes[i]]) hit = 1;
        c += (uint64_t)hit;
    }
    free(in_s);
    return c;
}

/* ------------------------------------------------------------------------ */
/* Constants (Table 1, Algorithms 1, 3, 4, Eq. 15).                          */
/* Pinned by hand-derived closed forms, by the paper's printed eps defaults  */
/* for eps = 0.1 and by Table 3's D-SSA sample counts.                       */
/* ------------------------------------------------------------------------ */

/* Upsilon(eps, delta) = (2 + 2 eps/3) ln(1/delta) / eps^2, with ln(1/delta)
 * passed directly so that delta / C(n,k) never underflows. */
static double upsilon_ln(double eps, double ln_inv_delta) {
    return (2.0 + 2.0 * eps / 3.0) * ln_inv_delta / (eps * eps);
}

double ora_upsilon(double eps, double delta) { return upsilon_ln(eps, log(1.0 / delta)); }

/* ln C(n,k) as the sum of ln((n-k+i)/i) for i = 1..k. */
double ora_ln_choose(uint32_t n, uint32_t k) {
    double s = 0.0;
    for (uint32_t i = 1; i <= k; ++i) s += log((double)(n - k + i) / (double)i);
    return s;
}

static int check_args(uint32_t n, uint32_t k, double eps, double delta) {
    const double one_minus_inv_e = 1.0 - exp(-1.0);
    if (n == 0 || k == 0 || k > n) return ORA_E_ARG;
    if (!(eps > 0.0 && eps < one_minus_inv_e)) return ORA_E_ARG;
    if (!(delta > 0.0 && delta < 1.0)) return ORA_E_ARG;
    return ORA_OK;
}

/* N_max of Algorithms 1 and 4: 8 (1-1/e)/(2+2eps/3) * Upsilon(eps, delta/6/C(n,k)) * n/k. */
static double n_max_of(uint32_t n, uint32_t k, double eps, double delta) {
    const double c = 1.0 - exp(-1.0);
    double ln_inv = log(6.0 / delta) + ora_ln_choose(n, k);
    return 8.0 * c / (2.0 + 2.0 * eps / 3.0) * upsilon_ln(eps, ln_inv) * (double)n / (double)k;
}

/* Eq. 14: the precision split of SSA is admissible when each eps_i is in  */
/* (0, 1) and (1-1/e)(eps1 + eps2 + eps1 eps2 + eps3) / ((1+eps1)(1+eps2))   */
/* does not exceed eps (a relative slack of 1e-12 admits Eq. 15's split,    */
/* which meets it with equality up to rounding).                             */
int ora_eps_admissible(double eps, double eps1, double eps2, double eps3) {
    if (!(eps1 > 0.0 && eps1 < 1.0 && eps2 > 0.0 && eps2 < 1.0 && eps3 > 0.0 && eps3 < 1.0)) return 0;
    const double c = 1.0 - exp(-1.0);
    const double lhs = c * (eps1 + eps2 + eps1 * eps2 + eps3) / ((1.0 + eps1) * (1.0 + eps2));
    return lhs <= eps * (1.0 + 1e-12);
}

static int ssa_constants_from(uint32_t n, uint32_t k, double eps, double eps1, double eps2, double eps3,
                              double delta, double out[8]) {
    int rc = check_args(n, k, eps, delta);
    if (rc) return rc;
    double nmax = n_max_of(n, k, eps, delta);
    double imax = ceil(log2(2.0 * nmax / ora_upsilon(eps, delta / 3.0)));
    double lambda = ora_upsilon(eps, delta / (3.0 * imax));
    double lambda1 = (1.0 + eps1) * (1.0 + eps2) * ora_upsilon(eps3, delta / (3.0 * imax));
    /* delta_2 is not defined in the paper; Lemma 5 uses delta/(3 i_max). */
    double delta2p = delta / (3.0 * imax);
    out[0] = eps1;
    out[1] = eps2;
    out[2] = eps3;
    out[3] = nmax;
    out[4] = imax;
    out[5] = lambda;
    out[6] = lambda1;
    out[7] = delta2p;
    return ORA_OK;
}

/* A caller's split must meet Eq. 14 with every eps_i in (0, 1). */
int ora_ssa_constants_eps(uint32_t n, uint32_t k, double eps, double eps1, double eps2, double eps3,
                          double delta, double out[8]) {
    if (!ora_eps_admissible(eps, eps1, eps2, eps3)) return ORA_E_ARG;
    return ssa_constants_from(n, k, eps, eps1, eps2, eps3, delta, out);
}

/* Eq. 15's default split, as printed (for eps near 1-1/e its eps1 exceeds 1). */
int ora_ssa_constants(uint32_t n, uint32_t k, double eps, double delta, double out[8]) {
    const double c = 1.0 - exp(-1.0);
    double eps2 = eps / (2.0 * c);
    double eps3 = eps2;
    double eps1 = (1.0 + eps / (2.0 * (c - eps))) / (1.0 + eps2) - 1.0;
    return ssa_constants_from(n, k, eps, eps1, eps2, eps3, delta, out);
}

/* The fixed RIS threshold of Section 3's simplified bound: with OPT_k >= k, */
/* theta = 8 (1-1/e) (ln(2/delta) + ln C(n,k)) n / (eps^2 k) RR sets give a   */
/* (1-1/e-eps)-approximation with probability at least 1-delta.             */
double ora_ris_theta(uint32_t n, uint32_t k, double eps, double delta) {
    const double c = 1.0 - exp(-1.0);
    return 8.0 * c * (log(2.0 / delta) + ora_ln_choose(n, k)) / (eps * eps) * (double)n / (double)k;
}

int ora_dssa_constants(uint32_t n, uint32_t k, double eps, double delta, double out[4]) {
    int rc = check_args(n, k, eps, delta);
    if (rc) return rc;
    double nmax = n_max_of(n, k, eps, delta);
    double tmax = ceil(log2(2.0 * nmax / ora_upsilon(eps, delta / 3.0)));
    double lambda = ora_upsilon(eps, delta / (3.0 * tmax));
    double lambda1 = 1.0 + (1.0 + eps) * ora_upsilon(eps, delta / (3.0 * tmax));
    out[0] = nmax;
    out[1] = tmax;
    out[2] = lambda;
    out[3] = lambda1;
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Estimate-Inf (Algorithm 3): draw RR sets R_1, R_2, ... from the stream    */
/* `key`, count those that S covers, and at the first T with count >=        */
/* Lambda2 = 1 + (1+eps')Upsilon(eps',delta') return n*Lambda2/T; give up    */
/* with -1 after floor(T_max) sets.                                          */
/* Pinned by Lemma 3's one-sided error rate on graphs with exact I(S) and by */
/* the forced -1 when T_max is too small.                                    */
/* ------------------------------------------------------------------------ */
double ora_estimate_inf(const ora_graph *g, const uint32_t *seeds, uint32_t k, double eps_p,
                        double delta_p, double t_max, uint64_t key, uint64_t *t_out,
                        uint64_t *edges) {
    double lambda2 = 1.0 + (1.0 + eps_p) * ora_upsilon(eps_p, delta_p);
    unsigned char *in_s = (unsigned char *)calloc(g->n, 1);
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    for (uint32_t i = 0; i < k; ++i) in_s[seeds[i]] = 1;
    uint64_t cov = 0, ex_total = 0;
    double result = -1.0;
    uint64_t t_last = (uint64_t)floor(t_max);
    uint64_t T;
    for (T = 1; T <= t_last; ++T) {
        uint64_t ex = 0;
        uint32_t size = ora_rr_set(g, key, T - 1, buf, &ex);
        ex_total += ex;
        int hit = 0;
        for (uint32_t i = 0; i < size; ++i)
            if (in_s[buf[i]]) hit = 1;
        cov += (uint64_t)hit;
        if ((double)cov >= lambda2) {
            result = estimate_scale(g) * lambda2 / (double)T;
            break;
        }
    }
    if (t_out) *t_out = (result < 0.0) ? t_last : T;
    if (edges) *edges = ex_total;
    free(in_s);
    free(buf);
    return result;
}

/* ------------------------------------------------------------------------ */
/* SSA (Algorithm 1) with the Eq. 15 defaults. Reading of the schedule: the  */
/* text and proofs (Section 4.1, Lemma 5) put |R| = Lambda 2^(t-1) at        */
/* iteration t, so the first check is at ceil(Lambda) sets and the count     */
/* doubles after each failed check. Verification at iteration t draws from   */
/* the derived stream K_t. The loop ends after the iteration whose |R|       */
/* reaches N_max, returning that iteration's seeds.                          */
/* Pinned by the (1-1/e-eps) guarantee against exhaustive OPT_k.             */
/* ------------------------------------------------------------------------ */
static int ssa_run(const ora_graph *g, uint32_t k, const double c[8], uint64_t key, uint32_t *seeds,
                   ora_stats *st) {
    int rc;
    double eps1 = c[0], eps2 = c[1], eps3 = c[2], nmax = c[3], imax = c[4], lambda = c[5],
           lambda1 = c[6], delta2p = c[7];
    memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    ora_pool pool;
    if (ora_pool_init(&pool, key)) return ORA_E_OOM;
    uint64_t n1 = (uint64_t)ceil(lambda);
    (void)imax;
    for (uint32_t t = 1;; ++t) {
        uint64_t size = n1 << (t - 1);
        if (ora_pool_extend(&pool, g, size)) return ORA_E_OOM;
        uint64_t cov = 0;
        rc = ora_max_coverage(&pool, 0, size, g->n, k, seeds, &cov);
        if (rc) return rc;
        double i_hat = estimate_scale(g) * (double)cov / (double)size;
        st->iterations = t;
        st->n_sets = size;
        st->cov = cov;
        st->i_hat = i_hat;
        if (t <= ORA_MAX_ITERS) {
            st->it_sets[t - 1] = size;
            st->it_cov[t - 1] = cov;
            st->it_eps_t[t - 1] = -1.0;
        }
        int done = 0;
        if ((double)cov >= lambda1) { /* condition C1 */
            double t_max = 2.0 * (double)size * (1.0 + eps2) / (1.0 - eps2) * (eps3 * eps3) / (eps2 * eps2);
            uint64_t T = 0, ex = 0;
            double ic = ora_estimate_inf(g, seeds, k, eps2, delta2p, t_max, ora_derived_key(key, t), &T, &ex);
            st->n_verify += T;
            st->edges += ex;
            st->cov_c = T;
            st->i_c = ic;
            if (t <= ORA_MAX_ITERS) {
                st->it_cov_c[t - 1] = T;
                st->it_eps_t[t - 1] = ic;
            }
            if (i_hat <= (1.0 + eps1) * ic) done = 1; /* condition C2 */
        }
        if (done) break;
        if ((double)size >= nmax) {
            st->stopped_by_cap = 1;
            break;
        }
    }
    st->eps1 = eps1;
    st->eps2 = eps2;
    st->eps3 = eps3;
    st->edges += pool.edges;
    ora_pool_free(&pool);
    return ORA_OK;
}

int ora_ssa(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key,
            uint32_t *seeds, ora_stats *st) {
    double c[8];
    int rc = ora_ssa_constants(g->n, k, eps, delta, c);
    if (rc) return rc;
    return ssa_run(g, k, c, key, seeds, st);
}

/* SSA with a caller's precision split (eps1, eps2, eps3) meeting Eq. 14.    */
int ora_ssa_eps(const ora_graph *g, uint32_t k, double eps, double eps1, double eps2, double eps3,
                double delta, uint64_t key, uint32_t *seeds, ora_stats *st) {
    double c[8];
    int rc = ora_ssa_constants_eps(g->n, k, eps, eps1, eps2, eps3, delta, c);
    if (rc) return rc;
    return ssa_run(g, k, c, key, seeds, st);
}

/* Fixed-threshold RIS: ceil(theta) RR sets of stream `key`, then one        */
/* Max-Coverage over all of them. n_sets = ceil(theta), cov, i_hat.          */
int ora_ris(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key, uint32_t *seeds,
            ora_stats *st) {
    int rc = check_args(g->n, k, eps, delta);
    if (rc) return rc;
    const double theta = ora_ris_theta(g->n, k, eps, delta);
    if (!(theta < 1e12)) return ORA_E_OOM;
    const uint64_t count = (uint64_t)ceil(theta);
    memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    ora_pool pool;
    if (ora_pool_init(&pool, key)) return ORA_E_OOM;
    if (ora_pool_extend(&pool, g, count)) {
        ora_pool_free(&pool);
        return ORA_E_OOM;
    }
    uint64_t cov = 0;
    rc = ora_max_coverage(&pool, 0, count, g->n, k, seeds, &cov);
    if (rc == ORA_OK) {
        st->iterations = 1;
        st->n_sets = count;
        st->cov = cov;
        st->i_hat = estimate_scale(g) * (double)cov / (double)count;
        st->edges = pool.edges;
    }
    ora_pool_free(&pool);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* D-SSA (Algorithm 4). One stream R_1, R_2, ...; at iteration t the first   */
/* N_t = ceil(Lambda) 2^(t-1) sets find S_k and the next N_t verify it. D1:  */
/* Cov on the second half >= Lambda1; then eps1, eps2, eps3 and eps_t as     */
/* printed (with 2^(t-1)); D2: eps_t <= eps. The loop ends after the         */
/* iteration whose N_t reaches N_max. n_sets reports 2 N_t at the stop.      */
/* Pinned by the guarantee tests and by Table 3 (every D-SSA count there is  */
/* Lambda times a power of two).                                             */
/* ------------------------------------------------------------------------ */
int ora_dssa(const ora_graph *g, uint32_t k, double eps, double delta, uint64_t key,
             uint32_t *seeds, ora_stats *st) {
    double c[4];
    int rc = ora_dssa_constants(g->n, k, eps, delta, c);
    if (rc) return rc;
    const double one_minus_inv_e = 1.0 - exp(-1.0);
    double nmax = c[0], lambda = c[2], lambda1 = c[3];
    double n = estimate_scale(g);
    memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    ora_pool pool;
    if (ora_pool_init(&pool, key)) return ORA_E_OOM;
    uint64_t n1 = (uint64_t)ceil(lambda);
    for (uint32_t t = 1;; ++t) {
        uint64_t nt = n1 << (t - 1);
        if (ora_pool_extend(&pool, g, 2 * nt)) return ORA_E_OOM;
        uint64_t cov = 0;
        rc = ora_max_coverage(&pool, 0, nt, g->n, k, seeds, &cov);
        if (rc) return rc;
        double i_hat = n * (double)cov / (double)nt;
        uint64_t cov_c = ora_coverage(&pool, nt, 2 * nt, g->n, seeds, k);
        st->iterations = t;
        st->n_sets = 2 * nt;
        st->cov = cov;
        st->cov_c = cov_c;
        st->i_hat = i_hat;
        if (t <= ORA_MAX_ITERS) {
            st->it_sets[t - 1] = nt;
            st->it_cov[t - 1] = cov;
            st->it_cov_c[t - 1] = cov_c;
            st->it_eps_t[t - 1] = -1.0;
        }
        int done = 0;
        if ((double)cov_c >= lambda1) { /* condition D1 */
            double two_t1 = ldexp(1.0, (int)t - 1);
            double i_c = (double)cov_c * n / (double)nt;
            double eps1 = i_hat / i_c - 1.0;
            double eps2 = eps * sqrt(n * (1.0 + eps) / (two_t1 * i_c));
            double eps3 = eps * sqrt(n * (1.0 + eps) * (one_minus_inv_e - eps) / ((1.0 + eps / 3.0) * two_t1 * i_c));
            double eps_t = (eps1 + eps2 + eps1 * eps2) * (one_minus_inv_e - eps) + one_minus_inv_e * eps3;
            st->i_c = i_c;
            st->eps1 = eps1;
            st->eps2 = eps2;
            st->eps3 = eps3;
            st->eps_t = eps_t;
            if (t <= ORA_MAX_ITERS) st->it_eps_t[t - 1] = eps_t;
            if (eps_t <= eps) done = 1; /* condition D2 */
        }
        if (done) break;
        if ((double)nt >= nmax) {
            st->stopped_by_cap = 1;
            break;
        }
    }
    st->edges = pool.edges;
    ora_pool_free(&pool);
    return ORA_OK;
}
