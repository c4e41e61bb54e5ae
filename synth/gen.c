/*
 * Seeded synthetic input generators: directed graphs shaped like the
 * networks of the paper's experiments (Section 7, Table 2) and the edge
 * weights of its settings (Section 7.1: w(u,v) = 1/d_in(v)), plus the
 * other weight recipes of the workloads (IC trivalency, LT uniform
 * weights normalised per node).
 *
 * This module holds none of the influence-maximization arithmetic: no
 * thresholds, no coins, no RR sets. It only produces edge lists and fp32
 * weights, and both the oracle and the HIP library consume its output.
 *
 * Every random draw is a pure function of (seed, stream, index) through the
 * splitmix64 output function (Steele, Lea, Flood, OOPSLA 2014), so results
 * do not depend on the OpenMP thread count.
 *
 * Output convention: edges (src -> dst) sorted by (dst, src), no duplicate
 * pairs, no self-loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ST_PERM_OUT 1u
#define ST_PERM_IN 2u
#define ST_DRAW 3u
#define ST_KEEP 4u
#define ST_RMAT 5u
#define ST_PERM_RMAT 6u
#define ST_TRIVAL 7u
#define ST_LTW 8u
#define ST_NODEW 9u

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
    return mix64(mix64(seed + 0x9E3779B97F4A7C15ull) ^ (stream * 0xD1B54A32D192ED03ull));
}

static inline uint64_t rnd_at(uint64_t base, uint64_t i) {
    return mix64(base + (i + 1) * 0x9E3779B97F4A7C15ull);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

static inline uint32_t below(uint64_t r, uint32_t n) {
    return (uint32_t)(((unsigned __int128)r * n) >> 64);
}

/* fp32 value nearest to x that does not exceed it (x >= 0). */
static inline float f32_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, 0.0f);
    return f;
}

/* ---------------- permutations and alias tables ---------------- */

static void permutation(uint32_t n, uint64_t seed, uint32_t stream, uint32_t *p) {
    uint64_t b = stream_base(seed, stream);
    for (uint32_t i = 0; i < n; ++i) p[i] = i;
    for (uint32_t i = n; i > 1; --i) {
        uint32_t j = below(rnd_at(b, i), i);
        uint32_t t = p[i - 1];
        p[i - 1] = p[j];
        p[j] = t;
    }
}

/* Vose's alias method over n non-negative weights. */
static void alias_build(const double *w, uint32_t n, double *prob, uint32_t *alias) {
    double total = 0.0;
    for (uint32_t i = 0; i < n; ++i) total += w[i];
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t ns = 0, nl = 0;
    for (uint32_t i = 0; i < n; ++i) {
        prob[i] = w[i] * (double)n / total;
        alias[i] = i;
        if (prob[i] < 1.0) small[ns++] = i;
        else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        uint32_t s = small[--ns], l = large[nl - 1];
        alias[s] = l;
        prob[l] = (prob[l] + prob[s]) - 1.0;
        if (prob[l] < 1.0) {
            --nl;
            small[ns++] = l;
        }
    }
    while (nl > 0) prob[large[--nl]] = 1.0;
    while (ns > 0) prob[small[--ns]] = 1.0;
    free(small);
    free(large);
}

static inline uint32_t alias_draw(const double *prob, const uint32_t *alias, uint32_t n,
                                  uint64_t r1, uint64_t r2) {
    uint32_t i = below(r1, n);
    return u01(r2) < prob[i] ? i : alias[i];
}

/* ---------------- parallel LSD radix sort of u64 keys ---------------- */

#define RBITS 11
#define RBUCK (1u << RBITS)

static void radix_sort_u64(uint64_t *a, uint64_t *tmp, uint64_t len, int key_bits) {
    int nthr = omp_get_max_threads();
    uint64_t *hist = (uint64_t *)malloc(sizeof(uint64_t) * RBUCK * (size_t)nthr);
    uint64_t *src = a, *dst = tmp;
    for (int shift = 0; shift < key_bits; shift += RBITS) {
        memset(hist, 0, sizeof(uint64_t) * RBUCK * (size_t)nthr);
#pragma omp parallel num_threads(nthr)
        {
            int t = omp_get_thread_num();
            uint64_t lo = len * (uint64_t)t / (uint64_t)nthr, hi = len * (uint64_t)(t + 1) / (uint64_t)nthr;
            uint64_t *h = hist + (size_t)t * RBUCK;
            for (uint64_t i = lo; i < hi; ++i) h[(src[i] >> shift) & (RBUCK - 1)]++;
        }
        /* skip a pass whose digit is constant over the whole array */
        int trivial = 0;
        for (uint32_t d = 0; d < RBUCK; ++d) {
            uint64_t c = 0;
            for (int t = 0; t < nthr; ++t) c += hist[(size_t)t * RBUCK + d];
            if (c == len) trivial = 1;
            if (c) break;
        }
        if (trivial) continue;
        uint64_t run = 0;
        for (uint32_t d = 0; d < RBUCK; ++d)
            for (int t = 0; t < nthr; ++t) {
                uint64_t c = hist[(size_t)t * RBUCK + d];
                hist[(size_t)t * RBUCK + d] = run;
                run += c;
            }
#pragma omp parallel num_threads(nthr)
        {
            int t = omp_get_thread_num();
            uint64_t lo = len * (uint64_t)t / (uint64_t)nthr, hi = len * (uint64_t)(t + 1) / (uint64_t)nthr;
            uint64_t *h = hist + (size_t)t * RBUCK;
            for (uint64_t i = lo; i < hi; ++i) dst[h[(src[i] >> shift) & (RBUCK - 1)]++] = src[i];
        }
        uint64_t *x = src;
        src = dst;
        dst = x;
    }
    if (src != a) memcpy(a, src, sizeof(uint64_t) * len);
    free(hist);
}

static uint64_t unique_sorted(uint64_t *a, uint64_t len) {
    if (len == 0) return 0;
    uint64_t w = 1;
    for (uint64_t i = 1; i < len; ++i)
        if (a[i] != a[w - 1]) a[w++] = a[i];
    return w;
}

static int bits_for(uint64_t v) {
    int b = 1;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

/* Keep exactly m of the len sorted unique keys: the m with the smallest
 * hash mix64(key ^ salt), preserving sorted order (among equal hashes, the
 * earlier keys). The cut is found by a histogram of the hashes' top bits and
 * a sort of the one bucket that holds it, so no copy of the keys is made. */
static uint64_t keep_m_smallest_hash(uint64_t *keys, uint64_t len, uint64_t m, uint64_t salt) {
    if (len <= m) return len;
    const int hb = 20;
    const uint64_t nb = 1ull << hb;
    const int nthr = omp_get_max_threads();
    uint64_t *hist = (uint64_t *)calloc(nb * (size_t)(nthr + 1), sizeof(uint64_t));
#pragma omp parallel num_threads(nthr)
    {
        uint64_t *h = hist + nb * (size_t)(omp_get_thread_num() + 1);
#pragma omp for schedule(static)
        for (uint64_t i = 0; i < len; ++i) h[mix64(keys[i] ^ salt) >> (64 - hb)]++;
    }
    for (int t = 1; t <= nthr; ++t)
        for (uint64_t b = 0; b < nb; ++b) hist[b] += hist[nb * (size_t)t + b];
    uint64_t below = 0, bucket = 0;
    while (below + hist[bucket] < m) below += hist[bucket++];
    const uint64_t in_bucket = hist[bucket];
    free(hist);
    uint64_t *hv = (uint64_t *)malloc(sizeof(uint64_t) * (in_bucket ? in_bucket : 1));
    uint64_t c = 0;
    for (uint64_t i = 0; i < len; ++i) {
        const uint64_t h = mix64(keys[i] ^ salt);
        if ((h >> (64 - hb)) == bucket) hv[c++] = h;
    }
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (c ? c : 1));
    radix_sort_u64(hv, tmp, c, 64);
    free(tmp);
    const uint64_t cut = hv[m - below - 1];
    uint64_t below_cut = below;
    for (uint64_t i = 0; i < m - below; ++i) below_cut += (hv[i] < cut);
    free(hv);
    uint64_t need_eq = m - below_cut;
    uint64_t w = 0;
    for (uint64_t i = 0; i < len; ++i) {
        const uint64_t h = mix64(keys[i] ^ salt);
        if (h < cut || (h == cut && need_eq > 0)) {
            if (h == cut) --need_eq;
            keys[w++] = keys[i];
        }
    }
    return w;
}

static void split_keys(const uint64_t *keys, uint64_t len, uint32_t n, uint32_t *src, uint32_t *dst) {
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < len; ++i) {
        dst[i] = (uint32_t)(keys[i] / n);
        src[i] = (uint32_t)(keys[i] % n);
    }
}

/* ---------------- directed Chung-Lu power-law graph ---------------- */

static double top_degree(double i0, double alpha, uint32_t n, uint64_t m) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (uint32_t i = 0; i < n; ++i) s += pow((double)i + i0, -alpha);
    return (double)m * pow(i0, -alpha) / s;
}

/*
 * Directed Chung-Lu graph with n nodes and exactly m distinct edges (when
 * the draw stream can supply them). Out- and in-weights both follow
 * w_i = (i + i0)^(-1/(gamma-1)) over rank i, assigned to nodes through two
 * independent seeded permutations; i0 is set so the largest expected degree
 * is min(n-1, 10 sqrt(m)). Endpoints are drawn from alias tables, self-loops
 * and repeated pairs are rejected, and if more than m distinct pairs were
 * drawn the m with the smallest keyed hash are kept.
 * Returns the number of edges written (m), or -1 on allocation failure.
 */
int64_t synth_chung_lu(uint32_t n, uint64_t m, double gamma, uint64_t seed,
                       uint32_t *src_out, uint32_t *dst_out) {
    if (n < 2 || gamma <= 1.0) return -1;
    double alpha = 1.0 / (gamma - 1.0);
    double target = fmin((double)n - 1.0, 10.0 * sqrt((double)m));
    double lo = log(1e-9), hi = log(1e12);
    for (int it = 0; it < 50; ++it) {
        double mid = 0.5 * (lo + hi);
        if (top_degree(exp(mid), alpha, n, m) > target) lo = mid;
        else hi = mid;
    }
    double i0 = exp(0.5 * (lo + hi));

    double *w = (double *)malloc(sizeof(double) * n);
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
    double *prob_out = (double *)malloc(sizeof(double) * n), *prob_in = (double *)malloc(sizeof(double) * n);
    uint32_t *al_out = (uint32_t *)malloc(sizeof(uint32_t) * n), *al_in = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!w || !perm || !prob_out || !prob_in || !al_out || !al_in) return -1;

    double *wn = (double *)malloc(sizeof(double) * n);
    permutation(n, seed, ST_PERM_OUT, perm);
    for (uint32_t i = 0; i < n; ++i) w[i] = pow((double)i + i0, -alpha);
    for (uint32_t i = 0; i < n; ++i) wn[perm[i]] = w[i];
    alias_build(wn, n, prob_out, al_out);
    permutation(n, seed, ST_PERM_IN, perm);
    for (uint32_t i = 0; i < n; ++i) wn[perm[i]] = w[i];
    alias_build(wn, n, prob_in, al_in);
    free(wn);
    free(w);
    free(perm);

    int key_bits = bits_for((uint64_t)n * n - 1);
    uint64_t cap = m + m / 4 + 1024;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    uint64_t len = 0, drawn = 0, batch = m;
    uint64_t base = stream_base(seed, ST_DRAW);
    for (int round = 0; round < 64 && len < m; ++round) {
        if (len + batch > cap) {
            cap = len + batch;
            keys = (uint64_t *)realloc(keys, sizeof(uint64_t) * cap);
            if (!keys) return -1;
        }
        uint64_t *dst = keys + len;
#pragma omp parallel for schedule(static)
        for (uint64_t t = 0; t < batch; ++t) {
            uint64_t d = drawn + t;
            uint32_t u = alias_draw(prob_out, al_out, n, rnd_at(base, 4 * d), rnd_at(base, 4 * d + 1));
            uint32_t v = alias_draw(prob_in, al_in, n, rnd_at(base, 4 * d + 2), rnd_at(base, 4 * d + 3));
            dst[t] = (u == v) ? UINT64_MAX : (uint64_t)v * n + u;
        }
        drawn += batch;
        uint64_t tot = len + batch;
        uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * tot);
        if (!tmp) return -1;
        radix_sort_u64(keys, tmp, tot, 64);
        free(tmp);
        while (tot > 0 && keys[tot - 1] == UINT64_MAX) --tot;
        len = unique_sorted(keys, tot);
        if (len < m) {
            double yield = (double)len / (double)drawn;
            batch = (uint64_t)((double)(m - len) / (yield > 1e-3 ? yield : 1e-3) * 1.15) + 1024;
        }
    }
    (void)key_bits;
    free(prob_out);
    free(prob_in);
    free(al_out);
    free(al_in);
    len = keep_m_smallest_hash(keys, len, m, stream_base(seed, ST_KEEP));
    split_keys(keys, len, n, src_out, dst_out);
    free(keys);
    return (int64_t)len;
}

/* ---------------- R-MAT ---------------- */

/*
 * R-MAT graph on 2^scale nodes from `draws` recursive quadrant draws with
 * probabilities (a, b, c, 1-a-b-c); node ids are relabelled by a seeded
 * permutation; self-loops and repeated pairs are dropped. Output capacity
 * must be >= draws. Returns the number of distinct edges written.
 */
int64_t synth_rmat(int scale, uint64_t draws, double a, double b, double c, uint64_t seed,
                   uint32_t *src_out, uint32_t *dst_out) {
    if (scale < 1 || scale > 31) return -1;
    uint32_t n = 1u << scale;
    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * draws);
    if (!perm || !keys) return -1;
    permutation(n, seed, ST_PERM_RMAT, perm);
    uint64_t base = stream_base(seed, ST_RMAT);
    double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (uint64_t t = 0; t < draws; ++t) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            double r = u01(rnd_at(base, t * (uint64_t)scale + (uint64_t)l));
            uint32_t bu = (r >= ab), bv = (r >= a && r < ab) || (r >= abc);
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        u = perm[u];
        v = perm[v];
        keys[t] = (u == v) ? UINT64_MAX : (uint64_t)v * n + u;
    }
    free(perm);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * draws);
    if (!tmp) return -1;
    radix_sort_u64(keys, tmp, draws, 64);
    free(tmp);
    uint64_t tot = draws;
    while (tot > 0 && keys[tot - 1] == UINT64_MAX) --tot;
    uint64_t len = unique_sorted(keys, tot);
    split_keys(keys, len, n, src_out, dst_out);
    free(keys);
    return (int64_t)len;
}

/* ---------------- weights (indexed by the sorted edge order) ---------------- */

/* In-degree of every node from dst[] (edges sorted by dst). */
void synth_in_degree(uint32_t n, uint64_t m, const uint32_t *dst, uint32_t *deg) {
    memset(deg, 0, sizeof(uint32_t) * n);
    for (uint64_t e = 0; e < m; ++e) deg[dst[e]]++;
}

/* Weighted cascade: w(u,v) = 1/d_in(v), rounded down to fp32 so that the
 * weights into a node never sum above 1. */
void synth_weights_wc(uint32_t n, uint64_t m, const uint32_t *dst, float *w) {
    uint32_t *deg = (uint32_t *)malloc(sizeof(uint32_t) * n);
    synth_in_degree(n, m, dst, deg);
#pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < m; ++e) w[e] = f32_down(1.0 / (double)deg[dst[e]]);
    free(deg);
}

/* Trivalency: each edge's probability drawn uniformly from {0.1, 0.01, 0.001}. */
void synth_weights_trivalency(uint64_t m, uint64_t seed, float *w) {
    static const float vals[3] = {0.1f, 0.01f, 0.001f};
    uint64_t base = stream_base(seed, ST_TRIVAL);
#pragma omp parallel for schedule(static)
    for (uint64_t e = 0; e < m; ++e) w[e] = vals[below(rnd_at(base, e), 3)];
}

/* LT weights: a uniform(0,1) draw per edge, divided by the node's sum of
 * draws (FP64, in sorted edge order), rounded down to fp32 (sum <= 1). */
void synth_weights_lt_uniform(uint32_t n, uint64_t m, const uint32_t *dst, uint64_t seed, float *w) {
    (void)n;
    uint64_t base = stream_base(seed, ST_LTW);
    uint64_t e = 0;
    while (e < m) {
        uint64_t f = e;
        double s = 0.0;
        while (f < m && dst[f] == dst[e]) {
            s += u01(rnd_at(base, f)) + 0x1.0p-53;
            ++f;
        }
        for (uint64_t i = e; i < f; ++i) w[i] = f32_down((u01(rnd_at(base, i)) + 0x1.0p-53) / s);
        e = f;
    }
}

/* Integer node weights with a power-law spread, for weighted RR-set sources
 * (a user's topic relevance as a keyword count). Zero for a node outside the
 * target group; a seeded fraction `frac` of the nodes is in the group. */
void synth_node_weights(uint32_t n, double frac, double gamma, uint64_t seed, uint32_t *w) {
    uint64_t base = stream_base(seed, ST_NODEW);
    double alpha = 1.0 / (gamma - 1.0);
#pragma omp parallel for schedule(static)
    for (uint32_t v = 0; v < n; ++v) {
        double r = u01(rnd_at(base, 2 * (uint64_t)v));
        if (r >= frac) {
            w[v] = 0;
        } else {
            double x = u01(rnd_at(base, 2 * (uint64_t)v + 1)) + 0x1.0p-54;
            double c = floor(pow(x, -alpha));
            w[v] = c > 1e6 ? 1000000u : (uint32_t)c;
        }
    }
}
