/*
 * libim — influence maximization by Stop-and-Stare (SSA, D-SSA) on AMD
 * Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Nguyen, Thai, Dinh,
 * "Stop-and-Stare: Optimal Sampling Algorithms for Viral Marketing in
 * Billion-scale Networks", SIGMOD 2016): given a weighted digraph
 * G = (V, E, w), a diffusion model (IC or LT, Section 2.1) and a budget
 * 1 <= k <= |V|, return k seeds S_k that maximise the expected spread
 * (Section 2.2, Definition 1).
 *
 * Conventions for every entry point:
 *   - Pointer arguments are HOST pointers unless the name says `_dev`.
 *   - Handles own all the device memory they use; the caller owns host
 *     arrays and must keep them valid for the duration of the call only.
 *   - All device work runs on the stream given to im_ctx_create; an entry
 *     point that returns results to the host synchronises that stream.
 *   - Handles are not thread-safe: serialise calls on one context.
 *   - Return IM_OK (0) or a negative im_status; im_last_error() then holds
 *     a thread-local message. Outputs are untouched on error.
 */
#ifndef IM_H
#define IM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IM_OK = 0,
    IM_E_ARG = -1,             /* invalid argument (range, ordering, null) */
    IM_E_OOM = -2,             /* device or host allocation failed */
    IM_E_LT_WEIGHTS = -3,      /* LT in-weights of some node sum above 1 */
    IM_E_DEVICE = -4,          /* a HIP call failed */
    IM_E_STREAM_MISMATCH = -5, /* pool extended with a key it was not made for */
    IM_E_STATE = -6,           /* handle in the wrong state for the call */
} im_status;

typedef enum { IM_IC = 0, IM_LT = 1 } im_model;

typedef struct im_ctx im_ctx;
typedef struct im_graph im_graph;
typedef struct im_pool im_pool;

/* Device allocator hooks: alloc returns a device pointer of >= bytes
 * (256-byte aligned) or NULL; free releases it. */
typedef void *(*im_alloc_fn)(size_t bytes, void *user);
typedef void (*im_free_fn)(void *ptr, void *user);

/*
 * Create a context on HIP device `device` whose work is queued on `stream`
 * (a hipStream_t; NULL = the null stream). alloc/free may be NULL, in which
 * case hipMalloc/hipFree are used. Errors: IM_E_ARG (bad device),
 * IM_E_DEVICE.
 */
im_status im_ctx_create(int device, void *stream, im_alloc_fn alloc, im_free_fn free_, void *user,
                        im_ctx **out);
/* Free the context's own buffers. Every engine, pool and graph made on it
 * must be freed before (they use its allocator and stream). */
void im_ctx_free(im_ctx *ctx);
/* Wait until no work of the context is in flight: its stream, its
 * side-sampling stream, and the covers of later D-SSA iterations that a run
 * dropped when it stopped before them (im_dssa returns without waiting for
 * those; their pools are freed here, or when their helper is next needed,
 * their graph is freed, or the context is freed). Errors: IM_E_ARG,
 * IM_E_DEVICE. */
im_status im_ctx_sync(im_ctx *ctx);

/*
 * Load G = (V, E, w) (Section 2) into device memory as a reverse adjacency.
 * n = |V|; m = |E|; edge e is src[e] -> dst[e]. Edges must be sorted by
 * (dst, src) with no repeated pair (the canonical order that keys every
 * edge coin). w_ic[e] is the IC activation probability of edge e and
 * w_lt[e] its LT weight (Section 2.1); either may be NULL, but not both,
 * and a graph used with a model needs that model's weights.
 * Device form: off[n+1] u64; per edge {u32 src, u32 thr}:
 *   IC thr = floor(w * 2^32) clamped to 2^32-1 (live iff coin < thr; 2^32-1
 *      is always live);
 *   LT thr = floor(2^32 * (w_1 + ... + w_i)) clamped, FP64 sum left to right
 *      over the node's in-edges (edge i kept iff thr_{i-1} <= coin < thr_i).
 * Errors: IM_E_ARG (ids >= n, unsorted or repeated pairs, w outside [0,1],
 * n == 0), IM_E_LT_WEIGHTS (some node's LT weights sum above 1 + 1e-6),
 * IM_E_OOM.
 */
im_status im_graph_load(im_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                        const float *w_ic, const float *w_lt, im_graph **out);

/*
 * Weighted RR-set sources for targeted viral marketing (Section 7.3, WRIS):
 * node_w[v] >= 0 integer relevance of v, n entries, not all zero. After this
 * call RR sets of this graph pick their source v with probability
 * node_w[v] / sum(node_w); NULL restores uniform sources (Definition 2).
 * The objective becomes the weighted spread I_w(S) (expected total weight
 * of the nodes S reaches), and since I_w(S) = W Pr[S meets an RR set] with
 * W = sum(node_w), every reported estimate (i_hat, i_c, Estimate-Inf's I_c)
 * scales by W instead of n; stopping decisions do not depend on the scale.
 * Pools created before the call are unaffected only if they are not
 * extended again. Errors: IM_E_ARG (all zero), IM_E_OOM.
 */
im_status im_graph_set_source_weights(im_graph *g, const uint32_t *node_w);
void im_graph_free(im_graph *g);

/* Graph properties: n, m, which models it holds weights for (bit 0 IC,
 * bit 1 LT) and bit 2: every node's IC in-edges share one threshold (the
 * weighted cascade w(u,v) = 1/d_in(v) of Section 7 is such a graph), so
 * the device also holds the compact IC form: per node {first in-edge,
 * in-degree, thr} in 16 bytes, per edge its u32 src (built unless
 * IM_PARAM_IC_COMPACT was 0 at load, or its memory could not be had). IC
 * draws read that form (IM_PARAM_IC_COMPACT); their sets are the same in
 * either form. */
im_status im_graph_info(const im_graph *g, uint32_t *n, uint64_t *m, uint32_t *models);

/*
 * An empty collection R of RR sets (Section 3.1.1) of one stream: set j is
 * the RR set of sample j under `stream_key`, for model `model`.
 * Errors: IM_E_ARG (graph lacks the model's weights), IM_E_OOM.
 */
im_status im_pool_create(im_ctx *ctx, const im_graph *g, im_model model, uint64_t stream_key,
                         im_pool **out);
void im_pool_free(im_pool *p);

/*
 * Append the RR sets (Definition 2) of samples [count, count + n_sets) of
 * the pool's stream. Each set is a pure function of (graph, model, key,
 * sample index): random source, then the nodes that reach it through live
 * edges (IC: reverse breadth-first search; LT: reverse walk keeping at most
 * one in-edge per node, stopping at a node with none or on a revisit).
 * Errors: IM_E_STREAM_MISMATCH (stream_key or model differs from the
 * pool's), IM_E_ARG (graph is not the pool's), IM_E_OOM, IM_E_DEVICE.
 */
im_status im_sample_rr(const im_graph *g, im_model model, uint64_t n_sets, uint64_t stream_key,
                       im_pool *pool);

/*
 * The batched form of im_sample_rr: append n_sets[i] RR sets (Definition 2)
 * to pools[i], i < n_pools, all of one graph and model, drawing the sets of
 * every pool together in fused launches of the persistent sampler (one
 * device work queue of (pool stream, sample range) items; heavy samples
 * move to workgroup tiers), at most 2^24 IC or 2^20 LT samples per launch.
 * Each pool ends as im_sample_rr would leave it: set j of a pool is a pure
 * function of (graph, model, the pool's key, j). Errors: IM_E_ARG (null
 * arguments, a pool of another graph, a pool listed twice),
 * IM_E_STREAM_MISMATCH (a pool of another model), IM_E_OOM, IM_E_DEVICE.
 */
im_status im_sample_rr_multi(const im_graph *g, im_model model, uint32_t n_pools, im_pool *const *pools,
                             const uint64_t *n_sets);

/* Number of sets and total number of node entries in the pool. */
im_status im_pool_info(const im_pool *p, uint64_t *count, uint64_t *total_nodes);

/*
 * Copy sets [begin, end) to the host: off_out[0 .. end-begin] (u64, relative
 * to the first copied set) and nodes_out (u32, off_out[end-begin] entries,
 * each set's nodes in traversal order, not sorted). Pass nodes_out = NULL to
 * get the offsets only. Errors: IM_E_ARG (range).
 */
im_status im_pool_read(const im_pool *p, uint64_t begin, uint64_t end, uint64_t *off_out,
                       uint32_t *nodes_out);

/* Device views of the pool (valid until the pool next grows or is freed):
 * poff_dev[count+1] u64 and pnodes_dev[poff[count]] u32. */
im_status im_pool_device(const im_pool *p, const uint64_t **poff_dev, const uint32_t **pnodes_dev);

/*
 * Max-Coverage (Algorithm 2) over sets [begin, end) of the pool: k greedy
 * rounds, each adding the node that covers the most not-yet-covered sets;
 * ties go to the lowest node id, chosen nodes are never chosen again (when
 * every remaining gain is 0 the lowest unchosen id is taken). Writes
 * seeds_out[k] in selection order and *cov_out = Cov_R(S_k) (Eq. 1); the
 * estimate n * Cov / |R| of Algorithm 2 is left to the caller.
 * Errors: IM_E_ARG (k == 0 or k > n, bad range).
 */
im_status im_max_coverage(const im_pool *p, uint32_t k, uint32_t *seeds_out, uint64_t *cov_out);
im_status im_max_coverage_range(const im_pool *p, uint64_t begin, uint64_t end, uint32_t k,
                                uint32_t *seeds_out, uint64_t *cov_out);

/*
 * Cov over sets [begin, end) (Eq. 1) of the seed set seeds[k] (the D-SSA
 * stare step on R^c_t, Algorithm 4). Errors: IM_E_ARG.
 */
im_status im_coverage_range(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds,
                            uint32_t k, uint64_t *cov_out);

/*
 * The count of im_coverage_range (same arguments, same result) for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation. It calls no hipMalloc,
 * hipFree or allocating routine; its scratch (counter, seed list, seed
 * bitmap) is one fixed device array of about 8.3 MiB per GPU, whose address
 * im_ctx_create takes once per device and which stays held until the process
 * ends. Limits: the pool's graph has at most 2^26 nodes and k <= 2^16.
 * Every call on one GPU shares that array (each call clears what it needs),
 * so calls that overlap on one GPU, from any contexts or threads, race: the
 * caller must serialise them. Errors: IM_E_ARG (bad range, null pointers,
 * n or k beyond the limits, seed id >= n), IM_E_STATE (no scratch address
 * for the pool's device), IM_E_DEVICE.
 */
im_status im_coverage_range_noalloc(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds,
                                    uint32_t k, uint64_t *cov_out);

/*
 * Estimate-Inf (Algorithm 3): draw RR sets of samples 0, 1, 2, ... of
 * stream `stream_key`, and at the first T with #{j <= T : R_j meets S} >=
 * Lambda2 = 1 + (1 + eps_p) Upsilon(eps_p, delta_p) return
 * *ic_out = n Lambda2 / T (W Lambda2 / T with weighted sources) and
 * *t_out = T; after floor(t_max) sets without
 * reaching it return *ic_out = -1 and *t_out = floor(t_max).
 * Errors: IM_E_ARG (eps_p, delta_p outside (0,1), seeds out of range).
 */
im_status im_estimate_inf(const im_graph *g, im_model model, const uint32_t *seeds, uint32_t k,
                          double eps_p, double delta_p, double t_max, uint64_t stream_key,
                          double *ic_out, uint64_t *t_out);

#define IM_MAX_ITERS 64

/* Statistics of one SSA / D-SSA run (host FP64 checkpoint logic). */
typedef struct im_stats {
    uint32_t iterations;     /* checkpoints visited */
    uint32_t stopped_by_cap; /* 1 if the N_max cap ended the run */
    uint64_t n_sets;         /* SSA |R| at stop; D-SSA |R_t| + |R^c_t| at stop */
    uint64_t n_verify;       /* SSA: RR sets drawn by Estimate-Inf, all iterations */
    uint64_t cov;            /* Cov_R(S_k) at stop */
    uint64_t cov_c;          /* D-SSA Cov on R^c_t; SSA Estimate-Inf T at stop */
    double i_hat;            /* n Cov / |R| at stop */
    double i_c;              /* verification estimate at stop, -1 if none */
    double eps1, eps2, eps3, eps_t;
    uint64_t edges;          /* edges traversed by every RR set drawn */
    uint64_t it_sets[IM_MAX_ITERS];
    uint64_t it_cov[IM_MAX_ITERS];
    uint64_t it_cov_c[IM_MAX_ITERS]; /* D-SSA Cov_c; SSA Estimate-Inf T (0 = not run) */
    double it_eps_t[IM_MAX_ITERS];   /* D-SSA eps_t; SSA I_c (-1 = not run / failed) */
    double ms_sample, ms_cover, ms_verify, ms_total; /* wall time per stage */
} im_stats;

/*
 * SSA (Algorithm 1) with the default eps1, eps2, eps3 of Eq. 15. Checks
 * at |R| = ceil(Lambda) 2^(t-1), t = 1, 2, ... (the schedule of the text
 * and proofs of Section 4), condition C1 Cov >= Lambda1, then Estimate-Inf
 * on stream derived_key(key, t) and condition C2 n Cov/|R| <= (1+eps1) I_c;
 * stops after the iteration whose |R| reaches N_max. seeds_out[k].
 * Errors: IM_E_ARG (k outside [1,n], eps outside (0, 1-1/e), delta outside
 * (0,1), graph lacks the model).
 */
im_status im_ssa(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                 uint32_t *seeds_out, im_stats *st);

/*
 * SSA (Algorithm 1) with a caller's precision split eps1, eps2, eps3 instead
 * of Eq. 15's: each in (0, 1) and together meeting Eq. 14,
 * (1-1/e)(eps1 + eps2 + eps1 eps2 + eps3) / ((1+eps1)(1+eps2)) <= eps.
 * Otherwise as im_ssa. Errors: those of im_ssa; IM_E_ARG for a split that
 * breaks Eq. 14.
 */
im_status im_ssa_eps(const im_graph *g, im_model model, uint32_t k, double eps, double eps1, double eps2,
                     double eps3, double delta, uint64_t key, uint32_t *seeds_out, im_stats *st);

/*
 * A precision split for im_ssa_eps following the orderings Section 4.2
 * recommends per network size: IM_NET_SMALL eps1 = 2x (eps1 above the
 * others), IM_NET_MODERATE eps1 = x (all alike), IM_NET_LARGE eps1 = x/8
 * (eps1 well below eps2 and eps3), with eps2 = eps3 = x and x the largest
 * value meeting Eq. 14. out[3] receives (eps1, eps2, eps3).
 * Errors: IM_E_ARG (unknown regime, eps outside (0, 1-1/e)).
 */
enum { IM_NET_SMALL = 0, IM_NET_MODERATE = 1, IM_NET_LARGE = 2 };
im_status im_ssa_eps_preset(int regime, double eps, double *out);

/*
 * The fixed RIS threshold of Section 3's simplified bound, taking
 * OPT_k >= k: theta = 8 (1-1/e) (ln(2/delta) + ln C(n,k)) n / (eps^2 k).
 */
double im_ris_theta(uint32_t n, uint32_t k, double eps, double delta);

/*
 * Fixed-threshold RIS: draw ceil(theta) RR sets of stream `key` (Definition
 * 2), then one Max-Coverage (Algorithm 2) over all of them. st->n_sets =
 * ceil(theta), st->cov, st->i_hat = n Cov / ceil(theta). This is the
 * sample count the stopping rules of SSA / D-SSA are measured against.
 * Errors: those of im_ssa; IM_E_OOM when the sets do not fit.
 */
im_status im_ris(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                 uint32_t *seeds_out, im_stats *st);

/*
 * D-SSA (Algorithm 4): one stream; at iteration t the first
 * N_t = ceil(Lambda) 2^(t-1) sets find S_k, the next N_t verify it
 * (condition D1 Cov_c >= Lambda1, then eps_t <= eps, condition D2); stops
 * after the iteration whose N_t reaches N_max. Same errors as im_ssa.
 */
im_status im_dssa(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                  uint32_t *seeds_out, im_stats *st);

/*
 * Kernel timing for measurement. When enabled on a context, every launch of
 * the main RR-set sampler (the pass that draws the RR sets of Definition 2
 * into staging: for IC the wave pass and its workgroup tier, for LT the
 * lane pass) is bracketed by HIP events on the context's stream;
 * im_ctx_read_timing returns the totals since the last reset.
 *   sample_launches  number of timed sampler launches
 *   sample_ms        sum of their event-measured durations
 *   sample_sets      RR sets those launches completed (deferred ones excluded)
 *   sample_steps     their edges traversed: IC in-edges examined, LT nodes
 *                    whose in-list was consulted (walk steps)
 *   sample_nodes     node entries of the sets they completed
 *   model            model of the last timed launch (IM_IC or IM_LT)
 * and the same for the IC workgroup tier launch that follows each IC one
 * (samples are counted there, not in sample_sets).
 * Errors: IM_E_ARG (null handle), IM_E_DEVICE.
 */
typedef struct im_kernel_times {
    uint64_t sample_launches;
    double sample_ms;
    uint64_t sample_sets;
    uint64_t sample_steps;
    uint64_t sample_nodes;
    int32_t model;
    int32_t reserved;
    /* IC workgroup tier (samples a wave hands on): launches, event time,
     * samples it finished, their examined edges and BFS levels */
    uint64_t group_launches;
    double group_ms;
    uint64_t group_samples;
    uint64_t group_edges;
    uint64_t group_levels;
} im_kernel_times;

im_status im_ctx_set_timing(im_ctx *ctx, int enable);

/*
 * Launch parameters of a context (what an autotuner adjusts; results never
 * depend on them):
 *   IM_PARAM_GREEDY_WG_MAX_ENTRIES  a Max-Coverage range whose node entries
 *       are at most this runs all k rounds in one workgroup; a larger one
 *       launches grid-wide kernels every round (default 0: always grid);
 *   IM_PARAM_IC_TICKET_BLOCK        consecutive samples an IC wave takes per
 *       ticket, 1..64, or 0 for the automatic choice (default 0);
 *   IM_PARAM_DSSA_SPECULATE         1: im_dssa draws the next iteration's
 *       new RR sets on a second stream (own work buffers, from a helper
 *       thread) while the current iteration is covered, and drops them if
 *       it stops; 0: strictly one step after another (default 1). Runs
 *       that draw ahead (LT with IM_PARAM_DSSA_DRAW_AHEAD above 1, IC with
 *       IM_PARAM_DSSA_IC_MIN_DRAW above 0) never sample on the side, and
 *       may then use three helpers for later iterations' covers instead of
 *       two;
 *   IM_PARAM_GREEDY_MARK_MIN_CHUNKS per-round Max-Coverage launches on a
 *       graph with more than this many 64-node chunks have the cover step
 *       mark every chunk it touches and re-derive only those; on smaller
 *       graphs each chunk's maximum holder is re-checked instead (default
 *       65536, i.e. n above 4,194,304);
 *   IM_PARAM_GREEDY_COVER_BLOCKS    workgroups per job that cover a round's
 *       seed, 1..65535, or 0 for the automatic choice (default 0);
 *   IM_PARAM_IC_EDGE_BUDGET         the most in-edges an IC sample may examine
 *       in the one-wave pass: a sample whose next frontier batch would take
 *       it past this is handed to the workgroup tiers before that batch is
 *       expanded, 64..2^31 (default 16384);
 *   IM_PARAM_GREEDY_CANDIDATES      grid-wide Max-Coverage of one range
 *       (im_max_coverage*, im_ssa*, im_dssa, im_ris) keeps this many 64-node
 *       chunks as candidates, 1..64, together with a bound on every key
 *       outside them, and takes a round in one launch while the best
 *       candidate beats that bound (two more launches re-derive the index
 *       and the candidates when it does not); 0: two launches every round
 *       (default 0);
 *   IM_PARAM_GREEDY_CANDIDATES_BATCH the same for the engine's batched
 *       Max-Coverage of many queries (default 32);
 *   IM_PARAM_DSSA_DRAW_AHEAD        when im_dssa on the LT model must draw
 *       the RR sets of iteration t, it draws up to this many times 2 N_t
 *       sets in the same launches (the sets of later iterations are
 *       identical whenever they are drawn; a launch lasts about as long as
 *       its longest walk), 1..64 (default 8; IC draws are not affected).
 *       While it is above 1, LT runs do not draw the next iteration's sets
 *       on the side;
 *   IM_PARAM_DSSA_IC_MIN_DRAW       when im_dssa on the IC model must draw
 *       the RR sets of iteration t, it also draws later iterations' sets in
 *       the same launches, up to the largest 2 N_{t+j} not above this many
 *       sets (a small IC launch lasts about as long as its deepest samples,
 *       whatever its size); 0 or a value below 2 N_t: no more than
 *       iteration t's (default 262144). While it is above 0, IC runs do not
 *       draw the next iteration's sets on the side;
 *   IM_PARAM_GREEDY_GRAPH           1: the k rounds of a grid-wide
 *       Max-Coverage of one range (two launches per round) are replayed
 *       from a HIP graph built the second time the same round count and
 *       launch shape recur (kept per context, at most 32); 0: launched one
 *       by one (default 0: replay measured slower than stream launches);
 *   IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES a Max-Coverage range of one query
 *       with at most this many (set, node) entries runs its rounds in one
 *       workgroup over up to 512 candidate nodes, keeping only their gains
 *       current; when no candidate beats the bound on the other keys, the
 *       grid recounts every gain from the covered sets and picks new
 *       candidates; if a re-selection keeps fewer than 64 candidates (and
 *       fewer than the rounds left), the remaining rounds run grid-wide, two
 *       launches each (default: every range; 0: off). Takes precedence over
 *       IM_PARAM_GREEDY_CANDIDATES, IM_PARAM_GREEDY_GRAPH and
 *       IM_PARAM_GREEDY_WG_MAX_ENTRIES;
 *   IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS the first this many rounds of such
 *       a range run grid-wide, two launches each (they cover the most sets),
 *       before the one-workgroup rounds take over (default 16);
 *   IM_PARAM_DSSA_GREEDY_AHEAD    im_dssa covers up to this many later
 *       iterations (0..3) at once, each on a helper context with its own
 *       stream and thread, once the pool holds their sets: iteration t's
 *       Max-Coverage reads only R_t, so the result is the one the iteration
 *       would compute; if the run stops first it is dropped and im_dssa
 *       returns without waiting for it (see im_ctx_sync). A helper covers
 *       its own copy of R_t, except in LT runs that draw ahead, whose pool
 *       does not grow while a helper reads it (default 3);
 *   IM_PARAM_GREEDY_WG_CAND_BATCH  the engine's batched Max-Coverage runs
 *       IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS grid-wide rounds and then
 *       one-workgroup rounds over candidate nodes, a workgroup per query,
 *       when no range has more (set, node) entries than this (nor than
 *       IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES) and the graph has no more
 *       nodes than this (a re-selection passes over every node once per
 *       query); other batches use the batched schedules above (default
 *       2^21; 0: never);
 *   IM_PARAM_IC_PLAIN              1: IC draws run as plain launches, the
 *       baseline the batched sampler is measured against: every wave takes
 *       a fixed share of the samples (wave w of W: samples w, w + W, ...)
 *       instead of tickets from the device work queue, and there are no
 *       workgroup tiers, so a sample stays with its wave until it outgrows
 *       the wave's LDS queue or visited set and then goes to the long path
 *       (one wave per sample with global visited stamps); 0: the batched
 *       persistent sampler (default 0);
 *   IM_PARAM_GREEDY_FLAT_LEVELS    1: when a range's one-workgroup rounds
 *       hand over because the gains are flat (a cut keeps too few
 *       candidates), the remaining rounds go level by level: with g* the
 *       largest gain and L the unchosen nodes of gain g* in id order, a
 *       level takes, walking L in order, every node none of whose g*
 *       uncovered sets was covered earlier in the level (exactly the
 *       rounds' argmaxes), then the gains are recounted for the next level;
 *       levels with g* above 16 use the grid-wide rounds; 0: grid-wide
 *       rounds, two launches each (default 1);
 *   IM_PARAM_GREEDY_DENSE           1: Max-Coverage (k > 1) of a range holding
 *       fewer entries than half the graph's nodes runs over the nodes the range
 *       holds, numbered by rank in id order (the same picks: a node outside
 *       the range has gain 0, and the rounds after every set is covered
 *       take the lowest unpicked ids); 0: over all n nodes (default 1);
 *   IM_PARAM_IC_COMPACT            1: IC draws on a graph that holds the
 *       compact IC form (im_graph_info bit 2) read it: 16 bytes per
 *       expanded node and 4 per examined in-edge, against 16 + 8; 0: the
 *       {src, thr} records (default 1). The sets drawn are the same. The
 *       value when a graph is loaded decides whether the form is built
 *       (4 m + 16 n bytes, left out if that memory cannot be had).
 * Errors: IM_E_ARG (unknown parameter or value out of range).
 */
typedef enum {
    IM_PARAM_GREEDY_WG_MAX_ENTRIES = 0,
    IM_PARAM_IC_TICKET_BLOCK = 1,
    IM_PARAM_DSSA_SPECULATE = 2,
    IM_PARAM_GREEDY_MARK_MIN_CHUNKS = 3,
    IM_PARAM_GREEDY_COVER_BLOCKS = 4,
    IM_PARAM_IC_EDGE_BUDGET = 5,
    IM_PARAM_GREEDY_CANDIDATES = 6,
    IM_PARAM_GREEDY_CANDIDATES_BATCH = 7,
    IM_PARAM_DSSA_DRAW_AHEAD = 8,
    IM_PARAM_GREEDY_GRAPH = 9,
    IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES = 10,
    IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS = 11,
    IM_PARAM_DSSA_GREEDY_AHEAD = 12,
    IM_PARAM_GREEDY_WG_CAND_BATCH = 13,
    IM_PARAM_IC_PLAIN = 14,
    IM_PARAM_GREEDY_FLAT_LEVELS = 15,
    IM_PARAM_GREEDY_DENSE = 16,
    IM_PARAM_DSSA_IC_MIN_DRAW = 17,
    IM_PARAM_IC_COMPACT = 18
} im_param;
im_status im_ctx_set_param(im_ctx *ctx, im_param param, uint64_t value);
im_status im_ctx_get_param(const im_ctx *ctx, im_param param, uint64_t *value);
im_status im_ctx_read_timing(im_ctx *ctx, im_kernel_times *out, int reset);

/*
 * Multi-query engine. Many SSA (Algorithm 1) and D-SSA (Algorithm 4)
 * queries advance together: each engine step issues one fused sampler
 * launch per (graph, model) holding every active query's next RR sets
 * (Definition 2) on its own stream, one fused Estimate-Inf pass
 * (Algorithm 3) for the SSA queries that passed condition C1, and one
 * batched Max-Coverage (Algorithm 2, one workgroup per query) plus stare
 * step for the queries whose pool reached their checkpoint; the FP64
 * checkpoint conditions run per query on the host exactly as in im_ssa /
 * im_dssa. A query's seeds and statistics (except the ms_* wall times,
 * which here are the query's share of shared passes) equal those of im_ssa /
 * im_dssa with the same arguments, whatever else runs beside it.
 *
 * im_query: graph (loaded on the engine's context), model, algo, k, eps,
 * delta, key: the arguments of im_ssa / im_dssa.
 */
typedef enum { IM_ALGO_SSA = 0, IM_ALGO_DSSA = 1, IM_ALGO_ESTIMATE = 2 } im_algo;

typedef struct im_query {
    const im_graph *graph;
    im_model model;
    im_algo algo;
    uint32_t k;
    double eps, delta;
    uint64_t key;
} im_query;

typedef struct im_engine im_engine;

/*
 * Create an engine on ctx. Queued queries are admitted at the start of a
 * step while fewer than max_active are active and the device bytes of the
 * active queries' RR pools are below pool_budget_bytes (one query is always
 * admitted when none is active). The engine borrows ctx, which must outlive
 * it. Errors: IM_E_ARG (null ctx/out, max_active 0), IM_E_OOM.
 */
im_status im_engine_create(im_ctx *ctx, uint64_t pool_budget_bytes, uint32_t max_active, im_engine **out);

/* Free the engine and every query it still holds (finished or not). */
void im_engine_free(im_engine *e);

/*
 * Queue a query (copied; the graph must stay loaded until its result is
 * taken). *ticket receives its id (> 0). No device work happens here.
 * Errors: those of im_ssa / im_dssa's argument checks; IM_E_ARG for a graph
 * of another context or an unknown algo.
 */
im_status im_engine_submit(im_engine *e, const im_query *q, uint64_t *ticket);

/*
 * Queue an influence-estimate query: Estimate-Inf (Algorithm 3) of the seed
 * set seeds[k] (copied) on stream `key`, exactly as im_estimate_inf, run in
 * the engine's fused verification passes beside the other queries. Its
 * result (im_engine_result) carries the seeds back, st->i_c = I_c (-1 when
 * floor(t_max) sets did not reach Lambda2), st->cov_c = st->n_verify = T,
 * st->edges. Errors: IM_E_ARG (k == 0, seed out of range, eps_p or delta_p
 * outside (0,1), t_max < 0, graph of another context or without the
 * model's weights).
 */
im_status im_engine_submit_estimate(im_engine *e, const im_graph *g, im_model model, const uint32_t *seeds,
                                    uint32_t k, double eps_p, double delta_p, double t_max, uint64_t key,
                                    uint64_t *ticket);

/*
 * One engine step: admission, then the fused sampling, verification and
 * coverage passes and every active query's checkpoint. Synchronises the
 * context's stream. *n_active / *n_pending (either may be NULL) receive the
 * queries still active / queued after the step. On a device error every
 * active query is marked failed with that status, which is also returned.
 */
im_status im_engine_step(im_engine *e, uint32_t *n_active, uint32_t *n_pending);

/* Step until no query is active or queued. */
im_status im_engine_run(im_engine *e);

/*
 * *state = 0 while the query is queued or running, 1 once its result is
 * ready, a negative im_status if it failed. Errors: IM_E_ARG (unknown
 * ticket: never issued or result already taken).
 */
im_status im_engine_poll(im_engine *e, uint64_t ticket, int *state);

/*
 * Take a finished query's result: seeds_out[k] and *st (either may be NULL),
 * then forget the ticket. A failed query returns its error status (and is
 * forgotten). Errors: IM_E_ARG (unknown ticket), IM_E_STATE (not finished).
 */
im_status im_engine_result(im_engine *e, uint64_t ticket, uint32_t *seeds_out, im_stats *st);

/* The stream key of SSA iteration i's verification pool, derived from key. */
uint64_t im_derived_key(uint64_t key, uint64_t i);

/* Message of the last failed call on this thread ("" if none). */
const char *im_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
