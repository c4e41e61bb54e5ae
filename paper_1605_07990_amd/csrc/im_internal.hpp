// Host-side internals of libim: handles, device buffers, error reporting,
// and the launch entry points each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/im.h"

namespace im {

// Per-thread message behind im_last_error().
void set_error(const char *fmt, ...);
void clear_error();

#define IM_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t err__ = (call);                                                           \
        if (err__ != hipSuccess) {                                                           \
            ::im::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(err__), __FILE__, \
                            __LINE__);                                                       \
            return IM_E_DEVICE;                                                              \
        }                                                                                    \
    } while (0)

#define IM_TRY(expr)                          \
    do {                                      \
        im_status st__ = (expr);              \
        if (st__ != IM_OK) return st__;       \
    } while (0)

}  // namespace im

// A device allocation owned by a context.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

namespace im {
struct AheadCover;  // api.hip
}  // namespace im

struct im_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    im_alloc_fn alloc = nullptr;
    im_free_fn free_ = nullptr;
    void *user = nullptr;
    int cu_count = 0;
    size_t total_mem = 0;

    // Reusable work buffers, grown on demand and kept for the context's life.
    DevBuf stage;        // sampler staging: RR sets before compaction
    DevBuf sample_meta;  // per-sample size / staging offset / hit flags
    DevBuf handoff;      // IC search states handed from one sampler tier to the next
    DevBuf counters;     // small device counters (tickets, cursors, flags)
    DevBuf scan_tmp;     // scan partials
    DevBuf slots;        // long-path visited stamps + queues
    uint32_t slot_n = 0;      // n the slot arrays are laid out for
    uint32_t slot_count = 0;  // number of long-path slots
    uint64_t slot_epoch = 0;  // stamps handed out so far (host mirror)
    DevBuf lt_tables;    // LT per-lane visited tables
    uint32_t lt_lanes = 0;    // lanes the tables cover
    uint64_t lt_stamp = 1;    // next LT walk stamp (never 0: zeroed entries are free)
    DevBuf cover;        // incidence / greedy working arrays
    // Max-Coverage with k = 1 over growing prefixes of one pool: the counts
    // of node entries [0, k1_end) of pool k1_serial, then the argmax key
    DevBuf k1_cnt;
    uint64_t k1_serial = 0;  // 0: no counts held
    uint64_t k1_end = 0;
    DevBuf seedbits;     // seed-set bitmap (n bits)
    DevBuf flat;         // greedy rounds by gain level: state, node lists, tile counts
    DevBuf dense;        // greedy over the nodes a range holds: node bitmap, ranks, ranked entries, ids
    DevBuf prefix_off;   // a helper context's copy of the first sets of the pool it covers: offsets
    DevBuf prefix_nodes; //   and node entries
    DevBuf zflags;       // Estimate-Inf per-sample hit flags
    DevBuf items;        // fused sampler work queue + per-item accumulators
    DevBuf append_dst;   // per-item pool destinations of a fused append
    void *host_pinned = nullptr;  // small pinned staging for read-backs

    // launch parameters (im_param)
    uint64_t greedy_wg_max_entries = 0;  // grid rounds measured faster at every size tried
    uint32_t ic_ticket_block = 0;  // 0: automatic
    uint64_t greedy_mark_min_chunks = 1u << 16;
    uint32_t greedy_cover_blocks = 0;  // 0: automatic
    uint32_t ic_edge_budget = 16384;
    bool ic_plain = false;  // IC draws as plain launches (static assignment, no workgroup tiers)
    bool ic_compact = true;  // IC draws read the graph's compact form when it has one
    bool greedy_flat_levels = true;  // flat gains: rounds by gain level instead of grid-wide rounds
    bool greedy_dense = true;        // a range holding few of the nodes: the greedy over the nodes it holds
    uint32_t greedy_candidates = 0;         // one range; 0: two launches per grid-wide round
    uint32_t greedy_candidates_batch = 32;  // the engine's batched rounds
    uint32_t dssa_draw_ahead = 8;           // im_dssa on LT: a draw takes up to this many iterations' sets
    uint64_t dssa_ic_min_draw = 262144;     // im_dssa on IC: a draw takes later iterations' sets up to this many
    double greedy_stall_rate = 0.15;  // running share of rounds that re-derive the candidates
    bool greedy_graph = false;        // replay cached graphs of a range's per-round launches
    uint64_t greedy_wg_cand_max_entries = ~0ull;  // ranges up to this many entries: one-workgroup candidate rounds
    double greedy_wg_resel_rate = 0.02;           // running re-selections per round of those rounds
    uint32_t greedy_wg_cand_grid_rounds = 16;     // of which the first this many run on the grid
    uint64_t greedy_wg_cand_batch = 1ull << 21;    // batched Max-Coverage with every range up to this: a workgroup per job
    struct RoundGraphCache *round_graphs = nullptr;

    // optional event timing of the main sampler launches
    bool timing = false;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr, ev_group = nullptr;
    hipEvent_t ev_ready = nullptr;  // a helper context: its copy of a pool's sets is written
    im_kernel_times times{};

    // second sampling context on its own stream (same device and allocator,
    // own work buffers), used by a helper thread to draw the next D-SSA
    // iteration's sets while the current one is covered; created on first use
    im_ctx *aux = nullptr;
    // contexts on their own streams that run later D-SSA iterations'
    // Max-Coverage while the current one is covered; created on first use
    im_ctx *helpers[3] = {nullptr, nullptr, nullptr};
    // the work of each helper: a later iteration's cover, and, when the run
    // stopped before it, the pool it reads (freed once the cover is done)
    im::AheadCover *ahead = nullptr;
    uint32_t dssa_greedy_ahead = 3;  // later iterations covered at once (0..3)
    bool owns_stream = false;
    size_t slot_budget = 8ull << 30;  // long-path slot memory cap
    bool speculate = true;
};

// Destroys the cached greedy round graphs of a context (cover.hip).
void free_round_graphs(im_ctx *ctx);

namespace im {
// Takes the device address of the no-allocation scratch array on `device`
// (current), once per device; called by im_ctx_create (cover.hip).
im_status noalloc_scratch_init(int device);
}  // namespace im

struct im_graph {
    im_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t m = 0;
    uint32_t models = 0;         // bit 0: IC weights present, bit 1: LT weights present
    uint32_t max_in = 0;         // largest in-degree
    DevBuf off;                  // u64[n+1]
    DevBuf edges_ic;             // uint2 {src, thr}: m records, then zero records to whole 4-edge groups + 4
    DevBuf edges_lt;             // uint2[m] {src, cumulative thr}
    // IC thresholds that depend only on the target node: the compact form
    // (empty otherwise)
    DevBuf nodes_ic;             // uint4[n] {first in-edge low, high, in-degree, thr}
    DevBuf srcs_ic;              // u32 src per edge, zero-padded like edges_ic
    DevBuf src_cum;              // u64[n+1] cumulative integer source weights, or empty
    uint64_t src_total = 0;      // sum of the source weights (0: uniform sources)
    // IC, LT: mean RR-set size of the last draw (a staging estimate; draws of
    // one graph may run on several threads' contexts at once)
    mutable std::atomic<double> mean_set[2] = {0.0, 0.0};
};

// Scale of influence estimates (Lemma 1: I(S) = n Pr[S meets an RR set]).
// With sources drawn in proportion to node weights (WRIS, Section 7.3) the
// estimate is of the weighted spread, and Pr[S meets R] = I_w(S) / W with W
// the total weight, so W takes the place of n.
inline double estimate_scale(const im_graph *g) {
    return g->src_total ? double(g->src_total) : double(g->n);
}

struct im_pool {
    im_ctx *ctx = nullptr;
    const im_graph *g = nullptr;
    im_model model = IM_IC;
    uint64_t key = 0;
    uint64_t count = 0;      // sets held
    uint64_t total = 0;      // node entries held
    uint64_t edges = 0;      // edges traversed while drawing the held sets
    size_t cap_sets = 0;     // poff capacity (sets)
    size_t cap_nodes = 0;    // pnodes capacity
    DevBuf poff;             // u64[cap_sets+1]
    DevBuf pnodes;           // u32[cap_nodes]
    double mean_size = 0.0;  // running mean set size (staging estimate)
    uint64_t serial = 0;     // unique per pool made (a copy of a prefix keeps it: same sets)
};

namespace im {

// Device memory through the context's allocator (or hipMalloc).
im_status dev_alloc(im_ctx *ctx, DevBuf &b, size_t bytes);
void dev_free(im_ctx *ctx, DevBuf &b);
// Grow b to at least `bytes` (contents not preserved).
im_status dev_reserve(im_ctx *ctx, DevBuf &b, size_t bytes);
im_status to_host_sync(im_ctx *ctx, void *dst, const void *src_dev, size_t bytes);

// What a sampling pass produces.
enum class SampleMode : int {
    Pool = 0,  // store RR sets into the context's staging buffer
    Hits = 1,  // only decide whether each RR set meets the seed bitmap
};

struct SampleResult {
    uint64_t total_nodes = 0;  // Pool mode: sum of set sizes of the batch
    uint64_t edges = 0;        // edges traversed
    uint64_t deferred = 0;     // samples that took the long path
    uint64_t count = 0;        // samples drawn
};

// One query's share of a fused sampling launch: samples [s0, s0+count) of
// stream `key`; hits mode tests them against the device bitmap `seedbits`.
struct SampleItem {
    uint64_t key;
    uint64_t s0;
    uint64_t count;
    const uint32_t *seedbits;
};

struct ItemTotals {
    uint64_t nodes = 0;  // node entries of the item's sets
    uint64_t edges = 0;  // edges its samples traversed
};

// Where a fused batch's item goes: the next `count` staged slots (in item
// order) are appended to `pool`.
struct AppendItem {
    im_pool *pool;
    uint64_t count;
    uint64_t nodes;
    uint64_t edges;
};

// Draw every item in one launch (slots laid out item after item). Pool mode
// leaves the sets in ctx->stage with per-slot (offset, size) in
// ctx->sample_meta; Hits mode leaves one u8 flag per slot in ctx->zflags.
im_status sample_items(im_ctx *ctx, const im_graph *g, im_model model, const SampleItem *items, uint32_t nitems,
                       SampleMode mode, double size_hint, SampleResult *res, ItemTotals *per_item);

// Append a fused batch, item by item, to the items' pools in sample order.
im_status pool_append_items(im_ctx *ctx, const AppendItem *items, uint32_t nitems);
// In-edges the first `sets` IC sets of pool p examined (the sum of their
// nodes' in-degrees, what their draws counted), on p's context.
im_status pool_ic_edges(const im_pool *p, uint64_t sets, uint64_t *edges);

// Draw samples [s0, s0+count) of stream `key` for `model`. Pool mode leaves
// the sets in ctx->stage with per-sample (offset, size) in ctx->sample_meta;
// Hits mode leaves one u8 flag per sample in ctx->zflags (1 = meets seeds in
// ctx->seedbits).
im_status sample_batch(im_ctx *ctx, const im_graph *g, im_model model, uint64_t key, uint64_t s0,
                       uint64_t count, SampleMode mode, double size_hint, SampleResult *res);


// Max-Coverage (Algorithm 2) over pool sets [begin, end); seeds stay on
// device in ctx->cover too; seeds_host[k] and *cov are written.
im_status max_coverage(const im_pool *p, uint64_t begin, uint64_t end, uint32_t k, uint32_t *seeds_host,
                       uint64_t *cov);
// Cov of seeds over [begin, end).
im_status coverage_range(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds_host,
                         uint32_t k, uint64_t *cov);
// The same two on another context of the pool's device (its stream and
// buffers); the pool's sets in range must be complete and must not move
// while they run.
im_status max_coverage_on(im_ctx *ctx, const im_pool *p, uint64_t begin, uint64_t end, uint32_t k,
                          uint32_t *seeds_host, uint64_t *cov);
im_status coverage_range_on(im_ctx *ctx, const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds_host,
                            uint32_t k, uint64_t *cov);
// Wait for the helpers' covers (all of them, or those of graph g's pools)
// and free the pools of dropped ones.
void reap_ahead(im_ctx *ctx, const im_graph *g);
// Build ctx->seedbits from host seeds.
im_status set_seed_bits(im_ctx *ctx, uint32_t n, const uint32_t *seeds_host, uint32_t k);
// First index in zflags[0..count) where the running hit count reaches
// `need` (or -1), plus the number of hits in the range.
im_status first_crossing(im_ctx *ctx, uint64_t count, uint64_t need, int64_t *index, uint64_t *hits);

// One Max-Coverage job of a batch: greedy over pool sets [begin, end), then
// (if stare_end > stare_begin) the coverage of its seeds over
// [stare_begin, stare_end). seeds[k] is host memory.
struct CoverJob {
    const im_pool *pool;
    uint64_t begin, end;
    uint32_t k;
    uint64_t stare_begin, stare_end;
    uint32_t *seeds;
    uint64_t cov = 0;
    uint64_t cov_c = 0;
};

// Every job of one graph in one pass: a flattened incidence build, one
// workgroup per job for its k rounds, a flattened stare step.
im_status max_coverage_batch(im_ctx *ctx, const im_graph *g, CoverJob *jobs, uint32_t njobs);

// Estimate-Inf crossing search for many items of one hits-mode launch.
struct CrossItem {
    uint64_t start, count, need;
    int64_t *index;  // out: first index (relative) where the count reaches need, or -1
    uint64_t *hits;  // out: ones in the segment
};
im_status first_crossing_items(im_ctx *ctx, const CrossItem *items, uint32_t nitems);

// Estimate-Inf (Algorithm 3) with an optional expected-T hint for chunking.
im_status estimate_inf(const im_graph *g, im_model model, const uint32_t *seeds, uint32_t k, double eps_p,
                       double delta_p, double t_max, uint64_t key, double t_hint, double *ic_out,
                       uint64_t *t_out, uint64_t *edges_out);

// Graph construction kernels.
im_status graph_build(im_graph *g, const uint32_t *src, const uint32_t *dst, const float *w_ic,
                      const float *w_lt);
im_status graph_source_weights(im_graph *g, const uint32_t *node_w);

double now_ms();

// Constants of Algorithms 1 and 4 (Table 1's Upsilon; N_max, i_max = t_max,
// Lambda), computed in the order the paper writes them.
struct Caps {
    double n_max, i_max, lambda;
};
double ups_ln(double eps, double ln_inv_delta);
double upsilon(double eps, double delta);
double ln_choose(uint32_t n, uint32_t k);
Caps caps(uint32_t n, uint32_t k, double eps, double delta);
im_status check_query(const im_graph *g, im_model model, uint32_t k, double eps, double delta);
uint64_t derived_key(uint64_t key, uint64_t i);
uint64_t max_batch(im_model model);
// The context's auxiliary sampling context (created on first use).
im_status aux_ctx(im_ctx *ctx, im_ctx **out);
// Seed bitmap of n bits in `out` from host seeds.
im_status seed_bits_into(im_ctx *ctx, uint32_t n, const uint32_t *seeds_host, uint32_t k, DevBuf &out);

}  // namespace im
