// C-ABI entry points of libim and the host-side checkpoint logic of SSA
// (Algorithm 1) and D-SSA (Algorithm 4), kept in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <atomic>
#include <thread>
#include <vector>

#include "im_internal.hpp"

namespace im {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

im_status dev_alloc(im_ctx *ctx, DevBuf &b, size_t bytes) {
    b.ptr = nullptr;
    b.bytes = 0;
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (ctx->alloc) {
        p = ctx->alloc(bytes, ctx->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) {
        set_error("device allocation of %zu bytes failed", bytes);
        return IM_E_OOM;
    }
    b.ptr = p;
    b.bytes = bytes;
    return IM_OK;
}

void dev_free(im_ctx *ctx, DevBuf &b) {
    if (b.ptr) {
        if (ctx->free_) {
            ctx->free_(b.ptr, ctx->user);
        } else {
            (void)hipFree(b.ptr);
        }
    }
    b.ptr = nullptr;
    b.bytes = 0;
}

im_status dev_reserve(im_ctx *ctx, DevBuf &b, size_t bytes) {
    if (b.ptr && b.bytes >= bytes) return IM_OK;
    // the stream may still use the old buffer
    IM_HIP(hipStreamSynchronize(ctx->stream));
    dev_free(ctx, b);
    size_t want = bytes + bytes / 4;
    return dev_alloc(ctx, b, want);
}

im_status to_host_sync(im_ctx *ctx, void *dst, const void *src_dev, size_t bytes) {
    IM_HIP(hipMemcpyAsync(ctx->host_pinned, src_dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    IM_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(dst, ctx->host_pinned, bytes);
    return IM_OK;
}

// Philox4x32-10 on the host (Salmon et al., SC 2011), for derived keys.
static void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = uint64_t(0xD2511F53u) * c[0];
        const uint64_t pb = uint64_t(0xCD9E8D57u) * c[2];
        const uint32_t n0 = uint32_t(pb >> 32) ^ c[1] ^ k0;
        const uint32_t n1 = uint32_t(pb);
        const uint32_t n2 = uint32_t(pa >> 32) ^ c[3] ^ k1;
        const uint32_t n3 = uint32_t(pa);
        c[0] = n0;
        c[1] = n1;
        c[2] = n2;
        c[3] = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

uint64_t derived_key(uint64_t key, uint64_t i) {
    uint32_t c[4] = {uint32_t(i), uint32_t(i >> 32), 0u, 3u};
    philox_host(c, uint32_t(key), uint32_t(key >> 32));
    return uint64_t(c[0]) | (uint64_t(c[1]) << 32);
}

// ---- constants (Table 1, Algorithms 1, 3, 4, Eq. 15) ----

double ups_ln(double eps, double ln_inv_delta) {
    return (2.0 + 2.0 * eps / 3.0) * ln_inv_delta / (eps * eps);
}

double upsilon(double eps, double delta) { return ups_ln(eps, std::log(1.0 / delta)); }

double ln_choose(uint32_t n, uint32_t k) {
    double s = 0.0;
    for (uint32_t i = 1; i <= k; ++i) s += std::log(double(n - k + i) / double(i));
    return s;
}

// N_max = 8 (1-1/e)/(2+2eps/3) Upsilon(eps, delta/6/C(n,k)) n/k ;
// i_max = ceil(log2(2 N_max / Upsilon(eps, delta/3))) ;
// Lambda = Upsilon(eps, delta/(3 i_max)).
Caps caps(uint32_t n, uint32_t k, double eps, double delta) {
    const double one_m = 1.0 - std::exp(-1.0);
    Caps c;
    c.n_max = 8.0 * one_m / (2.0 + 2.0 * eps / 3.0) * ups_ln(eps, std::log(6.0 / delta) + ln_choose(n, k)) * double(n) /
              double(k);
    c.i_max = std::ceil(std::log2(2.0 * c.n_max / upsilon(eps, delta / 3.0)));
    c.lambda = upsilon(eps, delta / (3.0 * c.i_max));
    return c;
}

im_status check_query(const im_graph *g, im_model model, uint32_t k, double eps, double delta) {
    const double one_m = 1.0 - std::exp(-1.0);
    if (!g) {
        set_error("null graph");
        return IM_E_ARG;
    }
    if (model != IM_IC && model != IM_LT) {
        set_error("unknown model %d", int(model));
        return IM_E_ARG;
    }
    if (!(g->models & (model == IM_IC ? 1u : 2u))) {
        set_error("graph has no %s weights", model == IM_IC ? "IC" : "LT");
        return IM_E_ARG;
    }
    if (k == 0 || k > g->n) {
        set_error("k = %u outside [1, n = %u]", k, g->n);
        return IM_E_ARG;
    }
    if (!(eps > 0.0 && eps < one_m)) {
        set_error("eps = %g outside (0, 1-1/e)", eps);
        return IM_E_ARG;
    }
    if (!(delta > 0.0 && delta < 1.0)) {
        set_error("delta = %g outside (0, 1)", delta);
        return IM_E_ARG;
    }
    return IM_OK;
}

// Largest batch drawn at once: LT reserves a staging region per sample.
uint64_t max_batch(im_model model) { return model == IM_LT ? (1ull << 20) : (1ull << 24); }

// Max-Coverage of a later D-SSA iteration's R_t = [0, N_t) and its stare
// count over [N_t, 2 N_t), on a helper context in a thread of its own. The
// result depends only on those sets, so it is the iteration's own whenever
// the run gets there. If the run stops first, the cover is dropped but not
// waited for: the slot keeps the run's pool (`orphan`) until the thread has
// returned, and the pool is freed when the slot is next reaped.
struct AheadCover {
    std::thread th;
    bool running = false;            // started and not joined
    std::atomic<bool> done{false};   // the thread has returned
    const im_pool *pool = nullptr;   // the run's pool (which run the cover belongs to)
    im_pool *orphan = nullptr;       // owned: the run that started it has returned
    im_pool snap;                    // what it reads: a copy of the pool's first sets, or the pool as it was
    bool stared = false;             // that held [N_t, 2 N_t) too, and cov_c was counted
    im_status rc = IM_OK;
    std::string err;
    uint64_t nt = 0, cov = 0, cov_c = 0;
    std::vector<uint32_t> seeds;

    // `copy` describes what the helper reads: a pool over its own buffers
    // holding the first copy.count sets, or the run's pool itself (which
    // then does not move until the cover is joined)
    void start(im_ctx *h, const im_pool *p, const im_pool &copy, uint64_t n_t, uint32_t k) {
        nt = n_t;
        pool = p;
        snap = copy;
        stared = copy.count >= 2 * n_t;
        seeds.assign(k, 0u);
        rc = IM_OK;
        done = false;
        running = true;
        th = std::thread([this, h, k] {
            if (hipSetDevice(h->device) != hipSuccess) {
                rc = IM_E_DEVICE;
                err = "hipSetDevice failed in the cover thread";
            } else {
                rc = max_coverage_on(h, &snap, 0, nt, k, seeds.data(), &cov);
                if (rc == IM_OK && stared) rc = coverage_range_on(h, &snap, nt, 2 * nt, seeds.data(), k, &cov_c);
                if (rc == IM_OK) rc = hipStreamSynchronize(h->stream) == hipSuccess ? IM_OK : IM_E_DEVICE;
                if (rc != IM_OK) err = im_last_error();
            }
            done = true;
        });
    }
    bool busy() const { return running && !done; }
};

// Copy the first `upto` sets of pool p into helper h's prefix buffers, on
// the run's stream (after the work that wrote them), with h's stream made
// to wait for the copy, and describe the copy as a pool: a helper covers
// it, so the run's pool may grow and move meanwhile.
static im_status copy_prefix(im_ctx *ctx, const im_pool *p, im_ctx *h, uint64_t upto, im_pool *copy) {
    uint64_t tot = p->total;  // every set copied: all node entries
    if (upto < p->count) IM_TRY(to_host_sync(ctx, &tot, static_cast<const uint64_t *>(p->poff.ptr) + upto, 8));
    IM_TRY(dev_reserve(h, h->prefix_off, (upto + 1) * 8));
    IM_TRY(dev_reserve(h, h->prefix_nodes, std::max<uint64_t>(tot, 1) * 4));
    IM_HIP(hipMemcpyAsync(h->prefix_off.ptr, p->poff.ptr, (upto + 1) * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (tot) IM_HIP(hipMemcpyAsync(h->prefix_nodes.ptr, p->pnodes.ptr, tot * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (!h->ev_ready) IM_HIP(hipEventCreateWithFlags(&h->ev_ready, hipEventDisableTiming));
    IM_HIP(hipEventRecord(h->ev_ready, ctx->stream));
    IM_HIP(hipStreamWaitEvent(h->stream, h->ev_ready, 0));
    *copy = *p;
    copy->ctx = h;
    copy->poff = h->prefix_off;
    copy->pnodes = h->prefix_nodes;
    copy->count = upto;
    copy->total = tot;
    copy->cap_sets = upto;
    copy->cap_nodes = tot;
    return IM_OK;
}

constexpr int kAheadSlots = 3;

// Join slot i. A dropped cover's pool may be shared by several slots (the
// run left a cover in each): it is freed by the join that leaves no slot
// holding it. Only the thread that runs the queries calls this.
static im_status join_slot(AheadCover *a, int i) {
    AheadCover &s = a[i];
    if (!s.running) return IM_OK;
    s.th.join();
    s.running = false;
    s.pool = nullptr;
    if (s.orphan) {
        im_pool *p = s.orphan;
        s.orphan = nullptr;
        bool held = false;
        for (int j = 0; j < kAheadSlots; ++j) held = held || (a[j].running && a[j].orphan == p);
        if (!held) im_pool_free(p);
        return IM_OK;  // a dropped cover's outcome is not used
    }
    if (s.rc != IM_OK) set_error("%s", s.err.c_str());
    return s.rc;
}

static AheadCover *ahead_slots(im_ctx *ctx) {
    if (!ctx->ahead) ctx->ahead = new (std::nothrow) AheadCover[kAheadSlots];
    return ctx->ahead;
}

void reap_ahead(im_ctx *ctx, const im_graph *g) {
    if (!ctx->ahead) return;
    for (int i = 0; i < kAheadSlots; ++i) {
        AheadCover &a = ctx->ahead[i];
        if (a.running && (!g || !a.pool || a.pool->g == g)) (void)join_slot(ctx->ahead, i);
    }
    clear_error();
}

// A context on the same device and allocator with its own stream and work
// buffers (its launch parameters are copied from ctx on each use).
static im_status new_side_ctx(im_ctx *ctx, im_ctx **out) {
    auto *a = new (std::nothrow) im_ctx();
    if (!a) return IM_E_OOM;
    a->device = ctx->device;
    a->alloc = ctx->alloc;
    a->free_ = ctx->free_;
    a->user = ctx->user;
    a->cu_count = ctx->cu_count;
    a->total_mem = ctx->total_mem;
    a->slot_budget = ctx->slot_budget;
    a->speculate = false;
    if (hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking) != hipSuccess) {
        delete a;
        set_error("helper stream creation failed");
        return IM_E_DEVICE;
    }
    a->owns_stream = true;
    if (hipHostMalloc(&a->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(a->stream);
        delete a;
        set_error("pinned host allocation failed");
        return IM_E_OOM;
    }
    *out = a;
    return IM_OK;
}

static void copy_greedy_params(const im_ctx *from, im_ctx *to) {
    to->greedy_wg_max_entries = from->greedy_wg_max_entries;
    to->greedy_mark_min_chunks = from->greedy_mark_min_chunks;
    to->greedy_cover_blocks = from->greedy_cover_blocks;
    to->greedy_candidates = from->greedy_candidates;
    to->greedy_candidates_batch = from->greedy_candidates_batch;
    to->greedy_graph = from->greedy_graph;
    to->greedy_wg_cand_max_entries = from->greedy_wg_cand_max_entries;
    to->greedy_wg_cand_grid_rounds = from->greedy_wg_cand_grid_rounds;
    to->greedy_wg_cand_batch = from->greedy_wg_cand_batch;
    to->greedy_flat_levels = from->greedy_flat_levels;
    to->greedy_dense = from->greedy_dense;
}

// Helper context i (0..2) of ctx for later iterations' Max-Coverage.
static im_status helper_ctx(im_ctx *ctx, int i, im_ctx **out) {
    if (!ctx->helpers[i]) IM_TRY(new_side_ctx(ctx, &ctx->helpers[i]));
    copy_greedy_params(ctx, ctx->helpers[i]);
    *out = ctx->helpers[i];
    return IM_OK;
}

im_status aux_ctx(im_ctx *ctx, im_ctx **out) {
    if (!ctx->aux) IM_TRY(new_side_ctx(ctx, &ctx->aux));
    im_ctx *a = ctx->aux;
    if (ctx->timing && !a->ev_begin) {
        IM_HIP(hipEventCreate(&a->ev_begin));
        IM_HIP(hipEventCreate(&a->ev_end));
        IM_HIP(hipEventCreate(&a->ev_group));
    }
    a->timing = ctx->timing;
    copy_greedy_params(ctx, a);
    a->ic_edge_budget = ctx->ic_edge_budget;
    a->ic_ticket_block = ctx->ic_ticket_block;
    a->ic_plain = ctx->ic_plain;
    a->ic_compact = ctx->ic_compact;
    *out = a;
    return IM_OK;
}

static im_status pool_extend_to(im_pool *p, uint64_t target, double *ms) {
    const double t0 = now_ms();
    while (p->count < target) {
        const uint64_t count = std::min<uint64_t>(target - p->count, max_batch(p->model));
        SampleResult r;
        SampleItem it{p->key, p->count, count, nullptr};
        ItemTotals tot;
        IM_TRY(sample_items(p->ctx, p->g, p->model, &it, 1, SampleMode::Pool, p->mean_size > 0 ? p->mean_size : 0.0,
                            &r, &tot));
        AppendItem ap{p, count, tot.nodes, tot.edges};
        IM_TRY(pool_append_items(p->ctx, &ap, 1));
    }
    if (ms) *ms += now_ms() - t0;
    return IM_OK;
}

im_status estimate_inf(const im_graph *g, im_model model, const uint32_t *seeds, uint32_t k, double eps_p,
                       double delta_p, double t_max, uint64_t key, double t_hint, double *ic_out, uint64_t *t_out,
                       uint64_t *edges_out) {
    im_ctx *ctx = g->ctx;
    const double lambda2 = 1.0 + (1.0 + eps_p) * upsilon(eps_p, delta_p);
    const uint64_t need = uint64_t(std::ceil(lambda2));  // Cov >= Lambda2 for an integer Cov
    const uint64_t t_last = t_max >= 1.8e19 ? ~0ull : uint64_t(std::floor(t_max));
    IM_TRY(set_seed_bits(ctx, g->n, seeds, k));
    uint64_t done = 0, cov = 0, edges = 0;
    double guess = t_hint > 0 ? t_hint : 16.0 * double(need);
    uint64_t chunk = uint64_t(std::min(1.1 * guess + 1024.0, 4.0e8));
    while (done < t_last) {
        const uint64_t c = std::min<uint64_t>(std::min<uint64_t>(std::max<uint64_t>(chunk, 1024), max_batch(model)),
                                              t_last - done);
        SampleResult r;
        IM_TRY(sample_batch(ctx, g, model, key, done, c, SampleMode::Hits, 0.0, &r));
        edges += r.edges;
        int64_t idx = -1;
        uint64_t hits = 0;
        IM_TRY(first_crossing(ctx, c, need - cov, &idx, &hits));
        if (idx >= 0) {
            const uint64_t T = done + uint64_t(idx) + 1;
            *ic_out = estimate_scale(g) * lambda2 / double(T);
            *t_out = T;
            if (edges_out) *edges_out = edges;
            return IM_OK;
        }
        cov += hits;
        done += c;
        chunk = std::max<uint64_t>(uint64_t(0.25 * guess) + 1024, chunk / 2);
    }
    *ic_out = -1.0;
    *t_out = t_last;
    if (edges_out) *edges_out = edges;
    return IM_OK;
}

}  // namespace im

using namespace im;

// ------------------------------------------------------------- context ----

extern "C" im_status im_ctx_create(int device, void *stream, im_alloc_fn alloc, im_free_fn free_, void *user,
                                   im_ctx **out) {
    clear_error();
    if (!out) {
        set_error("null output");
        return IM_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("no HIP device %d (found %d)", device, ndev);
        return IM_E_ARG;
    }
    IM_HIP(hipSetDevice(device));
    IM_TRY(noalloc_scratch_init(device));
    hipDeviceProp_t prop;
    IM_HIP(hipGetDeviceProperties(&prop, device));
    auto *c = new (std::nothrow) im_ctx();
    if (!c) return IM_E_OOM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->alloc = alloc;
    c->free_ = free_;
    c->user = user;
    c->cu_count = prop.multiProcessorCount;
    c->total_mem = prop.totalGlobalMem;
    if (hipHostMalloc(&c->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        set_error("pinned host allocation failed");
        return IM_E_OOM;
    }
    *out = c;
    return IM_OK;
}

extern "C" im_status im_ctx_set_timing(im_ctx *c, int enable) {
    clear_error();
    if (!c) return IM_E_ARG;
    if (enable && !c->ev_begin) {
        IM_HIP(hipEventCreate(&c->ev_begin));
        IM_HIP(hipEventCreate(&c->ev_end));
        IM_HIP(hipEventCreate(&c->ev_group));
    }
    c->timing = enable != 0;
    return IM_OK;
}

extern "C" im_status im_ctx_set_param(im_ctx *c, im_param param, uint64_t value) {
    clear_error();
    if (!c) return IM_E_ARG;
    switch (param) {
    case IM_PARAM_GREEDY_WG_MAX_ENTRIES:
        c->greedy_wg_max_entries = value;
        return IM_OK;
    case IM_PARAM_IC_TICKET_BLOCK:
        if (value > 64) break;
        c->ic_ticket_block = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_DSSA_SPECULATE:
        if (value > 1) break;
        c->speculate = value != 0;
        return IM_OK;
    case IM_PARAM_GREEDY_MARK_MIN_CHUNKS:
        c->greedy_mark_min_chunks = value;
        return IM_OK;
    case IM_PARAM_GREEDY_COVER_BLOCKS:
        if (value > 65535) break;
        c->greedy_cover_blocks = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_IC_EDGE_BUDGET:
        if (value < 64 || value > (1ull << 31)) break;
        c->ic_edge_budget = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_GREEDY_CANDIDATES:
        if (value > 64) break;
        c->greedy_candidates = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_GREEDY_CANDIDATES_BATCH:
        if (value > 64) break;
        c->greedy_candidates_batch = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_DSSA_DRAW_AHEAD:
        if (value < 1 || value > 64) break;
        c->dssa_draw_ahead = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_GREEDY_GRAPH:
        if (value > 1) break;
        c->greedy_graph = value != 0;
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES:
        c->greedy_wg_cand_max_entries = value;
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS:
        if (value > (1ull << 31)) break;
        c->greedy_wg_cand_grid_rounds = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_DSSA_GREEDY_AHEAD:
        if (value > 3) break;
        c->dssa_greedy_ahead = static_cast<uint32_t>(value);
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_BATCH:
        c->greedy_wg_cand_batch = value;
        return IM_OK;
    case IM_PARAM_IC_PLAIN:
        if (value > 1) break;
        c->ic_plain = value != 0;
        return IM_OK;
    case IM_PARAM_GREEDY_FLAT_LEVELS:
        if (value > 1) break;
        c->greedy_flat_levels = value != 0;
        return IM_OK;
    case IM_PARAM_GREEDY_DENSE:
        if (value > 1) break;
        c->greedy_dense = value != 0;
        return IM_OK;
    case IM_PARAM_DSSA_IC_MIN_DRAW:
        c->dssa_ic_min_draw = value;
        return IM_OK;
    case IM_PARAM_IC_COMPACT:
        if (value > 1) break;
        c->ic_compact = value != 0;
        return IM_OK;
    }
    set_error("im_ctx_set_param: bad parameter %d or value %llu", int(param), static_cast<unsigned long long>(value));
    return IM_E_ARG;
}

extern "C" im_status im_ctx_get_param(const im_ctx *c, im_param param, uint64_t *value) {
    clear_error();
    if (!c || !value) return IM_E_ARG;
    switch (param) {
    case IM_PARAM_GREEDY_WG_MAX_ENTRIES:
        *value = c->greedy_wg_max_entries;
        return IM_OK;
    case IM_PARAM_IC_TICKET_BLOCK:
        *value = c->ic_ticket_block;
        return IM_OK;
    case IM_PARAM_DSSA_SPECULATE:
        *value = c->speculate ? 1 : 0;
        return IM_OK;
    case IM_PARAM_GREEDY_MARK_MIN_CHUNKS:
        *value = c->greedy_mark_min_chunks;
        return IM_OK;
    case IM_PARAM_GREEDY_COVER_BLOCKS:
        *value = c->greedy_cover_blocks;
        return IM_OK;
    case IM_PARAM_IC_EDGE_BUDGET:
        *value = c->ic_edge_budget;
        return IM_OK;
    case IM_PARAM_GREEDY_CANDIDATES:
        *value = c->greedy_candidates;
        return IM_OK;
    case IM_PARAM_GREEDY_CANDIDATES_BATCH:
        *value = c->greedy_candidates_batch;
        return IM_OK;
    case IM_PARAM_DSSA_DRAW_AHEAD:
        *value = c->dssa_draw_ahead;
        return IM_OK;
    case IM_PARAM_GREEDY_GRAPH:
        *value = c->greedy_graph ? 1 : 0;
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_MAX_ENTRIES:
        *value = c->greedy_wg_cand_max_entries;
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_GRID_ROUNDS:
        *value = c->greedy_wg_cand_grid_rounds;
        return IM_OK;
    case IM_PARAM_DSSA_GREEDY_AHEAD:
        *value = c->dssa_greedy_ahead;
        return IM_OK;
    case IM_PARAM_GREEDY_WG_CAND_BATCH:
        *value = c->greedy_wg_cand_batch;
        return IM_OK;
    case IM_PARAM_IC_PLAIN:
        *value = c->ic_plain ? 1 : 0;
        return IM_OK;
    case IM_PARAM_GREEDY_FLAT_LEVELS:
        *value = c->greedy_flat_levels ? 1 : 0;
        return IM_OK;
    case IM_PARAM_GREEDY_DENSE:
        *value = c->greedy_dense ? 1 : 0;
        return IM_OK;
    case IM_PARAM_DSSA_IC_MIN_DRAW:
        *value = c->dssa_ic_min_draw;
        return IM_OK;
    case IM_PARAM_IC_COMPACT:
        *value = c->ic_compact ? 1 : 0;
        return IM_OK;
    }
    set_error("im_ctx_get_param: bad parameter %d", int(param));
    return IM_E_ARG;
}

extern "C" im_status im_ctx_read_timing(im_ctx *c, im_kernel_times *out, int reset) {
    clear_error();
    if (!c || !out) return IM_E_ARG;
    *out = c->times;
    if (c->aux) {
        const im_kernel_times &a = c->aux->times;
        out->sample_launches += a.sample_launches;
        out->sample_ms += a.sample_ms;
        out->sample_sets += a.sample_sets;
        out->sample_steps += a.sample_steps;
        out->sample_nodes += a.sample_nodes;
        out->group_launches += a.group_launches;
        out->group_ms += a.group_ms;
        out->group_samples += a.group_samples;
        out->group_edges += a.group_edges;
        out->group_levels += a.group_levels;
        if (a.sample_launches) out->model = a.model;
        if (reset) c->aux->times = im_kernel_times{};
    }
    if (reset) c->times = im_kernel_times{};
    return IM_OK;
}

extern "C" im_status im_ctx_sync(im_ctx *c) {
    clear_error();
    if (!c) return IM_E_ARG;
    reap_ahead(c, nullptr);
    IM_HIP(hipStreamSynchronize(c->stream));
    if (c->aux) IM_HIP(hipStreamSynchronize(c->aux->stream));
    return IM_OK;
}

extern "C" void im_ctx_free(im_ctx *c) {
    if (!c) return;
    reap_ahead(c, nullptr);
    delete[] c->ahead;
    c->ahead = nullptr;
    if (c->aux) im_ctx_free(c->aux);
    for (im_ctx *h : c->helpers)
        if (h) im_ctx_free(h);
    (void)hipStreamSynchronize(c->stream);
    if (c->ev_begin) (void)hipEventDestroy(c->ev_begin);
    if (c->ev_end) (void)hipEventDestroy(c->ev_end);
    if (c->ev_group) (void)hipEventDestroy(c->ev_group);
    if (c->ev_ready) (void)hipEventDestroy(c->ev_ready);
    free_round_graphs(c);
    for (DevBuf *b : {&c->stage, &c->sample_meta, &c->handoff, &c->counters, &c->scan_tmp, &c->slots, &c->cover, &c->seedbits, &c->flat,
                      &c->prefix_off, &c->prefix_nodes, &c->dense, &c->zflags, &c->lt_tables, &c->items, &c->append_dst,
                      &c->k1_cnt})
        dev_free(c, *b);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    if (c->owns_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// --------------------------------------------------------------- graph ----

extern "C" im_status im_graph_load(im_ctx *ctx, uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                                   const float *w_ic, const float *w_lt, im_graph **out) {
    clear_error();
    if (!ctx || !out || n == 0 || n == 0xFFFFFFFFu || (m && (!src || !dst)) || (!w_ic && !w_lt)) {
        set_error("im_graph_load: bad arguments (n must be in [1, 2^32-2]; src, dst and one weight array required)");
        return IM_E_ARG;
    }
    auto *g = new (std::nothrow) im_graph();
    if (!g) return IM_E_OOM;
    g->ctx = ctx;
    g->n = n;
    g->m = m;
    im_status rc = graph_build(g, src, dst, w_ic, w_lt);
    if (rc != IM_OK) {
        im_graph_free(g);
        return rc;
    }
    *out = g;
    return IM_OK;
}

extern "C" im_status im_graph_set_source_weights(im_graph *g, const uint32_t *node_w) {
    clear_error();
    if (!g) return IM_E_ARG;
    return graph_source_weights(g, node_w);
}

extern "C" void im_graph_free(im_graph *g) {
    if (!g) return;
    reap_ahead(g->ctx, g);  // dropped covers of this graph's runs read g
    (void)hipStreamSynchronize(g->ctx->stream);
    dev_free(g->ctx, g->off);
    dev_free(g->ctx, g->edges_ic);
    dev_free(g->ctx, g->edges_lt);
    dev_free(g->ctx, g->nodes_ic);
    dev_free(g->ctx, g->srcs_ic);
    dev_free(g->ctx, g->src_cum);
    delete g;
}

extern "C" im_status im_graph_info(const im_graph *g, uint32_t *n, uint64_t *m, uint32_t *models) {
    clear_error();
    if (!g) return IM_E_ARG;
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (models) *models = g->models;
    return IM_OK;
}

// ---------------------------------------------------------------- pool ----

extern "C" im_status im_pool_create(im_ctx *ctx, const im_graph *g, im_model model, uint64_t stream_key,
                                    im_pool **out) {
    clear_error();
    if (!ctx || !g || !out || g->ctx != ctx) {
        set_error("im_pool_create: bad arguments");
        return IM_E_ARG;
    }
    if ((model != IM_IC && model != IM_LT) || !(g->models & (model == IM_IC ? 1u : 2u))) {
        set_error("im_pool_create: graph has no weights for model %d", int(model));
        return IM_E_ARG;
    }
    auto *p = new (std::nothrow) im_pool();
    if (!p) return IM_E_OOM;
    static std::atomic<uint64_t> pools_made{0};
    p->serial = pools_made.fetch_add(1, std::memory_order_relaxed) + 1;
    p->ctx = ctx;
    p->g = g;
    p->model = model;
    p->key = stream_key;
    im_status rc = IM_OK;
    // empty pool: poff = {0}
    p->cap_sets = 1024;
    p->cap_nodes = 1 << 16;
    if ((rc = dev_alloc(ctx, p->poff, (p->cap_sets + 1) * 8)) || (rc = dev_alloc(ctx, p->pnodes, p->cap_nodes * 4))) {
        im_pool_free(p);
        return rc;
    }
    if (hipMemsetAsync(p->poff.ptr, 0, 8, ctx->stream) != hipSuccess) {
        im_pool_free(p);
        set_error("memset failed");
        return IM_E_DEVICE;
    }
    *out = p;
    return IM_OK;
}

extern "C" void im_pool_free(im_pool *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->ctx->stream);
    dev_free(p->ctx, p->poff);
    dev_free(p->ctx, p->pnodes);
    delete p;
}

extern "C" im_status im_sample_rr(const im_graph *g, im_model model, uint64_t n_sets, uint64_t stream_key,
                                  im_pool *pool) {
    clear_error();
    if (!g || !pool) return IM_E_ARG;
    if (pool->g != g) {
        set_error("im_sample_rr: pool belongs to another graph");
        return IM_E_ARG;
    }
    if (pool->key != stream_key || pool->model != model) {
        set_error("im_sample_rr: pool stream (key %llu, model %d) differs from the call's (key %llu, model %d)",
                  static_cast<unsigned long long>(pool->key), int(pool->model),
                  static_cast<unsigned long long>(stream_key), int(model));
        return IM_E_STREAM_MISMATCH;
    }
    return pool_extend_to(pool, pool->count + n_sets, nullptr);
}

extern "C" im_status im_sample_rr_multi(const im_graph *g, im_model model, uint32_t n_pools, im_pool *const *pools,
                                        const uint64_t *n_sets) {
    clear_error();
    if (!g || (n_pools && (!pools || !n_sets))) {
        set_error("im_sample_rr_multi: null arguments");
        return IM_E_ARG;
    }
    for (uint32_t i = 0; i < n_pools; ++i) {
        const im_pool *p = pools[i];
        if (!p || p->g != g) {
            set_error("im_sample_rr_multi: pool %u is null or belongs to another graph", i);
            return IM_E_ARG;
        }
        if (p->model != model) {
            set_error("im_sample_rr_multi: pool %u is of model %d, the call's is %d", i, int(p->model), int(model));
            return IM_E_STREAM_MISMATCH;
        }
        for (uint32_t j = 0; j < i; ++j)
            if (pools[j] == p) {
                set_error("im_sample_rr_multi: pool %u appears twice", i);
                return IM_E_ARG;
            }
    }
    // fused launches of up to a batch cap of samples each, pools in order
    std::vector<uint64_t> left(n_sets, n_sets + n_pools);
    const uint64_t cap = max_batch(model);
    uint32_t i = 0;
    while (i < n_pools) {
        std::vector<SampleItem> items;
        std::vector<im_pool *> members;
        uint64_t total = 0;
        double hint = 0.0;
        for (; i < n_pools && total < cap; ++i) {
            if (left[i] == 0) continue;
            const uint64_t take = std::min<uint64_t>(left[i], cap - total);
            items.push_back(SampleItem{pools[i]->key, pools[i]->count, take, nullptr});
            members.push_back(pools[i]);
            total += take;
            left[i] -= take;
            hint = std::max(hint, pools[i]->mean_size);
            if (left[i]) break;  // the rest of this pool goes in the next launch
        }
        if (items.empty()) break;
        SampleResult r;
        std::vector<ItemTotals> tot(items.size());
        IM_TRY(sample_items(g->ctx, g, model, items.data(), uint32_t(items.size()), SampleMode::Pool, hint, &r,
                            tot.data()));
        std::vector<AppendItem> app(items.size());
        for (size_t j = 0; j < items.size(); ++j) app[j] = AppendItem{members[j], items[j].count, tot[j].nodes, tot[j].edges};
        IM_TRY(pool_append_items(g->ctx, app.data(), uint32_t(app.size())));
    }
    return IM_OK;
}

extern "C" im_status im_pool_info(const im_pool *p, uint64_t *count, uint64_t *total_nodes) {
    clear_error();
    if (!p) return IM_E_ARG;
    if (count) *count = p->count;
    if (total_nodes) *total_nodes = p->total;
    return IM_OK;
}

extern "C" im_status im_pool_read(const im_pool *p, uint64_t begin, uint64_t end, uint64_t *off_out,
                                  uint32_t *nodes_out) {
    clear_error();
    if (!p || !off_out || begin > end || end > p->count) {
        set_error("im_pool_read: bad range");
        return IM_E_ARG;
    }
    hipStream_t st = p->ctx->stream;
    const auto *poff = static_cast<const uint64_t *>(p->poff.ptr);
    IM_HIP(hipMemcpyAsync(off_out, poff + begin, (end - begin + 1) * 8, hipMemcpyDeviceToHost, st));
    IM_HIP(hipStreamSynchronize(st));
    const uint64_t first = off_out[0];
    const uint64_t len = off_out[end - begin] - first;
    for (uint64_t i = 0; i <= end - begin; ++i) off_out[i] -= first;
    if (nodes_out && len) {
        IM_HIP(hipMemcpyAsync(nodes_out, static_cast<const uint32_t *>(p->pnodes.ptr) + first, len * 4,
                              hipMemcpyDeviceToHost, st));
        IM_HIP(hipStreamSynchronize(st));
    }
    return IM_OK;
}

extern "C" im_status im_pool_device(const im_pool *p, const uint64_t **poff_dev, const uint32_t **pnodes_dev) {
    clear_error();
    if (!p) return IM_E_ARG;
    if (poff_dev) *poff_dev = static_cast<const uint64_t *>(p->poff.ptr);
    if (pnodes_dev) *pnodes_dev = static_cast<const uint32_t *>(p->pnodes.ptr);
    return IM_OK;
}

// ------------------------------------------------------------ coverage ----

extern "C" im_status im_max_coverage_range(const im_pool *p, uint64_t begin, uint64_t end, uint32_t k,
                                           uint32_t *seeds_out, uint64_t *cov_out) {
    clear_error();
    if (!p || !seeds_out || !cov_out || begin > end || end > p->count || k == 0 || k > p->g->n) {
        set_error("im_max_coverage: bad arguments (k must be in [1, n], range within the pool)");
        return IM_E_ARG;
    }
    return max_coverage(p, begin, end, k, seeds_out, cov_out);
}

extern "C" im_status im_max_coverage(const im_pool *p, uint32_t k, uint32_t *seeds_out, uint64_t *cov_out) {
    if (!p) return IM_E_ARG;
    return im_max_coverage_range(p, 0, p->count, k, seeds_out, cov_out);
}

extern "C" im_status im_coverage_range(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds,
                                       uint32_t k, uint64_t *cov_out) {
    clear_error();
    if (!p || !cov_out || begin > end || end > p->count || (k && !seeds)) {
        set_error("im_coverage_range: bad arguments");
        return IM_E_ARG;
    }
    return coverage_range(p, begin, end, seeds, k, cov_out);
}

extern "C" im_status im_estimate_inf(const im_graph *g, im_model model, const uint32_t *seeds, uint32_t k,
                                     double eps_p, double delta_p, double t_max, uint64_t stream_key, double *ic_out,
                                     uint64_t *t_out) {
    clear_error();
    if (!g || !ic_out || !t_out || (k && !seeds) || !(eps_p > 0 && eps_p < 1) || !(delta_p > 0 && delta_p < 1) ||
        !(t_max >= 0)) {
        set_error("im_estimate_inf: bad arguments");
        return IM_E_ARG;
    }
    if ((model != IM_IC && model != IM_LT) || !(g->models & (model == IM_IC ? 1u : 2u))) {
        set_error("im_estimate_inf: graph has no weights for model %d", int(model));
        return IM_E_ARG;
    }
    return estimate_inf(g, model, seeds, k, eps_p, delta_p, t_max, stream_key, 0.0, ic_out, t_out, nullptr);
}

extern "C" uint64_t im_derived_key(uint64_t key, uint64_t i) { return derived_key(key, i); }

extern "C" const char *im_last_error(void) { return g_err; }

// ------------------------------------------------------- SSA / D-SSA ----

// Eq. 14: a caller's split needs every eps_i in (0, 1) and
// (1-1/e)(eps1 + eps2 + eps1 eps2 + eps3) / ((1+eps1)(1+eps2)) <= eps
// (relative slack 1e-12, so that a split meeting it with equality passes).
static double eq14_lhs(double eps1, double eps2, double eps3) {
    const double one_m = 1.0 - std::exp(-1.0);
    return one_m * (eps1 + eps2 + eps1 * eps2 + eps3) / ((1.0 + eps1) * (1.0 + eps2));
}

static bool eq14_ok(double eps, double eps1, double eps2, double eps3) {
    return eps1 > 0.0 && eps1 < 1.0 && eps2 > 0.0 && eps2 < 1.0 && eps3 > 0.0 && eps3 < 1.0 &&
           eq14_lhs(eps1, eps2, eps3) <= eps * (1.0 + 1e-12);
}

// SSA (Algorithm 1) with a given precision split.
static im_status ssa_run(const im_graph *g, im_model model, uint32_t k, double eps, double eps1, double eps2,
                         double eps3, double delta, uint64_t key, uint32_t *seeds_out, im_stats *st) {
    const double t_start = now_ms();
    std::memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    const Caps c = caps(g->n, k, eps, delta);
    const double lambda1 = (1.0 + eps1) * (1.0 + eps2) * upsilon(eps3, delta / (3.0 * c.i_max));
    const double delta2p = delta / (3.0 * c.i_max);
    const double lambda2 = 1.0 + (1.0 + eps2) * upsilon(eps2, delta2p);
    const double n = estimate_scale(g);

    im_pool *pool = nullptr;
    IM_TRY(im_pool_create(g->ctx, g, model, key, &pool));
    std::vector<uint32_t> seeds(k);
    const uint64_t n1 = uint64_t(std::ceil(c.lambda));
    im_status rc = IM_OK;
    for (uint32_t t = 1;; ++t) {
        const uint64_t size = n1 << (t - 1);
        if ((rc = pool_extend_to(pool, size, &st->ms_sample))) break;
        uint64_t cov = 0;
        double t0 = now_ms();
        if ((rc = max_coverage(pool, 0, size, k, seeds.data(), &cov))) break;
        st->ms_cover += now_ms() - t0;
        const double i_hat = n * double(cov) / double(size);
        st->iterations = t;
        st->n_sets = size;
        st->cov = cov;
        st->i_hat = i_hat;
        if (t <= IM_MAX_ITERS) {
            st->it_sets[t - 1] = size;
            st->it_cov[t - 1] = cov;
            st->it_eps_t[t - 1] = -1.0;
        }
        bool done = false;
        if (double(cov) >= lambda1) {  // C1
            const double t_max = 2.0 * double(size) * (1.0 + eps2) / (1.0 - eps2) * (eps3 * eps3) / (eps2 * eps2);
            double ic = -1.0;
            uint64_t T = 0, ex = 0;
            t0 = now_ms();
            const double hint = lambda2 * double(size) / double(cov > 0 ? cov : 1);
            if ((rc = estimate_inf(g, model, seeds.data(), k, eps2, delta2p, t_max, derived_key(key, t), hint, &ic, &T,
                                   &ex)))
                break;
            st->ms_verify += now_ms() - t0;
            st->n_verify += T;
            st->edges += ex;
            st->cov_c = T;
            st->i_c = ic;
            if (t <= IM_MAX_ITERS) {
                st->it_cov_c[t - 1] = T;
                st->it_eps_t[t - 1] = ic;
            }
            if (i_hat <= (1.0 + eps1) * ic) done = true;  // C2
        }
        if (done) break;
        if (double(size) >= c.n_max) {
            st->stopped_by_cap = 1;
            break;
        }
    }
    if (rc == IM_OK) {
        st->eps1 = eps1;
        st->eps2 = eps2;
        st->eps3 = eps3;
        st->edges += pool->edges;
        std::memcpy(seeds_out, seeds.data(), 4ull * k);
    }
    im_pool_free(pool);
    st->ms_total = now_ms() - t_start;
    return rc;
}

extern "C" im_status im_ssa(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                            uint32_t *seeds_out, im_stats *st) {
    clear_error();
    IM_TRY(check_query(g, model, k, eps, delta));
    if (!seeds_out || !st) return IM_E_ARG;
    // Eq. 15 defaults
    const double one_m = 1.0 - std::exp(-1.0);
    const double eps2 = eps / (2.0 * one_m);
    const double eps3 = eps2;
    const double eps1 = (1.0 + eps / (2.0 * (one_m - eps))) / (1.0 + eps2) - 1.0;
    return ssa_run(g, model, k, eps, eps1, eps2, eps3, delta, key, seeds_out, st);
}

extern "C" im_status im_ssa_eps(const im_graph *g, im_model model, uint32_t k, double eps, double eps1, double eps2,
                                double eps3, double delta, uint64_t key, uint32_t *seeds_out, im_stats *st) {
    clear_error();
    IM_TRY(check_query(g, model, k, eps, delta));
    if (!seeds_out || !st) return IM_E_ARG;
    if (!eq14_ok(eps, eps1, eps2, eps3)) {
        set_error("im_ssa_eps: (%g, %g, %g) does not meet Eq. 14 for eps = %g", eps1, eps2, eps3, eps);
        return IM_E_ARG;
    }
    return ssa_run(g, model, k, eps, eps1, eps2, eps3, delta, key, seeds_out, st);
}

extern "C" im_status im_ssa_eps_preset(int regime, double eps, double *out) {
    clear_error();
    // eps1 = a x, eps2 = eps3 = x, with x the largest value meeting Eq. 14
    double a = 0.0;
    switch (regime) {
    case IM_NET_SMALL: a = 2.0; break;
    case IM_NET_MODERATE: a = 1.0; break;
    case IM_NET_LARGE: a = 0.125; break;
    default: break;
    }
    if (!out || a == 0.0 || !(eps > 0.0 && eps < 1.0 - std::exp(-1.0))) {
        set_error("im_ssa_eps_preset: bad regime %d or eps %g", regime, eps);
        return IM_E_ARG;
    }
    double lo = 0.0, hi = std::min(1.0, 1.0 / a) * (1.0 - 1e-9);
    if (eq14_lhs(a * hi, hi, hi) <= eps) {
        lo = hi;
    } else {
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (eq14_lhs(a * mid, mid, mid) <= eps) lo = mid;
            else hi = mid;
        }
    }
    if (!eq14_ok(eps, a * lo, lo, lo)) {
        set_error("im_ssa_eps_preset: no admissible split");
        return IM_E_ARG;
    }
    out[0] = a * lo;
    out[1] = lo;
    out[2] = lo;
    return IM_OK;
}

extern "C" double im_ris_theta(uint32_t n, uint32_t k, double eps, double delta) {
    const double one_m = 1.0 - std::exp(-1.0);
    return 8.0 * one_m * (std::log(2.0 / delta) + ln_choose(n, k)) / (eps * eps) * double(n) / double(k);
}

extern "C" im_status im_ris(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                            uint32_t *seeds_out, im_stats *st) {
    clear_error();
    IM_TRY(check_query(g, model, k, eps, delta));
    if (!seeds_out || !st) return IM_E_ARG;
    const double theta = im_ris_theta(g->n, k, eps, delta);
    if (!(theta < 4.0e12)) {
        set_error("im_ris: theta = %g RR sets", theta);
        return IM_E_OOM;
    }
    const double t_start = now_ms();
    std::memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    const uint64_t count = uint64_t(std::ceil(theta));
    im_pool *pool = nullptr;
    IM_TRY(im_pool_create(g->ctx, g, model, key, &pool));
    im_status rc = pool_extend_to(pool, count, &st->ms_sample);
    uint64_t cov = 0;
    if (rc == IM_OK) {
        const double t0 = now_ms();
        rc = max_coverage(pool, 0, count, k, seeds_out, &cov);
        st->ms_cover = now_ms() - t0;
    }
    if (rc == IM_OK) {
        st->iterations = 1;
        st->n_sets = count;
        st->cov = cov;
        st->i_hat = estimate_scale(g) * double(cov) / double(count);
        st->edges = pool->edges;
        st->it_sets[0] = count;
        st->it_cov[0] = cov;
        st->it_eps_t[0] = -1.0;
    }
    im_pool_free(pool);
    st->ms_total = now_ms() - t_start;
    return rc;
}

namespace {

// One speculative draw: samples [s0, s0+count) of a pool's stream, drawn on
// the auxiliary context by a helper thread into that context's staging.
struct Speculation {
    std::thread th;
    bool running = false;
    im_status rc = IM_OK;
    std::string err;
    uint64_t s0 = 0, count = 0;
    SampleResult res;
    ItemTotals tot;

    void start(im_ctx *aux, const im_pool *p, uint64_t first, uint64_t n) {
        s0 = first;
        count = n;
        running = true;
        const im_graph *g = p->g;
        const im_model model = p->model;
        const uint64_t key = p->key;
        const double hint = p->mean_size;
        th = std::thread([this, aux, g, model, key, hint] {
            if (hipSetDevice(aux->device) != hipSuccess) {
                rc = IM_E_DEVICE;
                err = "hipSetDevice failed in the sampling thread";
                return;
            }
            SampleItem it{key, s0, count, nullptr};
            rc = sample_items(aux, g, model, &it, 1, SampleMode::Pool, hint, &res, &tot);
            if (rc != IM_OK) err = im_last_error();
        });
    }
    // Wait for the draw; on failure the thread's message becomes this one's.
    im_status join() {
        if (!running) return IM_OK;
        th.join();
        running = false;
        if (rc != IM_OK) set_error("%s", err.c_str());
        return rc;
    }
};

}  // namespace

extern "C" im_status im_dssa(const im_graph *g, im_model model, uint32_t k, double eps, double delta, uint64_t key,
                             uint32_t *seeds_out, im_stats *st) {
    clear_error();
    IM_TRY(check_query(g, model, k, eps, delta));
    if (!seeds_out || !st) return IM_E_ARG;
    const double t_start = now_ms();
    std::memset(st, 0, sizeof(*st));
    st->i_c = -1.0;
    const double one_m = 1.0 - std::exp(-1.0);
    const Caps c = caps(g->n, k, eps, delta);  // t_max = i_max
    const double lambda1 = 1.0 + (1.0 + eps) * upsilon(eps, delta / (3.0 * c.i_max));
    const double n = estimate_scale(g);
    im_ctx *ctx = g->ctx;

    im_pool *pool = nullptr;
    IM_TRY(im_pool_create(ctx, g, model, key, &pool));
    // the side-sampling context, made on the first draw on the side (an LT
    // run drawing ahead never makes one, so its stream takes no hardware
    // queue from the helpers)
    im_ctx *aux = nullptr;
    bool aux_tried = false;
    Speculation spec;
    double ms_draw = 0.0, ms_cover_last = 0.0;  // wall time of the last own draw of N_t sets / last cover
    std::vector<uint32_t> seeds(k);
    const uint64_t n1 = uint64_t(std::ceil(c.lambda));
    // sets the last possible iteration uses: 2 N_t for the first N_t >= N_max
    uint64_t most = 2 * n1;
    while (double(most / 2) < c.n_max && most < (1ull << 62)) most *= 2;
    im_status rc = IM_OK;
    // later iterations' covers running on helper contexts (slot i = helper
    // i); a slot still busy with a dropped cover of an earlier run is left
    // alone until it is done
    // Side sampling (the next iteration's new sets drawn on a second stream
    // while this one is covered) is for runs that draw one iteration at a
    // time: a run that draws ahead (LT, or IC with a minimum draw) has the
    // next sets already, and a side draw it turns out not to need is still
    // waited for at its end. A run that may sample on the side keeps one
    // helper fewer (the run's stream, the side stream and two helpers fill
    // the four hardware queues).
    const bool draws_ahead =
        (model == IM_LT && ctx->dssa_draw_ahead > 1) || (model == IM_IC && ctx->dssa_ic_min_draw > 0);
    const bool side_sampling = ctx->speculate && !draws_ahead;
    AheadCover *ahead = ctx->dssa_greedy_ahead ? ahead_slots(ctx) : nullptr;
    const uint32_t ahead_max = side_sampling ? kAheadSlots - 1 : kAheadSlots;
    // A run that draws ahead (LT) has every set a helper needs long before
    // it is covered and grows its pool rarely: helpers read the pool itself,
    // and every cover of the run is joined before the pool may move. Other
    // runs grow the pool every iteration: each helper covers its own copy
    // of the greedy sets, started as soon as those are drawn (not for k = 1,
    // whose cover is one count and argmax, shorter than the copy's wait).
    const bool helper_copies = !(model == IM_LT && ctx->dssa_draw_ahead > 1);
    const uint32_t n_ahead =
        (ahead && !(helper_copies && k < 2)) ? std::min<uint32_t>(ctx->dssa_greedy_ahead, ahead_max) : 0u;
    auto join_ahead = [&]() {
        im_status r = IM_OK;
        if (helper_copies) return r;
        for (uint32_t i = 0; i < n_ahead; ++i) {
            if (ahead[i].pool != pool) continue;
            const im_status x = join_slot(ahead, int(i));
            if (r == IM_OK) r = x;
        }
        return r;
    };
    for (uint32_t t = 1;; ++t) {
        const uint64_t nt = n1 << (t - 1);
        double t0 = now_ms();
        if (spec.running) {
            // the previous iteration drew this one's new sets on the side
            if ((rc = spec.join())) break;
            if (spec.s0 == pool->count) {
                if ((rc = join_ahead())) break;
                AppendItem ap{pool, spec.count, spec.tot.nodes, spec.tot.edges};
                if ((rc = pool_append_items(aux, &ap, 1))) break;
            }
        }
        const double t_fresh = now_ms();
        // an LT sampler launch of one query lasts about as long as its
        // longest walk whatever its size, so a draw may also take the next
        // iterations' sets (identical sets: they depend only on their index)
        uint64_t target = 2 * nt;
        if (model == IM_LT && pool->count < target && ctx->dssa_draw_ahead > 1)
            target = std::max(target, std::min(most, 2 * nt * ctx->dssa_draw_ahead));
        // likewise an IC run while its draws are small (a small IC launch
        // lasts about as long as its deepest samples, whatever its size): up
        // to the largest 2 N_{t+j} within the minimum draw
        if (model == IM_IC && pool->count < target)
            while (2 * target <= ctx->dssa_ic_min_draw && 2 * target <= most) target *= 2;
        const bool drew = pool->count < target;
        if (drew && (rc = join_ahead())) break;
        if ((rc = pool_extend_to(pool, target, nullptr))) break;
        const double ms_fresh = drew ? now_ms() - t_fresh : 0.0;  // this iteration's own draw, if any
        st->ms_sample += now_ms() - t0;
        // draw the next iteration's new sets [2 N_t, 4 N_t) while this one is
        // covered (they are dropped if this iteration stops), when the cover
        // step is expected to take at least half as long as that draw: the
        // last iteration's cover time, or about 15 us per greedy round
        // (not for runs that draw ahead, above)
        if (ms_fresh > 0) ms_draw = ms_fresh;
        const double est_cover = std::max(ms_cover_last, 0.015 * k);
        if (side_sampling && double(nt) < c.n_max && 2 * nt <= max_batch(model) &&
            est_cover >= ms_draw && pool->count < 4 * nt) {
            if (!aux_tried) {
                aux_tried = true;
                if (aux_ctx(ctx, &aux) != IM_OK) aux = nullptr;  // run without speculation
                clear_error();
            }
            if (aux) spec.start(aux, pool, pool->count, 4 * nt - pool->count);
        }
        // the next iterations whose greedy sets [0, N) are drawn are covered
        // on the helper contexts meanwhile (at most one per helper); with
        // copies, an iteration whose stare sets [N, 2N) were not drawn yet
        // has its stare count taken here when it comes
        bool synced = false;
        for (uint32_t j = 1; j <= n_ahead; ++j) {
            const uint64_t nj = nt << j;
            if (double(nj >> 1) >= c.n_max || (helper_copies ? nj : 2 * nj) > pool->count) break;
            bool have = false;
            for (uint32_t i = 0; i < n_ahead; ++i) have = have || (ahead[i].pool == pool && ahead[i].nt == nj);
            if (have) continue;
            for (uint32_t i = 0; i < n_ahead; ++i) {
                if (ahead[i].running && ahead[i].pool == pool) continue;  // this run's, not yet used
                if (ahead[i].busy()) continue;                            // an earlier run's, still running
                if (ahead[i].running) (void)join_slot(ahead, int(i));     // an earlier run's dropped cover, done
                im_ctx *h = nullptr;
                if (helper_ctx(ctx, int(i), &h) != IM_OK) {
                    clear_error();
                    continue;  // go on without this helper
                }
                im_pool copy = *pool;
                if (helper_copies) {
                    rc = copy_prefix(ctx, pool, h, std::min<uint64_t>(pool->count, 2 * nj), &copy);
                } else if (!synced) {
                    // the pool's sets were written on this context's stream
                    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
                        set_error("stream synchronize failed");
                        rc = IM_E_DEVICE;
                    }
                    synced = true;
                }
                if (rc == IM_OK) ahead[i].start(h, pool, copy, nj, k);
                break;
            }
            if (rc != IM_OK) break;
        }
        if (rc != IM_OK) break;
        uint64_t cov = 0, cov_c = 0;
        int mine = -1;
        for (uint32_t i = 0; i < n_ahead; ++i)
            if (ahead[i].running && ahead[i].pool == pool && ahead[i].nt == nt) mine = int(i);
        t0 = now_ms();
        if (mine >= 0) {
            // covered on a helper since an earlier iteration
            if ((rc = join_slot(ahead, mine))) break;
            const AheadCover &m = ahead[mine];
            std::copy(m.seeds.begin(), m.seeds.end(), seeds.begin());
            cov = m.cov;
            cov_c = m.cov_c;
            ms_cover_last = now_ms() - t0;
            st->ms_cover += ms_cover_last;
            if (!m.stared) {  // its stare sets were drawn after it started
                t0 = now_ms();
                if ((rc = coverage_range(pool, nt, 2 * nt, seeds.data(), k, &cov_c))) break;
                st->ms_verify += now_ms() - t0;
            }
        } else {
            if ((rc = max_coverage(pool, 0, nt, k, seeds.data(), &cov))) break;
            ms_cover_last = now_ms() - t0;
            st->ms_cover += ms_cover_last;
            t0 = now_ms();
            if ((rc = coverage_range(pool, nt, 2 * nt, seeds.data(), k, &cov_c))) break;
            st->ms_verify += now_ms() - t0;
        }
        const double i_hat = n * double(cov) / double(nt);
        st->iterations = t;
        st->n_sets = 2 * nt;
        st->cov = cov;
        st->cov_c = cov_c;
        st->i_hat = i_hat;
        if (t <= IM_MAX_ITERS) {
            st->it_sets[t - 1] = nt;
            st->it_cov[t - 1] = cov;
            st->it_cov_c[t - 1] = cov_c;
            st->it_eps_t[t - 1] = -1.0;
        }
        bool done = false;
        if (double(cov_c) >= lambda1) {  // D1
            const double two_t1 = std::ldexp(1.0, int(t) - 1);
            const double i_c = double(cov_c) * n / double(nt);
            const double e1 = i_hat / i_c - 1.0;
            const double e2 = eps * std::sqrt(n * (1.0 + eps) / (two_t1 * i_c));
            const double e3 = eps * std::sqrt(n * (1.0 + eps) * (one_m - eps) / ((1.0 + eps / 3.0) * two_t1 * i_c));
            const double e_t = (e1 + e2 + e1 * e2) * (one_m - eps) + one_m * e3;
            st->i_c = i_c;
            st->eps1 = e1;
            st->eps2 = e2;
            st->eps3 = e3;
            st->eps_t = e_t;
            if (t <= IM_MAX_ITERS) st->it_eps_t[t - 1] = e_t;
            if (e_t <= eps) done = true;  // D2
        }
        if (done) break;
        if (double(nt) >= c.n_max) {
            st->stopped_by_cap = 1;
            break;
        }
    }
    const im_status rs = spec.join();  // a draw still running is waited for and dropped
    if (rc == IM_OK) rc = rs;
    // covers of iterations the run did not reach are dropped without waiting:
    // their slots keep the pool until they are done
    bool pool_kept = false;
    for (uint32_t i = 0; i < n_ahead; ++i) {
        if (ahead[i].running && ahead[i].pool == pool) {
            ahead[i].orphan = pool;
            pool_kept = true;
        }
    }
    if (rc == IM_OK) {
        st->edges = pool->edges;
        if (pool->count > st->n_sets) {
            // drawn ahead: the used sets' edges. An LT walk examines one
            // in-edge list per node it holds, so they are their sizes; an IC
            // set examines every in-edge of its nodes
            if (model == IM_LT)
                rc = to_host_sync(ctx, &st->edges, static_cast<const uint64_t *>(pool->poff.ptr) + st->n_sets, 8);
            else
                rc = pool_ic_edges(pool, st->n_sets, &st->edges);
        }
        std::memcpy(seeds_out, seeds.data(), 4ull * k);
    }
    if (!pool_kept) im_pool_free(pool);
    st->ms_total = now_ms() - t_start;
    return rc;
}
