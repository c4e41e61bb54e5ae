// Multi-query engine: many SSA (Algorithm 1) / D-SSA (Algorithm 4) queries
// in flight at once on one GPU.
//
// Each query is a host state machine holding its FP64 checkpoint logic and
// its own RR pool. A step gathers the device work of every active query and
// issues it as shared launches:
//   1. SSA verification: one fused hits-mode launch over every verifying
//      query's next chunk of its own derived stream, then one crossing search;
//   2. sampling: one fused sampler launch per (graph, model) whose work queue
//      holds every query's next range of samples, then one batched append;
//   3. coverage: one batched Max-Coverage (and D-SSA stare step) over every
//      query whose pool reached its checkpoint;
//   4. the checkpoint conditions on the host.
// Queued queries are admitted between steps while the active queries' pools
// stay under a byte budget, so new work joins work already on the device.
// Every query's result is a pure function of its own arguments: identical
// whether it runs alone or among others.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "im_internal.hpp"

namespace {

using namespace im;

enum Phase { kPending = 0, kSample = 1, kCover = 2, kVerify = 3, kDone = 4, kFailed = 5 };

struct Query {
    uint64_t ticket = 0;
    im_query q{};
    Phase phase = kPending;
    im_status err = IM_OK;
    im_pool *pool = nullptr;
    uint32_t t = 0;
    // checkpoint constants
    Caps c{};
    double lambda1 = 0, eps1 = 0, eps2 = 0, eps3 = 0, delta2p = 0, lambda2 = 0;
    uint64_t n1 = 0;      // ceil(Lambda)
    uint64_t target = 0;  // sets the pool must hold at this iteration
    std::vector<uint32_t> seeds;
    im_stats st{};
    uint64_t verify_edges = 0;
    // SSA Estimate-Inf progress
    uint64_t vkey = 0, vdone = 0, vcov = 0, vlast = 0, vneed = 0, vchunk = 0;
    double vhint = 0;
    // influence-estimate queries (Algorithm 3 for a given seed set)
    double est_eps = 0, est_delta = 0, est_tmax = 0;
    DevBuf vbits;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct im_engine {
    im_ctx *ctx = nullptr;
    uint64_t budget = 0;
    uint32_t max_active = 0;
    uint64_t next_ticket = 1;
    std::deque<Query *> pending;
    std::vector<Query *> active;
    std::map<uint64_t, Query *> all;
};

namespace {

// Device bytes a query's pool holds, or at least what its current target
// needs at one node per set (a just-admitted pool has reserved nothing yet).
uint64_t pool_bytes(const Query *q) {
    if (!q->pool) return 0;
    const uint64_t held = (q->pool->cap_sets + 1) * 8 + q->pool->cap_nodes * 4;
    return std::max<uint64_t>(held, 12 * q->target);
}

uint64_t active_bytes(const im_engine *e) {
    uint64_t b = 0;
    for (const Query *q : e->active) b += pool_bytes(q);
    return b;
}

void finish(im_engine *e, Query *q, Phase ph, im_status err) {
    q->phase = ph;
    q->err = err;
    q->t_done = now_ms();
    q->st.ms_total = q->t_done - q->t_submit;
    if (q->q.algo == IM_ALGO_SSA && ph == kDone) {
        q->st.eps1 = q->eps1;
        q->st.eps2 = q->eps2;
        q->st.eps3 = q->eps3;
    }
    if (q->pool) {
        q->st.edges = (q->q.algo == IM_ALGO_SSA ? q->verify_edges : 0) + q->pool->edges;
        im_pool_free(q->pool);
        q->pool = nullptr;
    } else if (q->q.algo == IM_ALGO_ESTIMATE) {
        q->st.edges = q->verify_edges;
    }
    dev_free(e->ctx, q->vbits);
}

// An influence-estimate query goes straight to verification on its own
// stream: samples 0, 1, 2, ... of `key` against its seed set.
im_status admit_estimate(im_engine *e, Query *q) {
    std::memset(&q->st, 0, sizeof(q->st));
    q->st.i_c = -1.0;
    q->lambda2 = 1.0 + (1.0 + q->est_eps) * upsilon(q->est_eps, q->est_delta);
    q->vkey = q->q.key;
    q->vdone = 0;
    q->vcov = 0;
    q->vlast = q->est_tmax >= 1.8e19 ? ~0ull : uint64_t(std::floor(q->est_tmax));
    q->vneed = uint64_t(std::ceil(q->lambda2));
    q->vhint = 16.0 * double(q->vneed);
    q->vchunk = uint64_t(std::min(1.1 * q->vhint + 1024.0, 4.0e8));
    IM_TRY(seed_bits_into(e->ctx, q->q.graph->n, q->seeds.data(), q->q.k, q->vbits));
    q->phase = kVerify;
    q->t_admit = now_ms();
    if (q->vlast == 0) finish(e, q, kDone, IM_OK);  // nothing may be drawn: -1 with T = 0
    return IM_OK;
}

im_status admit(im_engine *e, Query *q) {
    if (q->q.algo == IM_ALGO_ESTIMATE) return admit_estimate(e, q);
    const im_graph *g = q->q.graph;
    const uint32_t n = g->n, k = q->q.k;
    const double eps = q->q.eps, delta = q->q.delta;
    q->c = caps(n, k, eps, delta);
    const double one_m = 1.0 - std::exp(-1.0);
    if (q->q.algo == IM_ALGO_SSA) {
        // Eq. 15 defaults
        q->eps2 = eps / (2.0 * one_m);
        q->eps3 = q->eps2;
        q->eps1 = (1.0 + eps / (2.0 * (one_m - eps))) / (1.0 + q->eps2) - 1.0;
        q->lambda1 = (1.0 + q->eps1) * (1.0 + q->eps2) * upsilon(q->eps3, delta / (3.0 * q->c.i_max));
        q->delta2p = delta / (3.0 * q->c.i_max);
        q->lambda2 = 1.0 + (1.0 + q->eps2) * upsilon(q->eps2, q->delta2p);
    } else {
        q->lambda1 = 1.0 + (1.0 + eps) * upsilon(eps, delta / (3.0 * q->c.i_max));
    }
    q->n1 = uint64_t(std::ceil(q->c.lambda));
    q->seeds.assign(k, 0);
    std::memset(&q->st, 0, sizeof(q->st));
    q->st.i_c = -1.0;
    IM_TRY(im_pool_create(e->ctx, g, q->q.model, q->q.key, &q->pool));
    q->t = 1;
    q->target = (q->q.algo == IM_ALGO_SSA) ? q->n1 : 2 * q->n1;
    q->phase = kSample;
    q->t_admit = now_ms();
    return IM_OK;
}

void next_iteration(Query *q) {
    q->t += 1;
    const uint64_t size = q->n1 << (q->t - 1);
    q->target = (q->q.algo == IM_ALGO_SSA) ? size : 2 * size;
    q->phase = kSample;
}

// D-SSA checkpoint after the greedy and the stare step (Algorithm 4).
void check_dssa(im_engine *e, Query *q, uint64_t cov, uint64_t cov_c) {
    const double n = estimate_scale(q->q.graph), eps = q->q.eps;
    const double one_m = 1.0 - std::exp(-1.0);
    const uint32_t t = q->t;
    const uint64_t nt = q->n1 << (t - 1);
    im_stats &st = q->st;
    const double i_hat = n * double(cov) / double(nt);
    st.iterations = t;
    st.n_sets = 2 * nt;
    st.cov = cov;
    st.cov_c = cov_c;
    st.i_hat = i_hat;
    if (t <= IM_MAX_ITERS) {
        st.it_sets[t - 1] = nt;
        st.it_cov[t - 1] = cov;
        st.it_cov_c[t - 1] = cov_c;
        st.it_eps_t[t - 1] = -1.0;
    }
    bool done = false;
    if (double(cov_c) >= q->lambda1) {  // D1
        const double two_t1 = std::ldexp(1.0, int(t) - 1);
        const double i_c = double(cov_c) * n / double(nt);
        const double e1 = i_hat / i_c - 1.0;
        const double e2 = eps * std::sqrt(n * (1.0 + eps) / (two_t1 * i_c));
        const double e3 = eps * std::sqrt(n * (1.0 + eps) * (one_m - eps) / ((1.0 + eps / 3.0) * two_t1 * i_c));
        const double e_t = (e1 + e2 + e1 * e2) * (one_m - eps) + one_m * e3;
        st.i_c = i_c;
        st.eps1 = e1;
        st.eps2 = e2;
        st.eps3 = e3;
        st.eps_t = e_t;
        if (t <= IM_MAX_ITERS) st.it_eps_t[t - 1] = e_t;
        if (e_t <= eps) done = true;  // D2
    }
    if (done) {
        finish(e, q, kDone, IM_OK);
    } else if (double(nt) >= q->c.n_max) {
        st.stopped_by_cap = 1;
        finish(e, q, kDone, IM_OK);
    } else {
        next_iteration(q);
    }
}

// SSA after the greedy: condition C1 decides whether to verify.
im_status after_cover_ssa(im_engine *e, Query *q, uint64_t cov) {
    const double n = estimate_scale(q->q.graph);
    const uint32_t t = q->t;
    const uint64_t size = q->n1 << (t - 1);
    im_stats &st = q->st;
    const double i_hat = n * double(cov) / double(size);
    st.iterations = t;
    st.n_sets = size;
    st.cov = cov;
    st.i_hat = i_hat;
    if (t <= IM_MAX_ITERS) {
        st.it_sets[t - 1] = size;
        st.it_cov[t - 1] = cov;
        st.it_eps_t[t - 1] = -1.0;
    }
    if (double(cov) >= q->lambda1) {  // C1: verify on a fresh stream
        const double t_max =
            2.0 * double(size) * (1.0 + q->eps2) / (1.0 - q->eps2) * (q->eps3 * q->eps3) / (q->eps2 * q->eps2);
        q->vkey = derived_key(q->q.key, t);
        q->vdone = 0;
        q->vcov = 0;
        q->vlast = t_max >= 1.8e19 ? ~0ull : uint64_t(std::floor(t_max));
        q->vneed = uint64_t(std::ceil(q->lambda2));
        q->vhint = q->lambda2 * double(size) / double(cov > 0 ? cov : 1);
        q->vchunk = uint64_t(std::min(1.1 * q->vhint + 1024.0, 4.0e8));
        IM_TRY(seed_bits_into(e->ctx, q->q.graph->n, q->seeds.data(), q->q.k, q->vbits));
        q->phase = kVerify;
        return IM_OK;
    }
    if (double(size) >= q->c.n_max) {
        st.stopped_by_cap = 1;
        finish(e, q, kDone, IM_OK);
    } else {
        next_iteration(q);
    }
    return IM_OK;
}

// SSA after Estimate-Inf ended (ic = -1 when T_max was reached): C2. An
// influence-estimate query simply reports I_c and T.
void after_verify_ssa(im_engine *e, Query *q, double ic, uint64_t T) {
    im_stats &st = q->st;
    if (q->q.algo == IM_ALGO_ESTIMATE) {
        st.n_verify = T;
        st.cov_c = T;
        st.i_c = ic;
        finish(e, q, kDone, IM_OK);
        return;
    }
    const uint32_t t = q->t;
    st.n_verify += T;
    st.cov_c = T;
    st.i_c = ic;
    if (t <= IM_MAX_ITERS) {
        st.it_cov_c[t - 1] = T;
        st.it_eps_t[t - 1] = ic;
    }
    const uint64_t size = q->n1 << (t - 1);
    if (st.i_hat <= (1.0 + q->eps1) * ic) {  // C2
        finish(e, q, kDone, IM_OK);
    } else if (double(size) >= q->c.n_max) {
        st.stopped_by_cap = 1;
        finish(e, q, kDone, IM_OK);
    } else {
        next_iteration(q);
    }
}

using GroupKey = std::pair<const im_graph *, int>;

im_status sample_phase(im_engine *e) {
    std::map<GroupKey, std::vector<Query *>> groups;
    for (Query *q : e->active)
        if (q->phase == kSample) groups[{q->q.graph, int(q->q.model)}].push_back(q);
    for (auto &kv : groups) {
        const im_graph *g = kv.first.first;
        const im_model model = im_model(kv.first.second);
        const uint64_t cap = max_batch(model);
        // each query draws at most an eighth of a launch per step, so one
        // that needs many sets spreads them over several steps and the
        // queries beside it finish in between (its sets are the same either
        // way: set j depends only on its key and j)
        const uint64_t quota = std::max<uint64_t>(1, cap / 8);
        const std::vector<Query *> &qs = kv.second;
        size_t i = 0;
        while (i < qs.size()) {
            // one fused launch: as many queries' next chunks as fit the batch cap
            const double t0 = now_ms();
            std::vector<SampleItem> items;
            std::vector<Query *> members;
            uint64_t total = 0;
            double hint = 0;
            for (; i < qs.size(); ++i) {
                Query *q = qs[i];
                const uint64_t take = std::min<uint64_t>(q->target - q->pool->count, quota);
                if (!members.empty() && total + take > cap) break;
                items.push_back(SampleItem{q->pool->key, q->pool->count, take, nullptr});
                members.push_back(q);
                total += take;
                hint = std::max(hint, q->pool->mean_size);
            }
            SampleResult r;
            std::vector<ItemTotals> tot(items.size());
            IM_TRY(sample_items(e->ctx, g, model, items.data(), uint32_t(items.size()), SampleMode::Pool, hint, &r,
                                tot.data()));
            std::vector<AppendItem> app(items.size());
            for (size_t j = 0; j < items.size(); ++j)
                app[j] = AppendItem{members[j]->pool, items[j].count, tot[j].nodes, tot[j].edges};
            IM_TRY(pool_append_items(e->ctx, app.data(), uint32_t(app.size())));
            const double dt = now_ms() - t0;
            for (Query *q : members) {
                q->st.ms_sample += dt;
                if (q->pool->count >= q->target) q->phase = kCover;
            }
        }
    }
    return IM_OK;
}

im_status verify_phase(im_engine *e) {
    std::map<GroupKey, std::vector<Query *>> groups;
    for (Query *q : e->active)
        if (q->phase == kVerify) groups[{q->q.graph, int(q->q.model)}].push_back(q);
    for (auto &kv : groups) {
        const im_graph *g = kv.first.first;
        const im_model model = im_model(kv.first.second);
        std::vector<Query *> &qs = kv.second;
        const uint64_t cap = max_batch(model);
        size_t i = 0;
        while (i < qs.size()) {
            const double t0 = now_ms();
            std::vector<SampleItem> items;
            std::vector<Query *> members;
            uint64_t total = 0;
            for (; i < qs.size(); ++i) {
                Query *q = qs[i];
                const uint64_t c = std::min<uint64_t>(std::min<uint64_t>(std::max<uint64_t>(q->vchunk, 1024), cap),
                                                      q->vlast - q->vdone);
                if (!members.empty() && total + c > cap) break;
                items.push_back(SampleItem{q->vkey, q->vdone, c, static_cast<const uint32_t *>(q->vbits.ptr)});
                members.push_back(q);
                total += c;
            }
            SampleResult r;
            std::vector<ItemTotals> tot(items.size());
            IM_TRY(sample_items(e->ctx, g, model, items.data(), uint32_t(items.size()), SampleMode::Hits, 0.0, &r,
                                tot.data()));
            std::vector<CrossItem> cross(items.size());
            std::vector<int64_t> idx(items.size());
            std::vector<uint64_t> hits(items.size());
            uint64_t start = 0;
            for (size_t j = 0; j < items.size(); ++j) {
                cross[j] = CrossItem{start, items[j].count, members[j]->vneed - members[j]->vcov, &idx[j], &hits[j]};
                start += items[j].count;
            }
            IM_TRY(first_crossing_items(e->ctx, cross.data(), uint32_t(cross.size())));
            const double dt = now_ms() - t0;
            for (size_t j = 0; j < items.size(); ++j) {
                Query *q = members[j];
                q->st.ms_verify += dt;
                q->verify_edges += tot[j].edges;
                if (idx[j] >= 0) {
                    const uint64_t T = q->vdone + uint64_t(idx[j]) + 1;
                    after_verify_ssa(e, q, estimate_scale(g) * q->lambda2 / double(T), T);
                    continue;
                }
                q->vcov += hits[j];
                q->vdone += items[j].count;
                q->vchunk = std::max<uint64_t>(uint64_t(0.25 * q->vhint) + 1024, q->vchunk / 2);
                if (q->vdone >= q->vlast) after_verify_ssa(e, q, -1.0, q->vlast);
            }
        }
    }
    return IM_OK;
}

im_status cover_phase(im_engine *e) {
    std::map<const im_graph *, std::vector<Query *>> groups;
    for (Query *q : e->active)
        if (q->phase == kCover) groups[q->q.graph].push_back(q);
    for (auto &kv : groups) {
        std::vector<Query *> &qs = kv.second;
        std::vector<CoverJob> jobs(qs.size());
        for (size_t j = 0; j < qs.size(); ++j) {
            Query *q = qs[j];
            const uint64_t nt = q->n1 << (q->t - 1);
            CoverJob &cj = jobs[j];
            cj.pool = q->pool;
            cj.begin = 0;
            cj.end = nt;
            cj.k = q->q.k;
            cj.stare_begin = cj.stare_end = nt;
            if (q->q.algo == IM_ALGO_DSSA) cj.stare_end = 2 * nt;
            cj.seeds = q->seeds.data();
        }
        const double t0 = now_ms();
        if (jobs.size() == 1) {
            // a lone query takes the latency-oriented single-range path
            CoverJob &cj = jobs[0];
            IM_TRY(max_coverage(cj.pool, cj.begin, cj.end, cj.k, cj.seeds, &cj.cov));
            if (cj.stare_end > cj.stare_begin)
                IM_TRY(coverage_range(cj.pool, cj.stare_begin, cj.stare_end, cj.seeds, cj.k, &cj.cov_c));
        } else {
            IM_TRY(max_coverage_batch(e->ctx, kv.first, jobs.data(), uint32_t(jobs.size())));
        }
        const double dt = now_ms() - t0;
        for (size_t j = 0; j < qs.size(); ++j) {
            Query *q = qs[j];
            q->st.ms_cover += dt;
            if (q->q.algo == IM_ALGO_DSSA) check_dssa(e, q, jobs[j].cov, jobs[j].cov_c);
            else IM_TRY(after_cover_ssa(e, q, jobs[j].cov));
        }
    }
    return IM_OK;
}

}  // namespace

extern "C" im_status im_engine_create(im_ctx *ctx, uint64_t pool_budget_bytes, uint32_t max_active, im_engine **out) {
    clear_error();
    if (!ctx || !out || max_active == 0) {
        set_error("im_engine_create: bad arguments");
        return IM_E_ARG;
    }
    auto *e = new (std::nothrow) im_engine();
    if (!e) return IM_E_OOM;
    e->ctx = ctx;
    e->budget = pool_budget_bytes;
    e->max_active = max_active;
    *out = e;
    return IM_OK;
}

extern "C" void im_engine_free(im_engine *e) {
    if (!e) return;
    for (auto &kv : e->all) {
        Query *q = kv.second;
        if (q->pool) im_pool_free(q->pool);
        dev_free(e->ctx, q->vbits);
        delete q;
    }
    delete e;
}

extern "C" im_status im_engine_submit(im_engine *e, const im_query *query, uint64_t *ticket) {
    clear_error();
    if (!e || !query || !ticket) return IM_E_ARG;
    IM_TRY(check_query(query->graph, query->model, query->k, query->eps, query->delta));
    if (query->graph->ctx != e->ctx || (query->algo != IM_ALGO_SSA && query->algo != IM_ALGO_DSSA)) {
        set_error("im_engine_submit: graph of another context or unknown algorithm");
        return IM_E_ARG;
    }
    auto *q = new (std::nothrow) Query();
    if (!q) return IM_E_OOM;
    q->ticket = e->next_ticket++;
    q->q = *query;
    q->t_submit = now_ms();
    e->pending.push_back(q);
    e->all[q->ticket] = q;
    *ticket = q->ticket;
    return IM_OK;
}

extern "C" im_status im_engine_submit_estimate(im_engine *e, const im_graph *g, im_model model,
                                               const uint32_t *seeds, uint32_t k, double eps_p, double delta_p,
                                               double t_max, uint64_t key, uint64_t *ticket) {
    clear_error();
    if (!e || !g || !seeds || !ticket || k == 0 || g->ctx != e->ctx) {
        set_error("im_engine_submit_estimate: bad arguments");
        return IM_E_ARG;
    }
    if (model != IM_IC && model != IM_LT) {
        set_error("im_engine_submit_estimate: unknown model %d", int(model));
        return IM_E_ARG;
    }
    if (!(g->models & (1u << model))) {
        set_error("im_engine_submit_estimate: graph has no weights for model %d", int(model));
        return IM_E_ARG;
    }
    if (!(eps_p > 0.0 && eps_p < 1.0 && delta_p > 0.0 && delta_p < 1.0 && t_max >= 0.0)) {
        set_error("im_engine_submit_estimate: eps_p, delta_p must be in (0,1), t_max >= 0");
        return IM_E_ARG;
    }
    for (uint32_t i = 0; i < k; ++i)
        if (seeds[i] >= g->n) {
            set_error("im_engine_submit_estimate: seed %u out of range", seeds[i]);
            return IM_E_ARG;
        }
    auto *q = new (std::nothrow) Query();
    if (!q) return IM_E_OOM;
    q->ticket = e->next_ticket++;
    q->q = im_query{g, model, IM_ALGO_ESTIMATE, k, eps_p, delta_p, key};
    q->seeds.assign(seeds, seeds + k);
    q->est_eps = eps_p;
    q->est_delta = delta_p;
    q->est_tmax = t_max;
    q->t_submit = now_ms();
    e->pending.push_back(q);
    e->all[q->ticket] = q;
    *ticket = q->ticket;
    return IM_OK;
}

extern "C" im_status im_engine_step(im_engine *e, uint32_t *n_active, uint32_t *n_pending) {
    clear_error();
    if (!e) return IM_E_ARG;
    // admission: by slots and by the bytes the active pools hold
    while (!e->pending.empty() && e->active.size() < e->max_active &&
           (e->active.empty() || active_bytes(e) < e->budget)) {
        Query *q = e->pending.front();
        e->pending.pop_front();
        im_status rc = admit(e, q);
        if (rc != IM_OK) {
            finish(e, q, kFailed, rc);
            continue;
        }
        e->active.push_back(q);
    }
    im_status rc = IM_OK;
    // verification first, so a query whose C2 fails samples its next
    // iteration in this same step
    if ((rc = verify_phase(e)) == IM_OK && (rc = sample_phase(e)) == IM_OK) rc = cover_phase(e);
    if (rc != IM_OK) {
        for (Query *q : e->active)
            if (q->phase != kDone && q->phase != kFailed) finish(e, q, kFailed, rc);
    }
    std::vector<Query *> still;
    for (Query *q : e->active)
        if (q->phase != kDone && q->phase != kFailed) still.push_back(q);
    e->active.swap(still);
    if (n_active) *n_active = uint32_t(e->active.size());
    if (n_pending) *n_pending = uint32_t(e->pending.size());
    return rc;
}

extern "C" im_status im_engine_poll(im_engine *e, uint64_t ticket, int *state) {
    clear_error();
    if (!e || !state) return IM_E_ARG;
    auto it = e->all.find(ticket);
    if (it == e->all.end()) {
        set_error("im_engine_poll: unknown ticket %llu", static_cast<unsigned long long>(ticket));
        return IM_E_ARG;
    }
    const Query *q = it->second;
    *state = q->phase == kDone ? 1 : (q->phase == kFailed ? int(q->err) : 0);
    return IM_OK;
}

extern "C" im_status im_engine_result(im_engine *e, uint64_t ticket, uint32_t *seeds_out, im_stats *st) {
    clear_error();
    if (!e) return IM_E_ARG;
    auto it = e->all.find(ticket);
    if (it == e->all.end()) {
        set_error("im_engine_result: unknown ticket %llu", static_cast<unsigned long long>(ticket));
        return IM_E_ARG;
    }
    Query *q = it->second;
    if (q->phase == kFailed) {
        set_error("query %llu failed with status %d", static_cast<unsigned long long>(ticket), int(q->err));
        im_status err = q->err;
        e->all.erase(it);
        delete q;
        return err;
    }
    if (q->phase != kDone) {
        set_error("query %llu is not finished", static_cast<unsigned long long>(ticket));
        return IM_E_STATE;
    }
    if (seeds_out) std::memcpy(seeds_out, q->seeds.data(), 4ull * q->q.k);
    if (st) *st = q->st;
    e->all.erase(it);
    delete q;
    return IM_OK;
}

extern "C" im_status im_engine_run(im_engine *e) {
    clear_error();
    if (!e) return IM_E_ARG;
    uint32_t na = 0, np = 0;
    do {
        IM_TRY(im_engine_step(e, &na, &np));
    } while (na + np > 0);
    return IM_OK;
}
