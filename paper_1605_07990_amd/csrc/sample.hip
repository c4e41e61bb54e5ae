// RR-set sampling (Definition 2) on gfx950.
//
// Every RR set is a pure function of (key, sample index): the source and
// every coin are Philox words at counters naming (sample, edge group) or
// (sample, node). So samples can run in any order, on any lane, and be
// re-run, and the pool is identical to a sequential draw.
//
// IC  — one wave per sample: reverse breadth-first search whose frontier
//       (up to 64 queued nodes at a time) is expanded as one flat list of
//       aligned 4-edge groups spread over the wave's lanes; one Philox call
//       per group gives the four edge coins. Visited set: an LDS bitmap
//       (n <= 65536) or an LDS open-addressing hash; the queue lives in LDS.
// LT  — one lane per sample: the reverse walk keeps at most one in-edge per
//       node (interpolation search of the node's cumulative thresholds in
//       8-record windows); revisits are caught exactly by a per-lane bucketed
//       hash table in global memory whose entries carry the walk's stamp.
// Long path — samples that outgrow LDS (IC) or the per-sample staging
//       region (LT) are deferred and re-run from scratch by whole waves on
//       global epoch-stamped visited arrays and queues.
// Pool append — sizes are scanned into the CSR offsets in sample order and
//       each set is copied from staging into the flat pool.
#include <algorithm>
#include <cmath>
#include <vector>

#include "im_device.hpp"
#include "im_internal.hpp"

namespace {

using namespace imd;

constexpr int kIcWaves = 4;                  // waves per IC block
constexpr uint32_t kIcQcap = 1024;           // LDS queue entries per wave
constexpr uint32_t kIcHcap = 2048;           // LDS hash slots / bitmap words per wave
constexpr uint32_t kIcHbits = 11;            // log2(kIcHcap)
constexpr uint32_t kBitmapMaxN = kIcHcap * 32;
constexpr uint32_t kLtCap = 512;             // per-sample staging region (LT)
constexpr int kLongWaves = 4;
constexpr uint32_t kStageChunk = 1024;       // IC staging entries a wave reserves at once
// IC workgroup tiers: a sample the wave pass hands on goes to a 256-thread
// workgroup (five fit on a compute unit, so many heavy samples advance at
// once: their BFS levels are many and small); one too large for its LDS goes
// to a 1024-thread workgroup with four times the LDS, then to the long path.
struct GrpSmall {
    static constexpr int kThreads = 256;
    static constexpr uint32_t kQcap = 2048;  // LDS queue entries
    static constexpr uint32_t kHbits = 12;   // LDS hash slots: 4096
};
struct GrpLarge {
    static constexpr int kThreads = 1024;
    static constexpr uint32_t kQcap = 8192;
    static constexpr uint32_t kHbits = 14;  // 16384
};

// Hand-over records (IC): a sample the wave pass hands to the small tier, or
// the small tier to the large one, carries its search state, and the next
// tier resumes it instead of starting over. A record is a header [t, head,
// tail, edges low, edges high, 0, 0, 0] and queue[0, tail): the state at the
// start of the frontier batch that was not finished, so every node reached
// before that batch is queued and the first `head` of them are expanded (the
// set reached does not depend on the order of expansion). Samples handed on
// past the records available start over, as does the long path.
constexpr uint32_t kHoHdr = 8;
constexpr uint32_t kHoStrideWave = kHoHdr + kIcQcap;
constexpr uint32_t kHoStrideSmall = kHoHdr + GrpSmall::kQcap;
constexpr uint32_t kHoMaxWave = 1u << 16;  // records per launch
constexpr uint32_t kHoMaxSmall = 1u << 14;
static_assert(kIcQcap <= GrpSmall::kQcap && GrpSmall::kQcap <= GrpLarge::kQcap,
              "a tier must hold the queue of the tier before it");
static_assert((1u << GrpSmall::kHbits) >= 2 * kIcQcap && (1u << GrpLarge::kHbits) >= 2 * GrpSmall::kQcap,
              "a resumed queue must fit a tier's visited set");

struct Counters {
    uint32_t ticket;        // next sample of the main pass
    uint32_t defer_count;   // samples handed on by the main pass (IC: to the workgroup tier; LT: to the long path)
    uint32_t defer_ticket;  // next of them to take
    uint32_t large_count;   // IC samples the small workgroup tier hands to the large one
    uint32_t large_ticket;
    uint32_t long_count;    // IC samples the large workgroup tier hands to the long path
    uint32_t long_ticket;
    uint32_t overflow;      // staging too small: the batch must be re-run
    unsigned long long stage_cursor;
    unsigned long long edges;        // main pass
    unsigned long long total_nodes;  // main pass
    unsigned long long edges_long;   // long path
    unsigned long long nodes_long;   // long path
    unsigned long long grp_samples;  // IC workgroup tier: samples finished there
    unsigned long long grp_edges;    //   their examined edges
    unsigned long long grp_levels;   //   their BFS levels
};

// One entry of the device work queue: samples [s0, s0+count) of stream
// `key`, occupying global slots [start, start+count) of the launch.
struct WorkItem {
    uint64_t key;
    uint64_t s0;
    uint32_t start;
    uint32_t count;
    const uint32_t *seedbits;  // hits mode: the query's seed bitmap
    unsigned long long *acc;   // per item: [0] node entries drawn, [1] edges traversed
};

struct Params {
    const uint64_t *off;
    const uint2 *edges;
    const uint64_t *src_cum;  // weighted sources, or null
    uint32_t n;
    uint32_t count;  // slots over all items
    const WorkItem *items;
    uint32_t nitems;
    Counters *cnt;
    uint32_t *defer_list;
    uint32_t *large_list;  // IC: samples the small workgroup tier hands to the large one
    uint32_t *long_list;   // IC: samples the large workgroup tier hands to the long path
    uint32_t *stage;
    uint64_t stage_cap;
    uint64_t *stage_off;  // per sample
    uint32_t *sizes;      // per sample
    uint8_t *z;           // per sample (hits mode)
    uint32_t lt_cap;
    uint32_t ticket_block;  // IC: consecutive samples a wave takes per ticket
    uint32_t edge_budget;   // IC: the most in-edges a wave examines for one sample; larger ones go to a workgroup
    uint32_t plain;         // IC: 1 = static assignment (wave w takes samples w, w + W, ...), no tickets
    uint32_t *ho_wave;      // IC: hand-over records of the wave pass (kHoStrideWave words each)
    uint32_t *ho_small;     // IC: hand-over records of the small workgroup tier (kHoStrideSmall words each)
    uint32_t ho_wave_cap;   // records available in each (0: none)
    uint32_t ho_small_cap;
    // IC: the graph's compact form (null: read off and the records); the
    // long path always reads off and the records
    const uint4 *nodes;     // {first in-edge low, high, in-degree, thr}
    const uint32_t *srcs;   // src per edge, zero-padded to whole groups + 4
};

// The work item owning global slot t.
__device__ __forceinline__ const WorkItem &item_of(const Params &p, uint32_t t) {
    uint32_t lo = 0, hi = p.nitems - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (p.items[mid].start <= t) lo = mid;
        else hi = mid - 1;
    }
    return p.items[lo];
}

// The work item of slot t, reusing `cur` (an index) while t stays inside it:
// a wave's or lane's tickets increase, so the search runs once per item.
__device__ __forceinline__ const WorkItem &item_cached(const Params &p, uint32_t t, uint32_t &cur) {
    const WorkItem &c = p.items[cur];
    if (t >= c.start && t - c.start < c.count) return c;
    uint32_t lo = 0, hi = p.nitems - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (p.items[mid].start <= t) lo = mid;
        else hi = mid - 1;
    }
    cur = lo;
    return p.items[lo];
}

// Per-item totals (node entries, edges) held in registers while a lane or
// wave stays on one work item and added to the item's accumulator with two
// atomics when it moves to another item or ends: one item's accumulator is
// shared by every wave, so a per-sample atomic would serialise them.
struct ItemAcc {
    unsigned long long *acc = nullptr;
    uint64_t nodes = 0, edges = 0;

    __device__ __forceinline__ void flush() {
        if (acc) {
            if (nodes) atomicAdd(&acc[0], static_cast<unsigned long long>(nodes));
            if (edges) atomicAdd(&acc[1], static_cast<unsigned long long>(edges));
        }
        nodes = edges = 0;
    }
    // `owner`: whether this lane issues the flush (lane 0 when the totals are
    // wave-uniform)
    __device__ __forceinline__ void move_to(unsigned long long *a, bool owner) {
        if (a != acc) {
            if (owner) flush();
            nodes = edges = 0;
            acc = a;
        }
    }
};

// End of a lane-per-sample kernel: one atomic pair per wave when every lane
// with totals holds the same item, else one pair per lane.
__device__ __forceinline__ void flush_lanes(ItemAcc &ia) {
    const uint64_t has = __ballot((ia.nodes | ia.edges) != 0);
    if (has == 0) return;
    const uint64_t mine = reinterpret_cast<uint64_t>(ia.acc);
    const uint64_t first = __shfl(mine, __ffsll(static_cast<unsigned long long>(has)) - 1, kWave);
    const bool same = (ia.nodes | ia.edges) == 0 || mine == first;
    if (__ballot(!same) == 0) {
        const uint64_t nsum = wave_sum_u64(ia.nodes);
        const uint64_t esum = wave_sum_u64(ia.edges);
        if (lane_id() == 0) {
            auto *a = reinterpret_cast<unsigned long long *>(first);
            if (nsum) atomicAdd(&a[0], static_cast<unsigned long long>(nsum));
            if (esum) atomicAdd(&a[1], static_cast<unsigned long long>(esum));
        }
        ia.nodes = ia.edges = 0;
    } else {
        ia.flush();
    }
}

// Plain IC launches have no workgroup tiers: the samples the wave pass hands
// on go straight to the long path.
__global__ void plain_handoff_kernel(Counters *c) {
    c->long_count = c->defer_count;
    c->long_ticket = 0;
}

__global__ void init_counters_kernel(Counters *c, unsigned long long cursor0) {
    c->ticket = 0;
    c->defer_count = 0;
    c->defer_ticket = 0;
    c->large_count = 0;
    c->large_ticket = 0;
    c->long_count = 0;
    c->long_ticket = 0;
    c->overflow = 0;
    c->stage_cursor = cursor0;
    c->edges = 0;
    c->total_nodes = 0;
    c->edges_long = 0;
    c->nodes_long = 0;
    c->grp_samples = 0;
    c->grp_edges = 0;
    c->grp_levels = 0;
}

// ---------------------------------------------------------------- IC ----

// In-edges [a, a + deg) of frontier node v and, in the compact form, the
// threshold they share (one aligned 16-byte load instead of the offset
// pair).
__device__ __forceinline__ void ic_node(const Params &p, uint32_t v, uint64_t &a, uint32_t &deg, uint32_t &thr) {
    if (p.nodes) {
        const uint4 r = p.nodes[v];
        a = static_cast<uint64_t>(r.x) | (static_cast<uint64_t>(r.y) << 32);
        deg = r.z;
        thr = r.w;
    } else {
        a = p.off[v];
        deg = static_cast<uint32_t>(p.off[v + 1] - a);
        thr = 0u;
    }
}

// The live edges among the four in-edge records of 4-edge group g of a node
// whose in-edges are [ea, eb). The group's 32 bytes come in two 16-byte
// loads (the record array is padded to whole aligned groups, so they stay
// in it; records outside [ea, eb) belong to other nodes or the pad and are
// never live), and liveness is decided without a branch.
__device__ __forceinline__ void ic_group_live(const uint2 *edges, uint64_t g, uint64_t ea, uint64_t eb,
                                              const uint4 &coins, uint2 (&rec)[4], bool (&live)[4]) {
    if (eb <= ea) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            rec[q] = make_uint2(0u, 0u);
            live[q] = false;
        }
        return;
    }
    const uint4 *gp = reinterpret_cast<const uint4 *>(edges + (g << 2));
    const uint4 lo = gp[0], hi = gp[1];
    rec[0] = make_uint2(lo.x, lo.y);
    rec[1] = make_uint2(lo.z, lo.w);
    rec[2] = make_uint2(hi.x, hi.y);
    rec[3] = make_uint2(hi.z, hi.w);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint64_t e = (g << 2) + q;
        live[q] = (e >= ea) & (e < eb) & ic_live(word_of(coins, q), rec[q].y);
    }
}

// ic_group_live on either form: in the compact one the group's four
// sources are one aligned 16-byte load and `thr` is the node's threshold.
__device__ __forceinline__ void ic_group_read(const Params &p, uint64_t g, uint64_t ea, uint64_t eb, uint32_t thr,
                                              const uint4 &coins, uint2 (&rec)[4], bool (&live)[4]) {
    if (!p.srcs) {
        ic_group_live(p.edges, g, ea, eb, coins, rec, live);
        return;
    }
    if (eb <= ea) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            rec[q] = make_uint2(0u, 0u);
            live[q] = false;
        }
        return;
    }
    const uint4 s4 = reinterpret_cast<const uint4 *>(p.srcs)[g];
    rec[0] = make_uint2(s4.x, thr);
    rec[1] = make_uint2(s4.y, thr);
    rec[2] = make_uint2(s4.z, thr);
    rec[3] = make_uint2(s4.w, thr);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        const uint64_t e = (g << 2) + q;
        live[q] = (e >= ea) & (e < eb) & ic_live(word_of(coins, q), thr);
    }
}

template <bool kBitmap>
__device__ __forceinline__ bool vis_insert(uint32_t *vis, uint32_t u, bool &full) {
    if constexpr (kBitmap) {
        const uint32_t bit = 1u << (u & 31u);
        const uint32_t old = atomicOr(&vis[u >> 5], bit);
        return !(old & bit);
    } else {
        const uint32_t key = u + 1u;
        uint32_t h = (u * 2654435761u) >> (32 - kIcHbits);
        for (uint32_t probe = 0; probe < kIcHcap; ++probe) {
            const uint32_t old = atomicCAS(&vis[h], 0u, key);
            if (old == 0u) return true;
            if (old == key) return false;
            h = (h + 1u) & (kIcHcap - 1u);
        }
        full = true;
        return false;
    }
}

// vis_insert in two steps, so that a lane's first probes of several nodes
// are in flight together: vis_probe makes the first attempt (the old word),
// vis_settle decides from it and, on a slot held by another node, probes on.
template <bool kBitmap>
__device__ __forceinline__ uint32_t vis_probe(uint32_t *vis, uint32_t u) {
    if constexpr (kBitmap) {
        return atomicOr(&vis[u >> 5], 1u << (u & 31u));
    } else {
        return atomicCAS(&vis[(u * 2654435761u) >> (32 - kIcHbits)], 0u, u + 1u);
    }
}

template <bool kBitmap>
__device__ __forceinline__ bool vis_settle(uint32_t *vis, uint32_t u, uint32_t old, bool &full) {
    if constexpr (kBitmap) {
        return !(old & (1u << (u & 31u)));
    } else {
        const uint32_t key = u + 1u;
        if (old == 0u) return true;
        if (old == key) return false;
        uint32_t h = (u * 2654435761u) >> (32 - kIcHbits);
        for (uint32_t probe = 1; probe < kIcHcap; ++probe) {
            h = (h + 1u) & (kIcHcap - 1u);
            const uint32_t o = atomicCAS(&vis[h], 0u, key);
            if (o == 0u) return true;
            if (o == key) return false;
        }
        full = true;
        return false;
    }
}

template <bool kBitmap>
__device__ __forceinline__ uint32_t vis_slot(const uint32_t *vis, uint32_t u) {
    if constexpr (kBitmap) {
        return u >> 5;
    } else {
        const uint32_t key = u + 1u;
        uint32_t h = (u * 2654435761u) >> (32 - kIcHbits);
        for (uint32_t probe = 0; probe < kIcHcap; ++probe) {
            if (vis[h] == key) return h;
            h = (h + 1u) & (kIcHcap - 1u);
        }
        return kIcHcap;  // not found (cannot happen for an inserted node)
    }
}

// Clear the visited structure after a sample whose queued nodes are
// queue[0..tail) (every inserted node is queued unless `dirty`).
template <bool kBitmap>
__device__ __forceinline__ void vis_clear(uint32_t *vis, const uint32_t *queue, uint32_t tail, bool dirty,
                                          uint32_t lane) {
    if (dirty || tail > kWave) {
        for (uint32_t i = lane; i < kIcHcap; i += kWave) vis[i] = 0u;
    } else {
        uint32_t slot = kIcHcap;
        if (lane < tail) slot = vis_slot<kBitmap>(vis, queue[lane]);
        wave_sync();
        if (slot < kIcHcap) vis[slot] = 0u;
    }
    wave_sync();
}

template <int kMode, bool kBitmap>
__global__ __launch_bounds__(kIcWaves *kWave) void ic_main_kernel(Params p) {
    __shared__ uint32_t s_queue[kIcWaves][kIcQcap];
    __shared__ uint32_t s_vis[kIcWaves][kIcHcap];
    __shared__ uint32_t s_pre[kIcWaves][kWave];
    __shared__ uint64_t s_a[kIcWaves][kWave];
    __shared__ uint2 s_b[kIcWaves][kWave];  // {in-degree, thr}

    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    uint32_t *queue = s_queue[wave];
    uint32_t *vis = s_vis[wave];
    uint32_t *pre = s_pre[wave];
    uint64_t *fa = s_a[wave];
    uint2 *fb = s_b[wave];
    for (uint32_t i = lane; i < kIcHcap; i += kWave) vis[i] = 0u;
    wave_sync();
    uint64_t edges_acc = 0, nodes_acc = 0;
    ItemAcc ia;  // wave-uniform; lane 0 flushes
    // wave-uniform: the block of samples taken per ticket, the item cache and
    // the staging chunk carved up without further atomics
    uint32_t t_next = 0, t_end = 0, cur = 0;
    uint64_t chunk_pos = 0, chunk_end = 0;
    // plain launches: the wave's fixed share of the samples, no work queue
    const uint32_t waves_total = gridDim.x * kIcWaves;
    uint32_t plain_next = blockIdx.x * kIcWaves + wave;

    for (;;) {
        if (t_next == t_end) {
            uint32_t base = 0;
            if (p.plain) {
                base = plain_next;
                plain_next += waves_total;
            } else {
                if (lane == 0) base = atomicAdd(&p.cnt->ticket, p.ticket_block);
                base = __shfl(base, 0, kWave);
            }
            if (base >= p.count) break;
            t_next = base;
            t_end = p.plain ? base + 1 : min(base + p.ticket_block, p.count);
        }
        const uint32_t t = t_next++;
        const WorkItem &it = item_cached(p, t, cur);
        ia.move_to(it.acc, lane == 0);
        const Stream st(it.key);
        const uint32_t *seedbits = it.seedbits;
        const uint64_t s = it.s0 + (t - it.start);
        const uint32_t v0 = pick_source(st, s, p.src_cum, p.n);
        bool full = false;
        if (lane == 0) {
            vis_insert<kBitmap>(vis, v0, full);
            queue[0] = v0;
        }
        uint32_t head = 0, tail = 1;
        bool hit = (kMode == 1) && test_bit(seedbits, v0);
        uint64_t sample_edges = 0;
        wave_sync();

        bool heavy = false;
        // the state at the start of the current frontier batch (what a
        // hand-over record carries)
        uint32_t hb = 0, tb = 1;
        uint64_t eb = 0;
        while (head < tail && !hit) {
            hb = head;
            tb = tail;
            eb = sample_edges;
            const uint32_t nb = min(tail - head, static_cast<uint32_t>(kWave));
            uint32_t cg = 0, deg = 0, thr = 0;
            uint64_t a = 0;
            if (lane < nb) {
                ic_node(p, queue[head + lane], a, deg, thr);
                if (deg) cg = static_cast<uint32_t>(((a + deg - 1) >> 2) - (a >> 2) + 1);
            }
            const uint64_t batch_edges = wave_sum_small_u64(deg);
            // a workgroup finishes a sample that would examine more in-edges
            // than the budget; checked before the batch is expanded, so that
            // a batch holding a high in-degree node (hundreds of thousands of
            // in-edges on a power-law graph) is never expanded here first
            if (sample_edges + batch_edges > p.edge_budget) {
                heavy = true;
                break;
            }
            sample_edges += batch_edges;
            const uint32_t inc = wave_scan_u32(cg);
            const uint32_t groups = wave_scan_total(inc);
            pre[lane] = inc - cg;
            fa[lane] = a;
            fb[lane] = make_uint2(deg, thr);
            head += nb;
            wave_sync();

            bool stop = false;
            for (uint32_t base = 0; base < groups; base += kWave) {
                const uint32_t w = base + lane;
                uint32_t f0 = 0xFFFFFFFFu, f1 = 0xFFFFFFFFu, f2 = 0xFFFFFFFFu, f3 = 0xFFFFFFFFu;
                if (w < groups) {
                    // owner: last frontier slot whose first group index <= w
                    uint32_t lo = 0, hi = nb - 1;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi + 1) >> 1;
                        if (pre[mid] <= w) lo = mid;
                        else hi = mid - 1;
                    }
                    const uint64_t ea = fa[lo];
                    const uint2 db = fb[lo];
                    const uint64_t eb = ea + db.x;
                    const uint64_t g = (ea >> 2) + (w - pre[lo]);
                    const uint4 coins = ic_coins(st, s, g);
                    uint2 rec[4];
                    bool live[4];
                    ic_group_read(p, g, ea, eb, db.y, coins, rec, live);
                    // the first probes of the four records go out together;
                    // a probe that meets another node goes on alone
                    uint32_t old[4];
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) old[q] = live[q] ? vis_probe<kBitmap>(vis, rec[q].x) : 0u;
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        if (live[q] && vis_settle<kBitmap>(vis, rec[q].x, old[q], full)) {
                            if (q == 0) f0 = rec[q].x;
                            else if (q == 1) f1 = rec[q].x;
                            else if (q == 2) f2 = rec[q].x;
                            else f3 = rec[q].x;
                        }
                    }
                }
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q) {
                    const uint32_t f = (q == 0) ? f0 : (q == 1) ? f1 : (q == 2) ? f2 : f3;
                    const bool has = f != 0xFFFFFFFFu;
                    const uint64_t mask = __ballot(has);
                    if (mask) {
                        const uint32_t pos = tail + lanes_below(mask);
                        if (has) {
                            if (pos < kIcQcap) queue[pos] = f;
                            if (kMode == 1 && test_bit(seedbits, f)) hit = true;
                        }
                        tail += static_cast<uint32_t>(__popcll(mask));
                    }
                }
                if (kMode == 1) hit = __ballot(hit) != 0;
                if (tail > kIcQcap || __ballot(full) != 0 || hit) {
                    stop = true;
                    break;
                }
            }
            wave_sync();
            if (stop) break;
        }

        const bool overflow = (tail > kIcQcap) || (__ballot(full) != 0) || heavy;
        if (overflow && !hit) {
            uint32_t d = 0;
            if (lane == 0) {
                d = atomicAdd(&p.cnt->defer_count, 1u);
                p.defer_list[d] = t;
            }
            d = __shfl(d, 0, kWave);
            if (d < p.ho_wave_cap) {  // queue[0, tb) is untouched by the unfinished batch
                uint32_t *rec = p.ho_wave + static_cast<uint64_t>(d) * kHoStrideWave;
                for (uint32_t i = lane; i < tb; i += kWave) rec[kHoHdr + i] = queue[i];
                if (lane == 0) {
                    rec[0] = t;
                    rec[1] = hb;
                    rec[2] = tb;
                    rec[3] = static_cast<uint32_t>(eb);
                    rec[4] = static_cast<uint32_t>(eb >> 32);
                }
            }
        } else if (kMode == 1) {
            if (lane == 0) p.z[t] = hit ? 1 : 0;
            ia.edges += sample_edges;
            edges_acc += sample_edges;
        } else {
            if (chunk_end - chunk_pos < tail) {
                const uint64_t want = max(static_cast<uint64_t>(tail), static_cast<uint64_t>(kStageChunk));
                unsigned long long c0 = 0;
                if (lane == 0) c0 = atomicAdd(&p.cnt->stage_cursor, static_cast<unsigned long long>(want));
                chunk_pos = __shfl(c0, 0, kWave);
                chunk_end = chunk_pos + want;
            }
            const uint64_t base = chunk_pos;
            chunk_pos += tail;
            const bool fits = base + tail <= p.stage_cap;
            if (lane == 0) {
                if (!fits) atomicOr(&p.cnt->overflow, 1u);
                p.sizes[t] = fits ? tail : 0;
                p.stage_off[t] = fits ? base : 0;
            }
            if (fits)
                for (uint32_t i = lane; i < tail; i += kWave) p.stage[base + i] = queue[i];
            ia.nodes += tail;
            ia.edges += sample_edges;
            edges_acc += sample_edges;
            nodes_acc += tail;
        }
        vis_clear<kBitmap>(vis, queue, min(tail, kIcQcap), overflow || hit, lane);
    }
    if (lane == 0) {
        ia.flush();
        if (edges_acc) atomicAdd(&p.cnt->edges, static_cast<unsigned long long>(edges_acc));
        if (nodes_acc) atomicAdd(&p.cnt->total_nodes, static_cast<unsigned long long>(nodes_acc));
    }
}

// ---------------------------------------------------------------- LT ----

// Per-lane visited set: an open-addressed table of 64-byte buckets (8 u64
// entries: walk stamp << 32 | node) in global memory. Entries of earlier
// walks carry older stamps and count as free, so a table is never cleared.
// A lookup's bucket load is issued together with the next node's offsets.
constexpr uint32_t kLtBucketSlots = 8;
constexpr uint32_t kLtBuckets = 128;  // 1024 entries = 8 KiB per lane
constexpr uint32_t kLtTableSlots = kLtBuckets * kLtBucketSlots;
constexpr uint32_t kLtMaxWalk = 640;  // longer walks take the long path (load <= 5/8)

__device__ __forceinline__ uint32_t lt_bucket(uint32_t u) { return (u * 0x9E3779B1u) >> (32 - 7); }

__device__ __forceinline__ uint64_t lt_entry(uint32_t stamp, uint32_t u) {
    return (static_cast<uint64_t>(stamp) << 32) | u;
}

// The in-edge kept by node v's LT coin c: the first e in [a, b) whose
// cumulative threshold exceeds c, or b if none (a < b). Interpolation on the
// thresholds picks an 8-record window (one round trip); a probe that does not
// halve the interval makes the next probe a bisection.
__device__ __forceinline__ uint64_t lt_pick(const uint2 *edges, uint64_t a, uint64_t b, uint32_t c, uint32_t &u) {
    uint64_t lo = a, hi = b;             // answer in [lo, hi]
    uint64_t tlo = 0, thi = 1ull << 32;  // threshold of record lo-1 (0 at a); of record hi (2^32 past the end)
    uint32_t hi_src = 0;
    bool bisect = false;
    while (hi - lo > 8) {
        const uint64_t len = hi - lo;
        const uint64_t span = thi - tlo;
        // both ends still open (the first probe): the division by 2^32 is a shift
        const uint64_t g = bisect                  ? lo + len / 2
                           : span == (1ull << 32) ? lo + ((static_cast<uint64_t>(c) * len) >> 32)
                                                  : lo + (static_cast<uint64_t>(c) - tlo) * len / span;
        uint64_t ws = (g >= lo + 3) ? g - 3 : lo;
        if (ws + 8 > hi) ws = hi - 8;
        uint2 r[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = edges[ws + i];
        if (r[0].y > c) {
            hi = ws;
            thi = r[0].y;
            hi_src = r[0].x;
        } else if (r[7].y <= c) {
            lo = ws + 8;
            tlo = r[7].y;
        } else {
            uint64_t pick = ws + 7;
            uint32_t pu = r[7].x;
#pragma unroll
            for (int i = 6; i >= 1; --i) {
                if (r[i].y > c) {
                    pick = ws + i;
                    pu = r[i].x;
                }
            }
            u = pu;
            return pick;
        }
        bisect = (hi - lo) * 2 > len;
    }
    uint64_t pick = hi;
    uint32_t pu = hi_src;
    if (b >= 8) {
        // one window of eight records that covers [lo, hi), all loads in
        // flight at once (records outside [lo, hi) belong to neighbours and
        // are skipped)
        const uint64_t ws = lo < b - 8 ? lo : b - 8;
        uint2 r[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = edges[ws + i];
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            const uint64_t e = ws + i;
            if (e >= lo && e < hi && r[i].y > c) {
                pick = e;
                pu = r[i].x;
            }
        }
    } else {  // fewer than eight records before b in the whole edge array
        uint2 r[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint64_t e = lo + i;
            r[i] = (e < hi) ? edges[e] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int i = 7; i >= 0; --i) {
            if (r[i].y > c) {
                pick = lo + i;
                pu = r[i].x;
            }
        }
    }
    if (pick == b) return b;
    u = pu;
    return pick;
}

template <int kMode>
__global__ __launch_bounds__(kWave) void lt_main_kernel(Params p, uint64_t *tables, uint32_t stamp_base) {
    const uint32_t lane = lane_id();
    uint64_t *table = tables + (static_cast<uint64_t>(blockIdx.x) * kWave + lane) * kLtTableSlots;
    Stream st(0);
    const uint32_t *seedbits = nullptr;
    ItemAcc ia;        // per lane
    uint32_t cur = 0;  // per-lane item cache

    bool active = false, finished = false;
    uint32_t t = 0, v = 0, len = 0, stamp = 0;
    uint32_t cv = 0;  // LT coin of v, computed while v's offsets load
    uint64_t s = 0, a = 0, b = 0;
    uint32_t *region = nullptr;
    uint64_t edges_acc = 0, nodes_acc = 0;
    const uint32_t max_walk = min(kLtMaxWalk, p.lt_cap);

    for (;;) {
        const bool need = !active && !finished;
        const uint64_t mask = __ballot(need);
        if (mask) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&p.cnt->ticket, static_cast<uint32_t>(__popcll(mask)));
            base = __shfl(base, 0, kWave);
            if (need) {
                const uint32_t mine = base + lanes_below(mask);
                if (mine < p.count) {
                    t = mine;
                    const WorkItem &it = item_cached(p, t, cur);
                    st = Stream(it.key);
                    seedbits = it.seedbits;
                    ia.move_to(it.acc, true);
                    s = it.s0 + (t - it.start);
                    stamp = stamp_base + t;
                    v = pick_source(st, s, p.src_cum, p.n);
                    region = p.stage + static_cast<uint64_t>(t) * p.lt_cap;
                    region[0] = v;
                    len = 1;
                    // every entry is stale for a new stamp: the first slot is free
                    table[lt_bucket(v) * kLtBucketSlots] = lt_entry(stamp, v);
                    a = p.off[v];
                    b = p.off[v + 1];
                    cv = lt_coin(st, s, v);
                    active = true;
                    if (kMode == 1 && test_bit(seedbits, v)) {
                        p.z[t] = 1;
                        edges_acc += 1;
                        ia.edges += 1;
                        active = false;
                    }
                } else {
                    finished = true;
                }
            }
        }
        // every lane without a sample just tried to take one: done when
        // all lanes found the batch exhausted
        if (__ballot(!finished) == 0) break;
        if (!active) continue;

        bool stop = (a == b);
        uint32_t u = 0;
        uint64_t na = 0, nb = 0;
        if (!stop && lt_pick(p.edges, a, b, cv, u) == b) stop = true;
        if (!stop) {
            na = p.off[u];
            nb = p.off[u + 1];
            const uint64_t want = lt_entry(stamp, u);
            uint32_t bi = lt_bucket(u);
            const ulonglong2 *bucket = reinterpret_cast<const ulonglong2 *>(table + bi * kLtBucketSlots);
            ulonglong2 q0 = bucket[0], q1 = bucket[1], q2 = bucket[2], q3 = bucket[3];
            cv = lt_coin(st, s, u);  // the next step's coin, while the loads above are in flight
            asm volatile("" : "+v"(cv));  // keeps it here rather than after the probe
            for (uint32_t probe = 0; probe < kLtBuckets; ++probe) {
                if (probe) {
                    bucket = reinterpret_cast<const ulonglong2 *>(table + bi * kLtBucketSlots);
                    q0 = bucket[0];
                    q1 = bucket[1];
                    q2 = bucket[2];
                    q3 = bucket[3];
                }
                const uint64_t ent[8] = {q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
                int free_slot = -1;
                bool found = false;
#pragma unroll
                for (int i = 7; i >= 0; --i) {
                    if (ent[i] == want) found = true;
                    if (static_cast<uint32_t>(ent[i] >> 32) != stamp) free_slot = i;
                }
                if (found) {
                    stop = true;  // the walk closed a cycle
                    break;
                }
                if (free_slot >= 0) {
                    table[bi * kLtBucketSlots + free_slot] = want;
                    break;
                }
                bi = (bi + 1) & (kLtBuckets - 1);
            }
        }
        if (stop) {
            if (kMode == 1) {
                p.z[t] = 0;
            } else {
                p.sizes[t] = len;
                p.stage_off[t] = static_cast<uint64_t>(t) * p.lt_cap;
                nodes_acc += len;
                ia.nodes += len;
            }
            ia.edges += len;
            edges_acc += len;
            active = false;
            continue;
        }
        if (len == max_walk) {  // longer than the staging region / table budget: long path
            const uint32_t d = atomicAdd(&p.cnt->defer_count, 1u);
            p.defer_list[d] = t;
            active = false;
            continue;
        }
        region[len++] = u;
        v = u;
        a = na;
        b = nb;
        if (kMode == 1 && test_bit(seedbits, u)) {
            p.z[t] = 1;
            edges_acc += len;
            ia.edges += len;
            active = false;
        }
    }
    flush_lanes(ia);
    const uint64_t e_sum = wave_sum_u64(edges_acc);
    const uint64_t n_sum = wave_sum_u64(nodes_acc);
    if (lane == 0) {
        if (e_sum) atomicAdd(&p.cnt->edges, static_cast<unsigned long long>(e_sum));
        if (n_sum) atomicAdd(&p.cnt->total_nodes, static_cast<unsigned long long>(n_sum));
    }
}

// ------------------------------------------------------- IC workgroup ----

// LDS open-addressed set of node ids (key u + 1) for one workgroup.
template <uint32_t kHbits>
__device__ __forceinline__ bool grp_insert(uint32_t *vis, uint32_t u, bool &full) {
    constexpr uint32_t kHcap = 1u << kHbits;
    const uint32_t key = u + 1u;
    uint32_t h = (u * 2654435761u) >> (32 - kHbits);
    for (uint32_t probe = 0; probe < kHcap; ++probe) {
        const uint32_t old = atomicCAS(&vis[h], 0u, key);
        if (old == 0u) return true;
        if (old == key) return false;
        h = (h + 1u) & (kHcap - 1u);
    }
    full = true;
    return false;
}

// grp_insert in two steps (as vis_probe / vis_settle): the first attempt,
// then the decision from its old word, probing on past another node.
template <uint32_t kHbits>
__device__ __forceinline__ uint32_t grp_probe(uint32_t *vis, uint32_t u) {
    return atomicCAS(&vis[(u * 2654435761u) >> (32 - kHbits)], 0u, u + 1u);
}

template <uint32_t kHbits>
__device__ __forceinline__ bool grp_settle(uint32_t *vis, uint32_t u, uint32_t old, bool &full) {
    constexpr uint32_t kHcap = 1u << kHbits;
    const uint32_t key = u + 1u;
    if (old == 0u) return true;
    if (old == key) return false;
    uint32_t h = (u * 2654435761u) >> (32 - kHbits);
    for (uint32_t probe = 1; probe < kHcap; ++probe) {
        h = (h + 1u) & (kHcap - 1u);
        const uint32_t o = atomicCAS(&vis[h], 0u, key);
        if (o == 0u) return true;
        if (o == key) return false;
    }
    full = true;
    return false;
}

// IC samples handed on by the previous tier, one workgroup per sample: each
// level's frontier (up to kThreads nodes at a time) is laid out by a block
// scan of its aligned 4-edge groups, which all threads then expand. A sample
// with a hand-over record (in_rec, in_stride words each, the first in_cap of
// the list) resumes from it. Samples too large for this tier's LDS go on to
// the next tier's list, with a record of their own when out_cap allows.
template <int kMode, typename Tier>
__global__ __launch_bounds__(Tier::kThreads) void ic_group_kernel(Params p, const uint32_t *in_list,
                                                                  const uint32_t *in_count, uint32_t *in_ticket,
                                                                  uint32_t *out_list, uint32_t *out_count,
                                                                  const uint32_t *in_rec, uint32_t in_stride,
                                                                  uint32_t in_cap, uint32_t *out_rec,
                                                                  uint32_t out_stride, uint32_t out_cap) {
    constexpr int kGrpThreads = Tier::kThreads;
    constexpr uint32_t kGrpQcap = Tier::kQcap;
    constexpr uint32_t kGrpHbits = Tier::kHbits;
    constexpr uint32_t kGrpHcap = 1u << kGrpHbits;
    __shared__ uint32_t s_queue[kGrpQcap];
    __shared__ uint32_t s_vis[kGrpHcap];
    __shared__ uint64_t s_pre[kGrpThreads];
    __shared__ uint64_t s_a[kGrpThreads];
    __shared__ uint2 s_b[kGrpThreads];  // {in-degree, thr}
    __shared__ uint64_t s_scan[kGrpThreads / kWave];
    __shared__ unsigned long long s_edges;
    __shared__ uint32_t s_t, s_d, s_tail, s_flags;  // flags: 1 hit, 2 too large
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < kGrpHcap; i += blockDim.x) s_vis[i] = 0u;
    __syncthreads();
    for (;;) {
        if (tid == 0) {
            const uint32_t d = atomicAdd(in_ticket, 1u);
            s_t = d < *in_count ? in_list[d] : 0xFFFFFFFFu;
            s_d = d;
        }
        __syncthreads();
        const uint32_t t = s_t;
        if (t == 0xFFFFFFFFu) break;
        const uint32_t d = s_d;
        const WorkItem &it = item_of(p, t);
        const Stream st(it.key);
        const uint32_t *seedbits = it.seedbits;
        const uint64_t s = it.s0 + (t - it.start);
        uint32_t head = 0, levels = 0;
        // the sender's record, when it left one for this sample (its
        // queue holds no seed: a hit would have ended the sample there)
        const uint32_t *rec = (d < in_cap) ? in_rec + static_cast<uint64_t>(d) * in_stride : nullptr;
        const bool resume = rec != nullptr && rec[0] == t && rec[2] <= kGrpQcap && rec[1] < rec[2];
        if (resume) {
            const uint32_t rt = rec[2];
            head = rec[1];
            for (uint32_t i = tid; i < rt; i += blockDim.x) s_queue[i] = rec[kHoHdr + i];
            if (tid == 0) {
                s_tail = rt;
                s_flags = 0u;
                s_edges = static_cast<unsigned long long>(rec[3]) | (static_cast<unsigned long long>(rec[4]) << 32);
            }
            __syncthreads();
            bool full = false;  // cannot fill: the set is at least twice the largest record
            for (uint32_t i = tid; i < rt; i += blockDim.x) grp_insert<kGrpHbits>(s_vis, s_queue[i], full);
        } else if (tid == 0) {
            const uint32_t v0 = pick_source(st, s, p.src_cum, p.n);
            bool full = false;
            grp_insert<kGrpHbits>(s_vis, v0, full);
            s_queue[0] = v0;
            s_tail = 1;
            s_flags = (kMode == 1 && test_bit(seedbits, v0)) ? 1u : 0u;
            s_edges = 0;
        }
        __syncthreads();
        // the state at the start of the current frontier batch (what a
        // hand-over record carries)
        uint32_t hb = head, tb = 0;
        uint64_t eb = 0;
        for (;;) {
            const uint32_t tail = s_tail;
            if (head >= tail || s_flags != 0u) break;
            hb = head;
            tb = tail;
            eb = s_edges;  // this batch's edges are added after the scan's barriers
            ++levels;
            const uint32_t nb = min(tail - head, static_cast<uint32_t>(kGrpThreads));
            uint64_t a = 0, cg = 0;
            uint32_t deg = 0, thr = 0;
            if (tid < nb) {
                ic_node(p, s_queue[head + tid], a, deg, thr);
                if (deg) cg = ((a + deg - 1) >> 2) - (a >> 2) + 1;
            }
            const uint64_t de = deg;
            uint64_t groups = 0;
            const uint64_t pre = block_scan_excl(cg, s_scan, groups);
            // after the scan's barriers: every thread has read s_edges above
            if (de) atomicAdd(&s_edges, static_cast<unsigned long long>(de));
            s_pre[tid] = pre;
            s_a[tid] = a;
            s_b[tid] = make_uint2(deg, thr);
            __syncthreads();
            head += nb;
            for (uint64_t w = tid; w < groups; w += blockDim.x) {
                // owner: last frontier slot whose first group index <= w
                uint32_t lo = 0, hi = nb - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= w) lo = mid;
                    else hi = mid - 1;
                }
                const uint64_t ea = s_a[lo];
                const uint2 db = s_b[lo];
                const uint64_t eb = ea + db.x;
                const uint64_t g = (ea >> 2) + (w - s_pre[lo]);
                const uint4 coins = ic_coins(st, s, g);
                bool full = false;
                uint2 rec[4];
                bool live[4];
                ic_group_read(p, g, ea, eb, db.y, coins, rec, live);
                uint32_t old[4];
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q) old[q] = live[q] ? grp_probe<kGrpHbits>(s_vis, rec[q].x) : 0u;
                uint32_t fresh = 0;  // bit q: record q reached a new node
#pragma unroll
                for (uint32_t q = 0; q < 4; ++q)
                    if (live[q] && grp_settle<kGrpHbits>(s_vis, rec[q].x, old[q], full)) fresh |= 1u << q;
                if (fresh) {  // one queue reservation for the thread's new nodes
                    uint32_t pos = atomicAdd(&s_tail, static_cast<uint32_t>(__popc(fresh)));
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        if (fresh & (1u << q)) {
                            if (pos < kGrpQcap) s_queue[pos] = rec[q].x;
                            else atomicOr(&s_flags, 2u);
                            if (kMode == 1 && test_bit(seedbits, rec[q].x)) atomicOr(&s_flags, 1u);
                            ++pos;
                        }
                    }
                }
                if (full) atomicOr(&s_flags, 2u);
            }
            __syncthreads();
        }
        const uint32_t flags = s_flags;
        const uint32_t tail = min(s_tail, kGrpQcap);
        const uint64_t sample_edges = s_edges;
        if (tid == 0 && !((flags & 2u) && !(flags & 1u))) {
            atomicAdd(&p.cnt->grp_samples, 1ull);
            atomicAdd(&p.cnt->grp_edges, static_cast<unsigned long long>(sample_edges));
            atomicAdd(&p.cnt->grp_levels, static_cast<unsigned long long>(levels));
        }
        if ((flags & 2u) && !(flags & 1u)) {
            if (tid == 0) {
                const uint32_t d2 = atomicAdd(out_count, 1u);
                out_list[d2] = t;
                s_d = d2;
            }
            __syncthreads();
            const uint32_t d2 = s_d;
            if (d2 < out_cap) {  // s_queue[0, tb) is untouched by the unfinished batch
                uint32_t *orec = out_rec + static_cast<uint64_t>(d2) * out_stride;
                for (uint32_t i = tid; i < tb; i += blockDim.x) orec[kHoHdr + i] = s_queue[i];
                if (tid == 0) {
                    orec[0] = t;
                    orec[1] = hb;
                    orec[2] = tb;
                    orec[3] = static_cast<uint32_t>(eb);
                    orec[4] = static_cast<uint32_t>(eb >> 32);
                }
            }
        } else if (kMode == 1) {
            if (tid == 0) {
                p.z[t] = (flags & 1u) ? 1 : 0;
                atomicAdd(&it.acc[1], static_cast<unsigned long long>(sample_edges));
                atomicAdd(&p.cnt->edges, static_cast<unsigned long long>(sample_edges));
            }
        } else {
            __shared__ unsigned long long s_base;
            if (tid == 0) {
                const unsigned long long base = atomicAdd(&p.cnt->stage_cursor, static_cast<unsigned long long>(tail));
                s_base = base;
                const bool fits = base + tail <= p.stage_cap;
                if (!fits) atomicOr(&p.cnt->overflow, 1u);
                p.sizes[t] = fits ? tail : 0;
                p.stage_off[t] = fits ? base : 0;
                atomicAdd(&it.acc[0], static_cast<unsigned long long>(tail));
                atomicAdd(&it.acc[1], static_cast<unsigned long long>(sample_edges));
                atomicAdd(&p.cnt->edges, static_cast<unsigned long long>(sample_edges));
                atomicAdd(&p.cnt->total_nodes, static_cast<unsigned long long>(tail));
            }
            __syncthreads();
            const unsigned long long base = s_base;
            if (base + tail <= p.stage_cap)
                for (uint32_t i = tid; i < tail; i += blockDim.x) p.stage[base + i] = s_queue[i];
        }
        __syncthreads();
        // clear the visited set: entry by entry unless it may be incomplete
        if (flags != 0u) {
            for (uint32_t i = tid; i < kGrpHcap; i += blockDim.x) s_vis[i] = 0u;
        } else {
            for (uint32_t i = tid; i < tail; i += blockDim.x) {
                const uint32_t u = s_queue[i], key = u + 1u;
                uint32_t h = (u * 2654435761u) >> (32 - kGrpHbits);
                for (uint32_t probe = 0; probe < kGrpHcap; ++probe) {
                    if (s_vis[h] == key) {
                        s_vis[h] = 0u;
                        break;
                    }
                    h = (h + 1u) & (kGrpHcap - 1u);
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------- long path ----

// One wave per slot; each slot owns vis[n] (epoch stamps) and queue[n].
template <int kModel, int kMode>
__global__ __launch_bounds__(kLongWaves *kWave) void long_kernel(Params p, uint32_t *slot_mem, uint64_t n_stride,
                                                                 uint32_t nslots, uint32_t *slot_epoch) {
    __shared__ uint32_t s_pre[kLongWaves][kWave];
    __shared__ uint64_t s_a[kLongWaves][kWave];
    __shared__ uint64_t s_b[kLongWaves][kWave];
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    const uint32_t slot = blockIdx.x * kLongWaves + wave;
    if (slot >= nslots) return;
    uint32_t *vis = slot_mem + static_cast<uint64_t>(slot) * 2 * n_stride;
    uint32_t *queue = vis + n_stride;
    uint32_t *pre = s_pre[wave];
    uint64_t *fa = s_a[wave];
    uint64_t *fb = s_b[wave];
    uint64_t edges_acc = 0, nodes_acc = 0;

    // LT samples come straight from the main pass, IC ones from the
    // workgroup tier
    const uint32_t *list = (kModel == IM_IC) ? p.long_list : p.defer_list;
    uint32_t *ticket = (kModel == IM_IC) ? &p.cnt->long_ticket : &p.cnt->defer_ticket;
    const uint32_t *count = (kModel == IM_IC) ? &p.cnt->long_count : &p.cnt->defer_count;
    for (;;) {
        uint32_t d = 0;
        if (lane == 0) d = atomicAdd(ticket, 1u);
        d = __shfl(d, 0, kWave);
        if (d >= *count) break;
        const uint32_t t = list[d];
        const WorkItem &it = item_of(p, t);
        const Stream st(it.key);
        const uint32_t *seedbits = it.seedbits;
        const uint64_t s = it.s0 + (t - it.start);
        uint32_t stamp = 0;
        if (lane == 0) stamp = ++slot_epoch[slot];
        stamp = __shfl(stamp, 0, kWave);
        const uint32_t v0 = pick_source(st, s, p.src_cum, p.n);
        bool hit = (kMode == 1) && test_bit(seedbits, v0);
        uint32_t tail = 1;
        uint64_t sample_edges = 0;
        if (lane == 0) {
            queue[0] = v0;
            vis[v0] = stamp;
        }
        wave_sync();
        if (kModel == IM_LT) {
            // the main pass walked this sample's first max_walk nodes into
            // its staging region before handing it on; a walk's coins depend
            // on the node, not the step, so the walk goes on from the last of
            // them once they are all marked (on lane 0; the others wait)
            const uint32_t walked = min(kLtMaxWalk, p.lt_cap);
            const uint32_t *region = p.stage + static_cast<uint64_t>(t) * p.lt_cap;
            for (uint32_t i = lane; i < walked; i += kWave) {
                const uint32_t u = region[i];
                queue[i] = u;
                vis[u] = stamp;
            }
            __threadfence_block();
            wave_sync();
            tail = walked;
            sample_edges = walked - 1;  // the lists of all but the last were examined
            if (lane == 0 && !hit) {
                uint32_t v = queue[walked - 1];
                for (;;) {
                    sample_edges += 1;
                    const uint64_t a = p.off[v], b = p.off[v + 1];
                    if (a == b) break;
                    uint32_t u = 0;
                    if (lt_pick(p.edges, a, b, lt_coin(st, s, v), u) == b) break;
                    if (vis[u] == stamp) break;
                    vis[u] = stamp;
                    queue[tail++] = u;
                    v = u;
                    if (kMode == 1 && test_bit(seedbits, u)) {
                        hit = true;
                        break;
                    }
                }
            }
            tail = __shfl(tail, 0, kWave);
            hit = __shfl(static_cast<int>(hit), 0, kWave) != 0;
            sample_edges = __shfl(sample_edges, 0, kWave);
        } else {
            uint32_t head = 0;
            while (head < tail && !hit) {
                const uint32_t nb = min(tail - head, static_cast<uint32_t>(kWave));
                uint32_t cg = 0;
                uint64_t a = 0, b = 0;
                if (lane < nb) {
                    const uint32_t v = queue[head + lane];
                    a = p.off[v];
                    b = p.off[v + 1];
                    if (b > a) cg = static_cast<uint32_t>(((b - 1) >> 2) - (a >> 2) + 1);
                }
                const uint32_t inc = wave_inclusive_scan(cg);
                const uint32_t groups = __shfl(inc, kWave - 1, kWave);
                sample_edges += wave_sum_u64(b - a);
                pre[lane] = inc - cg;
                fa[lane] = a;
                fb[lane] = b;
                head += nb;
                wave_sync();
                for (uint32_t base = 0; base < groups; base += kWave) {
                    const uint32_t w = base + lane;
                    uint32_t f[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
                    if (w < groups) {
                        uint32_t lo = 0, hi = nb - 1;
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi + 1) >> 1;
                            if (pre[mid] <= w) lo = mid;
                            else hi = mid - 1;
                        }
                        const uint64_t ea = fa[lo], eb = fb[lo];
                        const uint64_t g = (ea >> 2) + (w - pre[lo]);
                        const uint4 coins = ic_coins(st, s, g);
                        uint2 rec[4];
                        bool live[4];
                        ic_group_live(p.edges, g, ea, eb, coins, rec, live);
#pragma unroll
                        for (uint32_t q = 0; q < 4; ++q) {
                            if (live[q] && atomicExch(&vis[rec[q].x], stamp) != stamp) f[q] = rec[q].x;
                        }
                    }
#pragma unroll
                    for (uint32_t q = 0; q < 4; ++q) {
                        const bool has = f[q] != 0xFFFFFFFFu;
                        const uint64_t mask = __ballot(has);
                        if (mask) {
                            if (has) {
                                queue[tail + lanes_below(mask)] = f[q];
                                if (kMode == 1 && test_bit(seedbits, f[q])) hit = true;
                            }
                            tail += static_cast<uint32_t>(__popcll(mask));
                        }
                    }
                    if (kMode == 1) hit = __ballot(hit) != 0;
                    if (hit) break;
                }
                __threadfence_block();
                wave_sync();
            }
        }
        if (kMode == 1) {
            if (lane == 0) {
                p.z[t] = hit ? 1 : 0;
                atomicAdd(&it.acc[1], static_cast<unsigned long long>(sample_edges));
            }
            edges_acc += sample_edges;
        } else {
            unsigned long long base = 0;
            if (lane == 0) {
                atomicAdd(&it.acc[0], static_cast<unsigned long long>(tail));
                atomicAdd(&it.acc[1], static_cast<unsigned long long>(sample_edges));
                base = atomicAdd(&p.cnt->stage_cursor, static_cast<unsigned long long>(tail));
                if (base + tail > p.stage_cap) {
                    atomicOr(&p.cnt->overflow, 1u);
                    p.sizes[t] = 0;
                    p.stage_off[t] = 0;
                } else {
                    p.sizes[t] = tail;
                    p.stage_off[t] = base;
                }
            }
            base = __shfl(base, 0, kWave);
            __threadfence_block();
            wave_sync();
            if (base + tail <= p.stage_cap)
                for (uint32_t i = lane; i < tail; i += kWave) p.stage[base + i] = queue[i];
            edges_acc += sample_edges;
            nodes_acc += tail;
        }
        wave_sync();
    }
    if (lane == 0) {
        if (edges_acc) atomicAdd(&p.cnt->edges_long, static_cast<unsigned long long>(edges_acc));
        if (nodes_acc) atomicAdd(&p.cnt->nodes_long, static_cast<unsigned long long>(nodes_acc));
    }
}

// ---------------------------------------------------------- pool append ----

constexpr int kScanThreads = 256;
constexpr int kScanTile = 1024;  // 4 items per thread

__device__ __forceinline__ uint64_t block_exclusive_scan_u64(uint64_t x, uint64_t *smem, uint64_t &total) {
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d, kWave);
        if (lane >= static_cast<uint32_t>(d)) inc += y;
    }
    if (lane == kWave - 1) smem[wave] = inc;
    __syncthreads();
    uint64_t wave_off = 0, tot = 0;
    const uint32_t nw = blockDim.x / kWave;
    for (uint32_t w = 0; w < nw; ++w) {
        if (w < wave) wave_off += smem[w];
        tot += smem[w];
    }
    __syncthreads();
    total = tot;
    return wave_off + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(const uint32_t *in, uint64_t count, uint64_t *tile_sum) {
    __shared__ uint64_t smem[kScanThreads / kWave];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 4;
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (base + i < count) x += in[base + i];
    uint64_t total = 0;
    block_exclusive_scan_u64(x, smem, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One block: exclusive scan of tile sums in place (any length).
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint64_t *tile_sum, uint64_t tiles) {
    __shared__ uint64_t smem[1024 / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < tiles; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t x = i < tiles ? tile_sum[i] : 0;
        uint64_t total = 0;
        const uint64_t ex = block_exclusive_scan_u64(x, smem, total);
        if (i < tiles) tile_sum[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
}

// out[i+1] = base + sum(in[0..i]) ; out[0] written by the caller's layout.
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t *in, uint64_t count,
                                                                   const uint64_t *tile_off, uint64_t base,
                                                                   uint64_t *out) {
    __shared__ uint64_t smem[kScanThreads / kWave];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kScanTile + threadIdx.x * 4;
    uint64_t v[4];
    uint64_t x = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = (b0 + i < count) ? in[b0 + i] : 0;
        x += v[i];
    }
    uint64_t total = 0;
    uint64_t run = base + tile_off[blockIdx.x] + block_exclusive_scan_u64(x, smem, total);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        run += v[i];
        if (b0 + i < count) out[b0 + i + 1] = run;
    }
}

__global__ void set_first_kernel(uint64_t *out, uint64_t value) { out[0] = value; }

__global__ void zero_u64_kernel(uint64_t *p, uint64_t count) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

__global__ void copy_u64_kernel(const uint64_t *src, uint64_t *dst, uint64_t count) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

__global__ void copy_u32_kernel(const uint32_t *src, uint32_t *dst, uint64_t count) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

// Destination of one work item's sets in its pool.
struct AppendDst {
    uint64_t *poff;    // the pool's offsets at its current count (poff[0] = its total)
    uint32_t *pnodes;  // the pool's node array
    uint64_t base;     // the pool's total before the append
    uint32_t start;    // the item's first slot in the batch
};

// 16 lanes per slot: write the slot's pool offset and copy its set.
__global__ __launch_bounds__(256) void compact_items_kernel(const uint32_t *stage, const uint64_t *stage_off,
                                                            const uint64_t *prefix, const AppendDst *dst,
                                                            uint32_t nitems, uint64_t count) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t group = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t t = group; t < count; t += groups) {
        uint32_t lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (dst[mid].start <= t) lo = mid;
            else hi = mid - 1;
        }
        const AppendDst d = dst[lo];
        const uint64_t rel = prefix[t] - prefix[d.start];
        const uint64_t len = prefix[t + 1] - prefix[t];
        if (sub == 0) d.poff[t - d.start + 1] = d.base + rel + len;
        const uint32_t *src = stage + stage_off[t];
        uint32_t *out = d.pnodes + d.base + rel;
        for (uint64_t j = sub; j < len; j += 16) out[j] = src[j];
    }
}

uint32_t blocks_for(uint64_t items, uint32_t per_block, uint32_t cap) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<uint32_t>(b);
}

// Per-sample metadata layout inside ctx->sample_meta for `count` samples.
struct Meta {
    uint64_t *stage_off;
    uint32_t *sizes;
    uint32_t *defer_list;
    uint32_t *large_list;
    uint32_t *long_list;
    uint8_t *z;
};

size_t meta_bytes(uint64_t count) { return count * (8 + 4 + 4 + 4 + 4 + 1) + 256; }

Meta meta_view(im_ctx *ctx, uint64_t count) {
    Meta m;
    char *base = static_cast<char *>(ctx->sample_meta.ptr);
    m.stage_off = reinterpret_cast<uint64_t *>(base);
    m.sizes = reinterpret_cast<uint32_t *>(base + count * 8);
    m.defer_list = reinterpret_cast<uint32_t *>(base + count * 12);
    m.large_list = reinterpret_cast<uint32_t *>(base + count * 16);
    m.long_list = reinterpret_cast<uint32_t *>(base + count * 20);
    m.z = reinterpret_cast<uint8_t *>(base + count * 24);
    return m;
}

}  // namespace

namespace im {

// Long-path slot arrays for a graph of n nodes: each slot holds vis[n]
// (epoch stamps, zeroed once) and queue[n].
static im_status ensure_slots(im_ctx *ctx, uint32_t n) {
    const uint64_t per_slot = 2ull * n * 4;
    const uint64_t budget = std::min<uint64_t>(ctx->slot_budget, ctx->total_mem / 16);
    uint64_t want = std::max<uint64_t>(1, std::min<uint64_t>(1024, budget / std::max<uint64_t>(per_slot, 1)));
    if (ctx->slots.ptr && ctx->slot_n == n && ctx->slot_count == want && ctx->slot_epoch < 0xF0000000ull)
        return IM_OK;
    dev_free(ctx, ctx->slots);
    IM_TRY(dev_alloc(ctx, ctx->slots, want * per_slot + want * 4 + 256));
    IM_HIP(hipMemsetAsync(ctx->slots.ptr, 0, want * per_slot + want * 4 + 256, ctx->stream));
    ctx->slot_n = n;
    ctx->slot_count = static_cast<uint32_t>(want);
    ctx->slot_epoch = 0;
    return IM_OK;
}

im_status sample_items(im_ctx *ctx, const im_graph *g, im_model model, const SampleItem *items, uint32_t nitems,
                       SampleMode mode, double size_hint, SampleResult *res, ItemTotals *per_item) {
    *res = SampleResult{};
    uint64_t count = 0;
    for (uint32_t i = 0; i < nitems; ++i) count += items[i].count;
    if (count == 0 || nitems == 0) {
        for (uint32_t i = 0; i < nitems; ++i) per_item[i] = ItemTotals{};
        return IM_OK;
    }
    if (count > 0xFFFFFFF0ull) {
        set_error("sample batch of %llu samples is too large", static_cast<unsigned long long>(count));
        return IM_E_ARG;
    }
    const DevBuf &edges = (model == IM_IC) ? g->edges_ic : g->edges_lt;
    hipStream_t st = ctx->stream;
    IM_TRY(dev_reserve(ctx, ctx->sample_meta, meta_bytes(count)));
    IM_TRY(dev_reserve(ctx, ctx->counters, 256));
    IM_TRY(dev_reserve(ctx, ctx->items, size_t(nitems) * (sizeof(WorkItem) + 16) + 256));
    if (mode == SampleMode::Hits) IM_TRY(dev_reserve(ctx, ctx->zflags, count + 64));
    IM_TRY(ensure_slots(ctx, g->n));
    if (model == IM_LT && !ctx->lt_tables.ptr) {
        const uint32_t lanes = static_cast<uint32_t>(ctx->cu_count) * 16 * kWave;
        const uint64_t words = uint64_t(lanes) * kLtTableSlots;
        IM_TRY(dev_alloc(ctx, ctx->lt_tables, words * 8));
        zero_u64_kernel<<<blocks_for(words, 256, ctx->cu_count * 16), 256, 0, st>>>(
            static_cast<uint64_t *>(ctx->lt_tables.ptr), words);
        ctx->lt_lanes = lanes;
        ctx->lt_stamp = 1;
    }
    Meta meta = meta_view(ctx, count);
    // hand-over records between the IC tiers (plain launches have no tiers)
    uint32_t ho_wave_cap = 0, ho_small_cap = 0;
    if (model == IM_IC && !ctx->ic_plain) {
        ho_wave_cap = static_cast<uint32_t>(std::min<uint64_t>(count, kHoMaxWave));
        ho_small_cap = static_cast<uint32_t>(std::min<uint64_t>(count, kHoMaxSmall));
        IM_TRY(dev_reserve(ctx, ctx->handoff,
                           (uint64_t(ho_wave_cap) * kHoStrideWave + uint64_t(ho_small_cap) * kHoStrideSmall) * 4 + 256));
    }
    auto *cnt = static_cast<Counters *>(ctx->counters.ptr);
    // device work queue: items, then their accumulators
    auto *ditems = static_cast<WorkItem *>(ctx->items.ptr);
    auto *dacc = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->items.ptr) +
                                                        ((size_t(nitems) * sizeof(WorkItem) + 255) & ~size_t(255)));
    std::vector<WorkItem> hitems(nitems);
    uint32_t start = 0;
    for (uint32_t i = 0; i < nitems; ++i) {
        hitems[i] = WorkItem{items[i].key, items[i].s0, start, static_cast<uint32_t>(items[i].count),
                             items[i].seedbits, dacc + 2ull * i};
        start += static_cast<uint32_t>(items[i].count);
    }
    IM_HIP(hipMemcpyAsync(ditems, hitems.data(), sizeof(WorkItem) * nitems, hipMemcpyHostToDevice, st));

    // staging capacity: LT reserves a region per sample, then a bump area
    // for long walks; IC bump-allocates every set.
    // expected set size: the caller's, else this graph's last draws of the
    // model, else a guess (a guess too small costs a re-run of the batch)
    const double seen = g->mean_set[model == IM_IC ? 0 : 1].load(std::memory_order_relaxed);
    const double hint = size_hint > 0 ? size_hint : seen > 0 ? seen : (model == IM_IC ? 16.0 : 64.0);
    uint64_t lt_regions = (model == IM_LT) ? count * kLtCap : 0;
    // IC waves reserve staging in chunks of kStageChunk: allow one partly
    // used chunk per wave on top of the expected sizes
    const uint64_t chunk_slack = (model == IM_IC) ? uint64_t(ctx->cu_count) * 8 * kIcWaves * kStageChunk : 0;
    uint64_t cap = lt_regions + static_cast<uint64_t>(std::ceil(hint * 1.5 * count)) + (1u << 20) + chunk_slack;
    if (mode == SampleMode::Hits && model == IM_IC) cap = 0;

    for (int attempt = 0; attempt < 8; ++attempt) {
        if (cap) {
            IM_TRY(dev_reserve(ctx, ctx->stage, cap * 4));
            cap = ctx->stage.bytes / 4;  // all of it: a buffer kept from a larger batch holds more
        }
        Params p{};
        p.off = static_cast<const uint64_t *>(g->off.ptr);
        p.edges = static_cast<const uint2 *>(edges.ptr);
        p.src_cum = static_cast<const uint64_t *>(g->src_cum.ptr);
        p.n = g->n;
        p.count = static_cast<uint32_t>(count);
        p.items = ditems;
        p.nitems = nitems;
        p.cnt = cnt;
        p.defer_list = meta.defer_list;
        p.large_list = meta.large_list;
        p.long_list = meta.long_list;
        p.stage = static_cast<uint32_t *>(ctx->stage.ptr);
        p.stage_cap = cap;
        p.stage_off = meta.stage_off;
        p.sizes = meta.sizes;
        p.z = (mode == SampleMode::Hits) ? static_cast<uint8_t *>(ctx->zflags.ptr) : meta.z;
        p.lt_cap = kLtCap;
        p.ticket_block = 1;
        p.edge_budget = ctx->ic_edge_budget;
        // plain IC launches: static assignment, no workgroup tiers (a sample
        // leaves the wave pass only when it outgrows the wave's LDS)
        const bool plain = model == IM_IC && ctx->ic_plain;
        p.plain = plain ? 1u : 0u;
        if (plain) p.edge_budget = 0xFFFFFFFFu;
        p.ho_wave = ho_wave_cap ? static_cast<uint32_t *>(ctx->handoff.ptr) : nullptr;
        p.ho_small = ho_small_cap ? p.ho_wave + uint64_t(ho_wave_cap) * kHoStrideWave : nullptr;
        p.ho_wave_cap = ho_wave_cap;
        if (model == IM_IC && ctx->ic_compact && g->nodes_ic.ptr) {
            p.nodes = static_cast<const uint4 *>(g->nodes_ic.ptr);
            p.srcs = static_cast<const uint32_t *>(g->srcs_ic.ptr);
        }
        p.ho_small_cap = ho_small_cap;

        init_counters_kernel<<<1, 1, 0, st>>>(cnt, lt_regions);
        zero_u64_kernel<<<1, 256, 0, st>>>(reinterpret_cast<uint64_t *>(dacc), 2ull * nitems);
        const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
        if (ctx->timing) IM_HIP(hipEventRecord(ctx->ev_begin, st));
        if (model == IM_IC) {
            const uint32_t grid = blocks_for(count, kIcWaves, cu * 8);
            // several samples per ticket once there are many per wave
            const uint64_t per_wave = count / (uint64_t(grid) * kIcWaves);
            p.ticket_block = ctx->ic_ticket_block
                                 ? ctx->ic_ticket_block
                                 : static_cast<uint32_t>(std::min<uint64_t>(16, std::max<uint64_t>(1, per_wave / 8)));
            const bool bitmap = g->n <= kBitmapMaxN;
            if (mode == SampleMode::Pool) {
                if (bitmap) ic_main_kernel<0, true><<<grid, kIcWaves * kWave, 0, st>>>(p);
                else ic_main_kernel<0, false><<<grid, kIcWaves * kWave, 0, st>>>(p);
            } else {
                if (bitmap) ic_main_kernel<1, true><<<grid, kIcWaves * kWave, 0, st>>>(p);
                else ic_main_kernel<1, false><<<grid, kIcWaves * kWave, 0, st>>>(p);
            }
        } else {
            const uint32_t grid = blocks_for(count, kWave, std::min<uint32_t>(cu * 16, ctx->lt_lanes / kWave));
            if (ctx->lt_stamp + count >= 0xFFFFFFF0ull) {
                zero_u64_kernel<<<blocks_for(uint64_t(ctx->lt_lanes) * kLtTableSlots, 256, cu * 16), 256, 0, st>>>(
                    static_cast<uint64_t *>(ctx->lt_tables.ptr), uint64_t(ctx->lt_lanes) * kLtTableSlots);
                ctx->lt_stamp = 1;
            }
            const uint32_t stamp_base = static_cast<uint32_t>(ctx->lt_stamp);
            ctx->lt_stamp += count;
            auto *tables = static_cast<uint64_t *>(ctx->lt_tables.ptr);
            if (mode == SampleMode::Pool) lt_main_kernel<0><<<grid, kWave, 0, st>>>(p, tables, stamp_base);
            else lt_main_kernel<1><<<grid, kWave, 0, st>>>(p, tables, stamp_base);
        }
        if (ctx->timing) IM_HIP(hipEventRecord(ctx->ev_end, st));
        if (model == IM_IC && plain) {
            plain_handoff_kernel<<<1, 1, 0, st>>>(cnt);
        } else if (model == IM_IC) {
            const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
            Counters *c = cnt;
            if (mode == SampleMode::Pool) {
                ic_group_kernel<0, GrpSmall><<<cu * 5, GrpSmall::kThreads, 0, st>>>(
                    p, p.defer_list, &c->defer_count, &c->defer_ticket, p.large_list, &c->large_count, p.ho_wave,
                    kHoStrideWave, p.ho_wave_cap, p.ho_small, kHoStrideSmall, p.ho_small_cap);
                ic_group_kernel<0, GrpLarge><<<cu, GrpLarge::kThreads, 0, st>>>(
                    p, p.large_list, &c->large_count, &c->large_ticket, p.long_list, &c->long_count, p.ho_small,
                    kHoStrideSmall, p.ho_small_cap, nullptr, 0, 0);
            } else {
                ic_group_kernel<1, GrpSmall><<<cu * 5, GrpSmall::kThreads, 0, st>>>(
                    p, p.defer_list, &c->defer_count, &c->defer_ticket, p.large_list, &c->large_count, p.ho_wave,
                    kHoStrideWave, p.ho_wave_cap, p.ho_small, kHoStrideSmall, p.ho_small_cap);
                ic_group_kernel<1, GrpLarge><<<cu, GrpLarge::kThreads, 0, st>>>(
                    p, p.large_list, &c->large_count, &c->large_ticket, p.long_list, &c->long_count, p.ho_small,
                    kHoStrideSmall, p.ho_small_cap, nullptr, 0, 0);
            }
            if (ctx->timing) IM_HIP(hipEventRecord(ctx->ev_group, st));
        }
        {
            const uint32_t nslots = ctx->slot_count;
            const uint32_t grid = (nslots + kLongWaves - 1) / kLongWaves;
            auto *slot_mem = static_cast<uint32_t *>(ctx->slots.ptr);
            auto *epochs = slot_mem + 2ull * g->n * nslots;
            if (model == IM_IC) {
                Params pl = p;
                if (plain) pl.long_list = p.defer_list;  // the wave pass's hand-ons, in its order
                if (mode == SampleMode::Pool) long_kernel<IM_IC, 0><<<grid, kLongWaves * kWave, 0, st>>>(pl, slot_mem, g->n, nslots, epochs);
                else long_kernel<IM_IC, 1><<<grid, kLongWaves * kWave, 0, st>>>(pl, slot_mem, g->n, nslots, epochs);
                // a plain launch's timing covers its long path, which does
                // the work the tiers do otherwise
                if (plain && ctx->timing) IM_HIP(hipEventRecord(ctx->ev_group, st));
            } else {
                if (mode == SampleMode::Pool) long_kernel<IM_LT, 0><<<grid, kLongWaves * kWave, 0, st>>>(p, slot_mem, g->n, nslots, epochs);
                else long_kernel<IM_LT, 1><<<grid, kLongWaves * kWave, 0, st>>>(p, slot_mem, g->n, nslots, epochs);
            }
        }
        IM_HIP(hipGetLastError());
        Counters hc{};
        std::vector<unsigned long long> hacc(2ull * nitems);
        IM_HIP(hipMemcpyAsync(hacc.data(), dacc, 16ull * nitems, hipMemcpyDeviceToHost, st));
        IM_TRY(to_host_sync(ctx, &hc, cnt, sizeof(hc)));
        ctx->slot_epoch += (model == IM_IC) ? hc.long_count : hc.defer_count;
        if (hc.overflow) {
            cap = std::max<uint64_t>(cap * 2, hc.stage_cursor + (1u << 20));
            continue;
        }
        for (uint32_t i = 0; i < nitems; ++i) per_item[i] = ItemTotals{hacc[2 * i], hacc[2 * i + 1]};
        res->total_nodes = hc.total_nodes + hc.nodes_long;
        if (mode == SampleMode::Pool && count)
            g->mean_set[model == IM_IC ? 0 : 1].store(double(res->total_nodes) / double(count),
                                                      std::memory_order_relaxed);
        res->edges = hc.edges + hc.edges_long;
        res->deferred = hc.defer_count;
        res->count = count;
        if (ctx->timing && mode == SampleMode::Pool) {
            // IC: the wave pass and the workgroup tier together (the counters
            // cover both); LT: the main pass. The long path is left out.
            float ms = 0.f;
            IM_HIP(hipEventElapsedTime(&ms, ctx->ev_begin, model == IM_IC ? ctx->ev_group : ctx->ev_end));
            ctx->times.sample_launches += 1;
            ctx->times.sample_ms += ms;
            ctx->times.sample_sets += count - (model == IM_IC ? hc.long_count : hc.defer_count);
            ctx->times.sample_steps += hc.edges;
            ctx->times.sample_nodes += hc.total_nodes;
            ctx->times.model = model;
            if (model == IM_IC) {
                float gms = 0.f;
                IM_HIP(hipEventElapsedTime(&gms, ctx->ev_end, ctx->ev_group));
                ctx->times.group_launches += 1;
                ctx->times.group_ms += gms;
                ctx->times.group_samples += hc.grp_samples;
                ctx->times.group_edges += hc.grp_edges;
                ctx->times.group_levels += hc.grp_levels;
            }
        }
        return IM_OK;
    }
    set_error("sampler staging kept overflowing");
    return IM_E_OOM;
}

im_status sample_batch(im_ctx *ctx, const im_graph *g, im_model model, uint64_t key, uint64_t s0, uint64_t count,
                       SampleMode mode, double size_hint, SampleResult *res) {
    SampleItem it{key, s0, count, static_cast<const uint32_t *>(ctx->seedbits.ptr)};
    ItemTotals tot;
    return sample_items(ctx, g, model, &it, 1, mode, size_hint, res, &tot);
}

static im_status grow_pool(im_pool *p, uint64_t need_sets, uint64_t need_nodes) {
    im_ctx *ctx = p->ctx;
    hipStream_t st = ctx->stream;
    if (need_sets > p->cap_sets) {
        size_t cap = std::max<size_t>(need_sets, p->cap_sets * 2);
        DevBuf nb;
        IM_TRY(dev_alloc(ctx, nb, (cap + 1) * 8));
        if (p->poff.ptr) {
            copy_u64_kernel<<<blocks_for(p->count + 1, 256, 4096), 256, 0, st>>>(
                static_cast<const uint64_t *>(p->poff.ptr), static_cast<uint64_t *>(nb.ptr), p->count + 1);
        } else {
            set_first_kernel<<<1, 1, 0, st>>>(static_cast<uint64_t *>(nb.ptr), 0);
        }
        IM_HIP(hipStreamSynchronize(st));
        dev_free(ctx, p->poff);
        p->poff = nb;
        p->cap_sets = cap;
    }
    if (need_nodes > p->cap_nodes) {
        size_t cap = std::max<size_t>(need_nodes, p->cap_nodes * 2);
        DevBuf nb;
        IM_TRY(dev_alloc(ctx, nb, cap * 4));
        if (p->pnodes.ptr && p->total)
            copy_u32_kernel<<<blocks_for(p->total, 256, 4096), 256, 0, st>>>(
                static_cast<const uint32_t *>(p->pnodes.ptr), static_cast<uint32_t *>(nb.ptr), p->total);
        IM_HIP(hipStreamSynchronize(st));
        dev_free(ctx, p->pnodes);
        p->pnodes = nb;
        p->cap_nodes = cap;
    }
    return IM_OK;
}

}  // namespace im

namespace {

// Sum of the in-degrees of pool entries [0, entries) into *out.
__global__ void ic_entry_edges_kernel(const uint32_t *pnodes, uint64_t entries, const uint64_t *off,
                                      unsigned long long *out) {
    uint64_t acc = 0;
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < entries;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t v = pnodes[e];
        acc += off[v + 1] - off[v];
    }
    acc = wave_sum_u64(acc);
    if (lane_id() == 0 && acc) atomicAdd(out, static_cast<unsigned long long>(acc));
}

}  // namespace

namespace im {

im_status pool_ic_edges(const im_pool *p, uint64_t sets, uint64_t *edges) {
    im_ctx *ctx = p->ctx;
    uint64_t entries = 0;
    IM_TRY(to_host_sync(ctx, &entries, static_cast<const uint64_t *>(p->poff.ptr) + sets, 8));
    IM_TRY(dev_reserve(ctx, ctx->counters, 256));
    // past the sampler's counters, which the same stream uses before and after
    auto *sum = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->counters.ptr) + 192);
    static_assert(sizeof(Counters) <= 192, "the edge sum sits after the sampler counters");
    zero_u64_kernel<<<1, 64, 0, ctx->stream>>>(reinterpret_cast<uint64_t *>(sum), 1);
    if (entries)
        ic_entry_edges_kernel<<<blocks_for(entries, 256, static_cast<uint32_t>(ctx->cu_count) * 8), 256, 0,
                                ctx->stream>>>(static_cast<const uint32_t *>(p->pnodes.ptr), entries,
                                               static_cast<const uint64_t *>(p->g->off.ptr), sum);
    IM_HIP(hipGetLastError());
    return to_host_sync(ctx, edges, sum, 8);
}

im_status pool_append_items(im_ctx *ctx, const AppendItem *items, uint32_t nitems) {
    if (nitems == 0) return IM_OK;
    hipStream_t st = ctx->stream;
    uint64_t count = 0;
    for (uint32_t i = 0; i < nitems; ++i) {
        const AppendItem &a = items[i];
        IM_TRY(grow_pool(a.pool, a.pool->count + a.count, a.pool->total + a.nodes + 1));
        count += a.count;
    }
    if (count == 0) return IM_OK;
    Meta meta = meta_view(ctx, count);
    // global exclusive prefix of the batch's set sizes: prefix[t] (count+1)
    const uint64_t tiles = (count + kScanTile - 1) / kScanTile;
    IM_TRY(dev_reserve(ctx, ctx->scan_tmp, (tiles + 1) * 8 + (count + 1) * 8 + 256));
    auto *tsum = static_cast<uint64_t *>(ctx->scan_tmp.ptr);
    auto *prefix = tsum + ((tiles + 1 + 31) & ~uint64_t(31));
    set_first_kernel<<<1, 1, 0, st>>>(prefix, 0);
    scan_tiles_kernel<<<static_cast<uint32_t>(tiles), kScanThreads, 0, st>>>(meta.sizes, count, tsum);
    scan_sums_kernel<<<1, 1024, 0, st>>>(tsum, tiles);
    scan_apply_kernel<<<static_cast<uint32_t>(tiles), kScanThreads, 0, st>>>(meta.sizes, count, tsum, 0, prefix);
    // per-item destinations
    std::vector<AppendDst> hd(nitems);
    uint32_t start = 0;
    for (uint32_t i = 0; i < nitems; ++i) {
        im_pool *pl = items[i].pool;
        hd[i] = AppendDst{static_cast<uint64_t *>(pl->poff.ptr) + pl->count, static_cast<uint32_t *>(pl->pnodes.ptr),
                          pl->total, start};
        start += static_cast<uint32_t>(items[i].count);
    }
    IM_TRY(dev_reserve(ctx, ctx->append_dst, sizeof(AppendDst) * nitems + 64));
    auto *dd = static_cast<AppendDst *>(ctx->append_dst.ptr);
    IM_HIP(hipMemcpyAsync(dd, hd.data(), sizeof(AppendDst) * nitems, hipMemcpyHostToDevice, st));
    compact_items_kernel<<<blocks_for(count * 16, 256, static_cast<uint32_t>(ctx->cu_count) * 16), 256, 0, st>>>(
        static_cast<const uint32_t *>(ctx->stage.ptr), meta.stage_off, prefix, dd, nitems, count);
    IM_HIP(hipGetLastError());
    for (uint32_t i = 0; i < nitems; ++i) {
        im_pool *pl = items[i].pool;
        pl->count += items[i].count;
        pl->total += items[i].nodes;
        pl->edges += items[i].edges;
        if (pl->count) pl->mean_size = double(pl->total) / double(pl->count);
    }
    if (nitems == 1) {  // cross-check the device offsets against the item totals
        uint64_t end = 0;
        im_pool *pl = items[0].pool;
        IM_TRY(to_host_sync(ctx, &end, static_cast<const uint64_t *>(pl->poff.ptr) + pl->count, 8));
        if (end != pl->total) {
            set_error("pool append: offsets end at %llu, expected %llu", static_cast<unsigned long long>(end),
                      static_cast<unsigned long long>(pl->total));
            return IM_E_DEVICE;
        }
    }
    return IM_OK;
}

}  // namespace im
