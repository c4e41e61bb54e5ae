// Graph residency (Section 2): the reverse adjacency of G with per-edge
// 32-bit thresholds, built on the device from an edge list sorted by
// (dst, src).
//
//   off[v] .. off[v+1]  in-edges of v, ascending src
//   edges[e] = {src, thr}
//     IC: thr = floor(w * 2^32), clamped to 2^32-1 (which means "always
//         live"); edge live iff coin < thr (Section 2.1, each edge fires
//         once with probability w).
//     LT: thr = floor(2^32 * (w_1 + ... + w_i)) clamped, the running sum
//         taken left to right in FP64 over the node's in-edges; in-edge i
//         is the one kept iff thr_{i-1} <= coin < thr_i (the live-edge form
//         of the threshold model, Kempe et al. 2003).
//
// When every in-edge of each node carries the same IC threshold (the
// weighted cascade w(u,v) = 1/d_in(v) of the paper's experiments is one
// such case) the IC sampler reads a second, compact form:
//   nodes[v] = {first in-edge (low, high word), in-degree, threshold}, one
//     aligned 16-byte load per expanded node instead of the offset pair;
//   srcs[e] = src of edge e (4 bytes instead of 8), padded like the records.
// The coins are compared with the same thresholds, so the sets drawn are
// the same in either form.
#include "im_device.hpp"
#include "im_internal.hpp"

namespace {

constexpr uint32_t kBadId = 1u;
constexpr uint32_t kBadOrder = 2u;
constexpr uint32_t kBadWeight = 4u;
constexpr uint32_t kLtSum = 8u;
constexpr uint32_t kIcMixed = 16u;  // some node's IC in-edges differ in threshold

struct BuildCounters {
    uint32_t flags;
    uint32_t max_in;
};

__device__ __forceinline__ uint32_t to_threshold(double x) {
    const double t = floor(x * 4294967296.0);
    if (t >= 4294967295.0) return 0xFFFFFFFFu;
    if (t <= 0.0) return 0u;
    return static_cast<uint32_t>(t);
}

__device__ __forceinline__ bool bad_weight(float w) { return !(w >= 0.0f && w <= 1.0f); }

__global__ void validate_kernel(const uint32_t *src, const uint32_t *dst, const float *w_ic, const float *w_lt,
                                uint64_t m, uint32_t n, BuildCounters *cnt) {
    uint32_t flags = 0;
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < m;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t s = src[e], d = dst[e];
        if (s >= n || d >= n) flags |= kBadId;
        if (e > 0) {
            const uint32_t ps = src[e - 1], pd = dst[e - 1];
            if (!(pd < d || (pd == d && ps < s))) flags |= kBadOrder;
        }
        if (w_ic && bad_weight(w_ic[e])) flags |= kBadWeight;
        if (w_lt && bad_weight(w_lt[e])) flags |= kBadWeight;
    }
    if (flags) atomicOr(&cnt->flags, flags);
}

// off[v] = first edge whose dst >= v. Edge e writes the offsets of the nodes
// in (dst[e-1], dst[e]]; one extra thread closes (dst[m-1], n].
__global__ void offsets_kernel(const uint32_t *dst, uint64_t m, uint32_t n, uint64_t *off) {
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e <= m;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const int64_t prev = (e == 0) ? -1 : static_cast<int64_t>(dst[e - 1]);
        const int64_t cur = (e == m) ? static_cast<int64_t>(n) : static_cast<int64_t>(dst[e]);
        for (int64_t v = prev + 1; v <= cur; ++v) off[v] = e;
    }
}

// IC records {src, threshold}, padded with zero records to whole aligned
// 4-edge groups (a sampler lane reads a group's 32 bytes with two 16-byte
// loads; the pad is never live: it lies past every node's in-edge range).
__host__ __device__ inline uint64_t ic_records(uint64_t m) { return ((m + 3) & ~3ull) + 4; }

__global__ void ic_edges_kernel(const uint32_t *src, const float *w, uint64_t m, uint2 *edges) {
    const uint64_t total = ic_records(m);
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        edges[e] = e < m ? make_uint2(src[e], to_threshold(static_cast<double>(w[e]))) : make_uint2(0u, 0u);
    }
}

// Whether some node's in-edges carry different IC thresholds: edge e is
// compared with edge e-1 when both enter the same node.
__global__ void ic_uniform_kernel(const uint32_t *dst, const uint2 *edges, uint64_t m, BuildCounters *cnt) {
    bool mixed = false;
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x + 1; e < m;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        mixed |= dst[e] == dst[e - 1] && edges[e].y != edges[e - 1].y;
    if (__ballot(mixed) != 0 && imd::lane_id() == 0) atomicOr(&cnt->flags, kIcMixed);
}

// The compact IC form: sources padded to whole groups, and per node its
// first in-edge, in-degree and threshold (0 for a node with no in-edges).
__global__ void ic_compact_srcs_kernel(const uint2 *edges, uint64_t m, uint32_t *srcs) {
    const uint64_t total = ic_records(m);
    for (uint64_t e = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        srcs[e] = e < m ? edges[e].x : 0u;
}

__global__ void ic_compact_nodes_kernel(const uint64_t *off, const uint2 *edges, uint32_t n, uint4 *nodes) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint64_t a = off[v], b = off[v + 1];
        nodes[v] = make_uint4(static_cast<uint32_t>(a), static_cast<uint32_t>(a >> 32), static_cast<uint32_t>(b - a),
                              b > a ? edges[a].y : 0u);
    }
}

// One thread per node: the running FP64 sum in edge order (so the rounding
// sequence is fixed), plus the in-degree maximum.
__global__ void lt_edges_kernel(const uint32_t *src, const float *w, const uint64_t *off, uint32_t n,
                                uint2 *edges, BuildCounters *cnt) {
    uint32_t flags = 0, dmax = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint64_t a = off[v], b = off[v + 1];
        double sum = 0.0;
        for (uint64_t e = a; e < b; ++e) {
            sum = sum + static_cast<double>(w[e]);
            edges[e] = make_uint2(src[e], to_threshold(sum));
        }
        if (sum > 1.0 + 1e-6) flags |= kLtSum;
        dmax = max(dmax, static_cast<uint32_t>(b - a));
    }
    if (flags) atomicOr(&cnt->flags, flags);
    if (dmax) atomicMax(&cnt->max_in, dmax);
}

__global__ void max_in_kernel(const uint64_t *off, uint32_t n, BuildCounters *cnt) {
    uint32_t dmax = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        dmax = max(dmax, static_cast<uint32_t>(off[v + 1] - off[v]));
    if (dmax) atomicMax(&cnt->max_in, dmax);
}

__global__ void zero_counters_kernel(BuildCounters *cnt) {
    cnt->flags = 0;
    cnt->max_in = 0;
}

__global__ void cum_weights_kernel(const uint32_t *w, uint32_t n, uint64_t *cum) {
    // single block: running prefix over n node weights in chunks of blockDim
    __shared__ uint64_t part[1024];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) {
        carry = 0;
        cum[0] = 0;
    }
    __syncthreads();
    for (uint32_t base = 0; base < n; base += blockDim.x) {
        const uint32_t v = base + threadIdx.x;
        part[threadIdx.x] = (v < n) ? w[v] : 0;
        __syncthreads();
        for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
            const uint64_t y = (threadIdx.x >= d) ? part[threadIdx.x - d] : 0;
            __syncthreads();
            part[threadIdx.x] += y;
            __syncthreads();
        }
        if (v < n) cum[v + 1] = carry + part[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += part[threadIdx.x];
        __syncthreads();
    }
}

uint32_t grid_for(uint64_t items, int cu) {
    const uint64_t blocks = (items + 255) / 256;
    const uint64_t cap = static_cast<uint64_t>(cu) * 16;
    return static_cast<uint32_t>(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
}

}  // namespace

namespace im {

im_status graph_build(im_graph *g, const uint32_t *src_h, const uint32_t *dst_h, const float *w_ic_h,
                      const float *w_lt_h) {
    im_ctx *ctx = g->ctx;
    const uint64_t m = g->m;
    const uint32_t n = g->n;
    hipStream_t st = ctx->stream;
    DevBuf d_src, d_dst, d_wic, d_wlt, d_cnt;
    auto cleanup = [&]() {
        dev_free(ctx, d_src);
        dev_free(ctx, d_dst);
        dev_free(ctx, d_wic);
        dev_free(ctx, d_wlt);
        dev_free(ctx, d_cnt);
    };
    const size_t mb = (m ? m : 1);
    im_status rc = IM_OK;
    if ((rc = dev_alloc(ctx, d_src, mb * 4)) || (rc = dev_alloc(ctx, d_dst, mb * 4)) ||
        (w_ic_h && (rc = dev_alloc(ctx, d_wic, mb * 4))) || (w_lt_h && (rc = dev_alloc(ctx, d_wlt, mb * 4))) ||
        (rc = dev_alloc(ctx, d_cnt, sizeof(BuildCounters))) || (rc = dev_alloc(ctx, g->off, (size_t(n) + 1) * 8)) ||
        (w_ic_h && (rc = dev_alloc(ctx, g->edges_ic, ic_records(m) * 8))) ||
        (w_lt_h && (rc = dev_alloc(ctx, g->edges_lt, mb * 8)))) {
        cleanup();
        return rc;
    }
    auto fail = [&](hipError_t e, const char *what) {
        set_error("%s: %s", what, hipGetErrorString(e));
        cleanup();
        return IM_E_DEVICE;
    };
    hipError_t e;
    if (m) {
        if ((e = hipMemcpyAsync(d_src.ptr, src_h, m * 4, hipMemcpyHostToDevice, st))) return fail(e, "copy src");
        if ((e = hipMemcpyAsync(d_dst.ptr, dst_h, m * 4, hipMemcpyHostToDevice, st))) return fail(e, "copy dst");
        if (w_ic_h && (e = hipMemcpyAsync(d_wic.ptr, w_ic_h, m * 4, hipMemcpyHostToDevice, st)))
            return fail(e, "copy w_ic");
        if (w_lt_h && (e = hipMemcpyAsync(d_wlt.ptr, w_lt_h, m * 4, hipMemcpyHostToDevice, st)))
            return fail(e, "copy w_lt");
    }
    auto *cnt = static_cast<BuildCounters *>(d_cnt.ptr);
    const auto *s32 = static_cast<const uint32_t *>(d_src.ptr);
    const auto *d32 = static_cast<const uint32_t *>(d_dst.ptr);
    const auto *wic = static_cast<const float *>(d_wic.ptr);
    const auto *wlt = static_cast<const float *>(d_wlt.ptr);
    auto *off = static_cast<uint64_t *>(g->off.ptr);
    const int cu = ctx->cu_count;
    zero_counters_kernel<<<1, 1, 0, st>>>(cnt);
    if (m) validate_kernel<<<grid_for(m, cu), 256, 0, st>>>(s32, d32, wic, wlt, m, n, cnt);
    BuildCounters hc{};
    IM_TRY(to_host_sync(ctx, &hc, cnt, sizeof(hc)));
    if (hc.flags & (kBadId | kBadOrder | kBadWeight)) {
        set_error("im_graph_load: %s%s%s", (hc.flags & kBadId) ? "node id >= n; " : "",
                  (hc.flags & kBadOrder) ? "edges not strictly sorted by (dst, src); " : "",
                  (hc.flags & kBadWeight) ? "weight outside [0,1]; " : "");
        cleanup();
        return IM_E_ARG;
    }
    offsets_kernel<<<grid_for(m + 1, cu), 256, 0, st>>>(d32, m, n, off);
    if (w_ic_h) {
        ic_edges_kernel<<<grid_for(ic_records(m), cu), 256, 0, st>>>(s32, wic, m, static_cast<uint2 *>(g->edges_ic.ptr));
        if (m > 1) ic_uniform_kernel<<<grid_for(m, cu), 256, 0, st>>>(d32, static_cast<const uint2 *>(g->edges_ic.ptr), m, cnt);
    }
    if (w_lt_h) {
        lt_edges_kernel<<<grid_for(n, cu), 256, 0, st>>>(s32, wlt, off, n, static_cast<uint2 *>(g->edges_lt.ptr), cnt);
    } else {
        max_in_kernel<<<grid_for(n, cu), 256, 0, st>>>(off, n, cnt);
    }
    if ((e = hipGetLastError())) return fail(e, "graph kernels");
    IM_TRY(to_host_sync(ctx, &hc, cnt, sizeof(hc)));
    cleanup();
    if (hc.flags & kLtSum) {
        set_error("im_graph_load: LT in-weights of some node sum above 1");
        return IM_E_LT_WEIGHTS;
    }
    // the compact IC form is optional: not built when the context's draws
    // would not read it, and left out when its memory is not there (draws
    // then read the records)
    if (w_ic_h && ctx->ic_compact && !(hc.flags & kIcMixed)) {
        if (dev_alloc(ctx, g->srcs_ic, ic_records(m) * 4) != IM_OK ||
            dev_alloc(ctx, g->nodes_ic, size_t(n) * 16) != IM_OK) {
            dev_free(ctx, g->srcs_ic);
            dev_free(ctx, g->nodes_ic);
            (void)hipGetLastError();  // a failed hipMalloc is reported once more here; not an error of the load
            clear_error();
        }
    }
    if (g->nodes_ic.ptr) {
        const auto *rec = static_cast<const uint2 *>(g->edges_ic.ptr);
        ic_compact_srcs_kernel<<<grid_for(ic_records(m), cu), 256, 0, st>>>(rec, m, static_cast<uint32_t *>(g->srcs_ic.ptr));
        ic_compact_nodes_kernel<<<grid_for(n, cu), 256, 0, st>>>(off, rec, n, static_cast<uint4 *>(g->nodes_ic.ptr));
        if ((e = hipGetLastError()) || (e = hipStreamSynchronize(st))) {
            set_error("compact IC form: %s", hipGetErrorString(e));
            return IM_E_DEVICE;
        }
    }
    g->max_in = hc.max_in;
    g->models = (w_ic_h ? 1u : 0u) | (w_lt_h ? 2u : 0u) | (g->nodes_ic.ptr ? 4u : 0u);
    return IM_OK;
}

im_status graph_source_weights(im_graph *g, const uint32_t *node_w) {
    im_ctx *ctx = g->ctx;
    dev_free(ctx, g->src_cum);
    g->src_total = 0;
    if (!node_w) return IM_OK;
    uint64_t total = 0;
    for (uint32_t v = 0; v < g->n; ++v) total += node_w[v];
    if (total == 0) {
        set_error("im_graph_set_source_weights: all weights are zero");
        return IM_E_ARG;
    }
    DevBuf d_w;
    IM_TRY(dev_alloc(ctx, d_w, size_t(g->n) * 4));
    im_status rc = dev_alloc(ctx, g->src_cum, (size_t(g->n) + 1) * 8);
    if (rc) {
        dev_free(ctx, d_w);
        return rc;
    }
    hipError_t e = hipMemcpyAsync(d_w.ptr, node_w, size_t(g->n) * 4, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        cum_weights_kernel<<<1, 1024, 0, ctx->stream>>>(static_cast<const uint32_t *>(d_w.ptr), g->n,
                                                         static_cast<uint64_t *>(g->src_cum.ptr));
        e = hipStreamSynchronize(ctx->stream);
    }
    dev_free(ctx, d_w);
    if (e != hipSuccess) {
        set_error("source weights: %s", hipGetErrorString(e));
        return IM_E_DEVICE;
    }
    g->src_total = total;
    return IM_OK;
}

}  // namespace im
