// Max-Coverage (Algorithm 2), coverage counts (Eq. 1) and the ordered
// stopping search of Estimate-Inf (Algorithm 3).
//
// Incidence (node -> sets holding it) is a counting sort of the pool range:
// a histogram of node ids, an exclusive scan, and a scatter of set ids. The
// greedy then runs k rounds of
//   argmax over unchosen v of (gain[v] << 32 | ~v)   (max gain, lowest id)
//   for each not-yet-covered set of the winner: mark covered, decrement the
//   gain of every member
// which is linear in the total size of the sets, as the paper notes.
#include <algorithm>

#include "im_device.hpp"
#include "im_internal.hpp"

namespace {

using namespace imd;

constexpr int kThreads = 256;

uint32_t grid_of(uint64_t items, uint32_t per_block, uint32_t cap) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<uint32_t>(b);
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t count, uint32_t value) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = value;
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t count, uint64_t value) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = value;
}

__global__ void histogram_kernel(const uint32_t *nodes, uint64_t begin, uint64_t end, uint32_t *cnt) {
    for (uint64_t i = begin + blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < end;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        atomicAdd(&cnt[nodes[i]], 1u);
}

// ---- exclusive scan of u32 counts into u64 offsets (n+1 entries) ----

__device__ __forceinline__ uint64_t block_scan_excl(uint64_t x, uint64_t *smem, uint64_t &total) {
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
    uint64_t off = 0, tot = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
        if (w < wave) off += smem[w];
        tot += smem[w];
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

constexpr uint32_t kTile = 1024;

__global__ __launch_bounds__(kThreads) void tile_sums_kernel(const uint32_t *in, uint64_t count, uint64_t *tsum) {
    __shared__ uint64_t smem[kThreads / kWave];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kTile + threadIdx.x * 4;
    uint64_t x = 0;
    for (int i = 0; i < 4; ++i)
        if (b0 + i < count) x += in[b0 + i];
    uint64_t total = 0;
    block_scan_excl(x, smem, total);
    if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void tile_scan_kernel(uint64_t *tsum, uint64_t tiles) {
    __shared__ uint64_t smem[1024 / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < tiles; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t x = i < tiles ? tsum[i] : 0;
        uint64_t total = 0;
        const uint64_t ex = block_scan_excl(x, smem, total);
        if (i < tiles) tsum[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
}

// out[0] = 0, out[i+1] = sum(in[0..i])
__global__ __launch_bounds__(kThreads) void tile_apply_kernel(const uint32_t *in, uint64_t count, const uint64_t *toff,
                                                              uint64_t *out) {
    __shared__ uint64_t smem[kThreads / kWave];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kTile + threadIdx.x * 4;
    uint64_t v[4], x = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (b0 + i < count) ? in[b0 + i] : 0;
        x += v[i];
    }
    uint64_t total = 0;
    uint64_t run = toff[blockIdx.x] + block_scan_excl(x, smem, total);
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    for (int i = 0; i < 4; ++i) {
        run += v[i];
        if (b0 + i < count) out[b0 + i + 1] = run;
    }
}

// 16 lanes per set: scatter the set's index into each member's list.
__global__ __launch_bounds__(kThreads) void scatter_kernel(const uint64_t *poff, const uint32_t *pnodes, uint64_t begin,
                                                           uint64_t nsets, const uint64_t *ioff, uint32_t *fill,
                                                           uint32_t *isets) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t j = grp; j < nsets; j += ngrp) {
        const uint64_t a = poff[begin + j], b = poff[begin + j + 1];
        for (uint64_t q = a + sub; q < b; q += 16) {
            const uint32_t v = pnodes[q];
            const uint32_t pos = atomicAdd(&fill[v], 1u);
            isets[ioff[v] + pos] = static_cast<uint32_t>(j);
        }
    }
}

// ---- greedy rounds ----

struct GreedyState {
    uint32_t *gain;     // uncovered sets holding v
    uint8_t *chosen;    // 1 once v is a seed
    uint32_t *covbits;  // covered flag per set (bit)
    const uint64_t *ioff;
    const uint32_t *isets;
    const uint64_t *poff;
    const uint32_t *pnodes;
    uint64_t begin;
    uint32_t n;
    unsigned long long *best;  // per round: packed argmax key
    uint32_t *seeds;           // per round
    unsigned long long *cov;   // covered sets so far
};

__global__ __launch_bounds__(kThreads) void argmax_kernel(GreedyState g, uint32_t round) {
    __shared__ unsigned long long smem[kThreads / kWave];
    unsigned long long best = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const unsigned long long key =
            g.chosen[v] ? 0ull : ((static_cast<unsigned long long>(g.gain[v]) << 32) | static_cast<unsigned long long>(~v));
        best = key > best ? key : best;
    }
    best = wave_max_u64(best);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / kWave; ++w) best = smem[w] > best ? smem[w] : best;
        atomicMax(&g.best[round], best);
    }
}

// Cover the winner's sets. 16 lanes per incidence entry.
__global__ __launch_bounds__(kThreads) void apply_kernel(GreedyState g, uint32_t round) {
    __shared__ unsigned long long smem[kThreads / kWave];
    const uint32_t v = ~static_cast<uint32_t>(g.best[round] & 0xFFFFFFFFull);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.seeds[round] = v;
        g.chosen[v] = 1;
    }
    const uint64_t a = g.ioff[v], b = g.ioff[v + 1];
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    unsigned long long newly = 0;
    for (uint64_t i = a + grp; i < b; i += ngrp) {
        const uint32_t j = g.isets[i];
        uint32_t fresh = 0;
        if (sub == 0) {
            const uint32_t bit = 1u << (j & 31u);
            fresh = (atomicOr(&g.covbits[j >> 5], bit) & bit) ? 0u : 1u;
        }
        fresh = __shfl(fresh, static_cast<int>(lane_id() & ~15u), kWave);
        if (fresh) {
            if (sub == 0) ++newly;
            const uint64_t sa = g.poff[g.begin + j], sb = g.poff[g.begin + j + 1];
            for (uint64_t q = sa + sub; q < sb; q += 16) atomicSub(&g.gain[g.pnodes[q]], 1u);
        }
    }
    newly = wave_sum_u64(newly);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = newly;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kThreads / kWave; ++w) tot += smem[w];
        if (tot) atomicAdd(g.cov, tot);
    }
}

// Sets in [begin, end) that contain a node of the seed bitmap.
__global__ __launch_bounds__(kThreads) void coverage_kernel(const uint64_t *poff, const uint32_t *pnodes, uint64_t begin,
                                                            uint64_t end, const uint32_t *seedbits,
                                                            unsigned long long *out) {
    __shared__ unsigned long long smem[kThreads / kWave];
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    unsigned long long hits = 0;
    for (uint64_t j = begin + grp; j < end; j += ngrp) {
        const uint64_t a = poff[j], b = poff[j + 1];
        bool any = false;
        for (uint64_t q = a + sub; q < b && !any; q += 16) any = test_bit(seedbits, pnodes[q]);
        // combine the 16 lanes of the group
        const uint64_t mask = __ballot(any);
        const uint32_t shift = lane_id() & ~15u;
        if (sub == 0 && ((mask >> shift) & 0xFFFFull)) ++hits;
    }
    hits = wave_sum_u64(hits);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = hits;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kThreads / kWave; ++w) tot += smem[w];
        if (tot) atomicAdd(out, tot);
    }
}

__global__ void seed_bits_kernel(const uint32_t *seeds, uint32_t k, uint32_t *bits, uint32_t *bad, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t v = seeds[i];
        if (v >= n) atomicOr(bad, 1u);
        else atomicOr(&bits[v >> 5], 1u << (v & 31u));
    }
}

// ---- ordered first crossing over per-sample hit flags ----

__global__ __launch_bounds__(kThreads) void flag_tiles_kernel(const uint8_t *z, uint64_t count, uint32_t *tcnt) {
    __shared__ uint32_t smem[kThreads / kWave];
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kTile + threadIdx.x * 4;
    uint32_t x = 0;
    for (int i = 0; i < 4; ++i)
        if (b0 + i < count) x += z[b0 + i];
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kThreads / kWave; ++w) t += smem[w];
        tcnt[blockIdx.x] = t;
    }
}

// Single block: walk tiles in order to the one where the running count
// reaches `need`, then scan that tile's flags. out[0] = index or -1,
// out[1] = hits in the whole range.
__global__ __launch_bounds__(1024) void crossing_kernel(const uint8_t *z, uint64_t count, const uint32_t *tcnt,
                                                        uint64_t tiles, uint64_t need, long long *out) {
    __shared__ uint64_t smem[1024 / kWave];
    __shared__ uint64_t carry;
    __shared__ long long found_tile;
    __shared__ uint64_t before;
    if (threadIdx.x == 0) {
        carry = 0;
        found_tile = -1;
        before = 0;
    }
    __syncthreads();
    for (uint64_t b0 = 0; b0 < tiles; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t x = i < tiles ? tcnt[i] : 0;
        uint64_t total = 0;
        const uint64_t ex = block_scan_excl(x, smem, total);
        const uint64_t c = carry;
        // the tile where the running count first reaches need: unique i with
        // c+ex < need <= c+ex+x
        if (i < tiles && found_tile < 0 && c + ex < need && need <= c + ex + x) {
            found_tile = static_cast<long long>(i);
            before = c + ex;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    __syncthreads();
    long long index = -1;
    if (found_tile >= 0) {
        // scan flags of the tile (1024 entries, one per thread)
        const uint64_t pos = static_cast<uint64_t>(found_tile) * kTile + threadIdx.x;
        const uint64_t x = (pos < count) ? z[pos] : 0;
        uint64_t total = 0;
        const uint64_t ex = block_scan_excl(x, smem, total);
        __shared__ long long idx;
        if (threadIdx.x == 0) idx = -1;
        __syncthreads();
        if (x && before + ex + 1 == need) idx = static_cast<long long>(pos);
        __syncthreads();
        index = idx;
    }
    if (threadIdx.x == 0) {
        out[0] = index;
        out[1] = static_cast<long long>(carry);
    }
}

}  // namespace

namespace im {

im_status set_seed_bits(im_ctx *ctx, uint32_t n, const uint32_t *seeds_host, uint32_t k) {
    const uint64_t words = (uint64_t(n) + 31) / 32;
    IM_TRY(dev_reserve(ctx, ctx->seedbits, words * 4 + 4 * uint64_t(k) + 64));
    auto *bits = static_cast<uint32_t *>(ctx->seedbits.ptr);
    auto *dseeds = bits + words;
    auto *bad = dseeds + k;
    hipStream_t st = ctx->stream;
    fill_u32_kernel<<<grid_of(words + 1, kThreads, 1024), kThreads, 0, st>>>(bits, words, 0u);
    fill_u32_kernel<<<1, 64, 0, st>>>(bad, 1, 0u);
    if (k) {
        IM_HIP(hipMemcpyAsync(dseeds, seeds_host, 4ull * k, hipMemcpyHostToDevice, st));
        seed_bits_kernel<<<grid_of(k, kThreads, 64), kThreads, 0, st>>>(dseeds, k, bits, bad, n);
    }
    uint32_t hbad = 0;
    IM_TRY(to_host_sync(ctx, &hbad, bad, 4));
    if (hbad) {
        set_error("seed id >= n");
        return IM_E_ARG;
    }
    return IM_OK;
}

im_status coverage_range(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds_host, uint32_t k,
                         uint64_t *cov) {
    im_ctx *ctx = p->ctx;
    IM_TRY(set_seed_bits(ctx, p->g->n, seeds_host, k));
    IM_TRY(dev_reserve(ctx, ctx->counters, 256));
    auto *out = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->counters.ptr) + 128);
    hipStream_t st = ctx->stream;
    fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(out), 1, 0);
    if (end > begin) {
        coverage_kernel<<<grid_of((end - begin) * 16, kThreads, ctx->cu_count * 16), kThreads, 0, st>>>(
            static_cast<const uint64_t *>(p->poff.ptr), static_cast<const uint32_t *>(p->pnodes.ptr), begin, end,
            static_cast<const uint32_t *>(ctx->seedbits.ptr), out);
    }
    IM_HIP(hipGetLastError());
    IM_TRY(to_host_sync(ctx, cov, out, 8));
    return IM_OK;
}

im_status max_coverage(const im_pool *p, uint64_t begin, uint64_t end, uint32_t k, uint32_t *seeds_host,
                       uint64_t *cov) {
    im_ctx *ctx = p->ctx;
    const uint32_t n = p->g->n;
    const uint64_t nsets = end - begin;
    const auto *poff = static_cast<const uint64_t *>(p->poff.ptr);
    const auto *pnodes = static_cast<const uint32_t *>(p->pnodes.ptr);
    uint64_t ebegin = 0, eend = 0;
    IM_TRY(to_host_sync(ctx, &ebegin, poff + begin, 8));
    IM_TRY(to_host_sync(ctx, &eend, poff + end, 8));
    const uint64_t entries = eend - ebegin;

    // layout of the working arrays in ctx->cover
    const uint64_t tiles = (uint64_t(n) + kTile - 1) / kTile;
    const uint64_t covwords = (nsets + 31) / 32 + 1;
    size_t off_gain = 0;
    size_t off_fill = off_gain + 4ull * n;
    size_t off_ioff = (off_fill + 4ull * n + 7) & ~size_t(7);
    size_t off_tsum = off_ioff + 8ull * (n + 1);
    size_t off_best = off_tsum + 8ull * (tiles + 1);
    size_t off_cov = off_best + 8ull * k;
    size_t off_seeds = off_cov + 8;
    size_t off_chosen = off_seeds + 4ull * k;
    size_t off_covbits = (off_chosen + n + 3) & ~size_t(3);
    size_t off_isets = off_covbits + 4ull * covwords;
    size_t bytes = off_isets + 4ull * (entries + 1);
    IM_TRY(dev_reserve(ctx, ctx->cover, bytes));
    char *base = static_cast<char *>(ctx->cover.ptr);
    auto *gain = reinterpret_cast<uint32_t *>(base + off_gain);
    auto *fill = reinterpret_cast<uint32_t *>(base + off_fill);
    auto *ioff = reinterpret_cast<uint64_t *>(base + off_ioff);
    auto *tsum = reinterpret_cast<uint64_t *>(base + off_tsum);
    auto *best = reinterpret_cast<unsigned long long *>(base + off_best);
    auto *dcov = reinterpret_cast<unsigned long long *>(base + off_cov);
    auto *dseeds = reinterpret_cast<uint32_t *>(base + off_seeds);
    auto *chosen = reinterpret_cast<uint8_t *>(base + off_chosen);
    auto *covbits = reinterpret_cast<uint32_t *>(base + off_covbits);
    auto *isets = reinterpret_cast<uint32_t *>(base + off_isets);

    hipStream_t st = ctx->stream;
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(gain, n, 0u);
    fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(fill, n, 0u);
    fill_u32_kernel<<<grid_of(n / 4 + 1, kThreads, cu * 8), kThreads, 0, st>>>(reinterpret_cast<uint32_t *>(chosen),
                                                                               (uint64_t(n) + 3) / 4, 0u);
    fill_u32_kernel<<<grid_of(covwords, kThreads, cu * 8), kThreads, 0, st>>>(covbits, covwords, 0u);
    fill_u64_kernel<<<1, 256, 0, st>>>(reinterpret_cast<uint64_t *>(best), k, 0);
    fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(dcov), 1, 0);
    if (entries)
        histogram_kernel<<<grid_of(entries, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, ebegin, eend, gain);
    tile_sums_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gain, n, tsum);
    tile_scan_kernel<<<1, 1024, 0, st>>>(tsum, tiles);
    tile_apply_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gain, n, tsum, ioff);
    if (nsets)
        scatter_kernel<<<grid_of(nsets * 16, kThreads, cu * 16), kThreads, 0, st>>>(poff, pnodes, begin, nsets, ioff,
                                                                                     fill, isets);
    GreedyState gs{gain, chosen, covbits, ioff, isets, poff, pnodes, begin, n, best, dseeds, dcov};
    const uint32_t agrid = grid_of(n, kThreads, cu * 4);
    const uint32_t pgrid = std::max<uint32_t>(1, std::min<uint32_t>(cu * 4, static_cast<uint32_t>((nsets * 16 + kThreads - 1) / kThreads)));
    for (uint32_t r = 0; r < k; ++r) {
        argmax_kernel<<<agrid, kThreads, 0, st>>>(gs, r);
        apply_kernel<<<pgrid, kThreads, 0, st>>>(gs, r);
    }
    IM_HIP(hipGetLastError());
    IM_HIP(hipMemcpyAsync(seeds_host, dseeds, 4ull * k, hipMemcpyDeviceToHost, st));
    IM_TRY(to_host_sync(ctx, cov, dcov, 8));
    return IM_OK;
}

im_status first_crossing(im_ctx *ctx, uint64_t count, uint64_t need, int64_t *index, uint64_t *hits) {
    const uint64_t tiles = (count + kTile - 1) / kTile;
    IM_TRY(dev_reserve(ctx, ctx->scan_tmp, tiles * 4 + 64));
    IM_TRY(dev_reserve(ctx, ctx->counters, 256));
    auto *tcnt = static_cast<uint32_t *>(ctx->scan_tmp.ptr);
    auto *out = reinterpret_cast<long long *>(static_cast<char *>(ctx->counters.ptr) + 160);
    hipStream_t st = ctx->stream;
    const auto *z = static_cast<const uint8_t *>(ctx->zflags.ptr);
    flag_tiles_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(z, count, tcnt);
    crossing_kernel<<<1, 1024, 0, st>>>(z, count, tcnt, tiles, need, out);
    IM_HIP(hipGetLastError());
    long long h[2];
    IM_TRY(to_host_sync(ctx, h, out, sizeof(h)));
    *index = h[0];
    *hits = static_cast<uint64_t>(h[1]);
    return IM_OK;
}

}  // namespace im
