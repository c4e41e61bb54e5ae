// Device-side building blocks: the counter-based generator, the coin
// layout that makes every RR set a pure function of (key, sample), and
// wave64 primitives.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace imd {

constexpr int kWave = 64;

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC 2011): each
// round multiplies words 0 and 2 by the two round multipliers, mixes the
// high halves with words 1 and 3 and the round key, and the key advances by
// the two Weyl constants between rounds.
struct Philox {
    static constexpr uint32_t kMulA = 0xD2511F53u;
    static constexpr uint32_t kMulB = 0xCD9E8D57u;
    static constexpr uint32_t kWeylA = 0x9E3779B9u;
    static constexpr uint32_t kWeylB = 0xBB67AE85u;

    __device__ __forceinline__ static uint4 block(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint32_t a_hi = __umulhi(kMulA, c.x);
            const uint32_t a_lo = kMulA * c.x;
            const uint32_t b_hi = __umulhi(kMulB, c.z);
            const uint32_t b_lo = kMulB * c.z;
            c = make_uint4(b_hi ^ c.y ^ k0, b_lo, a_hi ^ c.w ^ k1, a_lo);
            k0 += kWeylA;
            k1 += kWeylB;
        }
        return c;
    }
};

// Counter domains (last counter word): which decision a Philox block feeds.
constexpr uint32_t kDomSource = 0u;
constexpr uint32_t kDomIcEdge = 1u;
constexpr uint32_t kDomLtNode = 2u;
constexpr uint32_t kDomKey = 3u;
constexpr uint32_t kDomWeighted = 4u;

struct Stream {
    uint32_t k0, k1;
    __device__ __forceinline__ explicit Stream(uint64_t key)
        : k0(static_cast<uint32_t>(key)), k1(static_cast<uint32_t>(key >> 32)) {}
};

// Uniform source of sample s: high 64 bits of (64-bit draw) * n.
__device__ __forceinline__ uint32_t uniform_source(const Stream &st, uint64_t s, uint32_t n) {
    const uint4 w = Philox::block(make_uint4(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32), 0u,
                                             kDomSource),
                                  st.k0, st.k1);
    const uint64_t r = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
    return static_cast<uint32_t>(__umul64hi(r, static_cast<uint64_t>(n)));
}

// Source drawn in proportion to integer weights: cum[v] = weight of nodes
// before v (n+1 entries); the v with cum[v] <= target < cum[v+1].
__device__ __forceinline__ uint32_t weighted_source(const Stream &st, uint64_t s, const uint64_t *cum,
                                                    uint32_t n) {
    const uint4 w = Philox::block(make_uint4(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32), 0u,
                                             kDomWeighted),
                                  st.k0, st.k1);
    const uint64_t r = static_cast<uint64_t>(w.x) | (static_cast<uint64_t>(w.y) << 32);
    const uint64_t target = __umul64hi(r, cum[n]);
    uint32_t lo = 0, hi = n;  // answer in [lo, hi): largest v with cum[v] <= target
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (cum[mid] <= target) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t pick_source(const Stream &st, uint64_t s, const uint64_t *cum, uint32_t n) {
    return cum ? weighted_source(st, s, cum, n) : uniform_source(st, s, n);
}

// Four IC coins for the aligned edge group g (edges 4g .. 4g+3) of sample s.
__device__ __forceinline__ uint4 ic_coins(const Stream &st, uint64_t s, uint64_t g) {
    return Philox::block(make_uint4(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32),
                                    static_cast<uint32_t>(g), kDomIcEdge | (static_cast<uint32_t>(g >> 32) << 8)),
                         st.k0, st.k1);
}

// The LT coin of node v in sample s.
__device__ __forceinline__ uint32_t lt_coin(const Stream &st, uint64_t s, uint32_t v) {
    return Philox::block(make_uint4(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32), v, kDomLtNode),
                         st.k0, st.k1)
        .x;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &w, uint32_t i) {
    return i == 0 ? w.x : (i == 1 ? w.y : (i == 2 ? w.z : w.w));
}

// IC edge liveness: coin below the threshold; threshold 2^32-1 = always.
__device__ __forceinline__ bool ic_live(uint32_t coin, uint32_t thr) {
    return thr == 0xFFFFFFFFu || coin < thr;
}

// ---- wave64 helpers ----
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Order this wave's LDS/global accesses before what follows (lanes of one
// wave exchange data through LDS between these points).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
        if (lane >= static_cast<uint32_t>(d)) x += y;
    }
    return x;
}

// The same inclusive prefix sum with DPP row shifts inside each row of 16
// lanes, each row then adding the totals of the rows before it (read with
// v_readlane): VALU latency only, where every __shfl above is an LDS
// permute and a wait. Call it with every lane of the wave active.
__device__ __forceinline__ uint32_t wave_scan_u32(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, false));  // row_shr:1
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, false));  // row_shr:2
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, false));  // row_shr:4
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, false));  // row_shr:8
    const uint32_t r0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 15));
    const uint32_t r1 = r0 + static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 31));
    const uint32_t r2 = r1 + static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 47));
    const uint32_t row = lane_id() >> 4;
    return x + (row == 0 ? 0u : row == 1 ? r0 : row == 2 ? r1 : r2);
}

// The wave's total from an inclusive scan (its last lane).
__device__ __forceinline__ uint32_t wave_scan_total(uint32_t inc) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(inc), kWave - 1));
}

// Sum of a wave's 64-bit values: the DPP scan when every value is below
// 2^24 (the sum then fits 32 bits), else the shuffle reduction.
__device__ __forceinline__ uint64_t wave_sum_small_u64(uint64_t x) {
    if (__ballot(x >= (1ull << 24)) == 0) return wave_scan_total(wave_scan_u32(static_cast<uint32_t>(x)));
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const uint64_t y = __shfl_xor(x, d, kWave);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Block-wide exclusive prefix sum (every thread of the block calls it;
// smem holds one entry per wave); total receives the block's sum.
__device__ __forceinline__ uint64_t block_scan_excl(uint64_t x, uint64_t *smem, uint64_t &total) {
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    uint64_t inc = x;
    if (__ballot(x >= (1ull << 26)) == 0) {  // the wave's sum fits 32 bits: the DPP scan
        inc = wave_scan_u32(static_cast<uint32_t>(x));
    } else {
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint64_t y = __shfl_up(inc, d, kWave);
            if (lane >= static_cast<uint32_t>(d)) inc += y;
        }
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

__device__ __forceinline__ bool test_bit(const uint32_t *bits, uint32_t v) {
    return (bits[v >> 5] >> (v & 31u)) & 1u;
}

}  // namespace imd
