// Max-Coverage (Algorithm 2), coverage counts (Eq. 1) and the ordered
// stopping search of Estimate-Inf (Algorithm 3).
//
// Incidence (node -> sets holding it) is a counting sort of the pool range:
// a histogram of node ids, an exclusive scan, and a scatter of set ids. The
// greedy then runs k rounds of
//   argmax over unchosen v of (gain[v] << 32 | ~v)   (max gain, lowest id)
//   for each not-yet-covered set of the winner: mark covered, decrement the
//   gain of every member
// which is linear in the total size of the sets, as the paper notes. The
// argmax reads a two-level maximum index that each round patches only where
// the previous round's decrements landed; the first rounds (the largest
// covers) run as grid-wide kernels, the rest in one persistent workgroup.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

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

// 16 lanes per set: scatter the set's index into each member's list, alone
// (isets) or with the set's pool extent (iext: index, size, first member as
// two words), which spares a round the load of the extent.
template <bool kExt>
__global__ __launch_bounds__(kThreads) void scatter_kernel(const uint64_t *poff, const uint32_t *pnodes, uint64_t begin,
                                                           uint64_t nsets, const uint64_t *ioff, uint32_t *fill,
                                                           uint32_t *isets, uint4 *iext) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t j = grp; j < nsets; j += ngrp) {
        const uint64_t a = poff[begin + j], b = poff[begin + j + 1];
        for (uint64_t q = a + sub; q < b; q += 16) {
            const uint32_t v = pnodes[q];
            const uint32_t pos = atomicAdd(&fill[v], 1u);
            if constexpr (kExt)
                iext[ioff[v] + pos] = make_uint4(static_cast<uint32_t>(j), static_cast<uint32_t>(b - a),
                                                 static_cast<uint32_t>(a), static_cast<uint32_t>(a >> 32));
            else
                isets[ioff[v] + pos] = static_cast<uint32_t>(j);
        }
    }
}

// ---- greedy: two-level maximum index over node gains ----
//
// gain[v] = uncovered sets of the range holding v, bit 31 = v already chosen.
// key(v) = chosen ? 0 : gain << 32 | ~v, so the largest key is the largest
// gain with the lowest id, and keys are unique. m1[c] caches the largest key
// of nodes [64c, 64c+64), m2[d] the largest m1 of chunks [64d, 64d+64).
// Keys only fall, so a cached maximum is still right exactly when the node
// holding it still has that key; each round re-derives only the entries
// whose holder changed.

constexpr uint32_t kChosen = 0x80000000u;
constexpr uint32_t kL1Shift = 6;  // 64 nodes per m1 entry (one 256-byte line of gains)
constexpr uint32_t kL2Shift = 6;  // 64 m1 entries per m2 entry
constexpr int kPersistThreads = 1024;
constexpr uint32_t kPersistDirtyCap = 2048;     // chunks listed per round before a full refresh
constexpr uint32_t kPersistCovWords = 8192;     // covered-set bits kept in LDS (262,144 sets)
constexpr uint32_t kPersistGroupWords = 512;    // m2 entries tracked per round (n up to 2^26)

constexpr uint32_t kCandMax = 64;                       // candidate chunks at most
constexpr uint32_t kCandSlots = kCandMax << kL1Shift;   // nodes of the candidate chunks
constexpr uint32_t kCandNodes = 512;                    // candidate nodes at most
constexpr uint32_t kCandHashBits = 10;                  // LDS map node -> slot: 1024 entries
constexpr uint32_t kNoCand = 0xFFFFFFFFu;
enum : uint32_t { kStepRound = 0, kStepRefresh = 1, kStepSelect = 2, kStepDone = 3 };

// A job's step state. `thresh` bounds the key of every node outside the
// candidate chunks; `r` is the next round.
struct StepHdr {
    uint32_t phase, r, stalls, nnode;  // nnode: candidate nodes
    unsigned long long thresh;
    unsigned long long pad;
};

struct GreedyState {
    uint32_t *gain;
    unsigned long long *m1;
    unsigned long long *m2;
    uint32_t *covbits;  // covered flag per set of the range
    const uint64_t *ioff;
    const uint32_t *isets;
    const uint4 *iext;  // when set, the entries with their sets' extents (and isets is unused)
    const uint64_t *poff;
    const uint32_t *pnodes;
    uint64_t begin;
    uint32_t n, n1, n2, k;
    uint32_t *seeds;
    unsigned long long *cov;
    uint32_t *dirty;  // chunks whose m1 must be re-derived: bitmap (n1 bits), zeroed
    uint64_t nsets;   // sets in the range
    unsigned long long *bmax;  // per-round launches: each refresh block's largest key
    uint32_t nbmax;            // per-round launches: refresh blocks
    uint32_t mark;             // per-round launches: cover marks touched chunks in `dirty` (large n)
    // step launches (candidate chunks)
    struct StepHdr *hdr;  // [2]: the job's step state, by launch parity
    uint32_t *cnode;      // [kCandNodes] node of a slot
    uint32_t *cbase;      // [2][kCandNodes] candidate gains at the start of the round before
    uint32_t *cdec;       // [3][kCandNodes] drops of candidate nodes in one round
    uint32_t want;        // candidate chunks asked for
    // one-workgroup candidate rounds
    uint32_t *hist;       // [2][kSelBins] unchosen nodes per gain bin, by re-selection parity
    uint32_t *ccount;     // candidates listed
};

// Load flavours. State written by earlier kernels is read with plain loads.
// State that other waves of the same workgroup change inside the kernel (the
// persistent rounds) is read with workgroup-scope atomic loads, which skip
// the CU's L1 and hit the XCD's L2 (where the atomics landed); an L1 line
// could still hold the old value.
template <bool kWg, typename T>
__device__ __forceinline__ T ld(const T *p) {
    if constexpr (kWg) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else return *p;
}

template <bool kWg>
__device__ __forceinline__ unsigned long long node_key(const uint32_t *gain, uint32_t v) {
    const uint32_t gv = ld<kWg>(gain + v);
    return (gv & kChosen) ? 0ull : ((static_cast<unsigned long long>(gv) << 32) | static_cast<unsigned long long>(~v));
}

// Lane-local recompute of m1[c]: the chunk's 64 gains as 16 vector loads.
template <bool kWg>
__device__ __forceinline__ unsigned long long m1_lane(const GreedyState &g, uint32_t c) {
    const uint32_t a = c << kL1Shift;
    unsigned long long best = 0;
    if (a + (1u << kL1Shift) <= g.n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(g.gain + a);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            uint4 q;
            if constexpr (kWg) {
                const uint32_t *w = reinterpret_cast<const uint32_t *>(p + i);
                q = make_uint4(ld<true>(w), ld<true>(w + 1), ld<true>(w + 2), ld<true>(w + 3));
            } else {
                q = p[i];
            }
            const uint32_t gv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t v = a + 4 * i + j;
                const unsigned long long key =
                    (gv[j] & kChosen) ? 0ull
                                      : ((static_cast<unsigned long long>(gv[j]) << 32) | static_cast<unsigned long long>(~v));
                best = key > best ? key : best;
            }
        }
    } else {
        for (uint32_t v = a; v < g.n; ++v) {
            const unsigned long long key = node_key<kWg>(g.gain, v);
            best = key > best ? key : best;
        }
    }
    return best;
}

template <bool kWg>
__device__ __forceinline__ unsigned long long m2_lane(const GreedyState &g, uint32_t d) {
    const uint32_t a = d << kL2Shift;
    unsigned long long best = 0;
    if (!kWg && a + (1u << kL2Shift) <= g.n1) {
        const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(g.m1 + a);
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const ulonglong2 q = p[i];
            best = q.x > best ? q.x : best;
            best = q.y > best ? q.y : best;
        }
        return best;
    }
    const uint32_t b = min(a + (1u << kL2Shift), g.n1);
    for (uint32_t c = a; c < b; ++c) {
        const unsigned long long m = ld<kWg>(g.m1 + c);
        best = m > best ? m : best;
    }
    return best;
}

// Re-validate m1[c]: right as long as its holder still has that key.
template <bool kWg>
__device__ __forceinline__ void refresh_m1_one(const GreedyState &g, uint32_t c) {
    const unsigned long long m = ld<kWg>(g.m1 + c);
    if (m != 0ull && node_key<kWg>(g.gain, ~static_cast<uint32_t>(m)) != m) g.m1[c] = m1_lane<kWg>(g, c);
}

template <bool kWg>
__device__ __forceinline__ void refresh_m2_one(const GreedyState &g, uint32_t d) {
    const unsigned long long m = ld<kWg>(g.m2 + d);
    if (m != 0ull && ld<kWg>(g.m1 + ((~static_cast<uint32_t>(m)) >> kL1Shift)) != m) g.m2[d] = m2_lane<kWg>(g, d);
}

// Largest value over a wave with DPP row shifts (a running maximum inside
// each row of 16 lanes, then the four row maxima read with v_readlane): VALU
// latency only, where the shuffle reduction is twelve LDS permutes and waits
// for a 64-bit key. Call it with every lane of the wave active.
__device__ __forceinline__ uint32_t wave_max_u32_dpp(uint32_t x) {
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xF, 0xF, false)));
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xF, 0xF, false)));
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xF, 0xF, false)));
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xF, 0xF, false)));
    const uint32_t a = max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 15)),
                           static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 31)));
    const uint32_t b = max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 47)),
                           static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 63)));
    return max(a, b);
}

// The wave's largest 64-bit key: the largest high word, then the largest low
// word among the lanes that hold it.
__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long x) {
    const uint32_t hi = wave_max_u32_dpp(static_cast<uint32_t>(x >> 32));
    const uint32_t lo = wave_max_u32_dpp(static_cast<uint32_t>(x >> 32) == hi ? static_cast<uint32_t>(x) : 0u);
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long x, unsigned long long *smem) {
    x = wave_max_key(x);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = x;
    __syncthreads();
    unsigned long long m = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) m = smem[w] > m ? smem[w] : m;
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(kThreads) void init_m1_kernel(GreedyState g) {
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < g.n1; c += gridDim.x * blockDim.x)
        g.m1[c] = m1_lane<false>(g, c);
}

__global__ __launch_bounds__(kThreads) void init_m2_kernel(GreedyState g) {
    for (uint32_t d = blockIdx.x * blockDim.x + threadIdx.x; d < g.n2; d += gridDim.x * blockDim.x)
        g.m2[d] = m2_lane<false>(g, d);
}

// The seed of round r from m2 (all threads of one block): the argmax key's
// node, or, when every remaining gain is zero, the lowest id not yet chosen
// (at most r, since only r nodes are chosen).
// The seed of round r given the largest key `best` (all threads of one
// block). An unchosen node with no gain left still has key ~v, so when every
// gain is zero the largest key names the lowest unchosen id, as Algorithm
// 2's argmax is read here; best is 0 only if every node is chosen, which
// k <= n rules out (the scan over the chosen bits is kept for safety).
__device__ uint32_t choose_key(const GreedyState &g, uint32_t r, unsigned long long best, uint32_t *s_pick) {
    if (best == 0ull) {
        if (threadIdx.x == 0) *s_pick = 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < g.n; v += blockDim.x)
            if (!(ld<true>(g.gain + v) & kChosen)) atomicMin(s_pick, v);
    } else if (threadIdx.x == 0) {
        *s_pick = ~static_cast<uint32_t>(best & 0xFFFFFFFFull);
    }
    __syncthreads();
    const uint32_t v = *s_pick;
    __syncthreads();
    if (threadIdx.x == 0) {
        g.seeds[r] = v;
        atomicOr(&g.gain[v], kChosen);
    }
    return v;
}

// The seed of round r from m2 (all threads of one block).
template <bool kWg>
__device__ uint32_t choose(const GreedyState &g, uint32_t r, unsigned long long *smem, uint32_t *s_pick) {
    unsigned long long best = 0;
    for (uint32_t d = threadIdx.x; d < g.n2; d += blockDim.x) {
        const unsigned long long m = ld<true>(g.m2 + d);
        best = m > best ? m : best;
    }
    best = block_max_u64(best, smem);
    return choose_key(g, r, best, s_pick);
}

// Round step 1 body (grid-wide over one job's blocks): re-derive stale m1
// entries and record each block's largest key in bmax[blk]. No block waits
// for another: the next launch reads bmax.
__device__ __forceinline__ void refresh_block(const GreedyState &g, uint32_t r, uint32_t blk, uint32_t nblk,
                                              unsigned long long *smem) {
    unsigned long long best = 0;
    // A wave takes 64 consecutive chunks (one m2 group) at a time. 32
    // consecutive chunks share a dirty word and are read by 32 consecutive
    // lanes; the word's first lane clears it once it has the value.
    const uint32_t lane = lane_id();
    for (uint32_t c0 = blk * blockDim.x + (threadIdx.x - lane); c0 < g.n1; c0 += nblk * blockDim.x) {
        const uint32_t c = c0 + lane;
        unsigned long long m = 0;
        if (c < g.n1) {
            m = g.m1[c];
            if (r > 0 && g.mark) {
                // re-derive the chunks whose nodes lost gain
                const uint32_t word = g.dirty[c >> 5];
                if ((word >> (c & 31u)) & 1u) {
                    m = m1_lane<false>(g, c);
                    g.m1[c] = m;
                }
                if ((c & 31u) == 0 && word != 0u) g.dirty[c >> 5] = 0u;
            } else if (r > 0 && m != 0ull && node_key<false>(g.gain, ~static_cast<uint32_t>(m)) != m) {
                // re-derive the chunks whose maximum holder lost gain
                m = m1_lane<false>(g, c);
                g.m1[c] = m;
            }
        }
        best = m > best ? m : best;
        const unsigned long long gm = wave_max_key(m);
        if (lane == 0) g.m2[c0 >> kL2Shift] = gm;
    }
    best = block_max_u64(best, smem);
    if (threadIdx.x == 0) g.bmax[blk] = best;
}

struct RoundLds;
template <bool kCand>
__device__ void cover_seed(const GreedyState &g, uint32_t r, uint32_t v, uint32_t blk, uint32_t nblk, uint32_t nnode,
                           RoundLds *L);

// Round step 2 body (grid-wide over one job's blocks): every block takes the
// largest of the refresh blocks' maxima, so all agree on seed r without
// waiting for one another; block 0 records it. Then the seed's sets are
// covered, 16 lanes per incidence entry.
__device__ __forceinline__ void cover_block(const GreedyState &g, uint32_t r, uint32_t blk, uint32_t nblk,
                                            unsigned long long *smem, uint32_t *s_pick) {
    unsigned long long best = 0;
    for (uint32_t i = threadIdx.x; i < g.nbmax; i += blockDim.x) {
        const unsigned long long m = g.bmax[i];
        best = m > best ? m : best;
    }
    best = block_max_u64(best, smem);
    if (best == 0ull) {  // every node chosen: cannot happen for k <= n, kept for safety
        if (threadIdx.x == 0) *s_pick = 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t v = threadIdx.x; v < g.n; v += blockDim.x)
            if (!(g.gain[v] & kChosen)) atomicMin(s_pick, v);
    } else if (threadIdx.x == 0) {
        *s_pick = ~static_cast<uint32_t>(best & 0xFFFFFFFFull);
    }
    __syncthreads();
    const uint32_t v = *s_pick;
    if (blk == 0 && threadIdx.x == 0) {
        g.seeds[r] = v;
        atomicOr(&g.gain[v], kChosen);
        const uint32_t c = v >> kL1Shift;
        if (g.mark) atomicOr(&g.dirty[c >> 5], 1u << (c & 31u));  // the seed's key is now 0
    }
    cover_seed<false>(g, r, v, blk, nblk, 0u, nullptr);
}

// LDS of a candidate round: the candidate nodes' slots by node id (open
// addressing) and the drops this block gives each slot.
struct RoundLds {
    uint32_t key[1u << kCandHashBits];
    uint32_t slot[1u << kCandHashBits];
    uint32_t dec[kCandNodes];
};

__device__ __forceinline__ uint32_t cand_slot(const RoundLds &L, uint32_t u) {
    constexpr uint32_t kMask = (1u << kCandHashBits) - 1u;
    uint32_t h = (u * 2654435761u) >> (32 - kCandHashBits);
    for (uint32_t p = 0; p <= kMask; ++p) {
        const uint32_t k = L.key[h];
        if (k == u) return L.slot[h];
        if (k == kNoCand) break;
        h = (h + 1u) & kMask;
    }
    return kNoCand;
}

// Cover seed v of round r (grid-wide over one job's blocks): every set
// holding v not covered yet is marked, and each member's gain drops by one,
// 16 lanes per incidence entry. With candidates (L holds their slots by node
// and zeroed counts), the drops of candidate nodes (the nodes most sets
// share) are summed in LDS per block and applied once per node at the end,
// to the gain and to the round's dec buffer.
template <bool kCand>
__device__ void cover_seed(const GreedyState &g, uint32_t r, uint32_t v, uint32_t blk, uint32_t nblk, uint32_t nnode,
                           RoundLds *L) {
    const uint64_t a = g.ioff[v], b = g.ioff[v + 1];
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blk) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(nblk) * blockDim.x) >> 4;
    unsigned long long newly = 0;
    for (uint64_t i = a + grp; i < b; i += ngrp) {
        uint32_t j;
        uint64_t sa, sb;
        if (g.iext) {
            const uint4 x = g.iext[i];
            j = x.x;
            sa = static_cast<uint64_t>(x.z) | (static_cast<uint64_t>(x.w) << 32);
            sb = sa + x.y;
        } else {
            j = g.isets[i];
            sa = g.poff[g.begin + j];
            sb = g.poff[g.begin + j + 1];
        }
        // the set's extent, its covered flag and its first members are in
        // flight together; the flag decides whether they are used
        const uint32_t u0 = sa + sub < sb ? g.pnodes[sa + sub] : 0u;
        const uint32_t bit = 1u << (j & 31u);
        uint32_t prior = bit;
        if (sub == 0) prior = atomicOr(&g.covbits[j >> 5], bit);
        const uint32_t fresh = __shfl((prior & bit) ? 0u : 1u, static_cast<int>(lane_id() & ~15u), kWave);
        if (fresh) {
            if (sub == 0) ++newly;
            for (uint64_t q = sa + sub; q < sb; q += 16) {
                const uint32_t u = q == sa + sub ? u0 : g.pnodes[q];
                const uint32_t c = u >> kL1Shift;
                bool direct = true;
                if constexpr (kCand) {
                    const uint32_t slot = cand_slot(*L, u);
                    if (slot != kNoCand) {
                        atomicAdd(&L->dec[slot], 1u);
                        direct = false;
                    }
                }
                if (direct) {
                    atomicSub(&g.gain[u], 1u);
                    if (g.mark) atomicOr(&g.dirty[c >> 5], 1u << (c & 31u));
                }
            }
        }
    }
    newly = wave_sum_u64(newly);
    if (lane_id() == 0 && newly) atomicAdd(g.cov, newly);
    if constexpr (kCand) {
        __syncthreads();
        uint32_t *dec = g.cdec + (r % 3u) * kCandNodes;
        for (uint32_t i = threadIdx.x; i < nnode; i += blockDim.x) {
            const uint32_t d = L->dec[i];
            if (d) {
                const uint32_t u = g.cnode[i];
                const uint32_t c = u >> kL1Shift;
                atomicSub(&g.gain[u], d);
                atomicAdd(&dec[i], d);
                if (g.mark) atomicOr(&g.dirty[c >> 5], 1u << (c & 31u));
            }
        }
    }
}

// Round r, step 1 (grid-wide).
__global__ __launch_bounds__(kThreads) void refresh_kernel(GreedyState g, uint32_t r) {
    __shared__ unsigned long long smem[kThreads / kWave];
    refresh_block(g, r, blockIdx.x, gridDim.x, smem);
}

// Round r, step 2 (grid-wide).
__global__ __launch_bounds__(kThreads) void cover_kernel(GreedyState g, uint32_t r) {
    __shared__ unsigned long long smem[kThreads / kWave];
    __shared__ uint32_t s_pick;
    cover_block(g, r, blockIdx.x, gridDim.x, smem, &s_pick);
}

// Batched rounds: blockIdx.y is the job; jobs whose k is reached idle.
__global__ __launch_bounds__(kThreads) void batch_refresh_kernel(const GreedyState *jobs, uint32_t r) {
    __shared__ unsigned long long smem[kThreads / kWave];
    const GreedyState &g = jobs[blockIdx.y];
    if (r >= g.k) return;
    refresh_block(g, r, blockIdx.x, gridDim.x, smem);
}

__global__ __launch_bounds__(kThreads) void batch_cover_kernel(const GreedyState *jobs, uint32_t r) {
    __shared__ unsigned long long smem[kThreads / kWave];
    __shared__ uint32_t s_pick;
    const GreedyState &g = jobs[blockIdx.y];
    if (r >= g.k) return;
    cover_block(g, r, blockIdx.x, gridDim.x, smem, &s_pick);
}

// ---- greedy rounds as steps over candidate chunks ----
//
// Keys only fall. So if C is a set of chunks and thresh bounds the key of
// every node outside C (the largest m1 outside C when C was picked), then
// while the largest current key inside C exceeds thresh it is the argmax
// over all nodes, and a round needs no grid-wide maximum: every block reads
// the candidate nodes' gains and all reach the same seed. Those gains come
// from buffers no block of the same launch writes:
//   gain at the start of round r = cbase[r & 1] - cdec[(r - 1) % 3]
// where cbase[r & 1] holds the gains at the start of round r - 1 and
// cdec[q % 3] the drops round q gave candidate nodes. Round r writes
// cbase[(r + 1) & 1] (adding its seed's chosen bit), clears cdec[(r + 1) % 3]
// for round r + 1 and counts its own drops in cdec[r % 3]. When the test
// fails the job re-derives m1 and picks new candidates. Each launch moves
// every job one step:
//   REFRESH -> SELECT -> ROUND ... ROUND [-> REFRESH -> SELECT -> ROUND ...]
// and the step state is kept twice, by launch parity, so the blocks of a
// launch read what the previous launch left.

struct SelectLds {
    uint32_t hist[kThreads];
    uint64_t scan[kThreads / kWave];
    uint32_t list[kCandSlots];  // chunks, then node positions (chunk index << 6 | node bit)
    uint32_t groups[kCandMax + 1];
    uint32_t cand[kCandMax];
    unsigned long long mask[kCandMax];
    uint32_t start[kCandMax];
    uint32_t ngroups, nlist, ncand, nnode, bin;
    uint64_t above;
};

// The rank-th largest (1-based, counting repeats) of count keys get(i), by
// eight 8-bit passes from the top byte; 0 when count < rank. All threads of
// one 256-thread block.
template <typename Get>
__device__ unsigned long long block_kth_largest(Get get, uint32_t count, uint32_t rank, SelectLds &L) {
    if (count < rank) return 0ull;
    const uint32_t tid = threadIdx.x;
    unsigned long long prefix = 0, mask = 0;
    uint32_t need = rank;
    for (int shift = 56; shift >= 0; shift -= 8) {
        L.hist[tid] = 0u;
        __syncthreads();
        for (uint32_t i = tid; i < count; i += blockDim.x) {
            const unsigned long long x = get(i);
            if ((x & mask) == prefix) atomicAdd(&L.hist[(x >> shift) & 255u], 1u);
        }
        __syncthreads();
        // thread t holds bin 255 - t, so the scan counts the larger bins first
        const uint32_t bin = 255u - tid;
        const uint64_t h = L.hist[bin];
        uint64_t total = 0;
        const uint64_t above = block_scan_excl(h, L.scan, total);
        if (above < need && need <= above + h) {
            L.bin = bin;
            L.above = above;
        }
        __syncthreads();
        prefix |= static_cast<unsigned long long>(L.bin) << shift;
        mask |= 0xFFull << shift;
        need -= static_cast<uint32_t>(L.above);
        __syncthreads();
    }
    return prefix;
}

// Log-scale bin of a gain >= 1: eight bins per power of two, 1..255,
// non-decreasing in the gain.
__device__ __forceinline__ uint32_t gain_bin(uint32_t gain) {
    const uint32_t lz = 31u - static_cast<uint32_t>(__clz(gain));
    const uint32_t frac = lz >= 3u ? (gain >> (lz - 3u)) & 7u : (gain << (3u - lz)) & 7u;
    return min(255u, 1u + 8u * lz + frac);
}

// A threshold t = (gain_t << 32 | 0xFFFFFFFF) keeping as many of the count
// keys get(i) above it as whole gain bins allow without passing cap (keys
// above t are exactly those with gain above gain_t). ok is false when no key
// has a gain or the top bin alone holds more than cap keys. Two passes and a
// scan; all threads of one 256-thread block.
template <typename Get>
__device__ unsigned long long block_gain_cut(Get get, uint32_t count, uint32_t cap, SelectLds &L, bool &ok) {
    const uint32_t tid = threadIdx.x;
    L.hist[tid] = 0u;
    if (tid == 0) L.bin = kNoCand;
    __syncthreads();
    for (uint32_t i = tid; i < count; i += blockDim.x) {
        const uint32_t gain = static_cast<uint32_t>(get(i) >> 32);
        if (gain) atomicAdd(&L.hist[gain_bin(gain)], 1u);
    }
    __syncthreads();
    const uint32_t bin = 255u - tid;
    const uint64_t h = L.hist[bin];
    uint64_t total = 0;
    const uint64_t above = block_scan_excl(h, L.scan, total);
    // the lowest bin whose keys, with those of the bins above, fit in cap
    if (bin >= 1u && above + h <= cap && above + h > 0) atomicMin(&L.bin, bin);
    __syncthreads();
    const uint32_t cut = L.bin;
    ok = cut != kNoCand;
    if (!ok) return 0ull;
    unsigned long long below = 0;
    for (uint32_t i = tid; i < count; i += blockDim.x) {
        const uint32_t gain = static_cast<uint32_t>(get(i) >> 32);
        if (gain && gain_bin(gain) < cut && gain > below) below = gain;
    }
    below = block_max_u64(below, reinterpret_cast<unsigned long long *>(L.scan));
    return (below << 32) | 0xFFFFFFFFull;
}

// SELECT (block 0 of the job), from the refreshed m1 and the group maxima
// m2. Chunks: those whose maximum beats the (want+1)-th largest group
// maximum t0 (they lie in the `want` leading groups); if more than kCandMax
// qualify, the `want` largest, with the threshold raised to the next one.
// Nodes: those of the chosen chunks whose key beats the threshold; if more
// than kCandNodes, the kCandNodes largest, raising the threshold again.
// Every node left out has a key at most the threshold. Then the
// candidates' gains are copied for round h.r.
__device__ void step_select(const GreedyState &g, const StepHdr &h, StepHdr *out, SelectLds &L) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        L.ngroups = 0;
        L.nlist = 0;
        L.ncand = 0;
        L.nnode = 0;
    }
    if (tid < kCandMax) L.mask[tid] = 0ull;
    __syncthreads();
    // thresholds come from gain bins, or exactly by rank when bins cannot split
    bool ok = false;
    auto group_key = [&](uint32_t i) { return g.m2[i]; };
    unsigned long long t0 = block_gain_cut(group_key, g.n2, g.want, L, ok);
    if (!ok) t0 = block_kth_largest(group_key, g.n2, g.want + 1u, L);
    for (uint32_t d = tid; d < g.n2; d += blockDim.x)
        if (g.m2[d] > t0) L.groups[atomicAdd(&L.ngroups, 1u)] = d;
    __syncthreads();
    const uint32_t ng = L.ngroups;
    for (uint32_t i = tid; i < (ng << kL2Shift); i += blockDim.x) {
        const uint32_t c = (L.groups[i >> kL2Shift] << kL2Shift) | (i & 63u);
        if (c < g.n1 && g.m1[c] > t0) L.list[atomicAdd(&L.nlist, 1u)] = c;
    }
    __syncthreads();
    const uint32_t nl = L.nlist;
    unsigned long long thresh = t0;
    if (nl > kCandMax) {
        auto chunk_key = [&](uint32_t i) { return g.m1[L.list[i]]; };
        unsigned long long t1 = block_gain_cut(chunk_key, nl, kCandMax, L, ok);
        if (!ok) t1 = block_kth_largest(chunk_key, nl, kCandMax + 1u, L);
        thresh = t1 > thresh ? t1 : thresh;
    }
    for (uint32_t i = tid; i < nl; i += blockDim.x) {
        const uint32_t c = L.list[i];
        if (g.m1[c] > thresh) L.cand[atomicAdd(&L.ncand, 1u)] = c;
    }
    __syncthreads();
    const uint32_t nc = L.ncand;
    // nodes of the chosen chunks above the threshold
    for (uint32_t i = tid; i < (nc << kL1Shift); i += blockDim.x) {
        const uint32_t v = (L.cand[i >> kL1Shift] << kL1Shift) | (i & 63u);
        if (v < g.n && node_key<false>(g.gain, v) > thresh) L.list[atomicAdd(&L.nnode, 1u)] = i;
    }
    __syncthreads();
    const uint32_t nn = L.nnode;
    auto key_at = [&](uint32_t idx) {
        const uint32_t i = L.list[idx];
        return node_key<false>(g.gain, (L.cand[i >> kL1Shift] << kL1Shift) | (i & 63u));
    };
    if (nn > kCandNodes) {
        unsigned long long t2 = block_gain_cut(key_at, nn, kCandNodes, L, ok);
        if (!ok) t2 = block_kth_largest(key_at, nn, kCandNodes + 1u, L);
        thresh = t2 > thresh ? t2 : thresh;
    }
    for (uint32_t idx = tid; idx < nn; idx += blockDim.x) {
        const uint32_t i = L.list[idx];
        if (key_at(idx) > thresh) atomicOr(&L.mask[i >> kL1Shift], 1ull << (i & 63u));
    }
    __syncthreads();
    // slots follow chunk order, then bit order
    if (tid < kWave) {
        const uint64_t cnt = tid < nc ? static_cast<uint64_t>(__popcll(L.mask[tid])) : 0ull;
        uint64_t inc = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint64_t y = __shfl_up(inc, d, kWave);
            if (tid >= static_cast<uint32_t>(d)) inc += y;
        }
        L.start[tid] = static_cast<uint32_t>(inc - cnt);
        if (tid == kWave - 1) L.nnode = static_cast<uint32_t>(inc);
    }
    __syncthreads();
    const uint32_t slots = L.nnode;
    uint32_t *base = g.cbase + (h.r & 1u) * kCandNodes;
    uint32_t *dec_prev = g.cdec + ((h.r + 2u) % 3u) * kCandNodes;
    uint32_t *dec_cur = g.cdec + (h.r % 3u) * kCandNodes;
    for (uint32_t i = tid; i < (nc << kL1Shift); i += blockDim.x) {
        const uint32_t ci = i >> kL1Shift, j = i & 63u;
        const unsigned long long m = L.mask[ci];
        if ((m >> j) & 1ull) {
            const uint32_t slot = L.start[ci] + static_cast<uint32_t>(__popcll(m & ((1ull << j) - 1ull)));
            const uint32_t v = (L.cand[ci] << kL1Shift) | j;
            g.cnode[slot] = v;
            base[slot] = g.gain[v];
            dec_prev[slot] = 0u;
            dec_cur[slot] = 0u;
        }
    }
    if (tid == 0) {
        StepHdr o = h;
        o.phase = kStepRound;
        o.nnode = slots;
        o.thresh = thresh;
        *out = o;
    }
}

// ROUND (grid-wide over one job's blocks).
__device__ void step_round(const GreedyState &g, const StepHdr &h, StepHdr *out, uint32_t blk, uint32_t nblk,
                           unsigned long long *smem, RoundLds &L) {
    const uint32_t r = h.r;
    const uint32_t nn = h.nnode;
    const uint32_t *base = g.cbase + (r & 1u) * kCandNodes;
    const uint32_t *dec_prev = g.cdec + ((r + 2u) % 3u) * kCandNodes;
    constexpr uint32_t kMask = (1u << kCandHashBits) - 1u;
    for (uint32_t i = threadIdx.x; i <= kMask; i += blockDim.x) L.key[i] = kNoCand;
    for (uint32_t i = threadIdx.x; i < nn; i += blockDim.x) L.dec[i] = 0u;
    __syncthreads();
    // the largest candidate key; the candidates' slots go into the LDS map
    unsigned long long best = 0;
    for (uint32_t s = threadIdx.x; s < nn; s += blockDim.x) {
        const uint32_t x = base[s] - dec_prev[s];
        const uint32_t u = g.cnode[s];
        uint32_t hh = (u * 2654435761u) >> (32 - kCandHashBits);
        for (uint32_t p = 0; p <= kMask; ++p) {
            if (atomicCAS(&L.key[hh], kNoCand, u) == kNoCand) {
                L.slot[hh] = s;
                break;
            }
            hh = (hh + 1u) & kMask;
        }
        if (!(x & kChosen)) {
            const unsigned long long key = (static_cast<unsigned long long>(x) << 32) | static_cast<unsigned long long>(~u);
            best = key > best ? key : best;
        }
    }
    best = block_max_u64(best, smem);  // its barriers also publish the map
    if (best <= h.thresh) {
        // a node outside the candidates may lead now: refresh and re-select
        if (blk == 0 && threadIdx.x == 0) {
            StepHdr o = h;
            o.phase = kStepRefresh;
            ++o.stalls;
            *out = o;
        }
        return;
    }
    const uint32_t v = ~static_cast<uint32_t>(best & 0xFFFFFFFFull);
    uint32_t *base_next = g.cbase + ((r + 1u) & 1u) * kCandNodes;
    uint32_t *dec_next = g.cdec + ((r + 1u) % 3u) * kCandNodes;
    for (uint32_t s = blk * blockDim.x + threadIdx.x; s < nn; s += nblk * blockDim.x) {
        base_next[s] = (base[s] - dec_prev[s]) | (g.cnode[s] == v ? kChosen : 0u);
        dec_next[s] = 0u;
    }
    if (blk == 0 && threadIdx.x == 0) {
        g.seeds[r] = v;
        atomicOr(&g.gain[v], kChosen);
        const uint32_t c = v >> kL1Shift;
        if (g.mark) atomicOr(&g.dirty[c >> 5], 1u << (c & 31u));
        StepHdr o = h;
        o.r = r + 1u;
        o.phase = r + 1u >= g.k ? kStepDone : kStepRound;
        *out = o;
    }
    cover_seed<true>(g, r, v, blk, nblk, nn, &L);
}

// One step of every job (blockIdx.y = job). REFRESH uses the first nbmax
// blocks of a job, SELECT its block 0, ROUND all of them.
__global__ __launch_bounds__(kThreads) void greedy_step_kernel(const GreedyState *jobs, uint32_t step) {
    __shared__ unsigned long long smem[kThreads / kWave];
    __shared__ union {
        SelectLds sel;
        RoundLds rnd;
    } lds;
    const GreedyState &g = jobs[blockIdx.y];
    const StepHdr h = g.hdr[step & 1u];
    StepHdr *out = g.hdr + ((step + 1u) & 1u);
    const uint32_t blk = blockIdx.x, nblk = gridDim.x;
    if (h.phase == kStepRound) {
        step_round(g, h, out, blk, nblk, smem, lds.rnd);
    } else if (h.phase == kStepRefresh) {
        if (blk < g.nbmax) refresh_block(g, h.r, blk, g.nbmax, smem);
        if (blk == 0 && threadIdx.x == 0) {
            StepHdr o = h;
            o.phase = kStepSelect;
            *out = o;
        }
    } else if (h.phase == kStepSelect) {
        if (blk == 0) step_select(g, h, out, lds.sel);
    } else if (blk == 0 && threadIdx.x == 0) {
        *out = h;
    }
}

// LDS of the one-workgroup rounds.
struct PersistLds {
    unsigned long long smem[kPersistThreads / kWave];
    uint64_t scan[kPersistThreads / kWave];
    uint64_t start[kPersistThreads];
    uint64_t pre[kPersistThreads];
    uint32_t dlist[kPersistDirtyCap];
    uint32_t groups[kPersistGroupWords];
    uint32_t cov[kPersistCovWords];
    uint32_t pick, dcount, dall;
};

// Rounds [r0, k) of one job in one workgroup. Each round chooses from m2,
// covers the winner's sets (the newly covered sets' members are decremented
// 1024 at a time, located through a block scan of the set sizes) and notes
// the chunks whose maximum holder lost gain; only those m1 entries, and the
// m2 entries above them, are re-derived before the next choice (all of them
// when more than kPersistDirtyCap chunks were hit). Covered-set bits live in
// LDS when the range is small enough.
template <bool kLdsCov>
__device__ void persist_rounds(const GreedyState &g, uint32_t r0, PersistLds &L) {
    const uint32_t tid = threadIdx.x;
    uint32_t *covbits = kLdsCov ? L.cov : g.covbits;
    const bool track = g.n2 <= kPersistGroupWords * 32;
    for (uint32_t w = tid; w < kPersistGroupWords; w += blockDim.x) L.groups[w] = 0u;
    if (tid == 0) {
        L.dcount = 0;
        L.dall = 0;
    }
    __syncthreads();
    // chunk c must be re-derived before the next choice
    auto mark = [&](uint32_t c) {
        const uint32_t bit = 1u << (c & 31u);
        if (!(atomicOr(&g.dirty[c >> 5], bit) & bit)) {
            const uint32_t slot = atomicAdd(&L.dcount, 1u);
            if (slot < kPersistDirtyCap) L.dlist[slot] = c;
            else L.dall = 1u;
        }
    };
    unsigned long long newly = 0;
    for (uint32_t r = r0; r < g.k; ++r) {
        if (r > r0) {
            __syncthreads();
            const uint32_t nd = L.dcount;
            const bool all = L.dall != 0;
            if (all) {
                for (uint32_t c = tid; c < g.n1; c += blockDim.x) {
                    g.m1[c] = m1_lane<true>(g, c);
                    if ((c & 31u) == 0) atomicAnd(&g.dirty[c >> 5], 0u);
                }
            } else {
                for (uint32_t i = tid; i < nd; i += blockDim.x) {
                    const uint32_t c = L.dlist[i];
                    g.m1[c] = m1_lane<true>(g, c);
                    atomicAnd(&g.dirty[c >> 5], ~(1u << (c & 31u)));
                    const uint32_t d = c >> kL2Shift;
                    if (track) atomicOr(&L.groups[d >> 5], 1u << (d & 31u));
                }
            }
            __threadfence_block();
            __syncthreads();
            const bool every = all || !track;
            for (uint32_t d = tid; d < g.n2; d += blockDim.x)
                if (every || ((L.groups[d >> 5] >> (d & 31u)) & 1u)) g.m2[d] = m2_lane<true>(g, d);
            __threadfence_block();
            __syncthreads();
            for (uint32_t w = tid; w < kPersistGroupWords; w += blockDim.x) L.groups[w] = 0u;
            if (tid == 0) {
                L.dcount = 0;
                L.dall = 0;
            }
            __syncthreads();
        }
        const uint32_t v = choose<true>(g, r, L.smem, &L.pick);
        if (tid == 0) mark(v >> kL1Shift);
        const uint64_t a = g.ioff[v], b = g.ioff[v + 1];
        for (uint64_t base = a; base < b; base += blockDim.x) {
            const uint64_t i = base + tid;
            uint64_t size = 0, start = 0;
            if (i < b) {
                const uint32_t j = g.isets[i];
                const uint32_t bit = 1u << (j & 31u);
                if (!(atomicOr(&covbits[j >> 5], bit) & bit)) {
                    start = g.poff[g.begin + j];
                    size = g.poff[g.begin + j + 1] - start;
                    ++newly;
                }
            }
            uint64_t members = 0;
            const uint64_t pre = block_scan_excl(size, L.scan, members);
            L.start[tid] = start;
            L.pre[tid] = pre;
            __syncthreads();
            for (uint64_t idx = tid; idx < members; idx += blockDim.x) {
                // the last slot whose prefix is <= idx owns member idx
                uint32_t lo = 0, hi = kPersistThreads - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) >> 1;
                    if (L.pre[mid] <= idx) lo = mid;
                    else hi = mid - 1;
                }
                const uint32_t u = g.pnodes[L.start[lo] + (idx - L.pre[lo])];
                const uint32_t c = u >> kL1Shift;
                const unsigned long long m = ld<true>(g.m1 + c);
                atomicSub(&g.gain[u], 1u);
                if (static_cast<uint32_t>(~m) == u) mark(c);
            }
            __syncthreads();
        }
    }
    newly = wave_sum_u64(newly);
    if (lane_id() == 0 && newly) atomicAdd(g.cov, newly);
}

// Job blockIdx.x, rounds [r0, k).
__global__ __launch_bounds__(kPersistThreads) void persist_kernel(const GreedyState *jobs, uint32_t r0) {
    __shared__ PersistLds L;
    const GreedyState g = jobs[blockIdx.x];
    const uint64_t words = (g.nsets + 31) / 32;
    if (r0 == 0 && words <= kPersistCovWords) {
        for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) L.cov[w] = 0u;
        __syncthreads();
        persist_rounds<true>(g, r0, L);
    } else {
        persist_rounds<false>(g, r0, L);
    }
}

// ---- rounds in one workgroup over candidate nodes ----
//
// The same candidate rule as the step launches (keys only fall, so the
// largest candidate key is the argmax while it beats a bound on every other
// node's key), with all the rounds of one candidate set inside one
// workgroup. Only the candidates' gains are kept current, in LDS: covering a
// set walks its members and drops the ones that are candidates. The other
// nodes' global gains go stale, so when the test fails the grid recounts
// every gain from the covered-set bits (clear, recount), bins the gains
// (hist), finds the bin cut that keeps at most kCandNodes nodes (cut) and
// lists them (collect). Between re-selections a round costs its own chain of
// loads and no launch. Every launch reads the job's header and does nothing
// unless the header is in its phase, so the host can queue cycles ahead.

constexpr int kWgThreads = 1024;
constexpr uint32_t kWgCovWords = 8192;  // covered-set bits kept in LDS (262,144 sets)
constexpr uint32_t kStepCollect = 4;     // header phase: candidates listed under thresh
constexpr uint32_t kStepGrid = 5;        // header phase: the remaining rounds go to the grid-wide path
constexpr uint32_t kStepZero = 6;        // header phase: every unchosen gain is zero
constexpr uint32_t kWgMinCand = 64;      // fewer candidates than this (and than rounds left): grid rounds
constexpr uint32_t kSelExact = 2048;     // gains below this have a bin of their own
constexpr uint32_t kSelBins = kSelExact + 8 * 20;  // then eight bins per power of two, up to 2^31

// Bin of a gain in [1, 2^31), non-decreasing in the gain.
__device__ __forceinline__ uint32_t sel_bin(uint32_t gain) {
    if (gain < kSelExact) return gain;
    const uint32_t lz = 31u - static_cast<uint32_t>(__clz(gain));  // 11..30
    return kSelExact + 8u * (lz - 11u) + ((gain >> (lz - 3u)) & 7u);
}

// The smallest gain of bin b >= 1.
__device__ __forceinline__ uint32_t sel_bin_low(uint32_t b) {
    if (b < kSelExact) return b;
    const uint32_t q = b - kSelExact, lz = 11u + q / 8u;
    return (8u + (q & 7u)) << (lz - 3u);
}

constexpr uint32_t kWgFilterShift = 16;  // candidate filter: 2^16 bits, one per hash value

__device__ __forceinline__ uint32_t wg_filter_bit(uint32_t u) { return (u * 2654435761u) >> (32 - kWgFilterShift); }

struct WgLds {
    unsigned long long smem[kWgThreads / kWave];
    uint32_t filter[(1u << kWgFilterShift) / 32];  // set for every candidate's hash value
    uint32_t key[1u << kCandHashBits];
    uint16_t slot[1u << kCandHashBits];
    uint32_t node[kCandNodes];
    uint32_t cg[kCandNodes];      // candidate gains, bit 31 = chosen
    uint64_t ia[kCandNodes];      // candidate's first incidence entry
    uint32_t ilen[kCandNodes];    // and entry count
    uint64_t fstart[kWgThreads];  // newly covered sets of one batch of entries: first member
    uint32_t fsize[kWgThreads];   // and size
    uint32_t cov[kWgCovWords];
    uint32_t nfresh[2];  // newly covered sets of a batch, by batch parity
};

__device__ __forceinline__ uint32_t wg_slot(const WgLds &L, uint32_t u) {
    constexpr uint32_t kMask = (1u << kCandHashBits) - 1u;
    uint32_t h = (u * 2654435761u) >> (32 - kCandHashBits);
    for (uint32_t p = 0; p <= kMask; ++p) {
        const uint32_t k = L.key[h];
        if (k == u) return L.slot[h];
        if (k == kNoCand) break;
        h = (h + 1u) & kMask;
    }
    return kNoCand;
}

// Pointers the compiler knows to be global: their loads and atomics become
// global instructions rather than flat ones, which also count against the
// LDS wait counter and so make every LDS wait also wait for them.
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u32 gconst_u4;
typedef __attribute__((address_space(1))) const uint32_t gconst_u32;
typedef __attribute__((address_space(1))) uint32_t gmem_u32;

template <bool kLdsCov>
__device__ void wg_rounds(const GreedyState &g, const StepHdr &h, uint64_t words, WgLds &L) {
    constexpr uint32_t kMask = (1u << kCandHashBits) - 1u;
    const uint32_t tid = threadIdx.x, bd = blockDim.x;
    const gconst_u4 *iext = (const gconst_u4 *)g.iext;
    const gconst_u32 *pnodes = (const gconst_u32 *)g.pnodes;
    gmem_u32 *gcov = (gmem_u32 *)g.covbits;
    gmem_u32 *gseeds = (gmem_u32 *)g.seeds;
    gmem_u32 *ggain = (gmem_u32 *)g.gain;
    if constexpr (kLdsCov)
        for (uint64_t w = tid; w < words; w += bd) L.cov[w] = g.covbits[w];
    for (uint32_t i = tid; i <= kMask; i += bd) L.key[i] = kNoCand;
    for (uint32_t i = tid; i < (1u << kWgFilterShift) / 32; i += bd) L.filter[i] = 0u;
    if (tid < 2) L.nfresh[tid] = 0u;
    uint32_t bp = 0;
    __syncthreads();
    const uint32_t nn = min(*g.ccount, kCandNodes);
    for (uint32_t s = tid; s < nn; s += bd) {
        const uint32_t u = g.cnode[s];
        const uint32_t fb = wg_filter_bit(u);
        atomicOr(&L.filter[fb >> 5], 1u << (fb & 31u));
        L.node[s] = u;
        L.cg[s] = g.cbase[s];
        const uint64_t ia = g.ioff[u];
        L.ia[s] = ia;
        L.ilen[s] = static_cast<uint32_t>(g.ioff[u + 1] - ia);
        uint32_t hh = (u * 2654435761u) >> (32 - kCandHashBits);
        for (uint32_t q = 0; q <= kMask; ++q) {
            if (atomicCAS(&L.key[hh], kNoCand, u) == kNoCand) {
                L.slot[hh] = static_cast<uint16_t>(s);
                break;
            }
            hh = (hh + 1u) & kMask;
        }
    }
    __syncthreads();
    unsigned long long newly = 0;
    uint32_t r = h.r;
    bool stalled = false;
    const uint32_t grp = tid >> 4, sub = tid & 15u, ngrp = bd >> 4;
    const uint32_t lane = lane_id();
    for (; r < g.k; ++r) {
        // every wave finds the largest candidate key itself (they all read
        // the same LDS, so they agree) and, from the lane holding it, its slot
        unsigned long long best = 0;
        uint32_t bslot = kNoCand;
        for (uint32_t s = lane; s < nn; s += kWave) {
            const uint32_t x = L.cg[s];
            if (!(x & kChosen)) {
                const unsigned long long key = (static_cast<unsigned long long>(x) << 32) | static_cast<unsigned long long>(~L.node[s]);
                if (key > best) {
                    best = key;
                    bslot = s;
                }
            }
        }
        const unsigned long long wbest = wave_max_key(best);
        if (wbest <= h.thresh) {  // the same value in every wave
            stalled = true;
            break;
        }
        const unsigned long long holder = __ballot(best == wbest);
        const uint32_t sv = static_cast<uint32_t>(
            __builtin_amdgcn_readlane(static_cast<int>(bslot), static_cast<int>(__ffsll(holder)) - 1));
        const uint32_t v = ~static_cast<uint32_t>(wbest & 0xFFFFFFFFull);
        if (tid == 0) {
            gseeds[r] = v;
            __hip_atomic_fetch_or(&ggain[v], kChosen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint64_t a = L.ia[sv], b = a + L.ilen[sv];
        if (a == b) {  // v is in no set (every gain left is zero): only its chosen bit
            __syncthreads();
            if (tid == 0) L.cg[sv] |= kChosen;
            __syncthreads();
            continue;
        }
        // cover v's sets, one batch of incidence entries at a time: first the
        // newly covered sets are listed, then 16 lanes walk each one's members
        for (uint64_t e0 = a; e0 < b; e0 += bd, bp ^= 1u) {
            // the count of this batch (parity bp) was cleared during the one before
            const uint64_t i = e0 + tid;
            if (i < b) {
                const v4u32 x = iext[i];
                const uint32_t j = x.x;
                const uint32_t bit = 1u << (j & 31u);
                uint32_t old;
                if constexpr (kLdsCov) old = atomicOr(&L.cov[j >> 5], bit);
                else old = __hip_atomic_fetch_or(&gcov[j >> 5], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (!(old & bit)) {
                    const uint32_t f = atomicAdd(&L.nfresh[bp], 1u);
                    L.fstart[f] = static_cast<uint64_t>(x.z) | (static_cast<uint64_t>(x.w) << 32);
                    L.fsize[f] = x.y;
                    ++newly;
                }
            }
            __syncthreads();
            const uint32_t nf = L.nfresh[bp];
            if (tid == 0) {
                L.nfresh[bp ^ 1u] = 0u;
                // every wave has read the candidates for this round's argmax
                if (e0 == a) atomicOr(&L.cg[sv], kChosen);
            }
            // a candidate among a set's members loses one gain
            auto drop = [&](uint32_t u) {
                if (u == kNoCand) return;
                const uint32_t fb = wg_filter_bit(u);
                if (!((L.filter[fb >> 5] >> (fb & 31u)) & 1u)) return;
                const uint32_t slot = wg_slot(L, u);
                if (slot != kNoCand) atomicSub(&L.cg[slot], 1u);
            };
            if (nf > ngrp) {
                // many sets: four per group at a time, so that a lane has the
                // members of all four in flight before any is used
                for (uint32_t f = grp; f < nf; f += 4 * ngrp) {
                    uint64_t sa[4];
                    uint32_t sz[4];
                    uint32_t mx = 0;
#pragma unroll
                    for (uint32_t w = 0; w < 4; ++w) {
                        const uint32_t ff = f + w * ngrp;
                        sa[w] = ff < nf ? L.fstart[ff] : 0ull;
                        sz[w] = ff < nf ? L.fsize[ff] : 0u;
                        mx = sz[w] > mx ? sz[w] : mx;
                    }
                    for (uint32_t q0 = 0; q0 < mx; q0 += 64) {
                        uint32_t u[16];
#pragma unroll
                        for (uint32_t w = 0; w < 4; ++w)
#pragma unroll
                            for (uint32_t t = 0; t < 4; ++t) {
                                const uint32_t q = q0 + sub + 16u * t;
                                u[4 * w + t] = q < sz[w] ? pnodes[sa[w] + q] : kNoCand;
                            }
#pragma unroll
                        for (uint32_t t = 0; t < 16; ++t) drop(u[t]);
                    }
                }
            } else {
                for (uint32_t f = grp; f < nf; f += ngrp) {
                    const uint64_t sa = L.fstart[f];
                    const uint32_t sz = L.fsize[f];
                    // a lane's members of the set are all in flight before any is used
                    for (uint32_t q0 = 0; q0 < sz; q0 += 128) {
                        uint32_t u[8];
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t) {
                            const uint32_t q = q0 + sub + 16u * t;
                            u[t] = q < sz ? pnodes[sa + q] : kNoCand;
                        }
#pragma unroll
                        for (uint32_t t = 0; t < 8; ++t) drop(u[t]);
                    }
                }
            }
            __syncthreads();
        }
    }
    if constexpr (kLdsCov) {
        if (stalled)
            for (uint64_t w = tid; w < words; w += bd) g.covbits[w] = L.cov[w];
    }
    newly = wave_sum_u64(newly);
    if (lane_id() == 0 && newly) atomicAdd(g.cov, newly);
    if (tid == 0) {
        g.hdr[0].r = r;
        if (stalled) {
            g.hdr[0].stalls = h.stalls + 1u;
            *g.ccount = 0u;  // for the next collect
        }
        g.hdr[0].phase = stalled ? kStepRefresh : kStepDone;
    }
}

// Job blockIdx.x: rounds over its listed candidates until done or the test fails.
__global__ __launch_bounds__(kWgThreads) void wg_round_kernel(const GreedyState *jobs) {
    __shared__ WgLds L;
    const GreedyState g = jobs[blockIdx.x];  // a copy: the rounds' loads must not wait on its fields
    StepHdr h = g.hdr[0];
    if (h.phase == kStepZero) {
        // every unchosen gain is zero: the argmax takes the unchosen ids in
        // order, so the candidates are the kCandNodes lowest and the bound is
        // the key of the next one (0 if there is none)
        __shared__ uint64_t zscan[kWgThreads / kWave];
        __shared__ unsigned long long s_t;
        if (threadIdx.x == 0) s_t = 0ull;
        uint64_t seen = 0;
        for (uint32_t base = 0; base < g.n; base += blockDim.x) {
            const uint32_t v = base + threadIdx.x;
            const uint64_t f = (v < g.n && !(g.gain[v] & kChosen)) ? 1u : 0u;
            uint64_t tot = 0;
            const uint64_t pre = block_scan_excl(f, zscan, tot);
            if (f && seen + pre < kCandNodes) {
                g.cnode[seen + pre] = v;
                g.cbase[seen + pre] = 0u;
            }
            if (f && seen + pre == kCandNodes) s_t = static_cast<unsigned long long>(~v);
            seen += tot;
            if (seen > kCandNodes) break;  // the same in every thread
        }
        __syncthreads();
        if (threadIdx.x == 0) *g.ccount = static_cast<uint32_t>(min<uint64_t>(seen, kCandNodes));
        h.thresh = s_t;
        __threadfence_block();
        __syncthreads();
    } else if (h.phase != kStepCollect) {
        return;
    }
    const uint64_t words = (g.nsets + 31) / 32;
    if (words <= kWgCovWords) wg_rounds<true>(g, h, words, L);
    else wg_rounds<false>(g, h, words, L);
}

// Re-selection, step 1 (grid, blockIdx.y = job): keep only the chosen bits.
__global__ __launch_bounds__(kThreads) void wg_clear_kernel(const GreedyState *jobs) {
    const GreedyState &g = jobs[blockIdx.y];
    if (g.hdr[0].phase != kStepRefresh) return;
    // four gains per 16-byte access where the job's gain array allows it
    const bool vec = (reinterpret_cast<uintptr_t>(g.gain) & 15u) == 0;
    const uint32_t n4 = vec ? g.n / 4u : 0u;
    uint4 *g4 = reinterpret_cast<uint4 *>(g.gain);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        const uint4 q = g4[i];
        g4[i] = make_uint4(q.x & kChosen, q.y & kChosen, q.z & kChosen, q.w & kChosen);
    }
    for (uint32_t v = 4u * n4 + blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x)
        g.gain[v] &= kChosen;
}

// Re-selection, step 2: every set not covered adds one to each member's
// gain, 16 lanes per set (a chosen node has no such set left).
__global__ __launch_bounds__(kThreads) void wg_recount_kernel(const GreedyState *jobs) {
    const GreedyState &g = jobs[blockIdx.y];
    if (g.hdr[0].phase != kStepRefresh) return;
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t step = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t j = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4; j < g.nsets; j += step) {
        if ((g.covbits[j >> 5] >> (j & 31u)) & 1u) continue;
        const uint64_t sa = g.poff[g.begin + j], sb = g.poff[g.begin + j + 1];
        for (uint64_t q = sa + sub; q < sb; q += 16) atomicAdd(&g.gain[g.pnodes[q]], 1u);
    }
}

// Re-selection, step 3: how many unchosen nodes have a gain in each bin,
// into the histogram of this re-selection's parity (the collect step of the
// one before left it zeroed).
__global__ __launch_bounds__(kThreads) void wg_hist_kernel(const GreedyState *jobs) {
    __shared__ uint32_t hl[kSelBins];
    const GreedyState &g = jobs[blockIdx.y];
    const StepHdr h = g.hdr[0];
    if (h.phase != kStepRefresh) return;
    uint32_t *hist = g.hist + (h.stalls & 1u) * kSelBins;
    for (uint32_t i = threadIdx.x; i < kSelBins; i += blockDim.x) hl[i] = 0u;
    __syncthreads();
    const bool vec = (reinterpret_cast<uintptr_t>(g.gain) & 15u) == 0;
    const uint32_t n4 = vec ? g.n / 4u : 0u;
    const uint4 *g4 = reinterpret_cast<const uint4 *>(g.gain);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        const uint4 q = g4[i];
        const uint32_t xs[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (uint32_t t = 0; t < 4; ++t)
            if (xs[t] && !(xs[t] & kChosen)) atomicAdd(&hl[sel_bin(xs[t])], 1u);
    }
    for (uint32_t v = 4u * n4 + blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += gridDim.x * blockDim.x) {
        const uint32_t x = g.gain[v];
        if (x && !(x & kChosen)) atomicAdd(&hl[sel_bin(x)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kSelBins; i += blockDim.x)
        if (hl[i]) atomicAdd(&hist[i], hl[i]);
}

// Re-selection, step 4 (grid, blockIdx.y = job): every block reads the
// histogram and finds the same cut: the lowest bin b whose nodes, with those
// of the bins above, number at most kCandNodes. The bound on the keys left
// out is then the largest key a gain below bin b can have, and each block
// lists its nodes whose key beats it. If every unchosen gain is zero the
// header goes to ZERO (the round kernel lists the lowest unchosen ids
// itself); if the cut keeps fewer than kWgMinCand nodes and fewer than the
// rounds left (flat gains: many nodes share the gain at the cut), to GRID,
// and the host finishes the range with grid-wide rounds, which need no
// candidates. Block 0 writes the header and clears the other parity's
// histogram for the next re-selection.
__global__ __launch_bounds__(kThreads) void wg_collect_kernel(const GreedyState *jobs) {
    constexpr uint32_t kPer = (kSelBins + kThreads - 1) / kThreads;
    __shared__ uint64_t scan[kThreads / kWave];
    __shared__ uint32_t s_cut;
    const GreedyState &g = jobs[blockIdx.y];
    const StepHdr h = g.hdr[0];
    // block 0 may already have moved the header on
    if (h.phase != kStepRefresh && h.phase != kStepCollect) return;
    const uint32_t tid = threadIdx.x;
    const uint32_t par = h.stalls & 1u;
    const uint32_t *hist = g.hist + par * kSelBins;
    // thread tid holds bins [c kPer, c kPer + kPer) with c = 255 - tid, so a
    // prefix over threads counts the bins above
    const uint32_t c = kThreads - 1u - tid;
    uint32_t cnt[kPer];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
        const uint32_t b = c * kPer + i;
        cnt[i] = (b >= 1u && b < kSelBins) ? hist[b] : 0u;
        sum += cnt[i];
    }
    if (tid == 0) s_cut = kNoCand;
    uint64_t total = 0;
    const uint64_t above = block_scan_excl(sum, scan, total);
    uint64_t run = above;
#pragma unroll
    for (int i = static_cast<int>(kPer) - 1; i >= 0; --i) {
        const uint32_t b = c * kPer + static_cast<uint32_t>(i);
        run += cnt[i];
        if (b >= 1u && b < kSelBins && run <= kCandNodes) atomicMin(&s_cut, b);
    }
    __syncthreads();
    const uint32_t cut = s_cut;
    uint64_t mine = 0;
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i)
        if (c * kPer + i >= cut) mine += cnt[i];
    uint64_t kept = 0;
    (void)block_scan_excl(mine, scan, kept);
    uint32_t phase = kStepCollect;
    if (total == 0) phase = kStepZero;
    else if (cut == kNoCand || (kept < kWgMinCand && kept < g.k - h.r)) phase = kStepGrid;
    const unsigned long long thresh =
        phase == kStepCollect ? (static_cast<unsigned long long>(sel_bin_low(cut) - 1u) << 32) | 0xFFFFFFFFull : 0ull;
    if (blockIdx.x == 0) {
        uint32_t *other = g.hist + (par ^ 1u) * kSelBins;
        for (uint32_t i = tid; i < kSelBins; i += blockDim.x) other[i] = 0u;
        if (tid == 0) {
            g.hdr[0].thresh = thresh;
            g.hdr[0].phase = phase;
        }
    }
    if (phase != kStepCollect) return;
    auto take = [&](uint32_t v, uint32_t x) {
        if (x & kChosen) return;
        const unsigned long long key = (static_cast<unsigned long long>(x) << 32) | static_cast<unsigned long long>(~v);
        if (key > thresh) {
            const uint32_t slot = atomicAdd(g.ccount, 1u);
            if (slot < kCandNodes) {
                g.cnode[slot] = v;
                g.cbase[slot] = x;
            }
        }
    };
    // four gains per 16-byte load where the job's gain array allows it
    const bool vec = (reinterpret_cast<uintptr_t>(g.gain) & 15u) == 0;
    const uint32_t n4 = vec ? g.n / 4u : 0u;
    const uint4 *g4 = reinterpret_cast<const uint4 *>(g.gain);
    for (uint32_t i = blockIdx.x * blockDim.x + tid; i < n4; i += gridDim.x * blockDim.x) {
        const uint4 q = g4[i];
        take(4u * i, q.x);
        take(4u * i + 1u, q.y);
        take(4u * i + 2u, q.z);
        take(4u * i + 3u, q.w);
    }
    for (uint32_t v = 4u * n4 + blockIdx.x * blockDim.x + tid; v < g.n; v += gridDim.x * blockDim.x) take(v, g.gain[v]);
}

// Max-Coverage with one seed: the packed key (count << 32 | ~v) of the node
// in the most sets (ties to the lowest id; every count zero gives node 0).
__global__ __launch_bounds__(kThreads) void argmax_count_kernel(const uint32_t *cnt, uint32_t n,
                                                                unsigned long long *out) {
    unsigned long long best = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned long long key = (static_cast<unsigned long long>(cnt[v]) << 32) | static_cast<uint32_t>(~v);
        best = key > best ? key : best;
    }
    best = wave_max_key(best);
    if (lane_id() == 0 && best) atomicMax(out, best);
}

// dst[0] = cnt[v]: one node's count, read on the stream between launches.
__global__ void pick_u32_kernel(const uint32_t *cnt, uint32_t v, uint32_t *dst) { dst[0] = cnt[v]; }

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


// ---- batched jobs: many pool ranges of one graph ----

struct JobTable {
    const uint64_t *poff;
    const uint32_t *pnodes;
    uint64_t begin;        // first set of the greedy range
    uint64_t ebegin;       // pnodes index of its first entry
    uint64_t set_start;    // flattened: sets of earlier jobs
    uint64_t entry_start;  // flattened: entries of earlier jobs
    uint64_t stare_begin;  // first set of the stare range
    uint64_t stare_start;  // flattened: stare sets of earlier jobs
    uint64_t seed_start;   // flattened: seeds of earlier jobs
    uint32_t *gain;
    uint32_t *fill;
    uint32_t *stare_bits;  // seed bitmap for the stare step
    unsigned long long *cov_c;
};

__device__ __forceinline__ uint32_t job_of(const JobTable *jt, uint32_t nj, uint64_t x, uint64_t JobTable::*field) {
    uint32_t lo = 0, hi = nj - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (jt[mid].*field <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// poff at the range ends of each job: out[4j..4j+3] = poff[begin], poff[end],
// poff[stare_begin], poff[stare_end].
__global__ void job_bounds_kernel(const uint64_t *const *poffs, const uint64_t *bounds, uint32_t nj, uint64_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < 4 * nj; i += gridDim.x * blockDim.x)
        out[i] = poffs[i / 4][bounds[i]];
}

__global__ __launch_bounds__(kThreads) void batch_histogram_kernel(const JobTable *jt, uint32_t nj, uint64_t total) {
    for (uint64_t x = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; x < total;
         x += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const JobTable &j = jt[job_of(jt, nj, x, &JobTable::entry_start)];
        atomicAdd(&j.gain[j.pnodes[j.ebegin + (x - j.entry_start)]], 1u);
    }
}

// 16 lanes per set; isets positions come from the global prefix over all
// jobs' counts (job j's counts occupy [j*n, j*n+n)).
template <bool kExt>
__global__ __launch_bounds__(kThreads) void batch_scatter_kernel(const JobTable *jt, uint32_t nj, uint64_t total_sets,
                                                                 const uint64_t *prefix, uint32_t n, uint32_t *isets,
                                                                 uint4 *iext) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t x = grp; x < total_sets; x += ngrp) {
        const uint32_t ji = job_of(jt, nj, x, &JobTable::set_start);
        const JobTable &j = jt[ji];
        const uint64_t js = x - j.set_start;
        const uint64_t a = j.poff[j.begin + js], b = j.poff[j.begin + js + 1];
        for (uint64_t q = a + sub; q < b; q += 16) {
            const uint32_t v = j.pnodes[q];
            const uint32_t pos = atomicAdd(&j.fill[v], 1u);
            if constexpr (kExt)
                iext[prefix[uint64_t(ji) * n + v] + pos] = make_uint4(
                    static_cast<uint32_t>(js), static_cast<uint32_t>(b - a), static_cast<uint32_t>(a),
                    static_cast<uint32_t>(a >> 32));
            else
                isets[prefix[uint64_t(ji) * n + v] + pos] = static_cast<uint32_t>(js);
        }
    }
}

__global__ __launch_bounds__(kThreads) void batch_init_m1_kernel(const GreedyState *gs, uint32_t nj, uint32_t n1) {
    const uint64_t total = uint64_t(nj) * n1;
    for (uint64_t x = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; x < total;
         x += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const GreedyState &g = gs[x / n1];
        const uint32_t c = static_cast<uint32_t>(x % n1);
        g.m1[c] = m1_lane<false>(g, c);
    }
}

__global__ __launch_bounds__(kThreads) void batch_init_m2_kernel(const GreedyState *gs, uint32_t nj, uint32_t n2) {
    const uint64_t total = uint64_t(nj) * n2;
    for (uint64_t x = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; x < total;
         x += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const GreedyState &g = gs[x / n2];
        const uint32_t d = static_cast<uint32_t>(x % n2);
        g.m2[d] = m2_lane<false>(g, d);
    }
}

__global__ void batch_seed_bits_kernel(const JobTable *jt, uint32_t nj, const uint32_t *seeds, uint64_t total) {
    for (uint64_t x = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; x < total;
         x += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const JobTable &j = jt[job_of(jt, nj, x, &JobTable::seed_start)];
        const uint32_t v = seeds[x];
        atomicOr(&j.stare_bits[v >> 5], 1u << (v & 31u));
    }
}

// Stare step of every job: its stare-range sets that meet its seed bitmap.
__global__ __launch_bounds__(kThreads) void batch_coverage_kernel(const JobTable *jt, uint32_t nj, uint64_t total_sets) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t grp = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const uint64_t ngrp = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t x = grp; x < total_sets; x += ngrp) {
        const JobTable &j = jt[job_of(jt, nj, x, &JobTable::stare_start)];
        const uint64_t js = x - j.stare_start;
        const uint64_t a = j.poff[j.stare_begin + js], b = j.poff[j.stare_begin + js + 1];
        bool any = false;
        for (uint64_t q = a + sub; q < b && !any; q += 16) any = test_bit(j.stare_bits, j.pnodes[q]);
        const uint64_t mask = __ballot(any);
        if (sub == 0 && ((mask >> (lane_id() & ~15u)) & 0xFFFFull)) atomicAdd(j.cov_c, 1ull);
    }
}

// Estimate-Inf crossing for many items: block i walks flags [start, start+count)
// in order, 1024 at a time, to the first index where the running count of
// ones reaches need[i]. out[2i] = that index (relative) or -1; out[2i+1] =
// ones in the whole segment.
__global__ __launch_bounds__(1024) void crossing_items_kernel(const uint8_t *z, const uint64_t *seg, long long *out) {
    __shared__ uint64_t smem[1024 / kWave];
    __shared__ long long s_idx;
    const uint64_t start = seg[3 * blockIdx.x], count = seg[3 * blockIdx.x + 1], need = seg[3 * blockIdx.x + 2];
    if (threadIdx.x == 0) s_idx = -1;
    __syncthreads();
    uint64_t run = 0;
    for (uint64_t b0 = 0; b0 < count; b0 += blockDim.x) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t x = (i < count) ? z[start + i] : 0;
        uint64_t total = 0;
        const uint64_t ex = block_scan_excl(x, smem, total);
        if (s_idx < 0 && x && run + ex + 1 == need) s_idx = static_cast<long long>(i);
        run += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = s_idx;
        out[2 * blockIdx.x + 1] = static_cast<long long>(run);
    }
}

// ---- greedy rounds level by level (flat gains) ----
//
// When the candidate cut keeps too few nodes (many nodes share the gain at
// the cut), the remaining rounds go by gain level. Let g* be the largest gain
// of an unchosen node and L the unchosen nodes with gain g*, in increasing id
// order. Gains only fall, so while a node of L still has g* uncovered sets it
// is a round's argmax, and the lowest-id such node is the seed. A node of L
// still has gain g* exactly when none of the sets it had uncovered when L was
// listed has been covered since. So a level walks L in order and takes every
// node whose sets are all still uncovered; the nodes it passes over now have
// less and wait for a later level. Once L is walked the largest gain is below
// g*: the gains are recounted from the sets still uncovered and the next
// level is listed. Only nodes that had a gain when the level rounds began
// (`act`, kept in id order) can have one later.

constexpr uint32_t kFlatMaxGain = 16;  // a larger g* goes back to the grid-wide rounds
constexpr uint32_t kFlatBatch = 256;   // candidates resolved per pass of the level kernel
constexpr uint32_t kFlatHash = 8192;   // LDS hash of the sets one pass covers (>= 2 x 256 x 16)
constexpr uint32_t kFlatTile = 2048;   // items per block of the ordered compactions
constexpr uint32_t kFlatEmpty = 0xFFFFFFFFu;

struct FlatState {
    unsigned int gstar;  // the level's g* (unchosen maximum)
    uint32_t r;          // rounds done
    uint32_t pad[6];
};

enum : int { kFlatAct = 0, kFlatLevel = 1, kFlatUnchosen = 2 };

// Which items an ordered compaction keeps: kFlatAct the unchosen nodes with a
// gain (items are node ids 0..n-1), kFlatLevel the unchosen nodes of `in`
// with gain g*, kFlatUnchosen every unchosen node (ids 0..n-1).
template <int kMode>
__device__ __forceinline__ bool flat_keep(const uint32_t *gain, uint32_t v, uint32_t gstar) {
    const uint32_t x = gain[v];
    if (x & kChosen) return false;
    if constexpr (kMode == kFlatAct) return x != 0u;
    else if constexpr (kMode == kFlatLevel) return x == gstar;
    else return true;
}

template <int kMode>
__device__ __forceinline__ uint32_t flat_item(const uint32_t *in, uint64_t i) {
    if constexpr (kMode == kFlatLevel) return in[i];
    else return static_cast<uint32_t>(i);
}

// Ordered compaction, pass 1: kept items per tile of kFlatTile (8 per thread).
template <int kMode>
__global__ __launch_bounds__(kThreads) void flat_count_kernel(const uint32_t *gain, const uint32_t *in,
                                                              const uint64_t *nin_p, uint64_t nin_fixed,
                                                              const FlatState *fs, uint64_t *bcount) {
    __shared__ uint64_t smem[kThreads / kWave];
    const uint64_t nin = nin_p ? *nin_p : nin_fixed;
    const uint32_t gstar = fs->gstar;
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kFlatTile + threadIdx.x * 8ull;
    uint64_t c = 0;
    for (uint32_t i = 0; i < 8; ++i)
        if (b0 + i < nin) c += flat_keep<kMode>(gain, flat_item<kMode>(in, b0 + i), gstar);
    uint64_t total = 0;
    block_scan_excl(c, smem, total);
    if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// Pass 3 (after the exclusive scan of the tile counts): write the kept items
// in order, at most cap of them.
template <int kMode>
__global__ __launch_bounds__(kThreads) void flat_write_kernel(const uint32_t *gain, const uint32_t *in,
                                                              const uint64_t *nin_p, uint64_t nin_fixed,
                                                              const FlatState *fs, const uint64_t *boff,
                                                              uint32_t *out, uint64_t cap) {
    __shared__ uint64_t smem[kThreads / kWave];
    const uint64_t nin = nin_p ? *nin_p : nin_fixed;
    const uint32_t gstar = fs->gstar;
    const uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * kFlatTile + threadIdx.x * 8ull;
    uint32_t keep = 0;
    uint64_t c = 0;
    for (uint32_t i = 0; i < 8; ++i)
        if (b0 + i < nin && flat_keep<kMode>(gain, flat_item<kMode>(in, b0 + i), gstar)) {
            keep |= 1u << i;
            ++c;
        }
    uint64_t total = 0;
    uint64_t pos = boff[blockIdx.x] + block_scan_excl(c, smem, total);
    for (uint32_t i = 0; i < 8; ++i)
        if ((keep >> i) & 1u) {
            if (pos < cap) out[pos] = flat_item<kMode>(in, b0 + i);
            ++pos;
        }
}

__global__ void flat_init_kernel(FlatState *fs, uint32_t r) {
    fs->gstar = 0;
    fs->r = r;
}

// g* = the largest gain of an unchosen node of act.
__global__ __launch_bounds__(kThreads) void flat_max_kernel(const uint32_t *gain, const uint32_t *act,
                                                            const uint64_t *nact_p, FlatState *fs) {
    const uint64_t nact = *nact_p;
    uint32_t best = 0;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nact;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t x = gain[act[i]];
        if (!(x & kChosen) && x > best) best = x;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const uint32_t y = __shfl_xor(best, d, kWave);
        best = y > best ? y : best;
    }
    if (lane_id() == 0 && best) atomicMax(&fs->gstar, best);
}

// Recount, step 1: the gains of act back to zero (chosen bits kept), and g*
// reset for the next level's maximum.
__global__ __launch_bounds__(kThreads) void flat_clear_kernel(uint32_t *gain, const uint32_t *act,
                                                              const uint64_t *nact_p, FlatState *fs) {
    const uint64_t nact = *nact_p;
    if (blockIdx.x == 0 && threadIdx.x == 0) fs->gstar = 0;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nact;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        gain[act[i]] &= kChosen;
}

// Recount, step 2: every set not covered adds one to each member's gain.
__global__ __launch_bounds__(kThreads) void flat_recount_kernel(GreedyState g) {
    const uint32_t sub = threadIdx.x & 15u;
    const uint64_t step = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 4;
    for (uint64_t j = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 4; j < g.nsets; j += step) {
        if ((g.covbits[j >> 5] >> (j & 31u)) & 1u) continue;
        const uint64_t sa = g.poff[g.begin + j], sb = g.poff[g.begin + j + 1];
        for (uint64_t q = sa + sub; q < sb; q += 16) atomicAdd(&g.gain[g.pnodes[q]], 1u);
    }
}

__device__ __forceinline__ uint32_t flat_hash(uint32_t j) { return (j * 0x9E3779B1u) >> (32 - 13); }

// One level: walk the listed nodes (gain g* when listed, in id order) in
// passes of kFlatBatch. Each pass gathers every candidate's uncovered sets,
// then wave 0 takes, in order, each candidate that still has g* of them and
// none covered earlier in the pass (an LDS hash of the pass's covered sets),
// and the block writes the pass's seeds, chosen bits and covered bits.
__global__ __launch_bounds__(1024) void flat_level_kernel(GreedyState g, const uint32_t *list,
                                                          const uint64_t *nlist_p, FlatState *fs) {
    __shared__ uint32_t s_sets[kFlatBatch][kFlatMaxGain];
    __shared__ uint32_t s_cnt[kFlatBatch];
    __shared__ uint32_t s_hash[kFlatHash];
    __shared__ uint32_t s_sel[kFlatBatch];
    __shared__ uint32_t s_nsel;
    const uint32_t gstar = fs->gstar;
    const uint64_t nlist = *nlist_p;
    uint32_t r = fs->r;
    if (gstar == 0 || gstar > kFlatMaxGain) return;
    for (uint32_t i = threadIdx.x; i < kFlatHash; i += blockDim.x) s_hash[i] = kFlatEmpty;
    for (uint64_t base = 0; base < nlist && r < g.k; base += kFlatBatch) {
        // gather: candidate t's sets not covered yet (covered bits come from
        // earlier passes' atomics, read past the L1)
        if (threadIdx.x < kFlatBatch) {
            const uint32_t t = threadIdx.x;
            uint32_t c = 0;
            if (base + t < nlist) {
                const uint32_t v = list[base + t];
                const uint64_t e0 = g.ioff[v], e1 = g.ioff[v + 1];
                for (uint64_t e = e0; e < e1; ++e) {
                    const uint32_t j = g.iext ? g.iext[e].x : g.isets[e];
                    if (!((ld<true>(g.covbits + (j >> 5)) >> (j & 31u)) & 1u)) {
                        if (c < kFlatMaxGain) s_sets[t][c] = j;
                        ++c;
                    }
                }
            }
            s_cnt[t] = c;
        }
        __syncthreads();
        // resolve the pass in order (wave 0)
        if (threadIdx.x < kWave) {
            const uint32_t lane = threadIdx.x;
            uint32_t nsel = 0;
            for (uint32_t i = 0; i < kFlatBatch && base + i < nlist && r + nsel < g.k; ++i) {
                if (s_cnt[i] != gstar) continue;  // its gain fell before this pass
                uint32_t j = 0, h = 0;
                bool seen = false;
                if (lane < gstar) {
                    j = s_sets[i][lane];
                    h = flat_hash(j);
                    for (;;) {
                        const uint32_t x = s_hash[h];
                        if (x == kFlatEmpty) break;
                        if (x == j) {
                            seen = true;
                            break;
                        }
                        h = (h + 1u) & (kFlatHash - 1u);
                    }
                }
                if (__ballot(seen)) continue;  // a set of it was covered earlier in the pass
                if (lane < gstar) {
                    // the sets of one node are distinct: claim a free slot each
                    for (;;) {
                        const uint32_t prev = atomicCAS(&s_hash[h], kFlatEmpty, j);
                        if (prev == kFlatEmpty) break;
                        h = (h + 1u) & (kFlatHash - 1u);
                    }
                }
                if (lane == 0) s_sel[nsel] = i;
                ++nsel;
            }
            if (lane == 0) s_nsel = nsel;
        }
        __syncthreads();
        const uint32_t nsel = s_nsel;
        for (uint32_t q = threadIdx.x; q < nsel * kFlatMaxGain; q += blockDim.x) {
            const uint32_t si = q / kFlatMaxGain, l = q % kFlatMaxGain;
            const uint32_t i = s_sel[si];
            if (l < gstar) {
                const uint32_t j = s_sets[i][l];
                atomicOr(&g.covbits[j >> 5], 1u << (j & 31u));
            }
            if (l == 0) {
                const uint32_t v = list[base + i];
                g.seeds[r + si] = v;
                atomicOr(&g.gain[v], kChosen);
            }
        }
        if (threadIdx.x == 0 && nsel) atomicAdd(g.cov, static_cast<unsigned long long>(nsel) * gstar);
        r += nsel;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kFlatHash; i += blockDim.x) s_hash[i] = kFlatEmpty;
        __syncthreads();
    }
    if (threadIdx.x == 0) fs->r = r;
}

// Every gain is zero: the remaining seeds (rounds r..k-1) are the lowest
// unchosen ids (listed in order), which cover nothing.
__global__ void flat_zero_kernel(GreedyState g, const uint32_t *list, uint32_t r) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; r + i < g.k; i += gridDim.x * blockDim.x) {
        const uint32_t v = list[i];
        g.seeds[r + i] = v;
        g.gain[v] |= kChosen;
    }
}

}  // namespace

namespace im {

im_status set_seed_bits(im_ctx *ctx, uint32_t n, const uint32_t *seeds_host, uint32_t k) {
    return seed_bits_into(ctx, n, seeds_host, k, ctx->seedbits);
}

im_status seed_bits_into(im_ctx *ctx, uint32_t n, const uint32_t *seeds_host, uint32_t k, DevBuf &out) {
    const uint64_t words = (uint64_t(n) + 31) / 32;
    IM_TRY(dev_reserve(ctx, out, words * 4 + 4 * uint64_t(k) + 64));
    auto *bits = static_cast<uint32_t *>(out.ptr);
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
    return coverage_range_on(p->ctx, p, begin, end, seeds_host, k, cov);
}

im_status coverage_range_on(im_ctx *ctx, const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds_host,
                            uint32_t k, uint64_t *cov) {
    const uint32_t n = p->g->n;
    if (k == 1 && seeds_host[0] < n && end > begin && ctx->k1_serial == p->serial && ctx->k1_cnt.ptr) {
        // one seed s, and the context holds the node counts of this pool's
        // entries up to exactly where the range starts (the stare step
        // after a one-seed Max-Coverage of [0, begin)): the sets of the
        // range that hold s are its count over the range's entries (a set
        // holds a node once), read before and after adding them, and the
        // counts then cover [0, end) for the next, doubled prefix
        const auto *poff = static_cast<const uint64_t *>(p->poff.ptr);
        uint64_t ends[2] = {0, 0};
        IM_TRY(to_host_sync(ctx, &ends[0], poff + begin, 8));
        IM_TRY(to_host_sync(ctx, &ends[1], poff + end, 8));
        if (ends[0] == ctx->k1_end) {
            auto *cnt = static_cast<uint32_t *>(ctx->k1_cnt.ptr);
            auto *two = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->k1_cnt.ptr) +
                                                     ((4ull * n + 255) & ~255ull) + 8);
            hipStream_t st = ctx->stream;
            const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
            ctx->k1_serial = 0;  // until the counts below are in
            pick_u32_kernel<<<1, 1, 0, st>>>(cnt, seeds_host[0], two);
            if (ends[1] > ends[0])
                histogram_kernel<<<grid_of(ends[1] - ends[0], kThreads, cu * 16), kThreads, 0, st>>>(
                    static_cast<const uint32_t *>(p->pnodes.ptr), ends[0], ends[1], cnt);
            pick_u32_kernel<<<1, 1, 0, st>>>(cnt, seeds_host[0], two + 1);
            IM_HIP(hipGetLastError());
            uint32_t h[2] = {0, 0};
            IM_TRY(to_host_sync(ctx, h, two, 8));
            ctx->k1_serial = p->serial;
            ctx->k1_end = ends[1];
            *cov = h[1] - h[0];
            return IM_OK;
        }
    }
    IM_TRY(set_seed_bits(ctx, n, seeds_host, k));
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

__global__ void step_init_kernel(const GreedyState *jobs, uint32_t nj) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nj) return;
    StepHdr h{};
    h.phase = jobs[j].k ? kStepRefresh : kStepDone;
    jobs[j].hdr[0] = h;
}

// Launch greedy steps on `dgs` (nj jobs, the step headers of job j at
// dhdr[2j], [2j+1]) until every job has its k seeds. Each pass launches
// what the slowest job needs at the context's running refresh rate, then
// reads the headers back once.
static im_status run_steps(im_ctx *ctx, const GreedyState *dgs, StepHdr *dhdr, const uint32_t *ks, uint32_t nj,
                           dim3 grid) {
    hipStream_t st = ctx->stream;
    step_init_kernel<<<(nj + 255) / 256, 256, 0, st>>>(dgs, nj);
    std::vector<StepHdr> hh(2ull * nj);
    uint32_t max_k = 0;
    for (uint32_t j = 0; j < nj; ++j) max_k = std::max(max_k, ks[j]);
    const uint64_t cap = 3ull * max_k + 64;  // a refresh pair always leads to a round
    uint32_t step = 0, remaining = max_k;
    bool first = true;
    for (;;) {
        const double rate = ctx->greedy_stall_rate;
        const uint32_t est = remaining + static_cast<uint32_t>(2.0 * rate * remaining + 0.999) + (first ? 4u : 2u);
        first = false;
        for (uint32_t i = 0; i < est; ++i) greedy_step_kernel<<<grid, kThreads, 0, st>>>(dgs, step++);
        IM_HIP(hipGetLastError());
        IM_HIP(hipMemcpyAsync(hh.data(), dhdr, sizeof(StepHdr) * 2 * nj, hipMemcpyDeviceToHost, st));
        IM_HIP(hipStreamSynchronize(st));
        remaining = 0;
        uint64_t stalls = 0, rounds = 0;
        for (uint32_t j = 0; j < nj; ++j) {
            const StepHdr &x = hh[2ull * j + (step & 1u)];
            if (x.phase != kStepDone) remaining = std::max<uint32_t>(remaining, ks[j] - std::min(ks[j], x.r));
            stalls += x.stalls;
            rounds += x.r;
        }
        if (remaining == 0) {
            bool all_done = true;
            for (uint32_t j = 0; j < nj; ++j) all_done = all_done && hh[2ull * j + (step & 1u)].phase == kStepDone;
            if (all_done) {
                if (rounds) ctx->greedy_stall_rate = 0.5 * ctx->greedy_stall_rate + 0.5 * double(stalls) / double(rounds);
                return IM_OK;
            }
            remaining = 1;
        }
        if (step > cap) {
            set_error("max coverage: greedy steps did not finish");
            return IM_E_DEVICE;
        }
    }
}

__global__ void wg_start_kernel(const GreedyState *jobs, uint32_t nj, uint32_t r0) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nj) return;
    StepHdr h{};
    h.r = r0;
    h.phase = r0 < jobs[j].k ? kStepRefresh : kStepDone;
    jobs[j].hdr[0] = h;
    *jobs[j].ccount = 0u;
}

// One-workgroup candidate rounds [r0, k) for nj jobs (job j's header at
// hdrs[j]), whose gains are exact. The first hist, collect and rounds run
// at once; then cycles (clear, recount, hist, collect, rounds) are
// queued at the context's running re-selection rate and the headers read
// back once per batch of cycles, until every job has its k seeds or its cut
// asked for grid-wide rounds: then grid_from[j] is job j's first round left
// to them, with every gain exact (else k).
static im_status run_wg_cycles(im_ctx *ctx, const GreedyState *dgs, StepHdr *const *hdrs, const uint32_t *ks,
                               uint32_t nj, uint32_t n, uint64_t max_sets, uint32_t r0, uint32_t *grid_from) {
    hipStream_t st = ctx->stream;
    for (uint32_t j = 0; j < nj; ++j) grid_from[j] = ks[j];
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    // node passes: the collect blocks each derive the cut from the whole
    // histogram, so they take more nodes per thread than the other passes
    const dim3 gn(grid_of(n, kThreads * 4, cu * 8), nj), gh(grid_of(n, kThreads * 8, cu * 4), nj),
        gs(grid_of(max_sets * 16, kThreads, cu * 16), nj), gc(grid_of(n, kThreads * 16, cu * 4), nj);
    wg_start_kernel<<<(nj + 255) / 256, 256, 0, st>>>(dgs, nj, r0);
    wg_hist_kernel<<<gh, kThreads, 0, st>>>(dgs);
    wg_collect_kernel<<<gc, kThreads, 0, st>>>(dgs);
    wg_round_kernel<<<nj, kWgThreads, 0, st>>>(dgs);
    uint32_t max_k = 0;
    for (uint32_t j = 0; j < nj; ++j) max_k = std::max(max_k, ks[j]);
    std::vector<StepHdr> hh(nj);
    uint64_t cycles = 1;
    uint32_t remaining = max_k - std::min(max_k, r0);
    for (;;) {
        const uint32_t est = 1u + static_cast<uint32_t>(ctx->greedy_wg_resel_rate * remaining);
        for (uint32_t i = 0; i < est; ++i) {
            wg_clear_kernel<<<gn, kThreads, 0, st>>>(dgs);
            wg_recount_kernel<<<gs, kThreads, 0, st>>>(dgs);
            wg_hist_kernel<<<gh, kThreads, 0, st>>>(dgs);
            wg_collect_kernel<<<gc, kThreads, 0, st>>>(dgs);
            wg_round_kernel<<<nj, kWgThreads, 0, st>>>(dgs);
        }
        cycles += est;
        IM_HIP(hipGetLastError());
        for (uint32_t j = 0; j < nj; ++j)
            IM_HIP(hipMemcpyAsync(&hh[j], hdrs[j], sizeof(StepHdr), hipMemcpyDeviceToHost, st));
        IM_HIP(hipStreamSynchronize(st));
        remaining = 0;
        uint64_t stalls = 0, rounds = 0;
        bool done = true;
        for (uint32_t j = 0; j < nj; ++j) {
            if (hh[j].phase != kStepDone) {
                done = false;
                remaining = std::max<uint32_t>(remaining, ks[j] - std::min(ks[j], hh[j].r));
            }
            stalls += hh[j].stalls;
            rounds += hh[j].r;
        }
        if (done) {
            if (rounds)
                ctx->greedy_wg_resel_rate = 0.5 * ctx->greedy_wg_resel_rate + 0.5 * double(stalls) / double(rounds);
            return IM_OK;
        }
        remaining = 0;
        for (uint32_t j = 0; j < nj; ++j)
            if (hh[j].phase != kStepDone && hh[j].phase != kStepGrid)
                remaining = std::max<uint32_t>(remaining, ks[j] - std::min(ks[j], hh[j].r));
        // jobs the cut handed to the grid-wide rounds are finished by the caller
        bool left = false;
        for (uint32_t j = 0; j < nj; ++j) left = left || (hh[j].phase != kStepDone && hh[j].phase != kStepGrid);
        if (!left) {
            for (uint32_t j = 0; j < nj; ++j)
                if (hh[j].phase == kStepGrid) grid_from[j] = hh[j].r;
            return IM_OK;
        }
        // every cycle chooses at least one seed: the cut keeps only keys above its bound
        if (cycles > uint64_t(max_k) + 2) {
            set_error("max coverage: one-workgroup rounds did not finish");
            return IM_E_DEVICE;
        }
    }
}

}  // namespace im

// Cached HIP graphs of the per-round launch pairs (refresh, cover) of one
// range: the kernels read the greedy state through a fixed device address,
// so a graph replays for any range with the same round count and launch
// shape. A shape is built into a graph the second time it is asked for.
struct RoundGraphCache {
    struct Entry {
        const void *dg;
        uint32_t k, rgrid, cgrid;
        uint64_t last;
        hipGraphExec_t exec;  // null: seen once
    };
    std::vector<Entry> e;
    uint64_t tick = 0;
};

void free_round_graphs(im_ctx *ctx) {
    if (!ctx->round_graphs) return;
    for (auto &x : ctx->round_graphs->e)
        if (x.exec) (void)hipGraphExecDestroy(x.exec);
    delete ctx->round_graphs;
    ctx->round_graphs = nullptr;
}

namespace im {

// The graph of rounds [0, k) for state dg, or null when this shape has not
// been seen before (the caller then launches the rounds itself).
static im_status round_graph(im_ctx *ctx, const GreedyState *dg, uint32_t k, uint32_t rgrid, uint32_t cgrid,
                      hipGraphExec_t *out) {
    constexpr size_t kMaxGraphs = 32;
    *out = nullptr;
    if (!ctx->round_graphs) ctx->round_graphs = new RoundGraphCache();
    RoundGraphCache &c = *ctx->round_graphs;
    ++c.tick;
    RoundGraphCache::Entry *hit = nullptr;
    for (auto &x : c.e)
        if (x.dg == dg && x.k == k && x.rgrid == rgrid && x.cgrid == cgrid) hit = &x;
    if (!hit) {
        if (c.e.size() >= kMaxGraphs) {
            auto old = std::min_element(c.e.begin(), c.e.end(),
                                        [](const auto &a, const auto &b) { return a.last < b.last; });
            if (old->exec) (void)hipGraphExecDestroy(old->exec);
            c.e.erase(old);
        }
        c.e.push_back({dg, k, rgrid, cgrid, c.tick, nullptr});
        return IM_OK;
    }
    hit->last = c.tick;
    if (!hit->exec) {
        hipGraph_t graph = nullptr;
        IM_HIP(hipGraphCreate(&graph, 0));
        hipGraphNode_t prev = nullptr;
        hipError_t e = hipSuccess;
        for (uint32_t r = 0; r < k && e == hipSuccess; ++r) {
            for (int step = 0; step < 2 && e == hipSuccess; ++step) {
                const GreedyState *arg_dg = dg;
                uint32_t arg_r = r;
                void *args[] = {&arg_dg, &arg_r};
                hipKernelNodeParams kp{};
                kp.func = step == 0 ? reinterpret_cast<void *>(batch_refresh_kernel)
                                    : reinterpret_cast<void *>(batch_cover_kernel);
                kp.gridDim = dim3(step == 0 ? rgrid : cgrid, 1, 1);
                kp.blockDim = dim3(kThreads, 1, 1);
                kp.sharedMemBytes = 0;
                kp.kernelParams = args;
                kp.extra = nullptr;
                hipGraphNode_t node = nullptr;
                e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
                prev = node;
            }
        }
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            set_error("max coverage round graph: %s", hipGetErrorString(e));
            return IM_E_DEVICE;
        }
        hit->exec = exec;
    }
    *out = hit->exec;
    return IM_OK;
}


// Rounds [*r, k) of one range level by level (see flat_level_kernel), with
// every gain exact on entry. Leaves *r < k when the largest gain is above
// kFlatMaxGain (the grid-wide rounds take over, gains still exact).
static im_status flat_rounds(im_ctx *ctx, const GreedyState &g, uint64_t entries, uint32_t *r_io) {
    const uint32_t n = g.n, k = g.k;
    const uint64_t cap = std::max<uint64_t>(std::min<uint64_t>(n, entries), k) + 1;
    const uint64_t nb_n = (uint64_t(n) + kFlatTile - 1) / kFlatTile;
    const uint64_t nb_c = (cap + kFlatTile - 1) / kFlatTile;
    const size_t o_act = 256 + (((nb_n + 1) * 8 + 255) & ~size_t(255));
    const size_t o_bl = o_act + ((cap * 4 + 255) & ~size_t(255));
    const size_t o_list = o_bl + (((nb_c + 1) * 8 + 255) & ~size_t(255));
    const size_t bytes = o_list + cap * 4 + 256;
    IM_TRY(dev_reserve(ctx, ctx->flat, bytes));
    char *base = static_cast<char *>(ctx->flat.ptr);
    auto *fs = reinterpret_cast<FlatState *>(base);
    auto *bc_n = reinterpret_cast<uint64_t *>(base + 256);  // tiles over node ids (act, zero tail)
    auto *act = reinterpret_cast<uint32_t *>(base + o_act);
    auto *bc_c = reinterpret_cast<uint64_t *>(base + o_bl);  // tiles over act (levels)
    auto *list = reinterpret_cast<uint32_t *>(base + o_list);
    const uint64_t *nact_p = bc_n + nb_n;    // after the act compaction's scan
    const uint64_t *nlist_p = bc_c + nb_c;   // after a level compaction's scan
    hipStream_t st = ctx->stream;
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    const uint32_t gb_n = static_cast<uint32_t>(std::max<uint64_t>(1, nb_n));
    const uint32_t gb_c = static_cast<uint32_t>(std::max<uint64_t>(1, nb_c));
    flat_init_kernel<<<1, 1, 0, st>>>(fs, *r_io);
    // act: the unchosen nodes with a gain, in id order
    fill_u64_kernel<<<1, 64, 0, st>>>(bc_n + nb_n, 1, 0);
    flat_count_kernel<kFlatAct><<<gb_n, kThreads, 0, st>>>(g.gain, nullptr, nullptr, n, fs, bc_n);
    tile_scan_kernel<<<1, 1024, 0, st>>>(bc_n, nb_n + 1);
    flat_write_kernel<kFlatAct><<<gb_n, kThreads, 0, st>>>(g.gain, nullptr, nullptr, n, fs, bc_n, act, cap);
    uint32_t r = *r_io;
    for (uint32_t level = 0; r < k; ++level) {
        if (level > 0) {
            flat_clear_kernel<<<grid_of(cap, kThreads, cu * 8), kThreads, 0, st>>>(g.gain, act, nact_p, fs);
            flat_recount_kernel<<<grid_of(g.nsets * 16, kThreads, cu * 16), kThreads, 0, st>>>(g);
        }
        flat_max_kernel<<<grid_of(cap, kThreads, cu * 8), kThreads, 0, st>>>(g.gain, act, nact_p, fs);
        fill_u64_kernel<<<1, 64, 0, st>>>(bc_c + nb_c, 1, 0);
        flat_count_kernel<kFlatLevel><<<gb_c, kThreads, 0, st>>>(g.gain, act, nact_p, 0, fs, bc_c);
        tile_scan_kernel<<<1, 1024, 0, st>>>(bc_c, nb_c + 1);
        flat_write_kernel<kFlatLevel><<<gb_c, kThreads, 0, st>>>(g.gain, act, nact_p, 0, fs, bc_c, list, cap);
        flat_level_kernel<<<1, 1024, 0, st>>>(g, list, nlist_p, fs);
        IM_HIP(hipGetLastError());
        FlatState h{};
        IM_TRY(to_host_sync(ctx, &h, fs, sizeof(h)));
        if (h.gstar == 0) {
            // every gain is zero: the lowest unchosen ids, in order
            fill_u64_kernel<<<1, 64, 0, st>>>(bc_n + nb_n, 1, 0);
            flat_count_kernel<kFlatUnchosen><<<gb_n, kThreads, 0, st>>>(g.gain, nullptr, nullptr, n, fs, bc_n);
            tile_scan_kernel<<<1, 1024, 0, st>>>(bc_n, nb_n + 1);
            flat_write_kernel<kFlatUnchosen><<<gb_n, kThreads, 0, st>>>(g.gain, nullptr, nullptr, n, fs, bc_n, list,
                                                                       cap);
            flat_zero_kernel<<<grid_of(k - r, kThreads, 64), kThreads, 0, st>>>(g, list, r);
            IM_HIP(hipGetLastError());
            r = k;
            break;
        }
        if (h.gstar > kFlatMaxGain) break;  // gains are exact: the grid-wide rounds go on
        if (h.r <= r) {
            set_error("max coverage: a gain level chose no seed");
            return IM_E_DEVICE;
        }
        r = h.r;
    }
    *r_io = r;
    return IM_OK;
}

im_status max_coverage(const im_pool *p, uint64_t begin, uint64_t end, uint32_t k, uint32_t *seeds_host,
                       uint64_t *cov) {
    return max_coverage_on(p->ctx, p, begin, end, k, seeds_host, cov);
}

// Algorithm 2 over sets [begin, end) of a pool whose node ids are below n,
// entries [ebegin, eend) of pnodes.
static im_status greedy_on(im_ctx *ctx, uint32_t n, const uint64_t *poff, const uint32_t *pnodes, uint64_t begin,
                           uint64_t end, uint64_t ebegin, uint64_t eend, uint32_t k, uint32_t *seeds_host,
                           uint64_t *cov) {
    const uint64_t nsets = end - begin;
    const uint64_t entries = eend - ebegin;

    if (k == 1) {
        // one round of Algorithm 2: the node in the most sets of the range;
        // its count is Cov (a node is in a set at most once). No incidence.
        IM_TRY(dev_reserve(ctx, ctx->cover, 4ull * n + 512));  // counts, then the key
        auto *cnt = static_cast<uint32_t *>(ctx->cover.ptr);
        auto *key = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->cover.ptr) +
                                                           ((4ull * n + 255) & ~255ull));
        hipStream_t st = ctx->stream;
        const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
        fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(cnt, n, 0u);
        fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(key), 1, 0);
        if (entries)
            histogram_kernel<<<grid_of(entries, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, ebegin, eend, cnt);
        argmax_count_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(cnt, n, key);
        IM_HIP(hipGetLastError());
        unsigned long long h = 0;
        IM_TRY(to_host_sync(ctx, &h, key, 8));
        seeds_host[0] = ~static_cast<uint32_t>(h);
        *cov = h >> 32;
        return IM_OK;
    }
    // layout of the working arrays in ctx->cover
    const uint64_t tiles = (uint64_t(n) + kTile - 1) / kTile;
    const uint32_t n1 = (n + (1u << kL1Shift) - 1) >> kL1Shift;
    const uint32_t n2 = (n1 + (1u << kL2Shift) - 1) >> kL2Shift;
    const uint64_t covwords = (nsets + 31) / 32 + 1;
    const bool wgc = k && entries <= ctx->greedy_wg_cand_max_entries;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    // the greedy state first: its address stays put from call to call, so
    // cached round graphs that read it through that address replay
    const size_t o_job = take(sizeof(GreedyState));
    const size_t o_gain = take(4ull * n), o_fill = take(4ull * n), o_ioff = take(8ull * (n + 1)),
                 o_tsum = take(8ull * (tiles + 1)), o_cov = take(8), o_seeds = take(4ull * k),
                 o_covbits = take(4ull * covwords), o_isets = take((wgc ? 16ull : 4ull) * (entries + 1)),
                 o_m1 = take(8ull * n1),
                 o_m2 = take(8ull * n2),
                 o_dirty = take(4ull * ((n1 + 31) / 32)), o_bmax = take(8ull * 4096),
                 o_hdr = take(2 * sizeof(StepHdr)), o_cnode = take(4ull * kCandNodes),
                 o_cbase = take(8ull * kCandNodes), o_cdec = take(12ull * kCandNodes),
                 o_hist = take(8ull * kSelBins), o_ccount = take(4);
    IM_TRY(dev_reserve(ctx, ctx->cover, off));
    char *base = static_cast<char *>(ctx->cover.ptr);
    auto at32 = [&](size_t o) { return reinterpret_cast<uint32_t *>(base + o); };
    auto *gain = at32(o_gain);
    auto *fill = at32(o_fill);
    auto *ioff = reinterpret_cast<uint64_t *>(base + o_ioff);
    auto *tsum = reinterpret_cast<uint64_t *>(base + o_tsum);
    auto *dcov = reinterpret_cast<unsigned long long *>(base + o_cov);
    auto *covbits = at32(o_covbits);
    auto *isets = at32(o_isets);

    GreedyState g{};
    g.gain = gain;
    g.m1 = reinterpret_cast<unsigned long long *>(base + o_m1);
    g.m2 = reinterpret_cast<unsigned long long *>(base + o_m2);
    g.covbits = covbits;
    g.ioff = ioff;
    g.isets = isets;
    g.poff = poff;
    g.pnodes = pnodes;
    g.begin = begin;
    g.n = n;
    g.n1 = n1;
    g.n2 = n2;
    g.k = k;
    g.seeds = at32(o_seeds);
    g.cov = dcov;
    g.dirty = at32(o_dirty);
    g.nsets = nsets;
    g.bmax = reinterpret_cast<unsigned long long *>(base + o_bmax);
    g.mark = n1 > ctx->greedy_mark_min_chunks ? 1u : 0u;

    hipStream_t st = ctx->stream;
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(gain, n, 0u);
    fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(fill, n, 0u);
    fill_u32_kernel<<<grid_of(covwords, kThreads, cu * 8), kThreads, 0, st>>>(covbits, covwords, 0u);
    fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(dcov), 1, 0);
    // incidence: counts, offsets, set ids per node
    if (entries)
        histogram_kernel<<<grid_of(entries, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, ebegin, eend, gain);
    tile_sums_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gain, n, tsum);
    tile_scan_kernel<<<1, 1024, 0, st>>>(tsum, tiles);
    tile_apply_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gain, n, tsum, ioff);
    if (wgc) g.iext = reinterpret_cast<const uint4 *>(isets);
    if (nsets && wgc)
        scatter_kernel<true><<<grid_of(nsets * 16, kThreads, cu * 16), kThreads, 0, st>>>(
            poff, pnodes, begin, nsets, ioff, fill, nullptr, reinterpret_cast<uint4 *>(isets));
    else if (nsets)
        scatter_kernel<false><<<grid_of(nsets * 16, kThreads, cu * 16), kThreads, 0, st>>>(
            poff, pnodes, begin, nsets, ioff, fill, isets, nullptr);
    if (wgc) {
        // the first rounds (the large covers) on the grid, two launches each,
        // which keep every gain exact; the rest in one workgroup over
        // candidate nodes
        const uint32_t lead = std::min<uint32_t>(k, ctx->greedy_wg_cand_grid_rounds);
        const uint32_t rg = grid_of(uint64_t(n1), kThreads, cu * 4);
        const uint32_t cg =
            ctx->greedy_cover_blocks
                ? ctx->greedy_cover_blocks
                : std::max<uint32_t>(1, std::min<uint32_t>(cu * 4, grid_of(nsets * 16, kThreads, cu * 4)));
        g.nbmax = rg;
        // grid-wide rounds [r0, r1) from exact gains
        auto grid_rounds = [&](uint32_t r0, uint32_t r1) {
            init_m1_kernel<<<grid_of(n1, kThreads, cu * 8), kThreads, 0, st>>>(g);
            if (g.mark)
                fill_u32_kernel<<<grid_of((n1 + 31) / 32, kThreads, cu), kThreads, 0, st>>>(g.dirty, (n1 + 31) / 32,
                                                                                           0u);
            for (uint32_t r = r0; r < r1; ++r) {
                refresh_kernel<<<rg, kThreads, 0, st>>>(g, r);
                cover_kernel<<<cg, kThreads, 0, st>>>(g, r);
            }
        };
        if (lead) grid_rounds(0, lead);
        g.hdr = reinterpret_cast<StepHdr *>(base + o_hdr);
        g.cnode = at32(o_cnode);
        g.cbase = at32(o_cbase);
        g.hist = at32(o_hist);
        g.ccount = at32(o_ccount);
        fill_u32_kernel<<<grid_of(2 * kSelBins, kThreads, 64), kThreads, 0, st>>>(g.hist, 2 * kSelBins, 0u);
        auto *dg = reinterpret_cast<GreedyState *>(base + o_job);
        IM_HIP(hipMemcpyAsync(dg, &g, sizeof(g), hipMemcpyHostToDevice, st));
        StepHdr *hdr = g.hdr;
        uint32_t grid_from = k;
        IM_TRY(run_wg_cycles(ctx, dg, &hdr, &k, 1, n, nsets, lead, &grid_from));
        // flat gains: level by level, then (if a level's gain is too large
        // for it) the grid-wide rounds
        if (grid_from < k && ctx->greedy_flat_levels) IM_TRY(flat_rounds(ctx, g, entries, &grid_from));
        if (grid_from < k) grid_rounds(grid_from, k);
        IM_HIP(hipGetLastError());
        IM_HIP(hipMemcpyAsync(seeds_host, g.seeds, 4ull * k, hipMemcpyDeviceToHost, st));
        IM_TRY(to_host_sync(ctx, cov, dcov, 8));
        return IM_OK;
    }
    // maximum index, then the rounds
    init_m1_kernel<<<grid_of(n1, kThreads, cu * 8), kThreads, 0, st>>>(g);
    // per-round launches pay for themselves once the cover work per round is
    // large; tiny problems keep every round in one workgroup (which chooses
    // from m2; the per-round launches reduce block maxima of m1 instead)
    const bool small = entries <= ctx->greedy_wg_max_entries;
    if (small) init_m2_kernel<<<grid_of(n2, kThreads, cu * 8), kThreads, 0, st>>>(g);
    const uint32_t big = small ? 0u : k;
    const uint32_t cgrid =
        ctx->greedy_cover_blocks
            ? ctx->greedy_cover_blocks
            : std::max<uint32_t>(1, std::min<uint32_t>(cu * 4, grid_of(nsets * 16, kThreads, cu * 4)));
    const uint32_t rgrid = grid_of(uint64_t(n1), kThreads, cu * 4);
    if (big)
        fill_u32_kernel<<<grid_of((n1 + 31) / 32, kThreads, cu), kThreads, 0, st>>>(g.dirty, (n1 + 31) / 32, 0u);
    g.nbmax = rgrid;
    const uint32_t want = std::min<uint32_t>(ctx->greedy_candidates, kCandMax);
    if (big && want) {
        g.hdr = reinterpret_cast<StepHdr *>(base + o_hdr);
        g.cnode = at32(o_cnode);
        g.cbase = at32(o_cbase);
        g.cdec = at32(o_cdec);
        g.want = want;
        auto *dg = reinterpret_cast<GreedyState *>(base + o_job);
        IM_HIP(hipMemcpyAsync(dg, &g, sizeof(g), hipMemcpyHostToDevice, st));
        IM_TRY(run_steps(ctx, dg, g.hdr, &k, 1, dim3(std::max(rgrid, cgrid), 1)));
    } else if (big) {
        hipGraphExec_t exec = nullptr;
        auto *dg = reinterpret_cast<GreedyState *>(base + o_job);
        if (ctx->greedy_graph) {
            IM_HIP(hipMemcpyAsync(dg, &g, sizeof(g), hipMemcpyHostToDevice, st));
            IM_TRY(round_graph(ctx, dg, big, rgrid, cgrid, &exec));
        }
        if (exec) {
            IM_HIP(hipGraphLaunch(exec, st));
        } else {
            for (uint32_t r = 0; r < big; ++r) {
                refresh_kernel<<<rgrid, kThreads, 0, st>>>(g, r);
                cover_kernel<<<cgrid, kThreads, 0, st>>>(g, r);
            }
        }
    }
    if (big < k) {
        fill_u32_kernel<<<grid_of((n1 + 31) / 32, kThreads, cu), kThreads, 0, st>>>(g.dirty, (n1 + 31) / 32, 0u);
        auto *dg = reinterpret_cast<GreedyState *>(base + o_job);
        IM_HIP(hipMemcpyAsync(dg, &g, sizeof(g), hipMemcpyHostToDevice, st));
        persist_kernel<<<1, kPersistThreads, 0, st>>>(dg, big);
    }
    IM_HIP(hipGetLastError());
    IM_HIP(hipMemcpyAsync(seeds_host, g.seeds, 4ull * k, hipMemcpyDeviceToHost, st));
    IM_TRY(to_host_sync(ctx, cov, dcov, 8));
    return IM_OK;
}

// ---- the greedy over the nodes a range holds ----
//
// Every per-node array and pass of the greedy (gains, incidence offsets,
// the maximum index, their scans) is sized by the graph's n. On a graph much
// larger than the range (a D-SSA iteration's sets on the Twitter-shaped
// graph hold a few million entries of its 41.7 M nodes), the greedy runs
// over the nodes the range holds instead, numbered by rank in id order, so
// that the lowest-id tie-break picks the same nodes. A node the range does
// not hold has gain 0, so it is picked only once every set is covered; the
// rounds from that point are filled here with the lowest unpicked ids, as
// Algorithm 2 over all of V picks them.

__global__ void mark_nodes_kernel(const uint32_t *pnodes, uint64_t eb, uint64_t ee, unsigned long long *bits) {
    for (uint64_t e = eb + blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < ee;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t v = pnodes[e];
        const unsigned long long m = 1ull << (v & 63u);
        // a node in many sets of the range sets its bit once, not once per set
        if (!(__atomic_load_n(&bits[v >> 6], __ATOMIC_RELAXED) & m)) atomicOr(&bits[v >> 6], m);
    }
}

__global__ void word_counts_kernel(const unsigned long long *bits, uint64_t words, uint32_t *cnt) {
    for (uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; w < words;
         w += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        cnt[w] = static_cast<uint32_t>(__popcll(bits[w]));
}

// rank[w]: the held nodes below word w
__global__ void dense_entries_kernel(const uint32_t *pnodes, uint64_t eb, uint64_t ee,
                                     const unsigned long long *bits, const uint64_t *rank, uint32_t *out) {
    for (uint64_t e = eb + blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; e < ee;
         e += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t v = pnodes[e];
        const unsigned long long below = bits[v >> 6] & ((1ull << (v & 63u)) - 1ull);
        out[e - eb] = static_cast<uint32_t>(rank[v >> 6] + static_cast<uint64_t>(__popcll(below)));
    }
}

__global__ void dense_ids_kernel(const unsigned long long *bits, uint64_t words, const uint64_t *rank, uint32_t *ids) {
    for (uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; w < words;
         w += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        unsigned long long b = bits[w];
        uint64_t r = rank[w];
        while (b) {
            ids[r++] = static_cast<uint32_t>(w * 64 + static_cast<uint64_t>(__ffsll(static_cast<long long>(b)) - 1));
            b &= b - 1ull;
        }
    }
}

// offsets of sets [begin, begin + nsets] relative to the first
__global__ void rebase_offsets_kernel(const uint64_t *poff, uint64_t begin, uint64_t nsets, uint64_t *out) {
    const uint64_t base = poff[begin];
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i <= nsets;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        out[i] = poff[begin + i] - base;
}

__global__ void map_ids_kernel(const uint32_t *ids, const uint32_t *dense, uint32_t k, uint32_t *out) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < k; r += gridDim.x * blockDim.x) out[r] = ids[dense[r]];
}

static im_status greedy_dense(im_ctx *ctx, const im_pool *p, uint64_t begin, uint64_t end, uint64_t ebegin,
                              uint64_t eend, uint32_t k, uint32_t *seeds_host, uint64_t *cov) {
    const uint32_t n = p->g->n;
    const uint64_t nsets = end - begin, entries = eend - ebegin;
    const uint64_t words = (uint64_t(n) + 63) / 64;
    const uint64_t tiles = (words + kTile - 1) / kTile;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    const size_t o_bits = take(8 * words), o_cnt = take(4 * words), o_rank = take(8 * (words + 1)),
                 o_tsum = take(8 * (tiles + 1)), o_ent = take(4 * (entries + 1)), o_off = take(8 * (nsets + 1)),
                 o_ids = take(4 * (std::min<uint64_t>(n, entries) + 1)), o_dseeds = take(4ull * k),
                 o_seeds = take(4ull * k);
    IM_TRY(dev_reserve(ctx, ctx->dense, off));
    char *base = static_cast<char *>(ctx->dense.ptr);
    auto *bits = reinterpret_cast<unsigned long long *>(base + o_bits);
    auto *cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
    auto *rank = reinterpret_cast<uint64_t *>(base + o_rank);
    auto *tsum = reinterpret_cast<uint64_t *>(base + o_tsum);
    auto *ent = reinterpret_cast<uint32_t *>(base + o_ent);
    auto *doff = reinterpret_cast<uint64_t *>(base + o_off);
    auto *ids = reinterpret_cast<uint32_t *>(base + o_ids);
    auto *dseeds = reinterpret_cast<uint32_t *>(base + o_dseeds);
    auto *oseeds = reinterpret_cast<uint32_t *>(base + o_seeds);
    const auto *poff = static_cast<const uint64_t *>(p->poff.ptr);
    const auto *pnodes = static_cast<const uint32_t *>(p->pnodes.ptr);
    hipStream_t st = ctx->stream;
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    fill_u64_kernel<<<grid_of(words, kThreads, cu * 8), kThreads, 0, st>>>(reinterpret_cast<uint64_t *>(bits), words,
                                                                           0);
    mark_nodes_kernel<<<grid_of(entries, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, ebegin, eend, bits);
    word_counts_kernel<<<grid_of(words, kThreads, cu * 8), kThreads, 0, st>>>(bits, words, cnt);
    tile_sums_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(cnt, words, tsum);
    tile_scan_kernel<<<1, 1024, 0, st>>>(tsum, tiles);
    tile_apply_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(cnt, words, tsum, rank);
    dense_entries_kernel<<<grid_of(entries, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, ebegin, eend, bits, rank,
                                                                                   ent);
    dense_ids_kernel<<<grid_of(words, kThreads, cu * 8), kThreads, 0, st>>>(bits, words, rank, ids);
    rebase_offsets_kernel<<<grid_of(nsets + 1, kThreads, cu * 4), kThreads, 0, st>>>(poff, begin, nsets, doff);
    IM_HIP(hipGetLastError());
    uint64_t held = 0;
    IM_TRY(to_host_sync(ctx, &held, rank + words, 8));
    if (held == 0 || held > n) {
        set_error("max coverage: %llu nodes held by a range of %llu entries", static_cast<unsigned long long>(held),
                  static_cast<unsigned long long>(entries));
        return IM_E_DEVICE;
    }
    // every held node picked covers every set: rounds past them have gain 0
    const uint32_t kd = static_cast<uint32_t>(std::min<uint64_t>(k, held));
    std::vector<uint32_t> picks(k);
    IM_TRY(greedy_on(ctx, static_cast<uint32_t>(held), doff, ent, 0, nsets, 0, entries, kd, picks.data(), cov));
    IM_HIP(hipMemcpyAsync(dseeds, picks.data(), 4ull * kd, hipMemcpyHostToDevice, st));
    map_ids_kernel<<<grid_of(kd, kThreads, 64), kThreads, 0, st>>>(ids, dseeds, kd, oseeds);
    IM_HIP(hipGetLastError());
    IM_HIP(hipMemcpyAsync(picks.data(), oseeds, 4ull * kd, hipMemcpyDeviceToHost, st));
    IM_HIP(hipStreamSynchronize(st));
    uint32_t positive = kd;
    if (*cov == nsets) {
        // the picks with a gain: the fewest whose sets cover the range
        uint32_t lo = 1, hi = kd;
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            uint64_t c = 0;
            IM_TRY(coverage_range_on(ctx, p, begin, end, picks.data(), mid, &c));
            if (c == nsets) hi = mid;
            else lo = mid + 1;
        }
        positive = nsets ? lo : 0;
    }
    std::copy(picks.begin(), picks.begin() + positive, seeds_host);
    if (positive < k) {  // gain 0 everywhere: the lowest ids not picked yet
        std::vector<uint32_t> taken(picks.begin(), picks.begin() + positive);
        std::sort(taken.begin(), taken.end());
        uint32_t r = positive, v = 0;
        size_t t = 0;
        while (r < k && v < n) {
            while (t < taken.size() && taken[t] < v) ++t;
            if (t < taken.size() && taken[t] == v) {
                ++v;
                continue;
            }
            seeds_host[r++] = v++;
        }
    }
    return IM_OK;
}

im_status max_coverage_on(im_ctx *ctx, const im_pool *p, uint64_t begin, uint64_t end, uint32_t k,
                          uint32_t *seeds_host, uint64_t *cov) {
    const uint32_t n = p->g->n;
    const auto *poff = static_cast<const uint64_t *>(p->poff.ptr);
    const auto *pnodes = static_cast<const uint32_t *>(p->pnodes.ptr);
    uint64_t ends[2] = {0, 0};
    IM_TRY(to_host_sync(ctx, &ends[0], poff + begin, 8));
    IM_TRY(to_host_sync(ctx, &ends[1], poff + end, 8));
    const uint64_t ebegin = ends[0], eend = ends[1];
    const uint64_t entries = eend - ebegin;
    if (k == 1 && begin == 0) {
        // one round over a prefix [0, end): SSA and D-SSA ask for prefixes
        // of one pool that double, so the counts of the last prefix are kept
        // and only the new sets' entries are added (integer counts: the
        // result is the full count's)
        const void *was = ctx->k1_cnt.ptr;
        IM_TRY(dev_reserve(ctx, ctx->k1_cnt, 4ull * n + 512));  // counts, then the key and two picks
        auto *cnt = static_cast<uint32_t *>(ctx->k1_cnt.ptr);
        auto *key = reinterpret_cast<unsigned long long *>(static_cast<char *>(ctx->k1_cnt.ptr) +
                                                           ((4ull * n + 255) & ~255ull));
        hipStream_t st = ctx->stream;
        const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
        uint64_t from = ctx->k1_end;
        if (ctx->k1_cnt.ptr != was || ctx->k1_serial != p->serial || eend < ctx->k1_end) {
            fill_u32_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(cnt, n, 0u);
            from = 0;
        }
        ctx->k1_serial = 0;  // until the counts below are in
        fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(key), 1, 0);
        if (eend > from)
            histogram_kernel<<<grid_of(eend - from, kThreads, cu * 16), kThreads, 0, st>>>(pnodes, from, eend, cnt);
        argmax_count_kernel<<<grid_of(n, kThreads, cu * 8), kThreads, 0, st>>>(cnt, n, key);
        IM_HIP(hipGetLastError());
        unsigned long long h = 0;
        IM_TRY(to_host_sync(ctx, &h, key, 8));
        ctx->k1_serial = p->serial;
        ctx->k1_end = eend;
        seeds_host[0] = ~static_cast<uint32_t>(h);
        *cov = h >> 32;
        return IM_OK;
    }
    // the ranked form once the range holds fewer entries than half the nodes
    // (k = 1 is one count and argmax over the nodes, no cheaper that way)
    if (ctx->greedy_dense && k > 1 && entries && 2 * entries <= n)
        return greedy_dense(ctx, p, begin, end, ebegin, eend, k, seeds_host, cov);
    return greedy_on(ctx, n, poff, pnodes, begin, end, ebegin, eend, k, seeds_host, cov);
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


// Blocks per job of the batched round launches (at most 1024: bmax holds
// 1024 entries per job), and of their refresh step.
static uint32_t batch_blocks_per_job(uint32_t cu, uint32_t nj) {
    return std::min<uint32_t>(1024, std::max<uint32_t>(1, (cu * 4 + nj - 1) / nj));
}

static uint32_t batch_refresh_blocks(uint32_t cu, uint32_t nj, uint32_t n1) {
    return std::min<uint32_t>(batch_blocks_per_job(cu, nj), grid_of(uint64_t(n1), kThreads, cu * 4));
}

im_status max_coverage_batch(im_ctx *ctx, const im_graph *gr, CoverJob *jobs, uint32_t nj) {
    if (nj == 0) return IM_OK;
    const uint32_t n = gr->n;
    hipStream_t st = ctx->stream;
    const uint32_t cu = static_cast<uint32_t>(ctx->cu_count);
    // range ends of every job in one read-back
    std::vector<const uint64_t *> hpoffs(nj);
    std::vector<uint64_t> hb(4ull * nj), he(4ull * nj);
    for (uint32_t j = 0; j < nj; ++j) {
        hpoffs[j] = static_cast<const uint64_t *>(jobs[j].pool->poff.ptr);
        hb[4 * j] = jobs[j].begin;
        hb[4 * j + 1] = jobs[j].end;
        hb[4 * j + 2] = jobs[j].stare_begin;
        hb[4 * j + 3] = jobs[j].stare_end;
    }
    IM_TRY(dev_reserve(ctx, ctx->scan_tmp, nj * (8 + 32 + 32) + 1024));
    auto *d_poffs = static_cast<const uint64_t **>(ctx->scan_tmp.ptr);
    auto *d_b = reinterpret_cast<uint64_t *>(d_poffs + nj);
    auto *d_e = d_b + 4ull * nj;
    IM_HIP(hipMemcpyAsync(d_poffs, hpoffs.data(), 8ull * nj, hipMemcpyHostToDevice, st));
    IM_HIP(hipMemcpyAsync(d_b, hb.data(), 32ull * nj, hipMemcpyHostToDevice, st));
    job_bounds_kernel<<<grid_of(4ull * nj, kThreads, 64), kThreads, 0, st>>>(d_poffs, d_b, nj, d_e);
    IM_HIP(hipMemcpyAsync(he.data(), d_e, 32ull * nj, hipMemcpyDeviceToHost, st));
    IM_HIP(hipStreamSynchronize(st));

    const uint32_t n1 = (n + (1u << kL1Shift) - 1) >> kL1Shift;
    const uint32_t n2 = (n1 + (1u << kL2Shift) - 1) >> kL2Shift;
    const uint64_t words = (uint64_t(n) + 31) / 32;
    uint64_t tot_entries = 0, tot_sets = 0, tot_stare = 0, tot_seeds = 0, tot_cov = 0;
    std::vector<JobTable> jt(nj);
    std::vector<uint64_t> cov_off(nj);
    for (uint32_t j = 0; j < nj; ++j) {
        const CoverJob &cj = jobs[j];
        jt[j].begin = cj.begin;
        jt[j].ebegin = he[4 * j];
        jt[j].set_start = tot_sets;
        jt[j].entry_start = tot_entries;
        jt[j].stare_begin = cj.stare_begin;
        jt[j].stare_start = tot_stare;
        jt[j].seed_start = tot_seeds;
        cov_off[j] = tot_cov;
        tot_entries += he[4 * j + 1] - he[4 * j];
        tot_sets += cj.end - cj.begin;
        tot_stare += cj.stare_end - cj.stare_begin;
        tot_seeds += cj.k;
        tot_cov += (cj.end - cj.begin + 31) / 32 + 1;
    }
    uint64_t max_entries = 0, max_sets = 0;
    uint32_t max_k = 0;
    for (uint32_t j = 0; j < nj; ++j) {
        max_entries = std::max<uint64_t>(max_entries, he[4 * j + 1] - he[4 * j]);
        max_sets = std::max<uint64_t>(max_sets, jobs[j].end - jobs[j].begin);
        max_k = std::max(max_k, jobs[j].k);
    }
    // one-workgroup rounds over candidate nodes, a workgroup per job (each
    // re-selection passes over every node once per job, so the node count
    // is held to the same limit as the ranges)
    const bool wgc = max_k && max_entries <= ctx->greedy_wg_cand_batch && uint64_t(n) <= ctx->greedy_wg_cand_batch &&
                     max_entries <= ctx->greedy_wg_cand_max_entries;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = (off + bytes + 255) & ~size_t(255);
        return at;
    };
    const uint64_t cells = uint64_t(nj) * n;
    const uint64_t tiles = (cells + kTile - 1) / kTile;
    const size_t o_gain = take(4 * cells), o_fill = take(4 * cells), o_prefix = take(8 * (cells + 1)),
                 o_tsum = take(8 * (tiles + 1)), o_isets = take((wgc ? 16 : 4) * (tot_entries + 1)),
                 o_covbits = take(4 * tot_cov),
                 o_m1 = take(8ull * nj * n1), o_m2 = take(8ull * nj * n2), o_seeds = take(4 * (tot_seeds + 1)),
                 o_cov = take(8ull * nj), o_covc = take(8ull * nj), o_bits = take(4 * words * nj),
                 o_jt = take(sizeof(JobTable) * nj), o_gs = take(sizeof(GreedyState) * nj),
                 o_dirty = take(4ull * nj * ((n1 + 31) / 32)),
                 o_bmax = take(8ull * nj * 1024), o_hdr = take(2 * sizeof(StepHdr) * nj),
                 o_cnode = take(4ull * kCandNodes * nj), o_cbase = take(8ull * kCandNodes * nj), o_cdec = take(12ull * kCandNodes * nj),
                 o_hist = take(8ull * kSelBins * nj), o_ccount = take(4ull * nj);
    IM_TRY(dev_reserve(ctx, ctx->cover, off));
    char *base = static_cast<char *>(ctx->cover.ptr);
    auto *gains = reinterpret_cast<uint32_t *>(base + o_gain);
    auto *fills = reinterpret_cast<uint32_t *>(base + o_fill);
    auto *prefix = reinterpret_cast<uint64_t *>(base + o_prefix);
    auto *tsum = reinterpret_cast<uint64_t *>(base + o_tsum);
    auto *isets = reinterpret_cast<uint32_t *>(base + o_isets);
    auto *covbits = reinterpret_cast<uint32_t *>(base + o_covbits);
    auto *seeds = reinterpret_cast<uint32_t *>(base + o_seeds);
    auto *covs = reinterpret_cast<unsigned long long *>(base + o_cov);
    auto *covcs = reinterpret_cast<unsigned long long *>(base + o_covc);
    auto *bits = reinterpret_cast<uint32_t *>(base + o_bits);
    auto *djt = reinterpret_cast<JobTable *>(base + o_jt);
    auto *dgs = reinterpret_cast<GreedyState *>(base + o_gs);
    std::vector<GreedyState> gs(nj);
    for (uint32_t j = 0; j < nj; ++j) {
        const CoverJob &cj = jobs[j];
        jt[j].poff = static_cast<const uint64_t *>(cj.pool->poff.ptr);
        jt[j].pnodes = static_cast<const uint32_t *>(cj.pool->pnodes.ptr);
        jt[j].gain = gains + uint64_t(j) * n;
        jt[j].fill = fills + uint64_t(j) * n;
        jt[j].stare_bits = bits + uint64_t(j) * words;
        jt[j].cov_c = covcs + j;
        GreedyState &g = gs[j];
        g.gain = jt[j].gain;
        g.m1 = reinterpret_cast<unsigned long long *>(base + o_m1) + uint64_t(j) * n1;
        g.m2 = reinterpret_cast<unsigned long long *>(base + o_m2) + uint64_t(j) * n2;
        g.covbits = covbits + cov_off[j];
        g.ioff = prefix + uint64_t(j) * n;
        g.isets = isets;
        g.poff = jt[j].poff;
        g.pnodes = jt[j].pnodes;
        g.begin = cj.begin;
        g.n = n;
        g.n1 = n1;
        g.n2 = n2;
        g.k = cj.k;
        g.seeds = seeds + jt[j].seed_start;
        g.bmax = reinterpret_cast<unsigned long long *>(base + o_bmax) + 1024ull * j;
        g.nbmax = batch_refresh_blocks(cu, nj, n1);
        g.mark = n1 > ctx->greedy_mark_min_chunks ? 1u : 0u;
        g.cov = covs + j;
        g.dirty = reinterpret_cast<uint32_t *>(base + o_dirty) + uint64_t(j) * ((n1 + 31) / 32);
        g.nsets = cj.end - cj.begin;
        g.hdr = reinterpret_cast<StepHdr *>(base + o_hdr) + 2ull * j;
        g.cnode = reinterpret_cast<uint32_t *>(base + o_cnode) + uint64_t(kCandNodes) * j;
        g.cbase = reinterpret_cast<uint32_t *>(base + o_cbase) + 2ull * kCandNodes * j;
        g.cdec = reinterpret_cast<uint32_t *>(base + o_cdec) + 3ull * kCandNodes * j;
        g.want = std::min<uint32_t>(ctx->greedy_candidates_batch, kCandMax);
        if (wgc) {
            g.iext = reinterpret_cast<const uint4 *>(isets);
            g.hist = reinterpret_cast<uint32_t *>(base + o_hist) + 2ull * kSelBins * j;
            g.ccount = reinterpret_cast<uint32_t *>(base + o_ccount) + j;
        }
    }
    IM_HIP(hipMemcpyAsync(djt, jt.data(), sizeof(JobTable) * nj, hipMemcpyHostToDevice, st));
    IM_HIP(hipMemcpyAsync(dgs, gs.data(), sizeof(GreedyState) * nj, hipMemcpyHostToDevice, st));
    fill_u32_kernel<<<grid_of(cells, kThreads, cu * 8), kThreads, 0, st>>>(gains, cells, 0u);
    fill_u32_kernel<<<grid_of(cells, kThreads, cu * 8), kThreads, 0, st>>>(fills, cells, 0u);
    fill_u32_kernel<<<grid_of(tot_cov, kThreads, cu * 8), kThreads, 0, st>>>(covbits, tot_cov, 0u);
    fill_u32_kernel<<<grid_of(words * nj, kThreads, cu * 8), kThreads, 0, st>>>(bits, words * nj, 0u);
    fill_u32_kernel<<<grid_of(uint64_t(nj) * ((n1 + 31) / 32), kThreads, cu * 8), kThreads, 0, st>>>(
        reinterpret_cast<uint32_t *>(base + o_dirty), uint64_t(nj) * ((n1 + 31) / 32), 0u);
    fill_u64_kernel<<<1, 256, 0, st>>>(reinterpret_cast<uint64_t *>(covs), nj, 0);
    fill_u64_kernel<<<1, 256, 0, st>>>(reinterpret_cast<uint64_t *>(covcs), nj, 0);
    if (tot_entries)
        batch_histogram_kernel<<<grid_of(tot_entries, kThreads, cu * 16), kThreads, 0, st>>>(djt, nj, tot_entries);
    tile_sums_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gains, cells, tsum);
    tile_scan_kernel<<<1, 1024, 0, st>>>(tsum, tiles);
    tile_apply_kernel<<<static_cast<uint32_t>(tiles), kThreads, 0, st>>>(gains, cells, tsum, prefix);
    if (tot_sets && wgc)
        batch_scatter_kernel<true><<<grid_of(tot_sets * 16, kThreads, cu * 16), kThreads, 0, st>>>(
            djt, nj, tot_sets, prefix, n, nullptr, reinterpret_cast<uint4 *>(isets));
    else if (tot_sets)
        batch_scatter_kernel<false><<<grid_of(tot_sets * 16, kThreads, cu * 16), kThreads, 0, st>>>(
            djt, nj, tot_sets, prefix, n, isets, nullptr);
    batch_init_m1_kernel<<<grid_of(uint64_t(nj) * n1, kThreads, cu * 8), kThreads, 0, st>>>(dgs, nj, n1);
    batch_init_m2_kernel<<<grid_of(uint64_t(nj) * n2, kThreads, cu * 8), kThreads, 0, st>>>(dgs, nj, n2);
    // ranges up to the one-workgroup limit all run their rounds in one
    // launch; beyond it every round is two grid launches shared by all jobs
    if (wgc) {
        // the first rounds grid-wide (two launches each, shared by all jobs),
        // then a workgroup per job over candidate nodes; a job whose cut
        // keeps too few candidates finishes with grid-wide rounds of its own
        const uint32_t per = batch_blocks_per_job(cu, nj);
        const uint32_t rx = batch_refresh_blocks(cu, nj, n1);
        const uint32_t cx = std::min<uint32_t>(per, std::max<uint32_t>(1, grid_of(max_entries * 16, kThreads, cu * 4)));
        const uint32_t lead = std::min<uint32_t>(max_k, ctx->greedy_wg_cand_grid_rounds);
        for (uint32_t r = 0; r < lead; ++r) {
            batch_refresh_kernel<<<dim3(rx, nj), kThreads, 0, st>>>(dgs, r);
            batch_cover_kernel<<<dim3(cx, nj), kThreads, 0, st>>>(dgs, r);
        }
        fill_u32_kernel<<<grid_of(2ull * kSelBins * nj, kThreads, cu), kThreads, 0, st>>>(
            reinterpret_cast<uint32_t *>(base + o_hist), 2ull * kSelBins * nj, 0u);
        std::vector<StepHdr *> hdrs(nj);
        std::vector<uint32_t> ks(nj), from(nj);
        for (uint32_t j = 0; j < nj; ++j) {
            hdrs[j] = gs[j].hdr;
            ks[j] = jobs[j].k;
        }
        IM_TRY(run_wg_cycles(ctx, dgs, hdrs.data(), ks.data(), nj, n, max_sets, lead, from.data()));
        for (uint32_t j = 0; j < nj; ++j) {
            if (from[j] >= ks[j]) continue;
            GreedyState g = gs[j];
            const uint32_t rg = grid_of(uint64_t(n1), kThreads, cu * 4);  // at most 1024: bmax holds 1024 per job
            const uint32_t cg = std::max<uint32_t>(1, std::min<uint32_t>(cu * 4, grid_of(g.nsets * 16, kThreads, cu * 4)));
            g.nbmax = rg;
            init_m1_kernel<<<grid_of(n1, kThreads, cu * 8), kThreads, 0, st>>>(g);
            if (g.mark)
                fill_u32_kernel<<<grid_of((n1 + 31) / 32, kThreads, cu), kThreads, 0, st>>>(g.dirty, (n1 + 31) / 32,
                                                                                           0u);
            for (uint32_t r = from[j]; r < ks[j]; ++r) {
                refresh_kernel<<<rg, kThreads, 0, st>>>(g, r);
                cover_kernel<<<cg, kThreads, 0, st>>>(g, r);
            }
        }
    } else if (max_entries <= ctx->greedy_wg_max_entries) {
        persist_kernel<<<nj, kPersistThreads, 0, st>>>(dgs, 0);
    } else {
        const uint32_t per = batch_blocks_per_job(cu, nj);
        const uint32_t rx = batch_refresh_blocks(cu, nj, n1);
        const uint32_t cx = std::min<uint32_t>(per, std::max<uint32_t>(1, grid_of(max_entries * 16, kThreads, cu * 4)));
        if (ctx->greedy_candidates_batch) {
            std::vector<uint32_t> ks(nj);
            for (uint32_t j = 0; j < nj; ++j) ks[j] = jobs[j].k;
            IM_TRY(run_steps(ctx, dgs, reinterpret_cast<StepHdr *>(base + o_hdr), ks.data(), nj,
                             dim3(std::max(rx, cx), nj)));
        } else {
            for (uint32_t r = 0; r < max_k; ++r) {
                batch_refresh_kernel<<<dim3(rx, nj), kThreads, 0, st>>>(dgs, r);
                batch_cover_kernel<<<dim3(cx, nj), kThreads, 0, st>>>(dgs, r);
            }
        }
    }
    if (tot_stare) {
        batch_seed_bits_kernel<<<grid_of(tot_seeds, kThreads, cu * 4), kThreads, 0, st>>>(djt, nj, seeds, tot_seeds);
        batch_coverage_kernel<<<grid_of(tot_stare * 16, kThreads, cu * 16), kThreads, 0, st>>>(djt, nj, tot_stare);
    }
    IM_HIP(hipGetLastError());
    std::vector<uint32_t> hseeds(tot_seeds);
    std::vector<unsigned long long> hcov(2ull * nj);
    IM_HIP(hipMemcpyAsync(hseeds.data(), seeds, 4 * tot_seeds, hipMemcpyDeviceToHost, st));
    IM_HIP(hipMemcpyAsync(hcov.data(), covs, 8ull * nj, hipMemcpyDeviceToHost, st));
    IM_HIP(hipMemcpyAsync(hcov.data() + nj, covcs, 8ull * nj, hipMemcpyDeviceToHost, st));
    IM_HIP(hipStreamSynchronize(st));
    for (uint32_t j = 0; j < nj; ++j) {
        std::copy(hseeds.begin() + jt[j].seed_start, hseeds.begin() + jt[j].seed_start + jobs[j].k, jobs[j].seeds);
        jobs[j].cov = hcov[j];
        jobs[j].cov_c = hcov[nj + j];
    }
    return IM_OK;
}

im_status first_crossing_items(im_ctx *ctx, const CrossItem *items, uint32_t nitems) {
    if (nitems == 0) return IM_OK;
    hipStream_t st = ctx->stream;
    IM_TRY(dev_reserve(ctx, ctx->scan_tmp, 40ull * nitems + 256));
    auto *dseg = static_cast<uint64_t *>(ctx->scan_tmp.ptr);
    auto *dout = reinterpret_cast<long long *>(dseg + 3ull * nitems);
    std::vector<uint64_t> seg(3ull * nitems);
    for (uint32_t i = 0; i < nitems; ++i) {
        seg[3 * i] = items[i].start;
        seg[3 * i + 1] = items[i].count;
        seg[3 * i + 2] = items[i].need;
    }
    IM_HIP(hipMemcpyAsync(dseg, seg.data(), 24ull * nitems, hipMemcpyHostToDevice, st));
    crossing_items_kernel<<<nitems, 1024, 0, st>>>(static_cast<const uint8_t *>(ctx->zflags.ptr), dseg, dout);
    IM_HIP(hipGetLastError());
    std::vector<long long> out(2ull * nitems);
    IM_HIP(hipMemcpyAsync(out.data(), dout, 16ull * nitems, hipMemcpyDeviceToHost, st));
    IM_HIP(hipStreamSynchronize(st));
    for (uint32_t i = 0; i < nitems; ++i) {
        items[i].index[0] = out[2 * i];
        items[i].hits[0] = static_cast<uint64_t>(out[2 * i + 1]);
    }
    return IM_OK;
}
}  // namespace im

// ------------------------------------------- stare step, no allocation ----
//
// im_coverage_range_noalloc: the coverage count of im_coverage_range (Eq. 1,
// the D-SSA stare step) for callers that cannot allocate device memory. Its
// scratch (a counter, the bad-seed flag, the seed list and the seed bitmap)
// is the file-scope array below instead of context buffers. Each GPU the
// library runs on holds one copy of it until the process ends, and every
// call on that GPU shares it. Host code never passes `scratch` itself to a
// kernel or a copy: it uses the device address taken once per device by
// noalloc_scratch_init.

constexpr uint32_t kNaMaxN = 1u << 26;  // nodes: bitmap of 2^21 words (8 MiB)
constexpr uint32_t kNaMaxK = 1u << 16;  // seeds
constexpr size_t kNaHead = 256;         // u64 counter at 0, u32 bad-seed flag at 8
constexpr size_t kNaSeedBytes = 4ull * kNaMaxK;
constexpr size_t kNaBitBytes = 4ull * (kNaMaxN / 32);
constexpr size_t kNaBytes = kNaHead + kNaSeedBytes + kNaBitBytes;

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};
}  // namespace

namespace im {

im_status noalloc_scratch_init(int device) {
    if (device < 0 || device >= kNaMaxDevices) {
        set_error("device %d beyond the %d the no-allocation scratch table covers", device, kNaMaxDevices);
        return IM_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (g_na_ptr[device]) return IM_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        set_error("hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
        return IM_E_DEVICE;
    }
    g_na_ptr[device] = ptr;
    return IM_OK;
}

}  // namespace im

extern "C" im_status im_coverage_range_noalloc(const im_pool *p, uint64_t begin, uint64_t end, const uint32_t *seeds,
                                               uint32_t k, uint64_t *cov_out) {
    using namespace im;
    clear_error();
    if (!p || !cov_out || (k && !seeds) || begin > end || end > p->count) {
        set_error("im_coverage_range_noalloc: bad arguments");
        return IM_E_ARG;
    }
    const uint32_t n = p->g->n;
    if (n > kNaMaxN || k > kNaMaxK) {
        set_error("im_coverage_range_noalloc: n = %u, k = %u beyond its fixed scratch (n <= %u, k <= %u)", n, k,
                  kNaMaxN, kNaMaxK);
        return IM_E_ARG;
    }
    im_ctx *ctx = p->ctx;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_na_mu);
        if (ctx->device >= 0 && ctx->device < kNaMaxDevices) base = g_na_ptr[ctx->device];
    }
    if (!base) {
        set_error("im_coverage_range_noalloc: no scratch address for device %d", ctx->device);
        return IM_E_STATE;
    }
    char *b = static_cast<char *>(base);
    auto *cnt = reinterpret_cast<unsigned long long *>(b);
    auto *bad = reinterpret_cast<uint32_t *>(b + 8);
    auto *dseeds = reinterpret_cast<uint32_t *>(b + kNaHead);
    auto *bits = reinterpret_cast<uint32_t *>(b + kNaHead + kNaSeedBytes);
    const uint64_t words = (uint64_t(n) + 31) / 32;
    hipStream_t st = ctx->stream;
    // the array keeps the last call's contents: clear what starts at zero
    fill_u32_kernel<<<grid_of(words, kThreads, 1024), kThreads, 0, st>>>(bits, words, 0u);
    fill_u64_kernel<<<1, 64, 0, st>>>(reinterpret_cast<uint64_t *>(cnt), 1, 0);
    fill_u32_kernel<<<1, 64, 0, st>>>(bad, 1, 0u);
    IM_HIP(hipGetLastError());
    // seeds go through the context's pinned host buffer, 1024 at a time
    for (uint32_t off = 0; off < k; off += 1024) {
        const uint32_t c = std::min<uint32_t>(1024, k - off);
        std::memcpy(ctx->host_pinned, seeds + off, 4ull * c);
        IM_HIP(hipMemcpyAsync(dseeds + off, ctx->host_pinned, 4ull * c, hipMemcpyHostToDevice, st));
        IM_HIP(hipStreamSynchronize(st));
    }
    if (k) seed_bits_kernel<<<grid_of(k, kThreads, 64), kThreads, 0, st>>>(dseeds, k, bits, bad, n);
    if (end > begin) {
        coverage_kernel<<<grid_of((end - begin) * 16, kThreads, ctx->cu_count * 16), kThreads, 0, st>>>(
            static_cast<const uint64_t *>(p->poff.ptr), static_cast<const uint32_t *>(p->pnodes.ptr), begin, end,
            bits, cnt);
    }
    IM_HIP(hipGetLastError());
    uint64_t head[2] = {0, 0};
    IM_TRY(to_host_sync(ctx, head, b, 16));
    if (static_cast<uint32_t>(head[1])) {
        set_error("im_coverage_range_noalloc: seed id >= n");
        return IM_E_ARG;
    }
    *cov_out = head[0];
    return IM_OK;
}
