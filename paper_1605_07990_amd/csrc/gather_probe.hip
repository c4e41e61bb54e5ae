// Random-gather bandwidth probe: the memory roofline the RR-set samplers
// run against. Segments of a fixed size are read at hashed random
// segment-aligned offsets of a large device buffer (well beyond the 256 MB
// last-level cache) and folded into one word per lane, so every byte loaded
// is used. Reported bandwidth counts only the segment bytes.
//
// Two access shapes, and the faster one is the roofline:
//   lane  each lane reads a whole segment by itself (its 16-byte pieces one
//         after another), so one wave instruction touches 64 segments;
//   coop  the lanes of a wave split segments between them, 16 bytes per
//         lane, as the IC sampler reads an in-list: a 64-byte segment takes
//         4 lanes (16 segments per wave instruction), a 512-byte one 32.
//         Eight independent segments per lane are in flight at once.
// Segment indices come from a power-of-two mask of a 32-bit hash (the
// buffer holds a power-of-two number of segments), not a division.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kCoopBatch = 8;  // independent segments in flight per lane

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// lane shape: each lane gathers `reps` segments of kSeg16 x 16 bytes.
template <uint32_t kSeg16>
__global__ __launch_bounds__(kThreads) void gather_lane_kernel(const uint4 *buf, uint32_t seg_mask, uint32_t reps,
                                                                uint32_t seed, uint32_t *out) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
#pragma unroll 4
    for (uint32_t r = 0; r < reps; ++r) {
        const uint32_t idx = mix32(gid * 0x9E3779B9u + r * 0x85EBCA6Bu + seed) & seg_mask;
        const uint4 *p = buf + static_cast<uint64_t>(idx) * kSeg16;
#pragma unroll
        for (uint32_t i = 0; i < kSeg16; ++i) {
            const uint4 q = p[i];
            acc ^= q.x ^ q.y ^ q.z ^ q.w;
        }
    }
    out[gid] = acc;
}

// coop shape: kSeg16 consecutive lanes read one segment, 16 bytes each;
// every lane issues kCoopBatch independent segment loads per step.
template <uint32_t kSeg16>
__global__ __launch_bounds__(kThreads) void gather_coop_kernel(const uint4 *buf, uint32_t seg_mask, uint32_t reps,
                                                                uint32_t seed, uint32_t *out) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t group = gid / kSeg16;  // the lanes sharing a segment
    const uint32_t piece = gid % kSeg16;  // this lane's 16-byte piece of it
    uint32_t acc = 0;
    for (uint32_t r = 0; r < reps; r += kCoopBatch) {
        uint4 q[kCoopBatch];
#pragma unroll
        for (uint32_t b = 0; b < kCoopBatch; ++b) {
            const uint32_t idx = mix32(group * 0x9E3779B9u + (r + b) * 0x85EBCA6Bu + seed) & seg_mask;
            q[b] = buf[static_cast<uint64_t>(idx) * kSeg16 + piece];
        }
#pragma unroll
        for (uint32_t b = 0; b < kCoopBatch; ++b) acc ^= q[b].x ^ q[b].y ^ q[b].z ^ q[b].w;
    }
    out[gid] = acc;
}

bool launch_gather(bool coop, uint32_t seg16, uint32_t blocks, const uint4 *buf, uint32_t seg_mask, uint32_t reps,
                   uint32_t seed, uint32_t *out) {
#define IM_PROBE_CASE(S)                                                                         \
    case S:                                                                                      \
        if (coop)                                                                                \
            gather_coop_kernel<S><<<blocks, kThreads>>>(buf, seg_mask, reps, seed, out);         \
        else                                                                                     \
            gather_lane_kernel<S><<<blocks, kThreads>>>(buf, seg_mask, reps, seed, out);         \
        break;
    switch (seg16) {
        IM_PROBE_CASE(1)
        IM_PROBE_CASE(2)
        IM_PROBE_CASE(4)
        IM_PROBE_CASE(8)
        IM_PROBE_CASE(16)
        IM_PROBE_CASE(32)
    default: return false;
    }
#undef IM_PROBE_CASE
    return hipGetLastError() == hipSuccess;
}

__global__ void fill_kernel(uint4 *buf, uint64_t n16) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n16;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t v = static_cast<uint32_t>(i);
        buf[i] = make_uint4(v, v ^ 1u, v ^ 2u, v ^ 3u);
    }
}

}  // namespace

// Bandwidth (GB/s of segment bytes) of random gathers of `seg_bytes` (16,
// 32, 64, 128, 256 or 512) from a device buffer of `buffer_bytes` rounded
// down to a power-of-two number of segments (at most 2^32), on `device`;
// shape 0 = lane, 1 = coop (see above). Best of `trials` timed launches
// goes to *gbs_out. Returns 0, or -1 on a HIP error or bad argument. The
// buffer is allocated and freed here.
extern "C" int im_probe_gather_shape(int device, uint64_t buffer_bytes, uint32_t seg_bytes, uint32_t trials,
                                     int shape, double *gbs_out) {
    const uint32_t seg16 = seg_bytes / 16;
    if (!gbs_out || seg_bytes % 16 || (seg16 & (seg16 - 1)) || seg16 == 0 || seg16 > 32 || buffer_bytes < seg_bytes ||
        trials == 0 || (shape != 0 && shape != 1))
        return -1;
    uint64_t nseg = 1;
    while (nseg * 2 <= buffer_bytes / seg_bytes && nseg * 2 <= (1ull << 32)) nseg *= 2;
    const uint32_t seg_mask = static_cast<uint32_t>(nseg - 1);
    const uint64_t n16 = nseg * seg16;
    if (hipSetDevice(device) != hipSuccess) return -1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -1;
    uint4 *buf = nullptr;
    uint32_t *out = nullptr;
    const uint32_t blocks = static_cast<uint32_t>(prop.multiProcessorCount) * 16;
    const uint32_t lanes = blocks * kThreads;
    if (hipMalloc(&buf, n16 * 16) != hipSuccess) return -1;
    if (hipMalloc(&out, lanes * 4ull) != hipSuccess) {
        (void)hipFree(buf);
        return -1;
    }
    const bool coop = shape == 1;
    // segments per lane: the lane shape reads a whole segment per rep; the
    // coop shape one 16-byte piece of one, in batches of kCoopBatch
    const uint64_t bytes_per_rep = coop ? 16ull * lanes : static_cast<uint64_t>(lanes) * seg_bytes;
    uint32_t reps = static_cast<uint32_t>(std::max<uint64_t>(1, (4ull << 30) / bytes_per_rep));  // ~4 GB
    if (coop) reps = (reps + kCoopBatch - 1) / kCoopBatch * kCoopBatch;
    hipEvent_t b, e;
    int rc = -1;
    if (hipEventCreate(&b) == hipSuccess && hipEventCreate(&e) == hipSuccess) {
        fill_kernel<<<blocks, kThreads>>>(buf, n16);
        bool ok = launch_gather(coop, seg16, blocks, buf, seg_mask, coop ? kCoopBatch : 1, 7u, out);  // warm-up
        double best = 0.0;
        ok = ok && hipDeviceSynchronize() == hipSuccess;
        for (uint32_t t = 0; ok && t < trials; ++t) {
            ok = hipEventRecord(b, nullptr) == hipSuccess;
            ok = ok && launch_gather(coop, seg16, blocks, buf, seg_mask, reps, 1000u + t, out);
            ok = ok && hipEventRecord(e, nullptr) == hipSuccess && hipEventSynchronize(e) == hipSuccess;
            float ms = 0.f;
            ok = ok && hipEventElapsedTime(&ms, b, e) == hipSuccess;
            if (ok && ms > 0.f) {
                const double gbs = static_cast<double>(bytes_per_rep) * reps / (ms * 1e-3) / 1e9;
                best = gbs > best ? gbs : best;
            }
        }
        if (ok) {
            *gbs_out = best;
            rc = 0;
        }
        (void)hipEventDestroy(b);
        (void)hipEventDestroy(e);
    }
    (void)hipFree(out);
    (void)hipFree(buf);
    return rc;
}

// The lane shape alone (the form earlier measurements used).
extern "C" int im_probe_gather(int device, uint64_t buffer_bytes, uint32_t seg_bytes, uint32_t trials,
                               double *gbs_out) {
    return im_probe_gather_shape(device, buffer_bytes, seg_bytes, trials, 0, gbs_out);
}
