// Random-gather bandwidth probe: the memory roofline the RR-set samplers
// run against. Threads read segments of a fixed size at hashed random
// segment-aligned offsets of a large device buffer (well beyond the 256 MB
// last-level cache) and fold them into one word each, so every byte loaded
// is used. Reported bandwidth counts only the segment bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Each lane gathers `reps` segments of kSeg16 x 16 bytes; the loads of a
// segment, and of several segments, are independent and issued together.
template <uint32_t kSeg16>
__global__ __launch_bounds__(kThreads) void gather_kernel(const uint4 *buf, uint64_t nseg, uint32_t reps,
                                                           uint32_t seed, uint32_t *out) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
#pragma unroll 4
    for (uint32_t r = 0; r < reps; ++r) {
        const uint32_t h1 = mix32(gid * 0x9E3779B9u + r * 0x85EBCA6Bu + seed);
        const uint32_t h2 = mix32(h1 ^ 0x27d4eb2fu);
        const uint64_t idx = ((static_cast<uint64_t>(h1) << 32) | h2) % nseg;
        const uint4 *p = buf + idx * kSeg16;
#pragma unroll
        for (uint32_t i = 0; i < kSeg16; ++i) {
            const uint4 q = p[i];
            acc ^= q.x ^ q.y ^ q.z ^ q.w;
        }
    }
    out[gid] = acc;
}

bool launch_gather(uint32_t seg16, uint32_t blocks, const uint4 *buf, uint64_t nseg, uint32_t reps, uint32_t seed,
                   uint32_t *out) {
    switch (seg16) {
    case 1: gather_kernel<1><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    case 2: gather_kernel<2><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    case 4: gather_kernel<4><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    case 8: gather_kernel<8><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    case 16: gather_kernel<16><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    case 32: gather_kernel<32><<<blocks, kThreads>>>(buf, nseg, reps, seed, out); break;
    default: return false;
    }
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
// 32, 64, 128, 256 or 512) from a `buffer_bytes` device buffer on `device`, best of
// `trials` timed launches; *gbs_out receives it. Returns 0, or -1 on a HIP
// error or bad argument. The buffer is allocated and freed here.
extern "C" int im_probe_gather(int device, uint64_t buffer_bytes, uint32_t seg_bytes, uint32_t trials,
                               double *gbs_out) {
    const uint32_t seg16 = seg_bytes / 16;
    if (!gbs_out || seg_bytes % 16 || (seg16 & (seg16 - 1)) || seg16 == 0 || seg16 > 32 || buffer_bytes < seg_bytes ||
        trials == 0)
        return -1;
    if (hipSetDevice(device) != hipSuccess) return -1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return -1;
    const uint64_t n16 = buffer_bytes / 16;
    const uint64_t nseg = buffer_bytes / seg_bytes;
    uint4 *buf = nullptr;
    uint32_t *out = nullptr;
    const uint32_t blocks = static_cast<uint32_t>(prop.multiProcessorCount) * 16;
    const uint32_t lanes = blocks * kThreads;
    if (hipMalloc(&buf, n16 * 16) != hipSuccess) return -1;
    if (hipMalloc(&out, lanes * 4ull) != hipSuccess) {
        (void)hipFree(buf);
        return -1;
    }
    hipEvent_t b, e;
    int rc = -1;
    if (hipEventCreate(&b) == hipSuccess && hipEventCreate(&e) == hipSuccess) {
        fill_kernel<<<blocks, kThreads>>>(buf, n16);
        // about 4 GB of segment bytes per launch
        const uint32_t reps = static_cast<uint32_t>(
            std::max<uint64_t>(1, (4ull << 30) / (static_cast<uint64_t>(lanes) * seg_bytes)));
        bool ok = launch_gather(seg16, blocks, buf, nseg, 1, 7u, out);  // warm-up
        double best = 0.0;
        ok = ok && hipDeviceSynchronize() == hipSuccess;
        for (uint32_t t = 0; ok && t < trials; ++t) {
            ok = hipEventRecord(b, nullptr) == hipSuccess;
            ok = ok && launch_gather(seg16, blocks, buf, nseg, reps, 1000u + t, out);
            ok = ok && hipEventRecord(e, nullptr) == hipSuccess && hipEventSynchronize(e) == hipSuccess;
            float ms = 0.f;
            ok = ok && hipEventElapsedTime(&ms, b, e) == hipSuccess;
            if (ok && ms > 0.f) {
                const double gbs = static_cast<double>(lanes) * reps * seg_bytes / (ms * 1e-3) / 1e9;
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
