// Streaming read of device memory: the attainable HBM read bandwidth that the
// search's gathers are measured against (next to the vendor peak).  Not part
// of the search path.
#include "internal.h"

namespace hnsw {
namespace {

constexpr uint32_t kProbeThreads = 256, kProbeUnroll = 4;

// Every thread reads 16-byte words at stride (grid threads), four loads in
// flight per iteration, and folds them with XOR; one word per block is
// written, so no load can be dropped.
__global__ __launch_bounds__(kProbeThreads) void read_probe_kernel(const uint4 *buf, uint64_t words, uint32_t *out) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kProbeThreads;
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kProbeUnroll - 1) * stride < words; i += kProbeUnroll * stride) {
        uint4 v[kProbeUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; ++u) v[u] = buf[i + u * stride];
#pragma unroll
        for (uint32_t u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < words; i += stride) {
        const uint4 v = buf[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    __shared__ uint32_t red[kProbeThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (uint32_t s = kProbeThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace
}  // namespace hnsw

extern "C" hnsw_status hnsw_read_probe(const void *buf, uint64_t bytes, uint32_t *out, uint32_t blocks, void *stream) {
    using namespace hnsw;
    if (!buf || !out || bytes % 16 != 0 || blocks == 0 || blocks > 65536) return HNSW_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return HNSW_ERR_INVALID_ARG;
    if (!is_device_ptr(buf) || !is_device_ptr(out)) return HNSW_ERR_INVALID_ARG;
    hipLaunchKernelGGL(read_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint4 *>(buf), bytes / 16, out);
    if (hipGetLastError() != hipSuccess) return HNSW_ERR_DEVICE;
    return HNSW_OK;
}
