// Low-precision copies of the vector store for the traversal of a
// low-precision search: BF16 (round to nearest even) and OCP FP8-E4M3 with a
// per-vector fp32 scale s = max_j |x_j| / 448 (s = 1 for an all-zero row),
// codes = nearest E4M3 value to x_j / s, ties to even, saturating at 448.
// The 8-bit integer copy (an integer-valued store like SIFT's, which the
// paper searched with integer distance functions, Sec. 5.4): code = x rounded
// to the nearest integer (ties to even) and clamped to [0, 255].
// Row layouts (16-byte pieces): BF16 and 8-bit rows hold the values; FP8 rows
// hold the values, then the fp32 scale; all padded to a multiple of 64 bytes.
#include "internal.h"

namespace hnsw {
namespace {

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

// Nearest E4M3 code of a finite float (ties to even, |x| >= 448 -> 448).
__device__ __forceinline__ uint8_t to_e4m3(float x) {
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a < 448.0f)) return static_cast<uint8_t>(sign | 0x7Eu);
    if (a < 0x1.0p-6f) {
        // subnormal spacing 2^-9; m = 8 is the smallest normal, code 0x08
        const uint32_t m = static_cast<uint32_t>(rintf(a * 512.0f));
        return static_cast<uint8_t>(sign | m);
    }
    int e = static_cast<int>((__float_as_uint(a) >> 23) & 0xFFu) - 127;  // a = 2^e * 1.f
    const float frac = ldexpf(a, -e) - 1.0f;                            // exact, in [0, 1)
    uint32_t m = static_cast<uint32_t>(rintf(frac * 8.0f));             // exact scaling, ties to even
    if (m == 8u) {
        m = 0u;
        ++e;
    }
    return static_cast<uint8_t>(sign | (static_cast<uint32_t>(e + 7) << 3) | m);
}

__global__ void quantize_bf16_kernel(DevIndex ix, uint16_t *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ix.n) return;
    const float *x = ix.vec + static_cast<size_t>(i) * ix.stride4 * 4;
    uint16_t *o = out + static_cast<size_t>(i) * ix.bf16_stride16 * 8;
    for (uint32_t j = 0; j < ix.bf16_stride16 * 8; ++j) o[j] = j < ix.dim ? to_bf16(x[j]) : 0;
}

__global__ void quantize_fp8_kernel(DevIndex ix, uint8_t *out, uint8_t *scale) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ix.n) return;
    const float *x = ix.vec + static_cast<size_t>(i) * ix.stride4 * 4;
    uint8_t *o = out + static_cast<size_t>(i) * ix.fp8_stride16 * 16;
    float mx = 0.0f;
    for (uint32_t j = 0; j < ix.dim; ++j) mx = fmaxf(mx, fabsf(x[j]));
    const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
    for (uint32_t j = 0; j < ix.fp8_pieces * 16; ++j) o[j] = j < ix.dim ? to_e4m3(x[j] / s) : 0;
    *reinterpret_cast<float *>(scale + static_cast<size_t>(i) * ix.fp8_scale_stride) = s;
}

__global__ void quantize_u8_kernel(DevIndex ix, uint8_t *out, uint32_t *inexact) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ix.n) return;
    const float *x = ix.vec + static_cast<size_t>(i) * ix.stride4 * 4;
    uint8_t *o = out + static_cast<size_t>(i) * ix.u8_stride16 * 16;
    bool exact = true;
    for (uint32_t j = 0; j < ix.u8_pieces * 16; ++j) {
        if (j >= ix.dim) {
            o[j] = 0;
            continue;
        }
        const float r = fminf(fmaxf(rintf(x[j]), 0.0f), 255.0f);
        exact = exact && r == x[j];
        o[j] = static_cast<uint8_t>(r);
    }
    if (!exact) atomicOr(inexact, 1u);
}

}  // namespace

hipError_t launch_quantize_u8(const DevIndex &ix, uint8_t *out, uint32_t *inexact, hipStream_t stream) {
    hipLaunchKernelGGL(quantize_u8_kernel, dim3((ix.n + 255) / 256), dim3(256), 0, stream, ix, out, inexact);
    return hipGetLastError();
}

hipError_t launch_quantize_bf16(const DevIndex &ix, uint16_t *out, hipStream_t stream) {
    hipLaunchKernelGGL(quantize_bf16_kernel, dim3((ix.n + 255) / 256), dim3(256), 0, stream, ix, out);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(const DevIndex &ix, uint8_t *out, uint8_t *scale, hipStream_t stream) {
    hipLaunchKernelGGL(quantize_fp8_kernel, dim3((ix.n + 255) / 256), dim3(256), 0, stream, ix, out, scale);
    return hipGetLastError();
}

}  // namespace hnsw
