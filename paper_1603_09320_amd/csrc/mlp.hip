// The 24-64-64-2 perceptron of the learned stop rule: FP32 training kernels
// (forward, forward + backward with per-wave gradient partials, reduction,
// Adam) and the BF16 inference net used inside the search kernel.
//
// Parameter layout (fp32, flat): W1[64][24], b1[64], W2[64][64], b2[64],
// W3[2][64], b3[2].
// Loss over a batch of n samples with labels (y0, c, y1, m):
//   L = (1/n) sum_s [ c * BCE(z0, y0) + lambda * m * (z1 - y1)^2 ],
//   BCE(z, y) = log(1 + e^z) - y z.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "internal.h"

namespace hnsw {
namespace {

constexpr int kIn = kMlpIn, kHid = kMlpHid, kOut = kMlpOut;
constexpr int oW1 = 0, ob1 = oW1 + kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid, oW3 = ob2 + kHid,
              ob3 = oW3 + kOut * kHid;
constexpr int kSamplesPerWave = 64;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave handles kSamplesPerWave consecutive samples; lane j is hidden unit j.
// Weights are read from global memory (they stay in cache); gradients are
// accumulated in registers (lane j owns rows j of W1/W2, column j of W3) and
// written once per wave to partial[wave][kMlpParams].  loss_part[wave] gets the
// wave's summed loss.  With `grad` false only the forward outputs are written.
template <bool GRAD>
__global__ __launch_bounds__(256) void mlp_wave_kernel(const float *P, const float *X, const float *Y, uint32_t n,
                                                       float lambda, float *out, float *partial, float *loss_part) {
    __shared__ float hs[4][2][kHid];
    const int lane = lane_id();
    const int w = threadIdx.x / 64;
    const uint32_t wave = blockIdx.x * 4 + w;
    const uint32_t s0 = wave * kSamplesPerWave;
    float gW1[kIn], gW2[kHid], gW3[kOut], gb1 = 0.f, gb2 = 0.f, gb3[kOut] = {0.f, 0.f}, loss = 0.f;
    for (int i = 0; i < kIn; ++i) gW1[i] = 0.f;
    for (int i = 0; i < kHid; ++i) gW2[i] = 0.f;
    for (int o = 0; o < kOut; ++o) gW3[o] = 0.f;
    const float inv_n = 1.0f / static_cast<float>(n);
    for (uint32_t s = s0; s < min(n, s0 + kSamplesPerWave); ++s) {
        const float *x = X + static_cast<size_t>(s) * kIn;
        // layer 1
        float a1 = P[ob1 + lane];
        for (int i = 0; i < kIn; ++i) a1 = fmaf(P[oW1 + lane * kIn + i], x[i], a1);
        const float h1 = a1 > 0.f ? a1 : 0.f;
        hs[w][0][lane] = h1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // layer 2
        float a2 = P[ob2 + lane];
        for (int i = 0; i < kHid; ++i) a2 = fmaf(P[oW2 + lane * kHid + i], hs[w][0][i], a2);
        const float h2 = a2 > 0.f ? a2 : 0.f;
        // layer 3
        const float z0 = wave_sum(P[oW3 + lane] * h2) + P[ob3];
        const float z1 = wave_sum(P[oW3 + kHid + lane] * h2) + P[ob3 + 1];
        if (!GRAD) {
            if (lane < kOut) out[static_cast<size_t>(s) * kOut + lane] = lane == 0 ? z0 : z1;
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        const float y0 = Y[s * 4 + 0], c = Y[s * 4 + 1], y1 = Y[s * 4 + 2], m = Y[s * 4 + 3];
        const float sig = 1.0f / (1.0f + expf(-z0));
        const float bce = fmaxf(z0, 0.f) + log1pf(expf(-fabsf(z0))) - y0 * z0;
        loss += c * bce + lambda * m * (z1 - y1) * (z1 - y1);
        const float dz0 = c * (sig - y0) * inv_n;
        const float dz1 = 2.0f * lambda * m * (z1 - y1) * inv_n;
        gW3[0] = fmaf(dz0, h2, gW3[0]);
        gW3[1] = fmaf(dz1, h2, gW3[1]);
        gb3[0] += dz0;
        gb3[1] += dz1;
        const float dh2 = a2 > 0.f ? fmaf(P[oW3 + lane], dz0, P[oW3 + kHid + lane] * dz1) : 0.f;
        hs[w][1][lane] = dh2;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (int i = 0; i < kHid; ++i) gW2[i] = fmaf(dh2, hs[w][0][i], gW2[i]);
        gb2 += dh2;
        // dh1[lane] = sum_j W2[j][lane] * dh2[j]
        float dh1 = 0.f;
        for (int j = 0; j < kHid; ++j) dh1 = fmaf(P[oW2 + j * kHid + lane], hs[w][1][j], dh1);
        dh1 = a1 > 0.f ? dh1 : 0.f;
        for (int i = 0; i < kIn; ++i) gW1[i] = fmaf(dh1, x[i], gW1[i]);
        gb1 += dh1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if (!GRAD) return;
    float *pp = partial + static_cast<size_t>(wave) * kMlpParams;
    for (int i = 0; i < kIn; ++i) pp[oW1 + lane * kIn + i] = gW1[i];
    pp[ob1 + lane] = gb1;
    for (int i = 0; i < kHid; ++i) pp[oW2 + lane * kHid + i] = gW2[i];
    pp[ob2 + lane] = gb2;
    pp[oW3 + lane] = gW3[0];
    pp[oW3 + kHid + lane] = gW3[1];
    if (lane < kOut) pp[ob3 + lane] = gb3[lane];
    if (lane == 0) loss_part[wave] = loss;  // every lane holds the same per-sample sum
}

// grad[p] = sum over waves of partial[wave][p] (fixed order); loss likewise.
__global__ void mlp_reduce_kernel(const float *partial, const float *loss_part, uint32_t nwaves, uint32_t n,
                                  float *grad, float *loss) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float g = 0.f;
        for (uint32_t w = 0; w < nwaves; ++w) g += partial[static_cast<size_t>(w) * kMlpParams + p];
        grad[p] = g;
    }
    if (p == kMlpParams && loss) {
        float l = 0.f;
        for (uint32_t w = 0; w < nwaves; ++w) l += loss_part[w];
        *loss = l / static_cast<float>(n);
    }
}

__global__ void adam_kernel(float *P, const float *G, float *M, float *V, uint32_t np, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.f - b1) * g;
    const float v = b2 * V[p] + (1.f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace

hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t n, float *out, hipStream_t st) {
    const uint32_t waves = (n + kSamplesPerWave - 1) / kSamplesPerWave;
    hipLaunchKernelGGL(mlp_wave_kernel<false>, dim3((waves + 3) / 4), dim3(256), 0, st, P, X, nullptr, n, 0.f, out,
                       nullptr, nullptr);
    return hipGetLastError();
}

uint32_t mlp_grad_waves(uint32_t n) {
    const uint32_t waves = (n + kSamplesPerWave - 1) / kSamplesPerWave;
    return (waves + 3) / 4 * 4;
}

hipError_t launch_mlp_grad(const float *P, const float *X, const float *Y, uint32_t n, float lambda, float *grad,
                           float *loss, float *scratch, hipStream_t st) {
    const uint32_t waves = mlp_grad_waves(n);
    float *partial = scratch;
    float *loss_part = scratch + static_cast<size_t>(waves) * kMlpParams;
    hipLaunchKernelGGL(mlp_wave_kernel<true>, dim3(waves / 4), dim3(256), 0, st, P, X, Y, n, lambda, nullptr,
                       partial, loss_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st, partial, loss_part,
                       waves, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *G, float *M, float *V, uint32_t np, float lr, float b1, float b2,
                       float eps, uint32_t step, hipStream_t st) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, st, P, G, M, V, np, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace hnsw
