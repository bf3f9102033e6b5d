// Exact K-NN by brute force (the problem statement of Sec. 1 of
// arXiv:1603.09320; Table 1 reports its cost as "BF time"), used as the
// ground truth that recall is measured against.
//
// Stage 1 (bf_scan): a dense fp32 contraction on the matrix cores.  A block
// takes 32 queries and one chunk of the base set; each of its 4 waves
// computes 32 x 16 tiles of <q, x> with v_mfma_f32_16x16x4f32 over the
// (zero padded) dimension, forms the ranking value ||x||^2 - 2<q,x> (or
// -<q,x> for the inner-product metric), and offers it to a per-query
// candidate buffer in LDS guarded by a threshold: when a buffer fills, it is
// sorted, cut to the KP best, and the threshold becomes the KP-th key.  The
// KP best keys of every (query, chunk) pair go to a scratch array.
// Stage 2 (bf_merge): one wave per query sorts the chunk candidates, keeps the
// KP best, recomputes their distances exactly in fp64 from the fp32 vectors,
// and writes the k nearest in (fp64 distance, id) order.
// With KP >= 2k the fp32 ranking only has to place the true k nearest among
// the first KP, which holds unless more than KP - k elements lie within the
// fp32 rounding error of the k-th distance.
#include <climits>

#include "internal.h"

namespace hnsw {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kQT = 32;     // queries per block
constexpr int kWaves = 4;   // base tiles of 16 per block iteration
constexpr int kKSlice = 64; // floats of each base row staged at a time
constexpr uint64_t kMaxKey = ~0ull;

__device__ __forceinline__ uint32_t ord_of(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Bitonic sort of `seg` independent segments of `len` (power of two) keys,
// ascending, by all threads of the block.
__device__ void block_bitonic(uint64_t *a, int seg, int len) {
    const int total = seg * len;
    for (int k = 2; k <= len; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < total / 2; t += blockDim.x) {
                const int s = t / (len / 2), r = t % (len / 2);
                const int i = 2 * j * (r / j) + (r % j);
                const int l = i + j;
                const bool up = (i & k) == 0;
                uint64_t *b = a + static_cast<size_t>(s) * len;
                const uint64_t x = b[i], y = b[l];
                if ((x > y) == up) {
                    b[i] = y;
                    b[l] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Sorts the candidate buffers whose count exceeds the trigger, keeps the KP
// best and tightens the thresholds.  Called by all threads.
template <int KP>
__device__ void compact(uint64_t *cand, uint32_t *cnt, uint64_t *thr, uint32_t trigger) {
    constexpr int CAP = 2 * KP;
    __syncthreads();
    bool any = false;
    for (int q = 0; q < kQT; ++q) any |= cnt[q] > trigger;
    if (!any) return;
    // pad unused slots so whole segments can be sorted
    for (int t = threadIdx.x; t < kQT * CAP; t += blockDim.x) {
        const int q = t / CAP, i = t % CAP;
        if (static_cast<uint32_t>(i) >= cnt[q]) cand[t] = kMaxKey;
    }
    __syncthreads();
    block_bitonic(cand, kQT, CAP);
    if (threadIdx.x < kQT) {
        const int q = threadIdx.x;
        if (cnt[q] >= static_cast<uint32_t>(KP)) thr[q] = cand[q * CAP + KP - 1];
        cnt[q] = cnt[q] < static_cast<uint32_t>(KP) ? cnt[q] : KP;
    }
    __syncthreads();
}

template <int KP>
__global__ __launch_bounds__(256) void bf_scan(DevIndex ix, const float *Q, uint32_t nq, const float *xnorm,
                                               uint32_t chunk, uint32_t nchunks, uint64_t *partial) {
    constexpr int CAP = 2 * KP;
    extern __shared__ __align__(16) uint8_t smem[];
    uint64_t *cand = reinterpret_cast<uint64_t *>(smem);                // [kQT][CAP]
    uint64_t *thr = cand + kQT * CAP;                                    // [kQT]
    uint32_t *cnt = reinterpret_cast<uint32_t *>(thr + kQT);             // [kQT]
    float *tile = reinterpret_cast<float *>(cnt + kQT);                  // [kWaves][16][kKSlice + 1]

    const int lane = lane_id();
    const int wave = threadIdx.x / 64;
    const uint32_t q0 = blockIdx.x * kQT;
    const uint32_t ch = blockIdx.y;
    const uint32_t b_lo = ch * chunk;
    const uint32_t b_hi = min(ix.n, b_lo + chunk);
    const uint32_t dpad = ix.stride4 * 4;
    float *my_tile = tile + wave * 16 * (kKSlice + 1);

    for (int t = threadIdx.x; t < kQT; t += blockDim.x) {
        cnt[t] = 0;
        thr[t] = kMaxKey;
    }
    __syncthreads();

    const int iters = b_lo < b_hi ? static_cast<int>((b_hi - b_lo + 63) / 64) : 0;
    for (int it = 0; it < iters; ++it) {
        const uint32_t b0 = b_lo + it * 64 + wave * 16;
        v4f acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        for (uint32_t k0 = 0; k0 < dpad; k0 += kKSlice) {
            // stage 16 rows x kKSlice floats of this wave's base tile
            for (int e = lane; e < 16 * kKSlice; e += 64) {
                const int r = e / kKSlice, c = e % kKSlice;
                const uint32_t b = b0 + r, col = k0 + c;
                float v = 0.f;
                if (b < b_hi && col < dpad) v = ix.vec[static_cast<size_t>(b) * dpad + col];
                my_tile[r * (kKSlice + 1) + c] = v;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll 4
            for (int s = 0; s < kKSlice / 4; ++s) {
                const uint32_t col = k0 + 4 * s + lane / 16;
                const float bv = my_tile[(lane % 16) * (kKSlice + 1) + 4 * s + lane / 16];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t q = q0 + 16 * h + (lane % 16);
                    const float av = (q < nq && col < ix.dim) ? Q[static_cast<size_t>(q) * ix.dim + col] : 0.f;
                    acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[h], 0, 0, 0);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // D[i][j] of a 16x16x4 product sits in lane j + 16 * (i / 4), element i % 4.
        const uint32_t b = b0 + (lane % 16);
        const float xn = (b < b_hi && ix.metric == HNSW_L2SQ) ? xnorm[b] : 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qq = 16 * h + 4 * (lane / 16) + r;
                if (b < b_hi && q0 + qq < nq) {
                    const float dot = acc[h][r];
                    const float d = ix.metric == HNSW_L2SQ ? xn - 2.f * dot : -dot;
                    const uint64_t key = (static_cast<uint64_t>(ord_of(d)) << 32) | b;
                    if (key < thr[qq]) {
                        const uint32_t slot = atomicAdd(&cnt[qq], 1u);
                        if (slot < static_cast<uint32_t>(CAP)) cand[qq * CAP + slot] = key;
                    }
                }
            }
        // each iteration adds at most 64 keys per query
        compact<KP>(cand, cnt, thr, CAP - 64);
    }
    compact<KP>(cand, cnt, thr, 0);
    for (int t = threadIdx.x; t < kQT * KP; t += blockDim.x) {
        const int q = t / KP, i = t % KP;
        if (q0 + q < nq)
            partial[(static_cast<size_t>(q0 + q) * nchunks + ch) * KP + i] =
                static_cast<uint32_t>(i) < cnt[q] ? cand[q * CAP + i] : kMaxKey;
    }
}

// Wave-level bitonic sort of len keys in LDS (power of two).
__device__ void wave_bitonic(uint64_t *a, int len) {
    const int lane = lane_id();
    for (int k = 2; k <= len; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < len / 2; t += 64) {
                const int i = 2 * j * (t / j) + (t % j);
                const int l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t x = a[i], y = a[l];
                if ((x > y) == up) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
}

template <int KP>
__global__ __launch_bounds__(64) void bf_merge(DevIndex ix, const float *Q, uint32_t nq, uint32_t nchunks,
                                               uint32_t pow2, const uint64_t *partial, uint32_t k, int32_t *ids_out,
                                               double *d_out) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint64_t *a = reinterpret_cast<uint64_t *>(smem);  // [pow2]
    double *dd = reinterpret_cast<double *>(a + pow2); // [KP]
    uint32_t *ii = reinterpret_cast<uint32_t *>(dd + KP);
    const uint32_t q = blockIdx.x;
    const int lane = lane_id();
    const size_t tot = static_cast<size_t>(nchunks) * KP;
    for (uint32_t i = lane; i < pow2; i += 64) a[i] = i < tot ? partial[static_cast<size_t>(q) * tot + i] : kMaxKey;
    wave_bitonic(a, static_cast<int>(pow2));
    // exact fp64 distances of the KP best candidates
    const uint32_t dpad = ix.stride4 * 4;
    const float *qr = Q + static_cast<size_t>(q) * ix.dim;
    for (int i = lane; i < KP; i += 64) {
        const uint64_t key = a[i];
        double d = __longlong_as_double(0x7ff0000000000000ll);
        uint32_t id = 0xFFFFFFFFu;
        if (key != kMaxKey) {
            id = static_cast<uint32_t>(key);
            const float *xr = ix.vec + static_cast<size_t>(id) * dpad;
            double s = 0.0;
            if (ix.metric == HNSW_L2SQ) {
                for (uint32_t j = 0; j < ix.dim; ++j) {
                    const double t = static_cast<double>(qr[j]) - static_cast<double>(xr[j]);
                    s = __fma_rn(t, t, s);
                }
                d = s;
            } else {
                for (uint32_t j = 0; j < ix.dim; ++j) s = __fma_rn(static_cast<double>(qr[j]), static_cast<double>(xr[j]), s);
                d = 1.0 - s;
            }
        }
        dd[i] = d;
        ii[i] = id;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // rank each candidate by (fp64 distance, id); ranks are distinct
    for (int i = lane; i < KP; i += 64) {
        const double di = dd[i];
        const uint32_t idi = ii[i];
        int r = 0;
        for (int j = 0; j < KP; ++j) {
            const double dj = dd[j];
            r += (dj < di) || (dj == di && (ii[j] < idi || (ii[j] == idi && j < i)));
        }
        if (static_cast<uint32_t>(r) < k) {
            const size_t o = static_cast<size_t>(q) * k + r;
            ids_out[o] = idi == 0xFFFFFFFFu ? -1 : static_cast<int32_t>(idi);
            d_out[o] = di;
        }
    }
}

__global__ void row_norms(DevIndex ix, float *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ix.n) return;
    const float *xr = ix.vec + static_cast<size_t>(i) * ix.stride4 * 4;
    double s = 0.0;
    for (uint32_t j = 0; j < ix.dim; ++j) s = __fma_rn(static_cast<double>(xr[j]), static_cast<double>(xr[j]), s);
    out[i] = static_cast<float>(s);
}

template <int KP>
hipError_t bf_run(const DevIndex &ix, const float *Q, uint32_t nq, uint32_t k, const float *xnorm,
                  uint64_t *partial, uint32_t nchunks, uint32_t chunk, int32_t *ids, double *d, hipStream_t st) {
    const size_t lds1 = static_cast<size_t>(kQT) * 2 * KP * 8 + kQT * 8 + kQT * 4 + kWaves * 16 * (kKSlice + 1) * 4;
    if (lds1 > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&bf_scan<KP>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds1));
    dim3 g1((nq + kQT - 1) / kQT, nchunks);
    hipLaunchKernelGGL(bf_scan<KP>, g1, dim3(256), lds1, st, ix, Q, nq, xnorm, chunk, nchunks, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t pow2 = 1;
    while (pow2 < nchunks * KP) pow2 <<= 1;
    const size_t lds2 = static_cast<size_t>(pow2) * 8 + KP * 8 + KP * 4;
    if (lds2 > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&bf_merge<KP>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds2));
    hipLaunchKernelGGL(bf_merge<KP>, dim3(nq), dim3(64), lds2, st, ix, Q, nq, nchunks, pow2, partial, k, ids, d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_row_norms(const DevIndex &ix, float *out, hipStream_t st) {
    hipLaunchKernelGGL(row_norms, dim3((ix.n + 255) / 256), dim3(256), 0, st, ix, out);
    return hipGetLastError();
}

uint32_t bf_candidates(uint32_t k) { return k <= 32 ? 64 : (k <= 64 ? 128 : 256); }

void bf_plan(const DevIndex &ix, uint32_t nq, uint32_t k, uint32_t *nchunks, uint32_t *chunk) {
    const uint32_t tiles = (nq + kQT - 1) / kQT;
    uint32_t nc = (4096 + tiles - 1) / tiles;
    const uint32_t kp = bf_candidates(k);
    const uint32_t max_nc = 8192 / kp;  // bf_merge sorts nchunks * KP keys in LDS
    if (nc > max_nc) nc = max_nc;
    if (nc < 1) nc = 1;
    uint32_t ck = (ix.n + nc - 1) / nc;
    ck = (ck + 63) & ~63u;
    nc = (ix.n + ck - 1) / ck;
    *nchunks = nc;
    *chunk = ck;
}

hipError_t launch_bruteforce(const DevIndex &ix, const float *Q, uint32_t nq, uint32_t k, const float *xnorm,
                             uint64_t *partial, uint32_t nchunks, uint32_t chunk, int32_t *ids, double *d,
                             hipStream_t st) {
    switch (bf_candidates(k)) {
        case 64: return bf_run<64>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
        case 128: return bf_run<128>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
        default: return bf_run<256>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
    }
}

}  // namespace hnsw
