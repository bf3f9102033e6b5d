// The batched search kernels and their launch dispatch, shared by two
// translation units: search.hip instantiates them with buffered gathers
// (stores of at most 2 GiB, 32-bit offsets) and search_wide.hip with 64-bit
// addressed gathers for larger stores.
#pragma once

#include "search_device.h"

namespace hnsw {
namespace {


template <int G, int F, int METRIC, int KIND, bool LEARN, bool BUF>
__device__ __forceinline__ void search_query(const DevIndex &ix, const SearchArgs &a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t qi = blockIdx.x;
    if (qi >= a.nq) return;
    Job job;
    job.q = a.queries + static_cast<size_t>(qi) * ix.dim;
    job.k = a.k;
    job.ef = a.ef;
    job.ids = a.ids + static_cast<size_t>(qi) * a.k;
    job.dists = a.dists + static_cast<size_t>(qi) * a.k;
    job.counters = a.counters ? a.counters + static_cast<size_t>(qi) * 4 : nullptr;
    job.trace = LEARN && a.ckpt_trace ? a.ckpt_trace + static_cast<size_t>(qi) * a.mlp.max_ckpt * (kMlpIn + 2)
                                      : nullptr;
    search_one<G, F, METRIC, KIND, LEARN, BUF>(ix, a, job, carve<LEARN>(smem, a));
}

// Waves per SIMD the register allocation is held to: six for the fp32 and
// BF16 stores (80 registers, no spills), five for FP8 (its decode needs more).
template <int G, int F, int METRIC, int KIND, bool BUF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KIND == kFP8 ? 5 : 6))) void search_kernel(
    DevIndex ix, SearchArgs a) {
    search_query<G, F, METRIC, KIND, false, BUF>(ix, a);
}

// The learned stop rule: also six waves per SIMD (its checkpoint keeps its
// addresses and constants out of the expansion loop, see learned_checkpoint).
template <int G, int F, int METRIC, bool BUF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void search_kernel_learned(DevIndex ix,
                                                                                                    SearchArgs a) {
    search_query<G, F, METRIC, kF32, true, BUF>(ix, a);
}

template <int G, int F, int KIND, bool BUF>
hipError_t launch_gfk(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a, KIND == kF32 && a.mode == HNSW_MODE_LEARNED);
    if constexpr (KIND == kF32) {
        if (a.mode == HNSW_MODE_LEARNED) {
            if (ix.metric == HNSW_IP)
                hipLaunchKernelGGL((search_kernel_learned<G, F, HNSW_IP, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
            else
                hipLaunchKernelGGL((search_kernel_learned<G, F, HNSW_L2SQ, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
            return hipGetLastError();
        }
    }
    if (ix.metric == HNSW_IP)
        hipLaunchKernelGGL((search_kernel<G, F, HNSW_IP, KIND, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    else
        hipLaunchKernelGGL((search_kernel<G, F, HNSW_L2SQ, KIND, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    return hipGetLastError();
}

template <int KIND, bool BUF>
hipError_t launch_kind(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const TileShape t = tile_for(KIND, ix.dim);
    switch (t.G * 16 + t.F) {
        case 1 * 16 + 1: return launch_gfk<1, 1, KIND, BUF>(ix, a, stream);
        case 2 * 16 + 1: return launch_gfk<2, 1, KIND, BUF>(ix, a, stream);
        case 2 * 16 + 2: return launch_gfk<2, 2, KIND, BUF>(ix, a, stream);
        case 4 * 16 + 1: return launch_gfk<4, 1, KIND, BUF>(ix, a, stream);
        case 4 * 16 + 2: return launch_gfk<4, 2, KIND, BUF>(ix, a, stream);
        case 8 * 16 + 1: return launch_gfk<8, 1, KIND, BUF>(ix, a, stream);
        case 8 * 16 + 2: return launch_gfk<8, 2, KIND, BUF>(ix, a, stream);
        case 16 * 16 + 1: return launch_gfk<16, 1, KIND, BUF>(ix, a, stream);
        case 16 * 16 + 2: return launch_gfk<16, 2, KIND, BUF>(ix, a, stream);
        case 16 * 16 + 4: return launch_gfk<16, 4, KIND, BUF>(ix, a, stream);
        default: return hipErrorInvalidValue;
    }
}

// Entry of one translation unit: every store kind of the search.
template <bool BUF>
hipError_t launch_search_stores(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    switch (a.mode) {
        case HNSW_MODE_BF16: return launch_kind<kBF16, BUF>(ix, a, stream);
        case HNSW_MODE_FP8: return launch_kind<kFP8, BUF>(ix, a, stream);
        default: return launch_kind<kF32, BUF>(ix, a, stream);
    }
}

}  // namespace
}  // namespace hnsw
