// Batched K-NN-SEARCH (Alg. 5 of arXiv:1603.09320) for gfx950: one workgroup
// of one wavefront per query; the search itself is search_one in
// search_device.h.
#include "search_device.h"

namespace hnsw {
namespace {

template <int G, int F, int METRIC, int KIND, bool LEARN>
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
    search_one<G, F, METRIC, KIND, LEARN>(ix, a, job, carve(smem, a));
}

// Waves per SIMD the register allocation is held to: six for the fp32 and
// BF16 stores (80 registers, no spills), five for FP8 (its decode needs more).
template <int G, int F, int METRIC, int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KIND == kFP8 ? 5 : 6))) void search_kernel(
    DevIndex ix, SearchArgs a) {
    search_query<G, F, METRIC, KIND, false>(ix, a);
}

// The learned stop rule: also six waves per SIMD (its checkpoint keeps its
// addresses and constants out of the expansion loop, see learned_checkpoint).
template <int G, int F, int METRIC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void search_kernel_learned(DevIndex ix,
                                                                                                    SearchArgs a) {
    search_query<G, F, METRIC, kF32, true>(ix, a);
}

template <int G, int F, int KIND>
hipError_t launch_gfk(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const size_t lds = search_lds_bytes(a);
    if constexpr (KIND == kF32) {
        if (a.mode == HNSW_MODE_LEARNED) {
            if (ix.metric == HNSW_IP)
                hipLaunchKernelGGL((search_kernel_learned<G, F, HNSW_IP>), dim3(a.nq), dim3(64), lds, stream, ix, a);
            else
                hipLaunchKernelGGL((search_kernel_learned<G, F, HNSW_L2SQ>), dim3(a.nq), dim3(64), lds, stream, ix, a);
            return hipGetLastError();
        }
    }
    if (ix.metric == HNSW_IP)
        hipLaunchKernelGGL((search_kernel<G, F, HNSW_IP, KIND>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    else
        hipLaunchKernelGGL((search_kernel<G, F, HNSW_L2SQ, KIND>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const TileShape t = tile_for(KIND, ix.dim);
    switch (t.G * 16 + t.F) {
        case 1 * 16 + 1: return launch_gfk<1, 1, KIND>(ix, a, stream);
        case 2 * 16 + 1: return launch_gfk<2, 1, KIND>(ix, a, stream);
        case 2 * 16 + 2: return launch_gfk<2, 2, KIND>(ix, a, stream);
        case 4 * 16 + 1: return launch_gfk<4, 1, KIND>(ix, a, stream);
        case 4 * 16 + 2: return launch_gfk<4, 2, KIND>(ix, a, stream);
        case 8 * 16 + 1: return launch_gfk<8, 1, KIND>(ix, a, stream);
        case 8 * 16 + 2: return launch_gfk<8, 2, KIND>(ix, a, stream);
        case 16 * 16 + 1: return launch_gfk<16, 1, KIND>(ix, a, stream);
        case 16 * 16 + 2: return launch_gfk<16, 2, KIND>(ix, a, stream);
        case 16 * 16 + 4: return launch_gfk<16, 4, KIND>(ix, a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// Lane-group tile for a store: G lanes per vector, F pieces per lane.
// fp32 rows use two pieces per lane up to 128 dimensions; low-precision
// rows (8 or 16 values per piece) use one piece per lane up to 16 pieces.
TileShape tile_for(int kind, uint32_t dim) {
    const uint32_t vpp = kind == kF32 ? 4 : (kind == kBF16 ? 8 : 16);
    const uint32_t pieces = (dim + vpp - 1) / vpp;
    if (kind == kF32) {
        if (pieces <= 1) return {1, 1};
        if (pieces <= 4) return {2, 2};
        if (pieces <= 8) return {4, 2};
        if (pieces <= 16) return {8, 2};
        if (pieces <= 32) return {16, 2};
        return {16, 4};
    }
    if (pieces <= 1) return {1, 1};
    if (pieces <= 2) return {2, 1};
    if (pieces <= 4) return {4, 1};
    if (pieces <= 8) return {8, 1};
    if (pieces <= 16) return {16, 1};
    return {16, 2};
}

size_t search_lds_bytes(const SearchArgs &a) {
    return static_cast<size_t>(a.wpow2) * 8 + 64 * 8 + 64 * 4 * 2 + 128 * 4 +
           (static_cast<size_t>(1) << a.ht_log2) * 4;
}

hipError_t launch_search(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    switch (a.mode) {
        case HNSW_MODE_BF16: return launch_kind<kBF16>(ix, a, stream);
        case HNSW_MODE_FP8: return launch_kind<kFP8>(ix, a, stream);
        default: return launch_kind<kF32>(ix, a, stream);
    }
}

}  // namespace hnsw
