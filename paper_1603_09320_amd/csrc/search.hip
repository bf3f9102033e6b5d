// Batched K-NN-SEARCH (Alg. 5 of arXiv:1603.09320) for gfx950: one workgroup
// of one wavefront per query; the search itself is search_one in
// search_device.h.  This unit holds the buffered-gather kernels (stores of at
// most 2 GiB); search_wide.hip holds those for larger stores.
#include <stdlib.h>

#include "search_kernels.h"

namespace hnsw {

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

size_t search_lds_bytes(const SearchArgs &a, bool learned) {
    return static_cast<size_t>(a.wpow2) * 8 + 64 * 8 + 64 * 4 + (learned ? 64 * 4 + 128 * 4 : 0) +
           (static_cast<size_t>(1) << a.ht_log2) * 4;
}

bool stores_buffered(const DevIndex &ix) {
    auto fits = [&](const void *p, uint32_t stride16) {
        return !p || (static_cast<uint64_t>(ix.n) + 1) * stride16 * 16 <= kBufferedMaxBytes;
    };
    return fits(ix.vec, ix.stride4) && fits(ix.vbf16, ix.bf16_stride16) && fits(ix.vfp8, ix.fp8_stride16);
}

// HNSW_WIDE_GATHERS=1 sends every launch through the 64-bit addressed kernels
// (they are otherwise taken only for stores above 2 GiB), so that tests can
// check them on small indices.
hipError_t launch_search(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const char *w = getenv("HNSW_WIDE_GATHERS");
    const bool force_wide = w && w[0] == '1';
    if (stores_buffered(ix) && !force_wide) return launch_search_stores<true>(ix, a, stream);
    return launch_search_wide(ix, a, stream);
}

}  // namespace hnsw
