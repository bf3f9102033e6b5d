// The batched search kernels with 64-bit addressed gathers, for indices
// whose vector stores exceed what 32-bit buffer offsets address.
#include "search_kernels.h"

namespace hnsw {

hipError_t launch_search_wide(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    return launch_search_stores<false>(ix, a, stream);
}

}  // namespace hnsw
