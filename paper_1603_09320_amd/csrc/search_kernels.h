// The batched search kernels and their launch dispatch, shared by two
// translation units: search.hip instantiates them with buffered gathers
// (stores of at most 2 GiB, 32-bit offsets) and search_wide.hip with 64-bit
// addressed gathers for larger stores.
#pragma once

#include "search_device.h"

namespace hnsw {
namespace {


__device__ __forceinline__ Job job_of(const DevIndex &ix, const SearchArgs &a, uint32_t qi, bool learn) {
    Job job;
    job.q = a.queries + static_cast<size_t>(qi) * ix.dim;
    job.k = a.k;
    job.ef = a.ef;
    job.ids = a.ids + static_cast<size_t>(qi) * a.k;
    job.dists = a.dists + static_cast<size_t>(qi) * a.k;
    job.counters = a.counters ? a.counters + static_cast<size_t>(qi) * 4 : nullptr;
    job.trace = learn && a.ckpt_trace ? a.ckpt_trace + static_cast<size_t>(qi) * a.mlp.max_ckpt * (kMlpIn + 2)
                                      : nullptr;
    return job;
}

template <int G, int F, int METRIC, int KIND, bool LEARN, bool BUF>
__device__ __forceinline__ void search_query(const DevIndex &ix, const SearchArgs &a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t qi = blockIdx.x;
    if (qi >= a.nq) return;
    search_one<G, F, METRIC, KIND, LEARN, BUF>(ix, a, job_of(ix, a, qi, LEARN), carve<LEARN>(smem, a));
}

// Waves per SIMD the register allocation is held to: six for the fp32 and
// BF16 stores (80 registers, no spills), five for FP8 and the 8-bit store
// (their 16 values per piece need more; six would spill); six for an exact
// 8-bit store of one piece per lane (78 registers without the re-rank).
template <int G, int F, int METRIC, int KIND, bool BUF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KIND == kFP8 || KIND == kU8 || (KIND == kU8E && F > 1) ? 5 : 6))) void search_kernel(
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

// ------------------------------------------------ scheduled launches
//
// A batch larger than the waves the chip holds at once finishes when its
// slowest queries do, and a query started late that needs many layer-0
// expansions decides the end.  The scheduled form runs every query's descent
// first (descent_kernel), then starts the layer-0 searches of the quarter of
// queries whose descent ended farthest from them (their layer-0 searches tend
// to be the longest) before the others (order_kernel, layer0_kernel).  It also
// places queries whose descents passed through the same node of layer
// ix.cell_level, which gather many of the same rows, on the same XCD at about
// the same time, so that those rows come from that XCD's L2 rather than from
// HBM.  Each query's arithmetic is that of the one-kernel path; only the order
// in which queries occupy the chip changes.

template <int G, int F, int METRIC, int KIND, bool BUF>
__global__ __launch_bounds__(64) void descent_kernel(DevIndex ix, SearchArgs a) {
    __shared__ uint64_t keys[64];
    __shared__ uint32_t ids[64];
    const uint32_t qi = blockIdx.x;
    if (qi >= a.nq) return;
    WaveLds s{};
    s.keys = keys;
    s.ids = ids;
    const RowSource src = rows_of(ix, a, KIND);
    QueryRegs<G, F, KIND> Q;
    load_query<G, F, KIND>(a.queries + static_cast<size_t>(qi) * ix.dim, ix.dim, Q);
    const Descent d = descend<G, F, METRIC, KIND, BUF>(ix, src, Q, s);
    if (lane_id() == 0) {
        a.sched_start[qi] = d.cur;
        a.sched_up[2 * static_cast<size_t>(qi)] = d.n_dist;
        a.sched_up[2 * static_cast<size_t>(qi) + 1] = d.n_exp;
        a.sched_cell[qi] = d.cell;
    }
}

// One workgroup of 1024 threads (16 waves).  The long queries are those whose
// descent ended at or beyond the distance ranked at a quarter of a sample of
// at most 512 descents (every nq/ns-th query, bitonic-sorted in LDS, largest
// first).  A counting sort over 2 x kCellBins bins (the long queries' bins
// first, then the others'; within each part, a hash of the query's cell)
// ranks the batch.  Workgroups go to the kXcds XCDs round robin (block b runs
// on XCD b % kXcds), so the long part and the rest are each cut into kXcds
// consecutive runs of nearly equal size, and XCD x takes the x-th run of each,
// its long run first: block kXcds * j + x gets the j-th query of XCD x's
// sequence.  Each XCD thus receives a share of the long queries at the start
// and queries from few cells at a time.  Queries that share a bin land in the
// order of their atomics, which changes when the chip runs them, never what
// they return.  Loads go in rounds of kOrderTiles tiles of 1024 consecutive
// queries (thread t reads query tile * 1024 + t of each tile, coalesced, all
// in flight together); a batch of one round keeps its bins in registers
// between the counting and the placing pass.
constexpr uint32_t kOrderThreads = 1024, kOrderSample = 512, kOrderTiles = 16;
constexpr uint32_t kCellBinsLog2 = 10, kCellBins = 1u << kCellBinsLog2, kXcds = 8;
static_assert(kCellBins == kOrderThreads, "the scan takes two bins per thread");

__global__ __launch_bounds__(1024) void order_kernel(const uint64_t *start, const uint32_t *cell, uint32_t nq,
                                                     uint32_t *order) {
    __shared__ uint32_t samp[kOrderSample];
    __shared__ uint32_t bins[2 * kCellBins];
    __shared__ uint32_t wsum[kOrderThreads / 64];
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    const uint32_t *dist_bits = reinterpret_cast<const uint32_t *>(start) + 1;  // high word of each key
    const uint32_t ns = nq < kOrderSample ? nq : kOrderSample;
    if (t < kOrderSample) samp[t] = t < ns ? dist_bits[2 * (static_cast<uint64_t>(t) * nq / ns)] : 0u;
    for (uint32_t i = t; i < 2 * kCellBins; i += kOrderThreads) bins[i] = 0u;
    __syncthreads();
    for (uint32_t k = 2; k <= kOrderSample; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (t < kOrderSample / 2) {
                const uint32_t i = 2 * j * (t / j) + (t % j), l = i + j;
                const bool down = (i & k) == 0;  // largest first
                const uint32_t x = samp[i], y = samp[l];
                if ((x < y) == down) {
                    samp[i] = y;
                    samp[l] = x;
                }
            }
            __syncthreads();
        }
    const uint32_t thr = samp[ns / 4];
    // bin of query r0 + i * 1024 + t (clamped loads, all in flight first)
    auto bins_of = [&](uint32_t r0, uint32_t (&b)[kOrderTiles]) {
        uint32_t hi[kOrderTiles], c[kOrderTiles];
#pragma unroll
        for (uint32_t i = 0; i < kOrderTiles; ++i) {
            const uint32_t q = min(r0 + i * kOrderThreads + t, nq - 1u);
            hi[i] = dist_bits[2 * static_cast<size_t>(q)];
            c[i] = cell[q];
        }
#pragma unroll
        for (uint32_t i = 0; i < kOrderTiles; ++i)
            b[i] = (hi[i] >= thr ? 0u : kCellBins) + ((c[i] * 0x9E3779B1u) >> (32 - kCellBinsLog2));
    };
    constexpr uint32_t kRound = kOrderTiles * kOrderThreads;
    uint32_t b[kOrderTiles];
    for (uint32_t r0 = 0; r0 < nq; r0 += kRound) {
        bins_of(r0, b);
#pragma unroll
        for (uint32_t i = 0; i < kOrderTiles; ++i)
            if (r0 + i * kOrderThreads + t < nq) atomicAdd(&bins[b[i]], 1u);
    }
    __syncthreads();
    // exclusive scan of the 2048 bin counts, two per thread
    const uint32_t c0 = bins[2 * t], c1 = bins[2 * t + 1];
    uint32_t incl = c0 + c1;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= static_cast<uint32_t>(o)) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t base = incl - (c0 + c1);
    for (uint32_t w = 0; w < wv; ++w) base += wsum[w];
    bins[2 * t] = base;
    bins[2 * t + 1] = base + c0;
    __syncthreads();
    const uint32_t nl = bins[kCellBins];  // queries in the long part
    __syncthreads();                      // read before the placing atomics move it
    // XCD x's sequence: la + (x < lb) long queries, then ca + (x < cb) in all
    const uint32_t la = nl / kXcds, lb = nl % kXcds, ca = nq / kXcds, cb = nq % kXcds;
    for (uint32_t r0 = 0; r0 < nq; r0 += kRound) {
        if (nq > kRound) bins_of(r0, b);  // else b still holds the only round's bins
#pragma unroll
        for (uint32_t i = 0; i < kOrderTiles; ++i) {
            const uint32_t q = r0 + i * kOrderThreads + t;
            if (q >= nq) continue;
            const uint32_t r = atomicAdd(&bins[b[i]], 1u);  // rank in the sorted batch
            uint32_t x, j;
            if (r < nl) {
                // runs of la + 1 for the first lb XCDs, then runs of la
                const uint32_t big = lb * (la + 1);
                if (r < big) {
                    x = r / (la + 1);
                    j = r % (la + 1);
                } else {
                    x = lb + (r - big) / la;  // la > 0 here: r < nl = lb when la == 0
                    j = (r - big) % la;
                }
            } else {
                uint32_t rest = r - nl;
                x = 0;
                while (x + 1 < kXcds && rest >= ca + (x < cb) - (la + (x < lb))) {
                    rest -= ca + (x < cb) - (la + (x < lb));
                    ++x;
                }
                j = la + (x < lb) + rest;
            }
            order[kXcds * j + x] = q;
        }
    }
}

template <int G, int F, int METRIC, int KIND, bool LEARN, bool BUF>
__device__ __forceinline__ void layer0_query(const DevIndex &ix, const SearchArgs &a) {
    extern __shared__ __align__(16) uint8_t smem[];
    if (blockIdx.x >= a.nq) return;
    const uint32_t qi = __builtin_amdgcn_readfirstlane(a.sched_order[blockIdx.x]);
    const Job job = job_of(ix, a, qi, LEARN);
    const RowSource src = rows_of(ix, a, KIND);
    QueryRegs<G, F, KIND> Q;
    load_query<G, F, KIND>(job.q, ix.dim, Q);
    const uint64_t cur = a.sched_start[qi];
    Descent d;
    d.cur = (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(cur >> 32))) << 32) |
            __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(cur));
    d.n_dist = __builtin_amdgcn_readfirstlane(a.sched_up[2 * static_cast<size_t>(qi)]);
    d.n_exp = __builtin_amdgcn_readfirstlane(a.sched_up[2 * static_cast<size_t>(qi) + 1]);
    search_layer0<G, F, METRIC, KIND, LEARN, BUF>(ix, a, job, carve<LEARN>(smem, a), src, Q, d);
}

template <int G, int F, int METRIC, int KIND, bool BUF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KIND == kFP8 || KIND == kU8 || (KIND == kU8E && F > 1) ? 5 : 6))) void layer0_kernel(
    DevIndex ix, SearchArgs a) {
    layer0_query<G, F, METRIC, KIND, false, BUF>(ix, a);
}

template <int G, int F, int METRIC, bool BUF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) void layer0_kernel_learned(DevIndex ix,
                                                                                                    SearchArgs a) {
    layer0_query<G, F, METRIC, kF32, true, BUF>(ix, a);
}

// The launches of one form (the one-kernel form, or the scheduled three).
template <int G, int F, int METRIC, int KIND, bool BUF>
hipError_t launch_form(const DevIndex &ix, const SearchArgs &a, hipStream_t stream, bool sched, bool learned,
                       size_t lds) {
    if (!sched) {
        if (learned)
            hipLaunchKernelGGL((search_kernel_learned<G, F, METRIC, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
        else
            hipLaunchKernelGGL((search_kernel<G, F, METRIC, KIND, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((descent_kernel<G, F, METRIC, KIND, BUF>), dim3(a.nq), dim3(64), 0, stream, ix, a);
    hipLaunchKernelGGL(order_kernel, dim3(1), dim3(kOrderThreads), 0, stream, a.sched_start, a.sched_cell, a.nq,
                       a.sched_order);
    if (learned)
        hipLaunchKernelGGL((layer0_kernel_learned<G, F, METRIC, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    else
        hipLaunchKernelGGL((layer0_kernel<G, F, METRIC, KIND, BUF>), dim3(a.nq), dim3(64), lds, stream, ix, a);
    return hipGetLastError();
}

// One metric: the one-kernel launch or the scheduled three.  A batch larger
// than the waves of the one-kernel form resident at once takes the form
// tuned_form picks for it (a.sched 1); a.sched 2 forces the scheduled form.
template <int G, int F, int METRIC, int KIND, bool BUF>
hipError_t launch_gfkm(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    const bool learned = KIND == kF32 && a.mode == HNSW_MODE_LEARNED;
    const size_t lds = search_lds_bytes(a, learned);
    const void *fused = learned ? reinterpret_cast<const void *>(&search_kernel_learned<G, F, METRIC, BUF>)
                                : reinterpret_cast<const void *>(&search_kernel<G, F, METRIC, KIND, BUF>);
    bool sched = a.sched_order && a.sched == 2;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // set while tuned_form times this call
    if (a.sched_order && a.sched == 1) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused, 64, lds) == hipSuccess &&
            hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            static_cast<uint64_t>(a.nq) > static_cast<uint64_t>(per_cu) * static_cast<uint64_t>(cus))
            sched = tuned_form(ix, a, stream, &ev0, &ev1);
        (void)hipGetLastError();
    }
    if (ev0) (void)hipEventRecord(ev0, stream);
    hipError_t err = launch_form<G, F, METRIC, KIND, BUF>(ix, a, stream, sched, learned, lds);
    if (ev1) (void)hipEventRecord(ev1, stream);
    return err;
}

template <int G, int F, int KIND, bool BUF>
hipError_t launch_gfk(const DevIndex &ix, const SearchArgs &a, hipStream_t stream) {
    if (ix.metric == HNSW_IP) return launch_gfkm<G, F, HNSW_IP, KIND, BUF>(ix, a, stream);
    return launch_gfkm<G, F, HNSW_L2SQ, KIND, BUF>(ix, a, stream);
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
        case HNSW_MODE_U8: return ix.u8_exact ? launch_kind<kU8E, BUF>(ix, a, stream) : launch_kind<kU8, BUF>(ix, a, stream);
        default: return launch_kind<kF32, BUF>(ix, a, stream);
    }
}

}  // namespace
}  // namespace hnsw
