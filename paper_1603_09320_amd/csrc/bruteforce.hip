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


// ---------------------------------------------------------------- bf_tile
//
// The scan for k <= 32 (KP = 32 or 64 candidates per query and chunk).  A
// block of W waves takes 16 W queries; each wave owns 16 of them, holds their
// coordinates in registers as the A operand of v_mfma_f32_16x16x4f32 and keeps
// their candidate lists in its own part of LDS, so that the selection never
// waits for the other waves.  The block streams its chunk of the base set
// through one LDS tile of 32 rows: the next tile is loaded into registers
// while the waves multiply the current one, and stored between two block
// barriers.  The dimension is split over the four lane groups of a wave
// (group g holds coordinates [g S, g S + S) of its row, 4 S >= the padded
// dimension; coordinates past the stored row are zero in LDS and in the A
// operand), so one MFMA step s adds coordinates s, S + s, 2S + s and 3S + s
// of 16 queries x 16 rows, and every lane reads four steps of B with one
// 16-byte LDS load.  Rows in LDS are padded by 4 floats against bank
// conflicts.
//
// Candidate list of a query: its KP best keys so far, sorted, kept in the
// query's slot of the output array `partial` (global memory, +inf-keys at the
// start), and up to kTail unsorted admissions in LDS.  A ranking key below the
// threshold (the KP-th best key) is appended to the LDS tail; once the tail
// could overflow during the next tile, the wave sorts it, reads the sorted
// part into LDS, merges the two by rank (a binary search of each key in the
// other list), writes the KP best back and tightens the threshold: about one
// merge per kTail - kTRows admissions.  Keeping the sorted lists out of LDS
// lets three blocks share a CU (51 KB of LDS each at d = 128) instead of two.
constexpr int kTRows = 32;   // base rows per tile
constexpr int kTail = 64;    // unsorted admissions held beyond the KP best

// Waves per block (16 queries each).
constexpr int bf_tile_waves(int) { return 4; }

// Count of the n (power of two) sorted keys a[] that are < x (strict) or
// <= x, by a fixed-step binary search.
template <int N, bool kLessEq>
__device__ __forceinline__ int sorted_count(const uint64_t *a, uint64_t x) {
    int c = 0;
#pragma unroll
    for (int step = N / 2; step >= 1; step >>= 1) {
        const uint64_t v = a[c + step - 1];
        if (kLessEq ? v <= x : v < x) c += step;
    }
    const uint64_t v = a[c];
    return c + ((kLessEq ? v <= x : v < x) ? 1 : 0);
}

// Merge one query's LDS tail (count keys) into its sorted KP best, which sit
// in global memory at best[0..KP) (whole wave; scr: KP keys of LDS scratch).
// Each lane below KP reads and writes only best[lane].  Returns the new KP-th
// best key.
template <int KP>
__device__ uint64_t merge_tail(uint64_t *best, uint64_t *scr, uint64_t *tail, uint32_t count, int lane) {
    if (lane >= static_cast<int>(count)) tail[lane] = kMaxKey;  // kTail == 64 lanes
    if (lane < KP) scr[lane] = best[lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    wave_bitonic(tail, kTail);
    // stable merge (sorted part first on equal keys): ranks are distinct
    const uint64_t t = tail[lane];
    const int rt = lane + sorted_count<KP, true>(scr, t);
    uint64_t p = kMaxKey;
    int rp = KP;
    if (lane < KP) {
        p = scr[lane];
        rp = lane + sorted_count<kTail, false>(tail, p);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (rp < KP) scr[rp] = p;
    if (rt < KP) scr[rt] = t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < KP) best[lane] = scr[lane];
    return scr[KP - 1];
}

template <int KP, int S>
__global__ __launch_bounds__(256) void bf_tile(DevIndex ix, const float *Q, uint32_t nq, const float *xnorm,
                                               uint32_t chunk, uint32_t nchunks, uint64_t *partial) {
    constexpr int WAVES = bf_tile_waves(KP), THREADS = 64 * WAVES, kTQ = 16 * WAVES;
    constexpr int UPT = (kTRows * S + THREADS - 1) / THREADS;  // float4 units per thread and tile (at most)
    constexpr uint32_t RS = 4 * S + 4;  // LDS row stride (floats)
    extern __shared__ __align__(16) uint8_t smem[];
    float *tile = reinterpret_cast<float *>(smem);                            // [kTRows][RS]
    uint64_t *tails = reinterpret_cast<uint64_t *>(smem + kTRows * RS * 4);   // [kTQ][kTail]
    uint64_t *scrs = tails + kTQ * kTail;                                      // [WAVES][KP]
    uint64_t *thrs = scrs + WAVES * KP;                                        // [kTQ]
    uint32_t *cnts = reinterpret_cast<uint32_t *>(thrs + kTQ);                 // [kTQ]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const uint32_t q0 = blockIdx.x * kTQ + wave * 16;
    const uint32_t ch = blockIdx.y;
    const uint32_t b_lo = ch * chunk, b_hi = min(ix.n, b_lo + chunk);
    const uint32_t units_row = ix.stride4;  // float4 units per stored row
    uint64_t *mytail = tails + static_cast<size_t>(wave) * 16 * kTail;
    uint64_t *myscr = scrs + wave * KP;
    uint64_t *mythr = thrs + wave * 16;
    uint32_t *mycnt = cnts + wave * 16;
    // the sorted KP best of query q0 + qi (valid queries only)
    auto best_of = [&](int qi) { return partial + (static_cast<size_t>(q0 + qi) * nchunks + ch) * KP; };

    // A operand: query q0 + j, coordinates g*S + s
    float a[S];
    {
        const uint32_t q = q0 + j;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const uint32_t c = g * S + s;
            a[s] = (q < nq && c < ix.dim) ? Q[static_cast<size_t>(q) * ix.dim + c] : 0.f;
        }
    }
    // every list starts as KP +inf-keys (sorted) and an empty tail
    for (int qi = 0; qi < 16; ++qi)
        if (q0 + qi < nq && lane < KP) best_of(qi)[lane] = kMaxKey;
    if (lane < 16) {
        mycnt[lane] = 0;
        mythr[lane] = q0 + lane < nq ? kMaxKey : 0;  // a missing query admits nothing
    }
    // zero the tile once: columns beyond the stored row stay zero
    for (uint32_t e = tid; e < kTRows * RS; e += THREADS) tile[e] = 0.f;

    const uint32_t ntiles = b_lo < b_hi ? (b_hi - b_lo + kTRows - 1) / kTRows : 0;
    // the thread's part of every tile copy, fixed over the tiles: float4 unit
    // u is column unit c of row frow[u] (~0 when the thread has no unit u)
    uint32_t frow[UPT > 0 ? UPT : 1], goff[UPT > 0 ? UPT : 1], loff[UPT > 0 ? UPT : 1];
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
        const uint32_t un = static_cast<uint32_t>(tid) + static_cast<uint32_t>(THREADS) * u;
        const uint32_t r = un / units_row, c = un % units_row;
        frow[u] = un < kTRows * units_row ? r : ~0u;
        goff[u] = r * units_row + c;
        loff[u] = r * RS + 4 * c;
    }
    float4 stage[UPT > 0 ? UPT : 1];
    float xn_next[2] = {0.f, 0.f};
    const bool l2 = ix.metric == HNSW_L2SQ;
    auto fetch = [&](uint32_t t) {
        const uint32_t r0 = b_lo + t * kTRows;
        const uint32_t lim = b_hi - r0;  // rows of the chunk left from r0 (>= 1)
        const float4 *src = reinterpret_cast<const float4 *>(ix.vec) + static_cast<size_t>(r0) * units_row;
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            stage[u] = frow[u] < lim ? src[goff[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t rr = 16 * h + j;
            xn_next[h] = (l2 && rr < lim) ? xnorm[r0 + rr] : 0.f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int u = 0; u < UPT; ++u)
            if (frow[u] != ~0u) *reinterpret_cast<float4 *>(tile + loff[u]) = stage[u];
    };
    float xn[2] = {0.f, 0.f};
    __syncthreads();
    if (ntiles) {
        fetch(0);
        store();
        xn[0] = xn_next[0];
        xn[1] = xn_next[1];
    }
    __syncthreads();
    // thresholds of the lane's four queries (4 g + r), kept in registers
    uint64_t thr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) thr[r] = mythr[4 * g + r];
    for (uint32_t t = 0; t < ntiles; ++t) {
        if (t + 1 < ntiles) fetch(t + 1);  // in flight during the products
        // four independent accumulation chains (two row halves x two halves
        // of the coordinate steps), interleaved so that no product waits for
        // the one before it
        v4f acc[2][2] = {{{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}, {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}}};
#pragma unroll
        for (int s = 0; s < S; s += 4) {
            const int p = (s >> 2) & 1;
            const float4 b0 = *reinterpret_cast<const float4 *>(tile + j * RS + g * S + s);
            const float4 b1 = *reinterpret_cast<const float4 *>(tile + (16 + j) * RS + g * S + s);
            acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b0.x, acc[0][p], 0, 0, 0);
            acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b1.x, acc[1][p], 0, 0, 0);
            acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 1], b0.y, acc[0][p], 0, 0, 0);
            acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 1], b1.y, acc[1][p], 0, 0, 0);
            acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 2], b0.z, acc[0][p], 0, 0, 0);
            acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 2], b1.z, acc[1][p], 0, 0, 0);
            acc[0][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 3], b0.w, acc[0][p], 0, 0, 0);
            acc[1][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s + 3], b1.w, acc[1][p], 0, 0, 0);
        }
        // D[i][c] of a 16x16x4 product: lane c + 16 * (i / 4), element i % 4
        // (i: query of the wave, c: row of the 16-row half)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t b = b_lo + t * kTRows + 16 * h + j;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dot = acc[h][0][r] + acc[h][1][r];
                const float d = l2 ? xn[h] - 2.f * dot : -dot;
                const uint64_t key = (static_cast<uint64_t>(ord_of(d)) << 32) | b;
                if (b < b_hi && key < thr[r]) {
                    const int qi = 4 * g + r;
                    const uint32_t slot = atomicAdd(&mycnt[qi], 1u);
                    if (slot < static_cast<uint32_t>(kTail)) mytail[qi * kTail + slot] = key;  // always: see the merge below
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // merge the tails that could overflow during the next tile (a tile
        // adds at most kTRows keys to a query)
        const uint64_t full = __ballot(lane < 16 && mycnt[lane] > static_cast<uint32_t>(kTail - kTRows));
        for (uint64_t m = full; m;) {
            const int qi = __ffsll(static_cast<unsigned long long>(m)) - 1;
            m &= m - 1;
            const uint64_t kth = merge_tail<KP>(best_of(qi), myscr, mytail + qi * kTail, mycnt[qi], lane);
            if (lane == 0) {
                mythr[qi] = kth;
                mycnt[qi] = 0;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (full) {
#pragma unroll
            for (int r = 0; r < 4; ++r) thr[r] = mythr[4 * g + r];
        }
        if (t + 1 < ntiles) {
            __syncthreads();  // every wave is done with the tile
            store();
            xn[0] = xn_next[0];
            xn[1] = xn_next[1];
            __syncthreads();
        }
    }
    // the last admissions of each query of the wave (a missing query has none)
    for (int qi = 0; qi < 16; ++qi)
        if (mycnt[qi] > 0) merge_tail<KP>(best_of(qi), myscr, mytail + qi * kTail, mycnt[qi], lane);
}

size_t bf_tile_lds(uint32_t S, int KP) {
    const size_t q = 16 * bf_tile_waves(KP);
    return static_cast<size_t>(kTRows) * (4 * S + 4) * 4 + q * kTail * 8 + bf_tile_waves(KP) * KP * 8 + q * 8 + q * 4;
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

template <int KP, int S>
hipError_t bf_tile_launch(const DevIndex &ix, const float *Q, uint32_t nq, const float *xnorm, uint32_t nchunks,
                          uint32_t chunk, uint64_t *partial, hipStream_t st) {
    const size_t lds = bf_tile_lds(S, KP);
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&bf_tile<KP, S>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    constexpr uint32_t qpb = 16 * bf_tile_waves(KP);
    dim3 g((nq + qpb - 1) / qpb, nchunks);
    hipLaunchKernelGGL((bf_tile<KP, S>), g, dim3(64 * bf_tile_waves(KP)), lds, st, ix, Q, nq, xnorm, chunk,
                       nchunks, partial);
    return hipGetLastError();
}

template <int KP>
hipError_t bf_run_tile(const DevIndex &ix, const float *Q, uint32_t nq, uint32_t k, const float *xnorm,
                       uint64_t *partial, uint32_t nchunks, uint32_t chunk, int32_t *ids, double *d,
                       hipStream_t st) {
    const uint32_t dpad = ix.stride4 * 4;
    // S: coordinates per lane group, 4 S >= the stored row (dpad <= 256)
    const uint32_t need = (dpad + 3) / 4;
    hipError_t e;
    if (need <= 4) e = bf_tile_launch<KP, 4>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else if (need <= 8) e = bf_tile_launch<KP, 8>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else if (need <= 16) e = bf_tile_launch<KP, 16>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else if (need <= 24) e = bf_tile_launch<KP, 24>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else if (need <= 32) e = bf_tile_launch<KP, 32>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else if (need <= 48) e = bf_tile_launch<KP, 48>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
    else e = bf_tile_launch<KP, 64>(ix, Q, nq, xnorm, nchunks, chunk, partial, st);
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

// Candidates kept per (query, chunk): 2k at least.  k <= 32 runs bf_tile
// (KP 32 or 64), larger k the block-synchronised bf_scan (KP 128 or 256).
uint32_t bf_candidates(uint32_t k) { return k <= 16 ? 32 : (k <= 32 ? 64 : (k <= 64 ? 128 : 256)); }

void bf_plan(const DevIndex &ix, uint32_t nq, uint32_t k, uint32_t *nchunks, uint32_t *chunk) {
    const bool tile = k <= 32;
    const uint32_t qpb = tile ? 16u * bf_tile_waves(static_cast<int>(bf_candidates(k))) : kQT;
    const uint32_t tiles = (nq + qpb - 1) / qpb;
    const uint32_t target = tile ? 2048u : 4096u;  // blocks of the scan
    uint32_t nc = (target + tiles - 1) / tiles;
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
        case 32: return bf_run_tile<32>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
        case 64: return bf_run_tile<64>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
        case 128: return bf_run<128>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
        default: return bf_run<256>(ix, Q, nq, k, xnorm, partial, nchunks, chunk, ids, d, st);
    }
}

}  // namespace hnsw
