// Device code of the batched K-NN-SEARCH (Alg. 5 of arXiv:1603.09320) for
// gfx950, shared by the batch kernel and the persistent serving kernel.
//
// One wavefront (64 lanes) answers one query:
//   1. the query is loaded into registers, split over lane groups;
//   2. greedy descent with ef = 1 through layers L..1: SEARCH-LAYER with
//      ef = 1 moves to the (dist, id)-smallest of the current element and its
//      neighbours until none is smaller, so no visited set is needed there;
//   3. SEARCH-LAYER (Alg. 2) on layer 0 with ef candidates;
//   4. the K nearest of W are written out.
//
// Layer-0 state per wave, all in LDS:
//   W    -- up to ef 64-bit keys sorted ascending; key = (ordered float bits
//           of the distance) << 32 | id << 1 | expanded-flag.  Alg. 2 keeps
//           the candidate set C and the list W; since an element that has
//           left W can never be expanded again (its key exceeds that of the
//           furthest element of W from then on), C is exactly the unexpanded
//           part of W, so one sorted list with a flag holds both.
//   ht   -- open-addressing visited table of element ids.  A probe run that
//           finds no free slot reports "not visited" without recording the
//           id: the table may forget (the element is scored again) but never
//           reports an unseen element as visited.  A re-scored element has
//           the same key; it is either in W (dropped by de-duplication) or
//           above the furthest element of W (rejected), so results do not
//           depend on the table size.
// Each expansion reads the candidate's adjacency row (one coalesced load of
// Mmax0 ids), filters it through ht, gathers the surviving vectors with G
// lanes per vector, reduces each distance across its lane group with
// cross-lane shuffles, then merges all new keys into W at once: W becomes the
// ef smallest of W and the new keys, which is what processing the
// neighbourhood one element at a time (Alg. 2, inner loop) produces.
#pragma once

#include <climits>

#include "internal.h"

namespace hnsw {
namespace {

// One query's inputs and outputs.
struct Job {
    const float *q;      // query row [dim]
    uint32_t k, ef;      // ef >= k
    int32_t *ids;        // [k]
    float *dists;        // [k]
    uint32_t *counters;  // [4] or null
    float *trace;        // learned mode: [max_ckpt][26] or null
};


constexpr int kProbes = 4;

__device__ __forceinline__ uint32_t ord_of(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;  // -0 orders as +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float float_of(uint32_t o) {
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(u);
}

__device__ __forceinline__ uint64_t make_key(float d, uint32_t id) {
    return (static_cast<uint64_t>(ord_of(d)) << 32) | (static_cast<uint64_t>(id) << 1);
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return static_cast<uint32_t>(k) >> 1; }
__device__ __forceinline__ float key_dist(uint64_t k) { return float_of(static_cast<uint32_t>(k >> 32)); }

// Keeps the compiler from moving LDS accesses across this point.  A wave's
// own LDS instructions are executed in issue order, so a later access (by
// any lane) sees every earlier one; only the compiler's order must be pinned
// (each workgroup is a single wave).
__device__ __forceinline__ void wave_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), lane);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int rank_in(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}

// Wave-wide minima.  Four DPP steps leave every lane with the minimum of its
// row of 16 (xor-1 and xor-2 swaps inside a quad, then the mirrored half-row
// and the mirrored row); the four row minima are then read into scalar
// registers, so the result is wave-uniform and known to the compiler as such
// (loop exits that depend on it stay uniform control flow).  No LDS traffic.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = dpp_u32<CTRL>(static_cast<uint32_t>(v)), hi = dpp_u32<CTRL>(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    uint64_t w;
    w = dpp_u64<0xB1>(v);   // quad_perm [1,0,3,2]
    v = w < v ? w : v;
    w = dpp_u64<0x4E>(v);   // quad_perm [2,3,0,1]
    v = w < v ? w : v;
    w = dpp_u64<0x141>(v);  // row_half_mirror
    v = w < v ? w : v;
    w = dpp_u64<0x140>(v);  // row_mirror
    v = w < v ? w : v;
    uint64_t m = readlane64(v, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) {
        const uint64_t x = readlane64(v, r);
        m = x < m ? x : m;
    }
    return m;
}

__device__ __forceinline__ int wave_min_int(int v) {
    v = min(v, static_cast<int>(dpp_u32<0xB1>(static_cast<uint32_t>(v))));
    v = min(v, static_cast<int>(dpp_u32<0x4E>(static_cast<uint32_t>(v))));
    v = min(v, static_cast<int>(dpp_u32<0x141>(static_cast<uint32_t>(v))));
    v = min(v, static_cast<int>(dpp_u32<0x140>(static_cast<uint32_t>(v))));
    const int a = min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16));
    const int b = min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48));
    return min(a, b);
}

// Test-and-set of `id` in the visited table.  Returns kSeen when the id was
// already there, kInserted when this call put it there, and kForgot when all
// kProbes slots were taken by other ids: the id is then treated as unseen
// (scored again).  The table only says which ids need no scoring, so any
// policy for a full table gives the same search results; it decides how often
// an id is scored twice.  Without REPLACE a forgotten id stays forgotten (slots
// are never cleared within a query), so an id that is inserted has never been
// scored before.  With REPLACE the id then takes its home slot (its older
// occupant is forgotten instead): ids met recently are the likeliest to be met
// again, and the longest queries, which fill the table, score fewer ids twice;
// an inserted id may then have been scored before.
constexpr int kSeen = 0, kInserted = 1, kForgot = 2;

// The home slot is the multiplicative hash of the id scaled onto [0, slots)
// (multiply-shift, so any slot count works); later probes step by a second
// hash of the id, 1..128 slots (below the smallest table, 256 slots), so that
// they do not fall in the runs that linear probing builds: at ef = 56 on
// sift_like this forgets fewer ids than linear steps (738 against 746
// distance evaluations per query, 1,216 slots).
template <bool REPLACE>
__device__ __forceinline__ int visit(uint32_t *ht, uint32_t slots, uint32_t id) {
    const uint32_t h = static_cast<uint32_t>((static_cast<uint64_t>(id * 0x9E3779B1u) * slots) >> 32);
    const uint32_t step = 1u + ((id * 0x85EBCA6Bu) >> 25);
    uint32_t slot = h;
#pragma unroll
    for (int p = 0; p < kProbes; ++p) {
        if (p) {
            slot += step;
            slot = slot >= slots ? slot - slots : slot;
        }
        const uint32_t old = atomicCAS(&ht[slot], kNoLink, id);
        if (old == kNoLink) return kInserted;
        if (old == id) return kSeen;
    }
    if (REPLACE) atomicExch(&ht[h], id);
    return kForgot;
}

// One DPP move of both halves of a double (gfx9 DPP controls, full rows and
// banks).  Every lane has a source lane under the controls used here, so the
// bound-control form is taken: it needs no "old" value to be materialised.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(u), CTRL, 0xF, 0xF, true));
    const uint32_t hi =
        static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(u >> 32), CTRL, 0xF, 0xF, true));
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// Sum over aligned groups of G lanes (G in {1,2,4,8,16}); every lane of a
// group ends with the same bits: each step adds two equal-shaped partial sums
// (xor-1 and xor-2 swaps inside a quad, then the mirrored half-row and row).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    if (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
    if (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
    return v;
}

// Vector stores the traversal can read.  A row is a sequence of 16-byte
// pieces: 4 fp32, 8 bf16, 16 fp8-E4M3 or 16 unsigned 8-bit integer values;
// an FP8 row's fp32 scale sits in the row's padding when the codes leave 4
// bytes before the next 64-byte boundary, else in an array after the rows (a
// d = 128 row stays 128 bytes, two 64-byte requests, not three).  kU8E is
// the 8-bit store when it equals the fp32 one (integer data in [0, 255]): its
// distances are the fp32 ones, so its kernels carry no re-rank (and, without
// the re-rank's registers, hold six waves per SIMD).
enum StoreKind { kF32 = 0, kBF16 = 1, kFP8 = 2, kU8 = 3, kU8E = 4 };

template <int KIND>
struct Store;
template <>
struct Store<kF32> {
    static constexpr int VPP = 4;  // values per 16-byte piece
    using QT = double;             // query element as held in registers
};
template <>
struct Store<kBF16> {
    static constexpr int VPP = 8;
    using QT = float;
};
template <>
struct Store<kFP8> {
    static constexpr int VPP = 16;
    using QT = float;
};
template <>
struct Store<kU8> {
    static constexpr int VPP = 16;
    using QT = float;
};
template <>
struct Store<kU8E> : Store<kU8> {};

// Byte k of w as an OCP FP8-E4M3 code, decoded by the hardware conversion
// (exact: every code is a float; the store holds no NaN codes).
__device__ __forceinline__ float fp8_byte(uint32_t w, int k) {
    switch (k & 3) {
        case 0: return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(w), 0);
        case 1: return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(w), 1);
        case 2: return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(w), 2);
        default: return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(w), 3);
    }
}

// Value j of a 16-byte piece.
template <int KIND>
__device__ __forceinline__ float piece_value(const uint4 &p, int j) {
    const uint32_t w = j < Store<KIND>::VPP / 4 ? p.x : (j < Store<KIND>::VPP / 2 ? p.y : (j < 3 * Store<KIND>::VPP / 4 ? p.z : p.w));
    if (KIND == kF32) return __uint_as_float(w);
    if (KIND == kBF16) return __uint_as_float((j & 1) ? (w & 0xFFFF0000u) : (w << 16));
    if (KIND == kU8 || KIND == kU8E) return static_cast<float>((w >> (8 * (j & 3))) & 0xFFu);
    return fp8_byte(w, j);
}

template <int G, int F, int KIND>
struct QueryRegs {
    typename Store<KIND>::QT q[F][Store<KIND>::VPP];  // values of pieces c = sub + f*G
};

template <int G, int F, int KIND>
__device__ __forceinline__ void load_query(const float *qrow, uint32_t dim, QueryRegs<G, F, KIND> &Q) {
    constexpr int V = Store<KIND>::VPP;
    const int sub = lane_id() % G;
#pragma unroll
    for (int f = 0; f < F; ++f)
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const uint32_t e = static_cast<uint32_t>(V * (sub + f * G) + j);
            const float x = qrow[e < dim ? e : dim - 1];
            Q.q[f][j] = e < dim ? static_cast<typename Store<KIND>::QT>(x) : 0;
        }
}

// Where the pieces of a row live.
struct RowSource {
    const uint4 *base;   // piece 0 of row 0
    uint32_t stride;     // pieces per row
    uint32_t pieces;     // pieces holding values (the rest of the row is padding)
    const uint8_t *scale;   // FP8: scale of row i at scale + i * scale_stride, else null
    uint32_t scale_stride;
    __amdgpu_buffer_rsrc_t rsrc;  // raw buffer over the store (buffered kernels: the store spans <= 2 GiB)
};

// Raw buffer descriptor word 3 for gfx9-family targets (32-bit data, no
// swizzle); loads beyond num_records return zero.
constexpr int kBufferDword3 = 0x00020000;
// Largest store the buffered gathers address (32-bit offsets, with room for
// the out-of-range offset of a padding piece).
constexpr uint64_t kBufferedMaxBytes = 1ull << 31;

__device__ __forceinline__ RowSource make_source(const void *base, uint32_t stride, uint32_t pieces,
                                                 const uint8_t *scale, uint32_t scale_stride, uint32_t n) {
    RowSource r;
    r.base = reinterpret_cast<const uint4 *>(base);
    r.stride = stride;
    r.pieces = pieces;
    r.scale = scale;
    r.scale_stride = scale_stride;
    const uint64_t bytes = (static_cast<uint64_t>(n) + 1) * stride * 16;
    r.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0,
                                               static_cast<int>(bytes <= kBufferedMaxBytes ? bytes : 0), kBufferDword3);
    return r;
}

__device__ __forceinline__ RowSource rows_of(const DevIndex &ix, const SearchArgs &a, int kind) {
    if (kind == kF32) return make_source(ix.vec, ix.stride4, ix.stride4, nullptr, 0, ix.n);
    if (kind == kBF16) return make_source(ix.vbf16, ix.bf16_stride16, ix.bf16_stride16, nullptr, 0, ix.n);
    if (kind == kU8 || kind == kU8E) return make_source(ix.vu8, ix.u8_stride16, ix.u8_pieces, nullptr, 0, ix.n);
    return make_source(ix.vfp8, ix.fp8_stride16, ix.fp8_pieces, ix.fp8_scale, ix.fp8_scale_stride, ix.n);
}

__device__ __forceinline__ float row_scale(const RowSource &src, uint32_t id) {
    return *reinterpret_cast<const float *>(src.scale + static_cast<size_t>(id) * src.scale_stride);
}

// Scores ids[0..m) against the query; keys[slot] receives the key of ids[slot].
// Lane group grp = lane / G handles slots grp, grp + P, ... (P = 64 / G).
// Every load is unconditional so that all of a chunk's loads are in flight
// together: an unused slot, and a piece beyond a row's values, read from the
// all-zero row n instead (the address is chosen, not the value, so no load is
// split or predicated).  Distances: sum over coordinates of (q_j - s*x_j)^2,
// or 1 - sum q_j*s*x_j, in double (s = 1 except for FP8), rounded once to float.
template <int G, int F, int METRIC, int KIND, bool BUF>
__device__ __forceinline__ void score_ids(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, KIND> &Q,
                                          const uint32_t *ids, int m, uint64_t *keys) {
    constexpr int P = 64 / G;
    // rows in flight per lane group: up to 4, fewer when each lane holds
    // more than two pieces of a row (register budget)
    constexpr int BP = (32 / P) < (8 / F) ? (32 / P) : (8 / F);
    constexpr int B = BP < 1 ? 1 : (BP > 4 ? 4 : BP);
    constexpr int V = Store<KIND>::VPP;
    const int lane = lane_id();
    const int grp = lane / G, sub = lane % G;
    const size_t zero_row = static_cast<size_t>(ix.n) * src.stride;
    // byte offset of each of this lane's pieces within a row (buffered path);
    // 0x80000000 places a piece past the row's values beyond the store
    uint32_t coff[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const uint32_t c = static_cast<uint32_t>(sub + f * G);
        coff[f] = c < src.pieces ? c * 16u : 0x80000000u;
    }
    for (int base = 0; base < m; base += P * B) {
        // sub-batches holding at least one id (wave-uniform: m and base are)
        const int nb = min(B, (m - base + P - 1) / P);
        uint32_t idv[B];
#pragma unroll
        for (int b = 0; b < B; ++b) idv[b] = ids[(base + b * P + grp) & 63];
#pragma unroll
        for (int b = 0; b < B; ++b) idv[b] = base + b * P + grp < m ? idv[b] : ix.n;
        uint4 v[B][F];
        float sc[B];
        if constexpr (BUF) {
            // 32-bit offsets: one multiply per row; a piece past the row's
            // values gets an offset beyond the store, which reads as zero
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b >= nb) break;
                const uint32_t roff = idv[b] * (src.stride * 16u);
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const auto w = __builtin_amdgcn_raw_buffer_load_b128(src.rsrc, roff + coff[f], 0, 0);
                    v[b][f] = make_uint4(w[0], w[1], w[2], w[3]);
                }
                if (KIND == kFP8) sc[b] = row_scale(src, idv[b]);
            }
        } else {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b >= nb) break;
                const size_t row = static_cast<size_t>(idv[b]) * src.stride;
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const uint32_t c = static_cast<uint32_t>(sub + f * G);
                    v[b][f] = src.base[c < src.pieces ? row + c : zero_row];
                }
                if (KIND == kFP8) sc[b] = row_scale(src, idv[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (b >= nb) break;
            double acc = 0.0;
            const double s = KIND == kFP8 ? static_cast<double>(sc[b]) : 1.0;
#pragma unroll
            for (int f = 0; f < F; ++f)
#pragma unroll
                for (int j = 0; j < V; ++j) {
                    const double x = KIND == kFP8 ? s * static_cast<double>(piece_value<KIND>(v[b][f], j))
                                                  : static_cast<double>(piece_value<KIND>(v[b][f], j));
                    const double qj = static_cast<double>(Q.q[f][j]);
                    if (METRIC == HNSW_L2SQ) {
                        const double t = qj - x;
                        acc = __fma_rn(t, t, acc);
                    } else {
                        acc = __fma_rn(qj, x, acc);
                    }
                }
            acc = group_sum<G>(acc);
            const int slot = base + b * P + grp;
            if (sub == 0 && slot < m) {
                const double d = METRIC == HNSW_L2SQ ? acc : 1.0 - acc;
                keys[slot] = make_key(static_cast<float>(d), idv[b]);
            }
        }
    }
}

struct WaveLds {
    uint64_t *W;       // [wslots]
    uint64_t *keys;    // [64] keys of the current batch
    uint32_t *ids;     // [64] ids of the current batch
    uint32_t *prevk;   // [64] top-K ids at the previous checkpoint (learned mode)
    float *hid;        // [2][64] hidden layers of the stop-rule network
    uint32_t *ht;      // [ht_slots]
};

// The learned stop rule's buffer prevk is carved only for its kernels, so the
// others keep more waves per CU within the LDS; its hidden layers (and the
// features) reuse the keys of the current batch, which are dead during a
// checkpoint (the merge has consumed them; the next gather rewrites them).
template <bool LEARN>
__device__ __forceinline__ WaveLds carve(uint8_t *base, const SearchArgs &a) {
    WaveLds s;
    s.W = reinterpret_cast<uint64_t *>(base);
    s.keys = s.W + a.wslots;
    s.ids = reinterpret_cast<uint32_t *>(s.keys + 64);
    if (LEARN) {
        s.prevk = s.ids + 64;
        s.hid = reinterpret_cast<float *>(s.keys);  // [2][64] floats: the 512 bytes of keys
        s.ht = s.prevk + 64;
    } else {
        s.prevk = nullptr;
        s.hid = nullptr;
        s.ht = s.ids + 64;
    }
    return s;
}

// Merges keys[0..m) (lane j owns keys[j]) into the sorted list W of size
// wsize: W <- the ef smallest of W and the new keys, dropping keys whose
// (distance, id) is already in W.  Returns the insertion position of the
// smallest admitted key (INT_MAX when none was admitted).
// Positions: while W fits one 64-entry chunk, from wave-wide comparisons (for
// each admitted key, broadcast with readlane, a ballot over W counts the
// smaller entries and detects an equal one); for a longer W, from a binary
// search of W by every lane at once (log2(wsize) dependent LDS reads in place
// of a ballot per chunk and admitted key: on glove_like at ef = 272 the
// ballots were most of the kernel's scalar instructions).
// `forgot`: some id of this batch was forgotten by the visited table.  Only
// then can a new key already be in W (the id was scored before without being
// recorded) or equal another new key of the batch (an adjacency row that
// lists one id twice, both copies forgotten): such keys are dropped, so W
// never holds an id twice, as with the exact visited set of Alg. 2.
// Otherwise both checks are skipped.  The low-precision stores pass whether
// their batch forgot; the fp32 store, whose table replaces entries (see
// visit), always passes true: on the 10,000-query sift_like batch the leaner
// loop measured 2% faster with FP8 but 0.6% slower with fp32 (same GPU,
// alternating runs).
__device__ __forceinline__ int merge_into_w(const WaveLds &s, int m, uint32_t ef, uint32_t &wsize, bool forgot) {
    const int lane = lane_id();
    const int ws = static_cast<int>(wsize);
    if (ws <= 64) {
        // W fits one chunk: lane i holds W[i] in registers (read together with
        // the new keys), the threshold W[ef-1] comes from a lane of it, and one
        // pass over the admitted keys yields every count: the W entries below
        // each key (scalar, from a ballot), whether W already holds it, the
        // admitted keys below each W entry and below each admitted key.
        const uint64_t wf = lane < ws ? s.W[lane] : ~0ull;
        const uint64_t a = lane < m ? s.keys[lane] : ~0ull;
        const uint64_t wk = lane < ws ? (wf >> 1) : ~0ull;
        const uint64_t thr = wsize < ef ? ~0ull : readlane64(wf, static_cast<int>(ef) - 1);
        uint64_t cm = __ballot(lane < m && a < thr);
        if (cm == 0) return INT_MAX;
        uint64_t km = 0;
        int lbmin = INT_MAX, lb = 0, r = 0, shift = 0;
        if (!forgot) {
            // every new key is distinct and absent from W: all are admitted
            km = cm;
            while (cm) {
                const int t = __ffsll(static_cast<unsigned long long>(cm)) - 1;
                cm &= cm - 1;
                const uint64_t at = readlane64(a, t);
                const int below = __popcll(__ballot(wk < (at >> 1)));
                lbmin = min(lbmin, below);
                // lane t takes `below`; with a scalar value the lane select
                // must come from M0 (one scalar operand per vector instruction)
                asm("s_mov_b32 m0, %2\n\ts_nop 0\n\tv_writelane_b32 %0, %1, m0" : "+v"(lb) : "s"(below), "s"(t) : "m0");
                shift += at < wf;
                r += at < a;
            }
        } else {
            while (cm) {
                const int t = __ffsll(static_cast<unsigned long long>(cm)) - 1;
                cm &= cm - 1;
                const uint64_t at = readlane64(a, t);
                if (__ballot(wk == (at >> 1))) continue;  // (distance, id) already in W
                if (__ballot(((km >> lane) & 1ull) && a == at)) continue;  // admitted already from a lower lane
                const int below = __popcll(__ballot(wk < (at >> 1)));
                km |= 1ull << t;
                lbmin = min(lbmin, below);
                lb = lane == t ? below : lb;
                shift += at < wf;
                r += (at < a) || (at == a && t < lane);
            }
        }
        if (km == 0) return INT_MAX;
        const bool keep = (km >> lane) & 1ull;
        const int np = lane + shift;
        wave_sync();
        if (lane < ws && lane >= lbmin && np < static_cast<int>(ef)) s.W[np] = wf;
        if (keep && lb + r < static_cast<int>(ef)) s.W[lb + r] = a;
        wave_sync();
        wsize = min(ef, wsize + static_cast<uint32_t>(__popcll(km)));
        return lbmin;
    }
    const uint64_t thr = wsize < ef ? ~0ull : s.W[ef - 1];
    const uint64_t a = lane < m ? s.keys[lane] : ~0ull;
    const bool cand = lane < m && a < thr;
    const uint64_t cm = __ballot(cand);
    if (cm == 0) return INT_MAX;
    int lb = 0;
    bool dup = false;
    if (forgot) {
        // the same key on a lower candidate lane: only the lowest copy may stay
        uint64_t mm = cm;
        while (mm) {
            const int t = __ffsll(static_cast<unsigned long long>(mm)) - 1;
            mm &= mm - 1;
            const uint64_t at = readlane64(a, t);
            const uint64_t same = __ballot(cand && a == at);
            if (lane == t) dup = (same & ((1ull << t) - 1ull)) != 0;
        }
    }
    {
        // each lane's position in W: the entries whose (distance, id) is below
        // its key, by a binary search of W (the flag bit ignored; W is sorted,
        // so it is sorted by key >> 1 too), and whether W holds the key
        const uint64_t key = a >> 1;
        int pos = 0;
        for (int step = 1 << (31 - __clz(ws)); step > 0; step >>= 1) {
            const int probe = pos + step - 1;
            if (probe < ws && (s.W[probe] >> 1) < key) pos += step;
        }
        lb = pos;
        if (forgot && pos < ws) dup = dup || (s.W[pos] >> 1) == key;
    }
    const bool keep = cand && !dup;
    const uint64_t km = __ballot(keep);
    if (km == 0) return INT_MAX;
    const int cnt = __popcll(km);
    int r = 0;
    {
        uint64_t mm = km;
        while (mm) {
            const int t = __ffsll(static_cast<unsigned long long>(mm)) - 1;
            mm &= mm - 1;
            const uint64_t at = readlane64(a, t);
            r += (at < a) || (at == a && t < lane);
        }
    }
    const int lbmin = wave_min_int(keep ? lb : INT_MAX);
    // Old elements at positions >= lbmin move right by the number of admitted
    // keys below them; chunks are moved top first so no unread slot is overwritten.
    for (int cb = (ws - 1) & ~63; cb >= (lbmin & ~63); cb -= 64) {
        const int i = cb + lane;
        const bool live = i >= lbmin && i < ws;
        const uint64_t w = live ? s.W[i] : 0ull;
        int below = 0;
        uint64_t mm = km;
        while (mm) {
            const int t = __ffsll(static_cast<unsigned long long>(mm)) - 1;
            mm &= mm - 1;
            below += readlane64(a, t) < w;
        }
        const int np = i + below;
        wave_sync();
        if (live && np < static_cast<int>(ef)) s.W[np] = w;
        wave_sync();
    }
    if (keep && lb + r < static_cast<int>(ef)) s.W[lb + r] = a;
    wave_sync();
    wsize = min(ef, wsize + static_cast<uint32_t>(cnt));
    return lbmin;
}

// ------------------------------------------------ learned stop rule
//
// Every `period` layer-0 expansions (at most max_ckpt times) the wave forms 24
// features of the search state (IEEE float arithmetic only), runs the
// 24-64-64-2 perceptron (BF16 weights and activations, products exact in
// float, accumulation in float in input order, lane j = hidden unit j), and
// (1) at the first checkpoint halves ef j = clamp(floor(0.5 - out1), 0, jmax)
// times (W keeps its ef nearest), (2) stops the search when out0 > tau.

struct LearnState {
    uint32_t ckpt, n_prev, n_exp_upper;
    float d_start, d_best_prev, d_k_prev;
};

// a / (|b| + tiny) clamped to [-big, big]; big = 1e6, tiny = 1e-20 (passed in
// scalar registers so that the constants are not held in vector registers).
__device__ __forceinline__ float lratio(float a, float b, float big, float tiny) {
    const float den = fabsf(b) + tiny;
    const float r = a / den;
    return r > big ? big : (r < -big ? -big : r);
}

// A wave-uniform float held in a scalar register.
__device__ __forceinline__ float uniform_f(float v) {
    return __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(v)));
}

__device__ __forceinline__ float bf16_round(float f) {
    uint32_t u = __float_as_uint(f);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(u);
}


// BF16 value h (0..7) of a 16-byte piece, as a float (exact).
__device__ __forceinline__ float bf16_half(const uint4 &p, int h) {
    const uint32_t w = h < 2 ? p.x : (h < 4 ? p.y : (h < 6 ? p.z : p.w));
    return __uint_as_float((h & 1) ? (w & 0xFFFF0000u) : (w << 16));
}

// Returns true when the rule stops the search; may lower ef and wsize.
[[maybe_unused]] __device__ bool learned_checkpoint(const WaveLds &s, const DevMlp &net, LearnState &st, uint32_t n_exp0,
                                   uint32_t K, int cursor, uint32_t &ef, uint32_t &wsize, float *trace) {
    // The lane id is re-read here behind an empty asm barrier: addresses the
    // checkpoint derives from it are then formed inside the checkpoint instead
    // of being hoisted out of the expansion loop and kept live across it.
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
    float big = 1e6f, tiny = 1e-20f;
    asm volatile("" : "+s"(big), "+s"(tiny));
    // likewise the loop-invariant inputs of the features (K, the upper-layer
    // expansion count, the distance at the start of layer 0)
    asm volatile("" : "+s"(K));
    uint32_t n_exp_upper = st.n_exp_upper;
    float d_start = st.d_start;
    asm volatile("" : "+s"(n_exp_upper), "+s"(d_start));
    const uint32_t ck = ++st.ckpt;
    wave_sync();  // the batch keys that hid overlays are consumed
    const uint32_t n = wsize;
    const uint32_t kk = n < K ? n : K;
    const float d_best = uniform_f(key_dist(s.W[0])), d_k = uniform_f(key_dist(s.W[kk - 1])),
                d_f = uniform_f(key_dist(s.W[n - 1]));
    uint32_t pos = n;
    for (int cb = cursor; cb < static_cast<int>(n); cb += 64) {
        const int i = cb + lane;
        const uint64_t um = __ballot(i < static_cast<int>(n) && !(s.W[i] & 1ull));
        if (um) {
            pos = static_cast<uint32_t>(cb + __ffsll(static_cast<unsigned long long>(um)) - 1);
            break;
        }
    }
    uint32_t n_unexp = 0;
    for (int cb = 0; cb < static_cast<int>(n); cb += 64) {
        const int i = cb + lane;
        n_unexp += __popcll(__ballot(i < static_cast<int>(n) && !(s.W[i] & 1ull)));
    }
    const float d_next = pos < n ? uniform_f(key_dist(s.W[pos])) : d_f;
    bool fresh_top = false;
    uint32_t my_id = 0;
    if (lane < static_cast<int>(kk)) {
        my_id = key_id(s.W[lane]);
        bool seen = false;
        for (uint32_t j = 0; j < st.n_prev; ++j) seen |= s.prevk[j] == my_id;
        fresh_top = !seen;
    }
    const uint32_t changed = __popcll(__ballot(fresh_top));
    wave_sync();
    if (lane < static_cast<int>(kk)) s.prevk[lane] = my_id;
    st.n_prev = kk;
    if (ck == 1) {
        st.d_best_prev = d_best;
        st.d_k_prev = d_k;
    }
    // features go to LDS as they are formed (hid[64..87]: layer 2 writes
    // there only after layer 1 has read them), so few are live at once
    const float fe = static_cast<float>(ef);
    float *fs = s.hid + 64;
    if (lane == 0) {
        fs[0] = static_cast<float>(n_exp0) / fe;
        fs[1] = static_cast<float>(n_exp0) / 256.0f;
        fs[2] = static_cast<float>(n_exp_upper) / 16.0f;
        fs[3] = static_cast<float>(n) / fe;
        fs[4] = static_cast<float>(pos) / fe;
        fs[5] = static_cast<float>(n_unexp) / fe;
        fs[6] = static_cast<float>(changed) / static_cast<float>(K);
        fs[7] = static_cast<float>(ck) / 32.0f;
        fs[8] = lratio(d_best, d_start, big, tiny);
        fs[9] = lratio(d_k, d_start, big, tiny);
        fs[10] = lratio(d_f, d_start, big, tiny);
        fs[11] = lratio(d_next, d_start, big, tiny);
        fs[12] = lratio(d_best, d_k, big, tiny);
        fs[13] = lratio(d_k, d_f, big, tiny);
        fs[14] = lratio(d_next, d_k, big, tiny);
        fs[15] = lratio(st.d_k_prev, d_k, big, tiny);
        fs[16] = lratio(st.d_best_prev, d_best, big, tiny);
        fs[17] = lratio(d_k - d_best, d_f - d_best, big, tiny);
        fs[18] = fe / 512.0f;
        fs[19] = static_cast<float>(K) / 100.0f;
        fs[20] = lratio(d_next - d_k, d_f - d_best, big, tiny);
        fs[21] = d_next < d_k ? 1.0f : 0.0f;
        fs[22] = pos < K ? 1.0f : 0.0f;
        fs[23] = 1.0f;
    }
    st.d_best_prev = d_best;
    st.d_k_prev = d_k;
    wave_sync();
    if (trace && lane < kMlpIn) trace[static_cast<size_t>(ck - 1) * (kMlpIn + 2) + lane] = fs[lane];
    // layer 1 (lane = hidden unit), inputs in order; the unit's 24 BF16
    // weights are three 16-byte pieces, fetched together
    const uint4 *r1 = reinterpret_cast<const uint4 *>(net.w1) + lane * 3;
    const uint4 w10 = r1[0], w11 = r1[1], w12 = r1[2];
    float a = net.b1[lane];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) {
        const uint4 &p = i < 8 ? w10 : (i < 16 ? w11 : w12);
        a = fmaf(bf16_half(p, i & 7), bf16_round(fs[i]), a);
    }
    const float h1 = bf16_round(a > 0.0f ? a : 0.0f);
    wave_sync();
    s.hid[lane] = h1;
    wave_sync();
    // layer 2: 64 weights per unit, eight pieces in two groups of four
    a = net.b2[lane];
    {
        const uint4 *r2 = reinterpret_cast<const uint4 *>(net.w2) + lane * 8;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const uint4 q0 = r2[4 * g], q1 = r2[4 * g + 1], q2 = r2[4 * g + 2], q3 = r2[4 * g + 3];
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint4 &p = i < 8 ? q0 : (i < 16 ? q1 : (i < 24 ? q2 : q3));
                a = fmaf(bf16_half(p, i & 7), s.hid[32 * g + i], a);
            }
        }
    }
    s.hid[64 + lane] = bf16_round(a > 0.0f ? a : 0.0f);
    wave_sync();
    // layer 3: lanes 0 and 1 hold the two outputs (the others repeat row 0)
    const int o = lane < kMlpOut ? lane : 0;
    a = net.b3[o];
    {
        const uint4 *r3 = reinterpret_cast<const uint4 *>(net.w3) + o * 8;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const uint4 q0 = r3[4 * g], q1 = r3[4 * g + 1], q2 = r3[4 * g + 2], q3 = r3[4 * g + 3];
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const uint4 &p = i < 8 ? q0 : (i < 16 ? q1 : (i < 24 ? q2 : q3));
                a = fmaf(bf16_half(p, i & 7), s.hid[64 + 32 * g + i], a);
            }
        }
    }
    const float out0 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(a), 0));
    const float out1 = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(a), 1));
    wave_sync();
    if (trace && lane == 0) {
        float *t = trace + static_cast<size_t>(ck - 1) * (kMlpIn + 2);
        t[kMlpIn] = out0;
        t[kMlpIn + 1] = out1;
    }
    if (ck == 1 && net.jmax > 0) {
        int j = static_cast<int>(floorf(0.5f - out1));
        j = j < 0 ? 0 : (j > net.jmax ? net.jmax : j);
        uint32_t ne = ef >> j;
        if (ne < K) ne = K;
        if (ne < ef) {
            ef = ne;
            if (wsize > ne) wsize = ne;
        }
    }
    return out0 > net.tau;
}

// Sorts W[0..n) ascending in LDS (n <= cap, cap a power of two; the tail is
// padded with the largest key).
__device__ __forceinline__ void sort_w(uint64_t *W, uint32_t n, uint32_t cap) {
    const int lane = lane_id();
    for (uint32_t i = n + lane; i < cap; i += 64) W[i] = ~0ull;
    wave_sync();
    for (uint32_t k = 2; k <= cap; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = lane; t < cap / 2; t += 64) {
                const uint32_t i = 2 * j * (t / j) + (t % j), l = i + j;
                const bool up = (i & k) == 0;
                const uint64_t x = W[i], y = W[l];
                if ((x > y) == up) {
                    W[i] = y;
                    W[l] = x;
                }
            }
            wave_sync();
        }
}

// Where the greedy descent of one query ends (the layer-0 entry, with its
// key) and the work it took.
struct Descent {
    uint64_t cur;
    uint32_t n_dist, n_exp;
    uint32_t cell;  // the node the walk reached on layer ix.cell_level (the entry point if that is 0)
};

// The first part of K-NN-SEARCH (Alg. 5): the entry point's distance, then a
// greedy walk (SEARCH-LAYER with ef = 1) through layers L..1.  Uses s.ids and
// s.keys only.
template <int G, int F, int METRIC, int KIND, bool BUF>
__device__ Descent descend(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, KIND> &Q,
                           const WaveLds &s) {
    const int lane = lane_id();
    Descent d{0ull, 0u, 0u, ix.entry};
    if (lane == 0) s.ids[0] = ix.entry;
    wave_sync();
    score_ids<G, F, METRIC, KIND, BUF>(ix, src, Q, s.ids, 1, s.keys);
    wave_sync();
    uint64_t cur = s.keys[0];
    d.n_dist = 1;
    for (int lc = static_cast<int>(ix.max_level); lc >= 1; --lc) {
        for (;;) {
            const uint32_t cid = key_id(cur);
            const size_t row = static_cast<size_t>(ix.uoff[cid]) + static_cast<size_t>(lc - 1);
            const uint32_t ld = ix.adjU[row * ix.Mmax + min(lane, static_cast<int>(ix.Mmax) - 1)];
            const uint32_t e = lane < static_cast<int>(ix.Mmax) ? ld : kNoLink;
            const bool valid = e != kNoLink;
            const uint64_t vm = __ballot(valid);
            const int m = __popcll(vm);
            if (valid) s.ids[rank_in(vm)] = e;
            wave_sync();
            score_ids<G, F, METRIC, KIND, BUF>(ix, src, Q, s.ids, m, s.keys);
            wave_sync();
            uint64_t best = cur;
            for (int i = lane; i < m; i += 64) best = s.keys[i] < best ? s.keys[i] : best;
            best = wave_min_u64(best);
            d.n_dist += m;
            d.n_exp += 1;
            wave_sync();
            if (best == cur) break;
            cur = best;
        }
        if (lc == static_cast<int>(ix.cell_level)) d.cell = key_id(cur);
    }
    d.cur = cur;
    return d;
}

// The rest of K-NN-SEARCH (Alg. 5) from the descent's result: SEARCH-LAYER on
// layer 0 with ef (Alg. 2), the exact rerank of low-precision traversals, and
// the K nearest of W written to the job's outputs.  `s` is the wave's LDS
// workspace, sized for a.wslots and a.ht_slots; job.ef >= job.k.
template <int G, int F, int METRIC, int KIND, bool LEARN, bool BUF>
__device__ void search_layer0(const DevIndex &ix, const SearchArgs &a, const Job &job, const WaveLds &s,
                              const RowSource &src, const QueryRegs<G, F, KIND> &Q, const Descent &dsc) {
    const int lane = lane_id();
    const float *qrow = job.q;
    const uint32_t ht_slots = a.ht_slots;
    for (uint32_t i = lane; i < ht_slots; i += 64) s.ht[i] = kNoLink;
    const uint64_t cur = dsc.cur;
    const uint32_t n_dist = dsc.n_dist, n_exp = dsc.n_exp;
    uint32_t n_dist0 = 0, n_exp0 = 0;

    // SEARCH-LAYER on layer 0 with ef candidates, starting from the descent's result.
    uint32_t ef = job.ef;
    LearnState lst{0u, 0u, n_exp, uniform_f(key_dist(cur)), 0.f, 0.f};
    if (lane == 0) {
        s.W[0] = cur;
        visit<false>(s.ht, ht_slots, key_id(cur));
    }
    wave_sync();
    uint32_t wsize = 1;
    int cursor = 0;  // every position below it is expanded
    n_dist0 = 1;
    // FP8 store: the links of the element most likely expanded next (the
    // second unexpanded element of W when the current one is taken; it comes
    // next unless a key admitted meanwhile is smaller, about 2 times in 3 on
    // sift_like) are loaded while the current element's neighbours are
    // gathered: when it does come next, its links are already in registers
    // and the expansion skips one dependent memory round trip.  pid: the
    // element whose row pl holds (kNoLink: none).  Alternating runs on one GPU
    // (10,000-query sift_like batch): FP8 3.5% faster; fp32 1.5% and BF16 2.3%
    // slower (their traversal moves 2-4 times the bytes and is limited by
    // bandwidth, not by the chain of round trips), so only FP8 does it.
    constexpr bool kPrefetch = KIND == kFP8;
    const int lsel = min(lane, static_cast<int>(ix.Mmax0) - 1);
    uint32_t pid = kNoLink, pl = 0;
    // fp32 store: a full visited table replaces (see visit).  Same-GPU
    // alternating runs, 10,000-query sift_like batch at ef 56: fp32 4.6%
    // faster (the longest queries, which end the batch, score fewer ids
    // twice); BF16 and FP8 0.4-1.6% slower (after a replacement their merge
    // must keep its duplicate checks), so they keep a forgetting table.
    // The low-precision stores replace too when the host asks (large ef, where
    // a forgetting table scores too many ids again).
    constexpr bool kReplace = KIND == kF32;
    const bool replace = kReplace || a.replace;
    for (;;) {
        int c = -1;
        uint64_t ck = 0;
        uint32_t nid = kNoLink;  // the second unexpanded element, if in the same 64-entry chunk
        for (int cb = cursor; cb < static_cast<int>(wsize); cb += 64) {
            const int i = cb + lane;
            const uint64_t w = i < static_cast<int>(wsize) ? s.W[i] : 1ull;
            const uint64_t um = __ballot(!(w & 1ull));
            if (um) {
                const int t = __ffsll(static_cast<unsigned long long>(um)) - 1;
                c = cb + t;
                ck = readlane64(w, t);
                const uint64_t um2 = um & (um - 1);
                if (kPrefetch && um2) nid = key_id(readlane64(w, __ffsll(static_cast<unsigned long long>(um2)) - 1));
                break;
            }
        }
        if (c < 0) break;  // every element of W has been expanded
        if (lane == 0) s.W[c] = ck | 1ull;
        cursor = c + 1;
        const uint32_t cid = key_id(ck);
        uint32_t ld;
        if (kPrefetch && cid == pid)
            ld = pl;
        else
            ld = ix.adj0[static_cast<size_t>(cid) * ix.Mmax0 + lsel];
        const uint32_t e = lane < static_cast<int>(ix.Mmax0) ? ld : kNoLink;
        const int vs = e == kNoLink ? kSeen
                       : (replace ? visit<true>(s.ht, ht_slots, e) : visit<false>(s.ht, ht_slots, e));
        const bool fresh = vs != kSeen;
        // with replacement an id that was inserted may have been scored before
        // (its slot was taken over), so the fp32 merge always keeps its checks
        const bool forgot = replace || __ballot(vs == kForgot) != 0;
        const uint64_t fm = __ballot(fresh);
        const int m = __popcll(fm);
        if (fresh) s.ids[rank_in(fm)] = e;
        wave_sync();
        // issued here, after the links above are used, so that no wait for them
        // also waits for it: it is in flight with the gathers below
        if (kPrefetch && nid != kNoLink) pl = ix.adj0[static_cast<size_t>(nid) * ix.Mmax0 + lsel];
        pid = nid;
        score_ids<G, F, METRIC, KIND, BUF>(ix, src, Q, s.ids, m, s.keys);
        wave_sync();
        n_dist0 += m;
        n_exp0 += 1;
        const int lbmin = merge_into_w(s, m, ef, wsize, forgot);
        if (lbmin < cursor) cursor = lbmin;
        if (LEARN && n_exp0 % a.mlp.period == 0 && lst.ckpt < a.mlp.max_ckpt &&
            learned_checkpoint(s, a.mlp, lst, n_exp0, job.k, cursor, ef, wsize, job.trace))
            break;
    }

    uint32_t n_rerank = 0;
    // an 8-bit copy that equals the fp32 store (integer data in [0, 255])
    // already gave the exact distances: nothing to re-rank
    if constexpr (KIND != kF32 && KIND != kU8E) {
        // Low-precision traversal: re-score every element of W exactly from the
        // fp32 vectors (the same grouped gather and arithmetic as the plain
        // path, pieces of 4 floats, so each lane holds VPP/4 times as many)
        // and keep the K nearest by that distance.
        constexpr int FX = F * (Store<KIND>::VPP / 4);
        QueryRegs<G, FX, kF32> QX;
        load_query<G, FX, kF32>(qrow, ix.dim, QX);
        const RowSource sx = rows_of(ix, a, kF32);
        // the traversal copy may fit the buffered gathers while the fp32 store
        // does not (10M x 96: 1.3-1.9 GB copies, a 3.8 GB store): then only
        // the re-rank takes the 64-bit addressed loads
        const bool fp32_buffered = (static_cast<uint64_t>(ix.n) + 1) * ix.stride4 * 16 <= kBufferedMaxBytes;
        for (uint32_t c0 = 0; c0 < wsize; c0 += 64) {
            const int cnt = static_cast<int>(min(64u, wsize - c0));
            if (lane < cnt) s.ids[lane] = key_id(s.W[c0 + lane]);
            wave_sync();
            if (BUF && fp32_buffered)
                score_ids<G, FX, METRIC, kF32, BUF>(ix, sx, QX, s.ids, cnt, s.keys);
            else
                score_ids<G, FX, METRIC, kF32, false>(ix, sx, QX, s.ids, cnt, s.keys);
            wave_sync();
            if (lane < cnt) s.W[c0 + lane] = s.keys[lane];
            wave_sync();
        }
        sort_w(s.W, wsize, a.wslots);
        n_rerank = wsize;
    }

    // The K nearest of W (Alg. 5, last line); W is sorted.
    for (uint32_t i = lane; i < job.k; i += 64) {
        if (i < wsize) {
            const uint64_t kk = s.W[i];
            job.ids[i] = static_cast<int32_t>(key_id(kk));
            job.dists[i] = key_dist(kk);
        } else {
            job.ids[i] = -1;
            job.dists[i] = __int_as_float(0x7f800000);
        }
    }
    if (job.counters && lane == 0) {
        uint32_t *c4 = job.counters;
        c4[0] = n_dist + n_dist0 + n_rerank;
        c4[1] = n_exp + n_exp0;
        c4[2] = n_dist0;
        c4[3] = n_exp0;
    }
}

// One query, answered by the calling wave (Alg. 5): descent, then layer 0.
template <int G, int F, int METRIC, int KIND, bool LEARN, bool BUF>
__device__ void search_one(const DevIndex &ix, const SearchArgs &a, const Job &job, const WaveLds &s) {
    const RowSource src = rows_of(ix, a, KIND);
    QueryRegs<G, F, KIND> Q;
    load_query<G, F, KIND>(job.q, ix.dim, Q);
    const Descent d = descend<G, F, METRIC, KIND, BUF>(ix, src, Q, s);
    search_layer0<G, F, METRIC, KIND, LEARN, BUF>(ix, a, job, s, src, Q, d);
}


}  // namespace
}  // namespace hnsw
