// Graph construction on the GPU: INSERT (Alg. 1 of arXiv:1603.09320) for
// batches of elements, with few synchronisation points (the paper's Sec. 4.1
// notes that construction parallelises this way, at the cost of a
// non-deterministic graph on CPU threads; here a batch schedule fixes it).
//
// Elements are inserted in id order, in batches.  Every element of a batch
// runs the per-element part of Alg. 1 against the graph as it stood before
// the batch, one wavefront per element (build_insert_kernel):
//   greedy descent with ef = 1 through the layers above its level l;
//   for each layer lc = min(L, l)..0: SEARCH-LAYER with efConstruction
//   candidates, entered from all of W of the layer above, then
//   SELECT-NEIGHBORS-HEURISTIC (Alg. 4) for M neighbours, which become the
//   element's list on lc (with extendCandidates, over the candidates and
//   their neighbours on lc, a list kept in global scratch).
// Its new links e <- q are then grouped by (lc, e) with a stable radix sort,
// and one wavefront per receiving element (build_link_kernel) appends them,
// or, when the list would exceed Mmax (Mmax0 on layer 0), selects the list
// again with the heuristic from e over its links and the new ones.  An
// element whose level exceeds the current top layer is inserted alone (it
// becomes the enter point).  With batches of one element this is Alg. 1 step
// for step: the lists equal those of the sequential INSERT.
//
// The heuristic runs in rounds that give exactly the sequential result:
// candidates are visited in increasing (distance, id) order; the first one not
// yet discarded is kept, and every later candidate nearer to it than to the
// base is discarded (one batched distance evaluation per kept element).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <hipcub/hipcub.hpp>
#include <vector>

#include "search_device.h"

namespace hnsw {

// One batch of insertions.
struct BuildArgs {
    const uint8_t *levels;   // [n] level of every element
    uint32_t first, end;     // elements [first, end)
    uint32_t entry, top;     // enter point and top layer L before the batch
    uint32_t M, efC;         // links per new element per layer, candidates of the layer searches
    uint32_t wpow2;          // LDS slots for W (power of two >= efC, >= 64)
    uint32_t ht_slots;       // visited-table slots (>= 256)
    int keep_pruned;         // Alg. 4 keepPrunedConnections
    int simple;              // SELECT-NEIGHBORS-SIMPLE (Alg. 3) instead of the heuristic
    int extend;              // Alg. 4 extendCandidates
    uint64_t *ext;           // extendCandidates: [waves][ecap] keys of each wave's extended list
    uint32_t ecap;           // keys per wave (power of two >= efC * (max list width + 1))
    uint64_t upper_base;     // upper_off of the batch's first element with a layer >= 1 (row origin of its pairs)
    uint64_t *pair_key;      // [(batch + batch upper rows) * M] (lc << 32 | e), or kNoPair
    uint32_t *pair_val;      // the new element q of each pair
};

// Re-selection of the lists that receive links.
struct LinkArgs {
    const uint64_t *key;      // sorted unique keys of the runs
    const uint32_t *count;    // links per run
    const uint32_t *offset;   // first link of the run in val
    const uint32_t *val;      // new elements, grouped by run
    const uint32_t *n_runs;   // device scalar
    uint32_t wpow2;           // LDS slots of the candidate list (power of two, <= 1024)
    int keep_pruned;
    int simple;               // Alg. 3 instead of Alg. 4
    int extend;               // Alg. 4 extendCandidates
    uint64_t *ext;            // [grid][ecap] keys of each wave's extended list
    uint32_t ecap;            // power of two >= wpow2 * (max list width + 1)
    uint32_t *stage;          // extendCandidates: [runs][stage_w] new lists, written to the graph afterwards
    uint32_t stage_w;
};

namespace {

constexpr uint64_t kNoPair = ~0ull;

__device__ __forceinline__ uint32_t *row_of(const DevIndex &ix, uint32_t id, int lc) {
    uint32_t *p = const_cast<uint32_t *>(lc ? ix.adjU + (static_cast<size_t>(ix.uoff[id]) + lc - 1) * ix.Mmax
                                            : ix.adj0 + static_cast<size_t>(id) * ix.Mmax0);
    return p;
}

__device__ __forceinline__ const float *vec_row(const DevIndex &ix, uint32_t id) {
    return ix.vec + static_cast<size_t>(id) * ix.stride4 * 4;
}

// LDS of one build wave: the search state of search_device.h plus the
// positions of the candidates being tested and the kept list R.
struct BuildLds {
    WaveLds s;      // W [wpow2], keys [64], ids [64], ht [ht_slots]
    uint32_t *pos;  // [64]
    uint32_t *R;    // [64]
};

__device__ __forceinline__ BuildLds carve_build(uint8_t *base, uint32_t wpow2) {
    BuildLds b;
    b.s.W = reinterpret_cast<uint64_t *>(base);
    b.s.keys = b.s.W + wpow2;
    b.s.ids = reinterpret_cast<uint32_t *>(b.s.keys + 64);
    b.pos = b.s.ids + 64;
    b.R = b.pos + 64;
    b.s.ht = b.R + 64;
    b.s.prevk = nullptr;
    b.s.hid = nullptr;
    return b;
}

size_t build_lds_bytes(uint32_t wpow2, uint32_t ht_slots) {
    return static_cast<size_t>(wpow2) * 8 + 64 * 8 + 3 * 64 * 4 + static_cast<size_t>(ht_slots) * 4;
}

// Stores of one wave to global memory complete and are seen by the wave's
// later loads from any lane (the workgroup is the one wave).
__device__ __forceinline__ void global_sync() {
    __threadfence_block();
    wave_sync();
}

template <bool GW>
__device__ __forceinline__ void list_sync() {
    if constexpr (GW)
        global_sync();
    else
        wave_sync();
}

// SELECT-NEIGHBORS-HEURISTIC (Alg. 4) over the candidates W[0..m), sorted by
// (distance to the base, id) with clear flags: R receives at most Mk ids.  A
// candidate is kept when its distance to the base is smaller (strictly) than
// its distance to every element kept before it.  Rounds: the first candidate
// not discarded is kept; every later candidate not discarded is then scored
// against it and discarded unless it is nearer to the base.  keep_pruned
// fills the rest of R with discarded candidates, nearest first.  W keeps its
// keys; flags are set on kept and discarded candidates.  GW: W is in global
// memory (an extended candidate list), so flag stores are fenced before other
// lanes read them.
template <int G, int F, int METRIC, bool BUF, bool GW = false>
__device__ uint32_t select_heuristic_w(const DevIndex &ix, const RowSource &src, const BuildLds &b, uint32_t m,
                                       uint32_t Mk, bool keep_pruned) {
    const int lane = lane_id();
    uint32_t r = 0;
    int cursor = 0;
    while (r < Mk) {
        int c = -1;
        uint64_t ck = 0;
        for (int cb = cursor; cb < static_cast<int>(m); cb += 64) {
            const int i = cb + lane;
            const uint64_t w = i < static_cast<int>(m) ? b.s.W[i] : 1ull;
            const uint64_t am = __ballot(!(w & 1ull));
            if (am) {
                const int t = __ffsll(static_cast<unsigned long long>(am)) - 1;
                c = cb + t;
                ck = readlane64(w, t);
                break;
            }
        }
        if (c < 0) break;
        const uint32_t cid = key_id(ck);
        if (lane == 0) {
            b.R[r] = cid;
            b.s.W[c] = ck | 1ull;
        }
        list_sync<GW>();
        ++r;
        cursor = c + 1;
        if (r == Mk) break;
        // discard the later candidates nearer to the kept element than to the base
        QueryRegs<G, F, kF32> QC;
        load_query<G, F, kF32>(vec_row(ix, cid), ix.dim, QC);
        for (int cb = cursor; cb < static_cast<int>(m); cb += 64) {
            const int i = cb + lane;
            const bool alive = i < static_cast<int>(m) && !(b.s.W[i] & 1ull);
            const uint64_t am = __ballot(alive);
            if (!am) continue;
            const int cnt = __popcll(am);
            if (alive) {
                const int k = rank_in(am);
                b.s.ids[k] = key_id(b.s.W[i]);
                b.pos[k] = static_cast<uint32_t>(i);
            }
            wave_sync();
            score_ids<G, F, METRIC, kF32, BUF>(ix, src, QC, b.s.ids, cnt, b.s.keys);
            wave_sync();
            if (lane < cnt) {
                const uint32_t p = b.pos[lane];
                const uint64_t w = b.s.W[p];
                // keep test: distance to the base < distance to the kept element
                if (!(key_dist(w) < key_dist(b.s.keys[lane]))) b.s.W[p] = w | 1ull;
            }
            list_sync<GW>();
        }
    }
    if (keep_pruned && r < Mk) {
        // the kept ones are in R: the others with a flag were discarded, in key order
        const uint32_t rl = lane < static_cast<int>(r) ? b.R[lane] : kNoLink;
        for (int cb = 0; cb < static_cast<int>(m) && r < Mk; cb += 64) {
            const int i = cb + lane;
            const uint64_t w = i < static_cast<int>(m) ? b.s.W[i] : 0ull;
            bool pruned = (w & 1ull) != 0;
            uint64_t pm = __ballot(pruned);
            while (pm && r < Mk) {
                const int t = __ffsll(static_cast<unsigned long long>(pm)) - 1;
                pm &= pm - 1;
                const uint32_t id = key_id(readlane64(w, t));
                if (__ballot(rl == id)) continue;  // kept, not discarded
                if (lane == 0) b.R[r] = id;
                ++r;
            }
        }
        wave_sync();
    }
    return r;
}

// SELECT-NEIGHBORS-SIMPLE (Alg. 3): the Mk nearest of W[0..m) (sorted) into R.
__device__ __forceinline__ uint32_t select_simple_w(const BuildLds &b, uint32_t m, uint32_t Mk) {
    const int lane = lane_id();
    const uint32_t r = m < Mk ? m : Mk;
    if (lane < static_cast<int>(r)) b.R[lane] = key_id(b.s.W[lane]);
    wave_sync();
    return r;
}

// Alg. 3 or Alg. 4 on the sorted candidates W[0..m).
template <int G, int F, int METRIC, bool BUF>
__device__ __forceinline__ uint32_t select_w(const DevIndex &ix, const RowSource &src, const BuildLds &b, uint32_t m,
                                             uint32_t Mk, bool keep_pruned, bool simple) {
    if (simple) return select_simple_w(b, m, Mk);
    return select_heuristic_w<G, F, METRIC, BUF>(ix, src, b, m, Mk, keep_pruned);
}

// Ascending bitonic sort of E[0..cap) (cap a power of two >= 64) in global
// memory by one wave; four compare-exchanges per lane are loaded together.
__device__ void sort_global(uint64_t *E, uint32_t cap) {
    const int lane = lane_id();
    const uint32_t half = cap / 2;
    for (uint32_t k = 2; k <= cap; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t0 = lane; t0 < half; t0 += 256) {
                uint32_t ii[4];
                uint64_t x[4], y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t t = t0 + 64u * u;
                    ii[u] = 2 * j * (t / j) + (t % j);
                    if (t < half) {
                        x[u] = E[ii[u]];
                        y[u] = E[ii[u] + j];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t t = t0 + 64u * u;
                    if (t < half && (x[u] > y[u]) == ((ii[u] & k) == 0)) {
                        E[ii[u]] = y[u];
                        E[ii[u] + j] = x[u];
                    }
                }
            }
            global_sync();
        }
}

// Alg. 4's extendCandidates.  E receives the keys (distance to the base,
// computed as for every other candidate) of the candidates W[0..m) and of
// every neighbour on layer lc of a candidate, the base itself excepted, each
// element once, ascending, flags clear; returns their count.  E is the wave's
// global scratch of ecap >= m * (width + 1) keys.  An element met twice has
// the same key both times, so the repeats are adjacent after the sort and are
// dropped there.
template <int G, int F, int METRIC, bool BUF>
__device__ uint32_t extend_candidates(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, kF32> &QB,
                                      const BuildLds &b, uint32_t m, uint32_t base_id, int lc, uint64_t *E) {
    const int lane = lane_id();
    for (uint32_t i = lane; i < m; i += 64) E[i] = b.s.W[i] & ~1ull;
    uint32_t t = m;
    const uint32_t width = lc ? ix.Mmax : ix.Mmax0;
    const int lsel = min(lane, static_cast<int>(width) - 1);
    int pend = 0;  // neighbour ids waiting in b.s.ids
    for (uint32_t i = 0; i <= m; ++i) {
        uint64_t vm = 0;
        uint32_t e = kNoLink;
        if (i < m) {
            const uint32_t cid = key_id(b.s.W[i]);
            // a candidate that is not a member of layer lc has no list there
            if (lc == 0 || ix.uoff[cid] >= 0) {
                const uint32_t ld = row_of(ix, cid, lc)[lsel];
                e = lane < static_cast<int>(width) && ld != base_id ? ld : kNoLink;
                vm = __ballot(e != kNoLink);
            }
        }
        const int c = __popcll(vm);
        if (pend > 0 && (i == m || pend + c > 64)) {
            wave_sync();
            score_ids<G, F, METRIC, kF32, BUF>(ix, src, QB, b.s.ids, pend, b.s.keys);
            wave_sync();
            if (lane < pend) E[t + lane] = b.s.keys[lane];
            t += static_cast<uint32_t>(pend);
            pend = 0;
        }
        if (e != kNoLink) b.s.ids[pend + rank_in(vm)] = e;
        pend += c;
    }
    uint32_t p2 = 64;
    while (p2 < t) p2 <<= 1;
    for (uint32_t i = t + lane; i < p2; i += 64) E[i] = ~0ull;
    global_sync();
    sort_global(E, p2);
    // drop repeats in place: a key is kept unless it equals its predecessor
    // (~0ull, a flagged key, equals no candidate's)
    uint32_t u = 0;
    uint64_t last = ~0ull;
    for (uint32_t cb = 0; cb < t; cb += 64) {
        const uint32_t i = cb + lane;
        const uint64_t v = i < t ? E[i] : ~0ull;
        uint64_t prev = __shfl_up(v, 1, 64);
        if (lane == 0) prev = last;
        const bool keep = i < t && v != prev;
        const uint64_t km = __ballot(keep);
        last = readlane64(v, 63);
        if (keep) E[u + rank_in(km)] = v;
        u += static_cast<uint32_t>(__popcll(km));
    }
    global_sync();
    return u;
}

// Alg. 4 with extendCandidates on the sorted candidates W[0..m) of base_id on
// layer lc: the extended list is built in E, then selected from as W is.
template <int G, int F, int METRIC, bool BUF>
__device__ uint32_t select_extended(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, kF32> &QB,
                                    const BuildLds &b, uint32_t m, uint32_t Mk, bool keep_pruned, uint32_t base_id,
                                    int lc, uint64_t *E) {
    const uint32_t u = extend_candidates<G, F, METRIC, BUF>(ix, src, QB, b, m, base_id, lc, E);
    BuildLds g = b;
    g.s.W = E;
    return select_heuristic_w<G, F, METRIC, BUF, true>(ix, src, g, u, Mk, keep_pruned);
}

// SEARCH-LAYER (Alg. 2) on layer lc with ef candidates, entered from W[0..wsize)
// (sorted keys, flags clear, ids already in the visited table).
template <int G, int F, int METRIC, bool BUF>
__device__ void beam_layer(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, kF32> &Q, const BuildLds &b,
                           uint32_t ht_slots, uint32_t ef, uint32_t &wsize, int lc) {
    const int lane = lane_id();
    const uint32_t width = lc ? ix.Mmax : ix.Mmax0;
    const int lsel = min(lane, static_cast<int>(width) - 1);
    int cursor = 0;
    for (;;) {
        int c = -1;
        uint64_t ck = 0;
        for (int cb = cursor; cb < static_cast<int>(wsize); cb += 64) {
            const int i = cb + lane;
            const uint64_t w = i < static_cast<int>(wsize) ? b.s.W[i] : 1ull;
            const uint64_t um = __ballot(!(w & 1ull));
            if (um) {
                const int t = __ffsll(static_cast<unsigned long long>(um)) - 1;
                c = cb + t;
                ck = readlane64(w, t);
                break;
            }
        }
        if (c < 0) break;  // every element of W has been expanded
        if (lane == 0) b.s.W[c] = ck | 1ull;
        cursor = c + 1;
        const uint32_t ld = row_of(ix, key_id(ck), lc)[lsel];
        const uint32_t e = lane < static_cast<int>(width) ? ld : kNoLink;
        const int vs = e != kNoLink ? visit<true>(b.s.ht, ht_slots, e) : kSeen;
        const bool fresh = vs != kSeen;
        const uint64_t fm = __ballot(fresh);
        const int m = __popcll(fm);
        if (fresh) b.s.ids[rank_in(fm)] = e;
        wave_sync();
        score_ids<G, F, METRIC, kF32, BUF>(ix, src, Q, b.s.ids, m, b.s.keys);
        wave_sync();
        const int lbmin = merge_into_w(b.s, m, ef, wsize, true);
        if (lbmin < cursor) cursor = lbmin;
    }
}

// The per-element part of INSERT (Alg. 1) for element q of the batch.
template <int G, int F, int METRIC, bool BUF>
__global__ __launch_bounds__(64) void build_insert_kernel(DevIndex ix, BuildArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t q = a.first + blockIdx.x;
    if (q >= a.end) return;
    const int lane = lane_id();
    const BuildLds b = carve_build(smem, a.wpow2);
    const RowSource src = rows_of(ix, SearchArgs{}, kF32);
    QueryRegs<G, F, kF32> Q;
    load_query<G, F, kF32>(vec_row(ix, q), ix.dim, Q);
    const int l = a.levels[q];
    const int L = static_cast<int>(a.top);
    // distance to the enter point, then the greedy phase above the element's level
    if (lane == 0) b.s.ids[0] = a.entry;
    wave_sync();
    score_ids<G, F, METRIC, kF32, BUF>(ix, src, Q, b.s.ids, 1, b.s.keys);
    wave_sync();
    uint64_t cur = b.s.keys[0];
    for (int lc = L; lc > l; --lc) {
        for (;;) {
            const uint32_t ld = row_of(ix, key_id(cur), lc)[min(lane, static_cast<int>(ix.Mmax) - 1)];
            const uint32_t e = lane < static_cast<int>(ix.Mmax) ? ld : kNoLink;
            const uint64_t vm = __ballot(e != kNoLink);
            const int m = __popcll(vm);
            if (e != kNoLink) b.s.ids[rank_in(vm)] = e;
            wave_sync();
            score_ids<G, F, METRIC, kF32, BUF>(ix, src, Q, b.s.ids, m, b.s.keys);
            wave_sync();
            uint64_t best = cur;
            if (lane < m) best = b.s.keys[lane] < best ? b.s.keys[lane] : best;
            best = wave_min_u64(best);
            wave_sync();
            if (best == cur) break;
            cur = best;
        }
    }
    if (lane == 0) b.s.W[0] = cur;
    wave_sync();
    uint32_t wsize = 1;
    const uint32_t M = a.M;
    for (int lc = min(L, l); lc >= 0; --lc) {
        // entry set: all of W (its elements are members of this layer)
        for (uint32_t i = lane; i < a.ht_slots; i += 64) b.s.ht[i] = kNoLink;
        wave_sync();
        for (uint32_t i = lane; i < wsize; i += 64) {
            const uint64_t w = b.s.W[i] & ~1ull;
            b.s.W[i] = w;
            visit<true>(b.s.ht, a.ht_slots, key_id(w));
        }
        wave_sync();
        beam_layer<G, F, METRIC, BUF>(ix, src, Q, b, a.ht_slots, a.efC, wsize, lc);
        for (uint32_t i = lane; i < wsize; i += 64) b.s.W[i] &= ~1ull;
        wave_sync();
        const uint32_t r =
            a.extend && !a.simple
                ? select_extended<G, F, METRIC, BUF>(ix, src, Q, b, wsize, M, a.keep_pruned != 0, q, lc,
                                                     a.ext + static_cast<size_t>(blockIdx.x) * a.ecap)
                : select_w<G, F, METRIC, BUF>(ix, src, b, wsize, M, a.keep_pruned != 0, a.simple != 0);
        const uint32_t width = lc ? ix.Mmax : ix.Mmax0;
        uint32_t *row = row_of(ix, q, lc);
        if (lane < static_cast<int>(width)) row[lane] = lane < static_cast<int>(r) ? b.R[lane] : kNoLink;
        // the reverse links e <- q, in slots of their own
        const size_t slot0 = lc == 0 ? static_cast<size_t>(q - a.first) * M
                                     : static_cast<size_t>(a.end - a.first) * M +
                                           (static_cast<uint64_t>(ix.uoff[q]) + lc - 1 - a.upper_base) * M;
        if (lane < static_cast<int>(M)) {
            const bool has = lane < static_cast<int>(r);
            a.pair_key[slot0 + lane] = has ? (static_cast<uint64_t>(lc) << 32) | b.R[lane] : kNoPair;
            a.pair_val[slot0 + lane] = q;
        }
        wave_sync();
    }
    // layers above the current top (an element inserted alone): no links, no pairs
    for (int lc = l; lc > L && lc >= 1; --lc) {
        const size_t slot0 = static_cast<size_t>(a.end - a.first) * M +
                             (static_cast<uint64_t>(ix.uoff[q]) + lc - 1 - a.upper_base) * M;
        if (lane < static_cast<int>(M)) a.pair_key[slot0 + lane] = kNoPair;
    }
}

// Candidates' keys (distance to the base element) into W[off..off+cnt) from
// ids in b.s.ids[0..cnt); cnt <= 64.
template <int G, int F, int METRIC, bool BUF>
__device__ __forceinline__ void score_into_w(const DevIndex &ix, const RowSource &src, const QueryRegs<G, F, kF32> &QE,
                                             const BuildLds &b, int cnt, uint32_t off) {
    const int lane = lane_id();
    wave_sync();
    score_ids<G, F, METRIC, kF32, BUF>(ix, src, QE, b.s.ids, cnt, b.s.keys);
    wave_sync();
    if (lane < cnt) b.s.W[off + lane] = b.s.keys[lane];
    wave_sync();
}

// One element's list after the new links of a batch: appended when they fit,
// else selected again by the heuristic from the element over its links and the
// new ones (in chunks when more arrive than W holds).  With extendCandidates
// the new lists go to a.stage and build_commit_kernel writes them to the graph
// afterwards, so every extension reads the lists as they stood before the
// batch's links (no wave reads a list another wave is rewriting).
template <int G, int F, int METRIC, bool BUF>
__global__ __launch_bounds__(64) void build_link_kernel(DevIndex ix, LinkArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = lane_id();
    const BuildLds b = carve_build(smem, a.wpow2);
    const RowSource src = rows_of(ix, SearchArgs{}, kF32);
    const uint32_t runs = *a.n_runs;
    for (uint32_t run = blockIdx.x; run < runs; run += gridDim.x) {
        const uint64_t key = a.key[run];
        if (key == kNoPair) continue;
        const uint32_t e = static_cast<uint32_t>(key);
        const int lc = static_cast<int>(key >> 32);
        const uint32_t cnt = a.count[run], off = a.offset[run];
        const uint32_t cap = lc ? ix.Mmax : ix.Mmax0;
        const uint32_t *row = row_of(ix, e, lc);
        uint32_t *out = a.stage ? a.stage + static_cast<size_t>(run) * a.stage_w : row_of(ix, e, lc);
        const uint32_t cur = lane < static_cast<int>(cap) ? row[lane] : kNoLink;
        const uint64_t hm = __ballot(cur != kNoLink);
        uint32_t have = static_cast<uint32_t>(__popcll(hm));
        // the current list, compacted, in R
        if (cur != kNoLink) b.R[rank_in(hm)] = cur;
        wave_sync();
        if (have + cnt <= cap) {
            if (lane < static_cast<int>(cap))
                out[lane] = lane < static_cast<int>(have)         ? b.R[lane]
                            : lane < static_cast<int>(have + cnt) ? a.val[off + lane - have]
                                                                  : kNoLink;
            wave_sync();
            continue;
        }
        QueryRegs<G, F, kF32> QE;
        load_query<G, F, kF32>(vec_row(ix, e), ix.dim, QE);
        const uint32_t room = a.wpow2 - cap;  // new links taken per selection
        for (uint32_t done = 0; done < cnt;) {
            const uint32_t take = min(room, cnt - done);
            // candidates: the list (R) and the next `take` new links
            uint32_t m = 0;
            if (lane < static_cast<int>(have)) b.s.ids[lane] = b.R[lane];
            if (have) score_into_w<G, F, METRIC, BUF>(ix, src, QE, b, static_cast<int>(have), 0);
            m = have;
            for (uint32_t j = 0; j < take; j += 64) {
                const int c = static_cast<int>(min(64u, take - j));
                if (lane < c) b.s.ids[lane] = a.val[off + done + j + lane];
                score_into_w<G, F, METRIC, BUF>(ix, src, QE, b, c, m);
                m += static_cast<uint32_t>(c);
            }
            done += take;
            uint32_t p2 = 64;
            while (p2 < m) p2 <<= 1;
            sort_w(b.s.W, m, p2);
            have = a.extend && !a.simple
                       ? select_extended<G, F, METRIC, BUF>(ix, src, QE, b, m, cap, a.keep_pruned != 0, e, lc,
                                                            a.ext + static_cast<size_t>(blockIdx.x) * a.ecap)
                       : select_w<G, F, METRIC, BUF>(ix, src, b, m, cap, a.keep_pruned != 0, a.simple != 0);
        }
        if (lane < static_cast<int>(cap)) out[lane] = lane < static_cast<int>(have) ? b.R[lane] : kNoLink;
        wave_sync();
    }
}

// The staged lists of the runs (extendCandidates) into the graph.
__global__ __launch_bounds__(64) void build_commit_kernel(DevIndex ix, LinkArgs a) {
    const int lane = lane_id();
    const uint32_t runs = *a.n_runs;
    for (uint32_t run = blockIdx.x; run < runs; run += gridDim.x) {
        const uint64_t key = a.key[run];
        if (key == kNoPair) continue;
        const int lc = static_cast<int>(key >> 32);
        const uint32_t cap = lc ? ix.Mmax : ix.Mmax0;
        uint32_t *row = row_of(ix, static_cast<uint32_t>(key), lc);
        if (lane < static_cast<int>(cap)) row[lane] = a.stage[static_cast<size_t>(run) * a.stage_w + lane];
    }
}

// Explicit candidate lists (tests of the in-wave heuristic): base element
// base[i], candidates cand[i][0..nc) (kNoLink entries skipped), Mk kept into
// out[i][Mk] (kNoLink padded).  extend: extendCandidates on layer lc, with
// the extended list of base i in ext[i][ecap].
template <int G, int F, int METRIC, bool BUF>
__global__ __launch_bounds__(64) void select_kernel(DevIndex ix, const uint32_t *base, const uint32_t *cand,
                                                    uint32_t nb, uint32_t nc, uint32_t Mk, uint32_t wpow2,
                                                    int keep_pruned, int extend, int lc, uint64_t *ext, uint32_t ecap,
                                                    uint32_t *out) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t i = blockIdx.x;
    if (i >= nb) return;
    const int lane = lane_id();
    const BuildLds b = carve_build(smem, wpow2);
    const RowSource src = rows_of(ix, SearchArgs{}, kF32);
    QueryRegs<G, F, kF32> QE;
    load_query<G, F, kF32>(vec_row(ix, base[i]), ix.dim, QE);
    uint32_t m = 0;
    for (uint32_t j = 0; j < nc; j += 64) {
        const uint32_t v = j + lane < nc ? cand[static_cast<size_t>(i) * nc + j + lane] : kNoLink;
        const uint64_t vm = __ballot(v != kNoLink);
        const int c = __popcll(vm);
        if (v != kNoLink) b.s.ids[rank_in(vm)] = v;
        if (c) score_into_w<G, F, METRIC, BUF>(ix, src, QE, b, c, m);
        m += static_cast<uint32_t>(c);
    }
    sort_w(b.s.W, m, wpow2);
    const uint32_t r = extend ? select_extended<G, F, METRIC, BUF>(ix, src, QE, b, m, Mk, keep_pruned != 0, base[i], lc,
                                                                   ext + static_cast<size_t>(i) * ecap)
                              : select_heuristic_w<G, F, METRIC, BUF>(ix, src, b, m, Mk, keep_pruned != 0);
    for (uint32_t j = lane; j < Mk; j += 64) out[static_cast<size_t>(i) * Mk + j] = j < r ? b.R[j] : kNoLink;
}

template <int G, int F, int METRIC, bool BUF>
struct BuildKernels {
    static hipError_t insert(const DevIndex &ix, const BuildArgs &a, hipStream_t st) {
        const size_t lds = build_lds_bytes(a.wpow2, a.ht_slots);
        hipLaunchKernelGGL((build_insert_kernel<G, F, METRIC, BUF>), dim3(a.end - a.first), dim3(64), lds, st, ix, a);
        return hipGetLastError();
    }
    static hipError_t link(const DevIndex &ix, const LinkArgs &a, uint32_t grid, hipStream_t st) {
        const size_t lds = build_lds_bytes(a.wpow2, 0);
        hipLaunchKernelGGL((build_link_kernel<G, F, METRIC, BUF>), dim3(grid), dim3(64), lds, st, ix, a);
        if (a.stage) hipLaunchKernelGGL(build_commit_kernel, dim3(grid), dim3(64), 0, st, ix, a);
        return hipGetLastError();
    }
    static hipError_t select(const DevIndex &ix, const uint32_t *base, const uint32_t *cand, uint32_t nb, uint32_t nc,
                             uint32_t Mk, uint32_t wpow2, int keep_pruned, int extend, int lc, uint64_t *ext,
                             uint32_t ecap, uint32_t *out, hipStream_t st) {
        const size_t lds = build_lds_bytes(wpow2, 0);
        hipLaunchKernelGGL((select_kernel<G, F, METRIC, BUF>), dim3(nb), dim3(64), lds, st, ix, base, cand, nb, nc, Mk,
                           wpow2, keep_pruned, extend, lc, ext, ecap, out);
        return hipGetLastError();
    }
};

template <int G_, int F_>
struct GF {
    static constexpr int G = G_, F = F_;
};

// Calls fn with the kernel set of the index's tile shape, metric and addressing.
template <template <int, int, int, bool> class K, typename Fn>
hipError_t with_kernels(const DevIndex &ix, Fn &&fn) {
    const TileShape t = tile_for(kF32, ix.dim);
    const bool buf = stores_buffered(ix);
    auto pick_m = [&](auto gf) -> hipError_t {
        constexpr int G = decltype(gf)::G, F = decltype(gf)::F;
        if (ix.metric == HNSW_IP) {
            if (buf) return fn(K<G, F, HNSW_IP, true>{});
            return fn(K<G, F, HNSW_IP, false>{});
        }
        if (buf) return fn(K<G, F, HNSW_L2SQ, true>{});
        return fn(K<G, F, HNSW_L2SQ, false>{});
    };
    switch (t.G * 16 + t.F) {
        case 1 * 16 + 1: return pick_m(GF<1, 1>{});
        case 2 * 16 + 2: return pick_m(GF<2, 2>{});
        case 4 * 16 + 2: return pick_m(GF<4, 2>{});
        case 8 * 16 + 2: return pick_m(GF<8, 2>{});
        case 16 * 16 + 2: return pick_m(GF<16, 2>{});
        case 16 * 16 + 4: return pick_m(GF<16, 4>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace hnsw

// ------------------------------------------------------------ host driver

namespace {

using hnsw::kNoLink;

// The level draw of Alg. 1, l = floor(-ln(U) * mL), with U = (r + 1) * 2^-53 in
// (0, 1] and r the top 53 bits of splitmix64(seed XOR i) (Steele, Lea and
// Flood's SplitMix generator with Vigna's 64-bit finaliser constants).
uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

uint8_t level_of(uint64_t seed, uint32_t i, double mL) {
    const uint64_t r = splitmix64(seed ^ static_cast<uint64_t>(i)) >> 11;
    const double U = static_cast<double>(r + 1) * 0x1.0p-53;
    const double l = std::floor(-std::log(U) * mL);
    return static_cast<uint8_t>(l > 255.0 ? 255.0 : l);
}

uint32_t row_floats_of(uint32_t dim) {
    const uint32_t v4 = (dim + 3) / 4;
    if (v4 <= 1) return 4;
    return ((v4 + 3) / 4) * 16;
}

struct DevBuf {
    std::vector<void *> got;
    uint64_t bytes = 0;
    void *take(size_t sz) {
        void *p = nullptr;
        if (hipMalloc(&p, sz ? sz : 16) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        got.push_back(p);
        bytes += sz;
        return p;
    }
    void release() {
        for (void *p : got) hnsw::device_free(p);
        got.clear();
    }
};

}  // namespace

extern "C" {

hnsw_status hnsw_index_build(const float *vectors, uint32_t n, uint32_t dim, int metric,
                             const hnsw_build_params *pr, void *stream, hnsw_index **out) {
    using namespace hnsw;
    if (!out) return HNSW_ERR_INVALID_ARG;
    *out = nullptr;
    if (!vectors || !pr || n == 0 || n >= 0x7FFFFFFFu || dim == 0) return HNSW_ERR_INVALID_ARG;
    if (metric != HNSW_L2SQ && metric != HNSW_IP) return HNSW_ERR_INVALID_ARG;
    if (dim > HNSW_DIM_MAX || pr->Mmax > HNSW_DEG_MAX || pr->Mmax0 > HNSW_DEG_MAX) return HNSW_ERR_UNSUPPORTED;
    if (pr->M == 0 || pr->Mmax == 0 || pr->Mmax0 == 0 || pr->M > pr->Mmax0 || pr->M > pr->Mmax ||
        pr->efC == 0 || pr->efC > HNSW_EF_MAX || !(pr->mL >= 0.0) || pr->batch_div == 0)
        return HNSW_ERR_INVALID_ARG;
    if (!device_count_ok()) return HNSW_ERR_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t efC = pr->efC < pr->M ? pr->M : pr->efC;

    // levels and the rows of the upper layers (consecutive per element, in id order)
    std::vector<uint8_t> lv(n);
    std::vector<int32_t> uoff(n);
    std::vector<uint64_t> rows_before(static_cast<size_t>(n) + 1, 0);
    uint32_t top_level = 0;
    for (uint32_t i = 0; i < n; ++i) {
        lv[i] = level_of(pr->seed, i, pr->mL);
        if (lv[i] > top_level) top_level = lv[i];
        rows_before[i + 1] = rows_before[i] + lv[i];
    }
    if (rows_before[n] >= 0x7FFFFFFFull) return HNSW_ERR_UNSUPPORTED;
    for (uint32_t i = 0; i < n; ++i) uoff[i] = lv[i] ? static_cast<int32_t>(rows_before[i]) : -1;
    const uint64_t rows = rows_before[n];

    // batches: element 0 alone (the first enter point), then at most
    // 1/batch_div of the elements inserted so far (and batch_max); an element
    // above the current top layer is inserted alone
    uint32_t bmax_cfg = pr->batch_max ? pr->batch_max : 65536u;
    const uint32_t M = pr->M;
    // extendCandidates: a global list per wave of up to (candidates) x (list
    // width + 1) keys; batches and link grids are sized so that these lists
    // take at most kExtBytes, and the link phase re-selects at most 128
    // candidates at a time
    const bool extend = pr->extend_candidates != 0 && pr->select_simple == 0;
    constexpr size_t kExtBytes = size_t(512) << 20;
    const uint32_t wmax = pr->Mmax0 > pr->Mmax ? pr->Mmax0 : pr->Mmax;
    const uint32_t link_wpow2 = extend ? 128u : 512u;
    auto pow2_at_least = [](uint64_t v) {
        uint64_t p = 64;
        while (p < v) p <<= 1;
        return static_cast<uint32_t>(p);
    };
    const uint32_t ecap_i = extend ? pow2_at_least(static_cast<uint64_t>(efC) * (wmax + 1)) : 0u;
    const uint32_t ecap_l = extend ? pow2_at_least(static_cast<uint64_t>(link_wpow2) * (wmax + 1)) : 0u;
    uint32_t link_grid_max = 8192;
    if (extend) {
        const size_t bi = std::max<size_t>(1, kExtBytes / (static_cast<size_t>(ecap_i) * 8));
        if (bmax_cfg > bi) bmax_cfg = static_cast<uint32_t>(bi);
        link_grid_max = static_cast<uint32_t>(
            std::min<size_t>(8192, std::max<size_t>(1, kExtBytes / (static_cast<size_t>(ecap_l) * 8))));
    }

    const uint32_t rf = row_floats_of(dim);
    const size_t vec_bytes = (static_cast<size_t>(n) + 1) * rf * 4;
    DevBuf al;
    float *vec = static_cast<float *>(al.take(vec_bytes));
    uint32_t *adj0 = static_cast<uint32_t *>(al.take(static_cast<size_t>(n) * pr->Mmax0 * 4));
    int32_t *duoff = static_cast<int32_t *>(al.take(static_cast<size_t>(n) * 4));
    uint32_t *adjU = static_cast<uint32_t *>(al.take(static_cast<size_t>(rows) * pr->Mmax * 4));
    float *xnorm = static_cast<float *>(al.take(static_cast<size_t>(n) * 4));
    const uint64_t index_bytes = al.bytes;
    if (!vec || !adj0 || !duoff || !adjU || !xnorm) {
        al.release();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    // scratch of the build (freed at the end)
    uint32_t max_upper_rows = 0;  // upper rows of one batch, at most
    {
        // a batch spans at most bmax elements; bound its upper rows by a sliding maximum
        uint32_t lo = 0;
        for (uint32_t hi = 1; hi <= n; ++hi) {
            while (hi - lo > bmax_cfg) ++lo;
            const uint64_t r = rows_before[hi] - rows_before[lo];
            if (r > max_upper_rows) max_upper_rows = static_cast<uint32_t>(r);
        }
    }
    const size_t max_pairs = (static_cast<size_t>(bmax_cfg) + max_upper_rows) * M;
    DevBuf tmp;
    uint8_t *dlv = static_cast<uint8_t *>(tmp.take(n));
    uint64_t *pk = static_cast<uint64_t *>(tmp.take(max_pairs * 8));
    uint64_t *pk2 = static_cast<uint64_t *>(tmp.take(max_pairs * 8));
    uint32_t *pv = static_cast<uint32_t *>(tmp.take(max_pairs * 4));
    uint32_t *pv2 = static_cast<uint32_t *>(tmp.take(max_pairs * 4));
    uint64_t *ukey = static_cast<uint64_t *>(tmp.take(max_pairs * 8));
    uint32_t *ucnt = static_cast<uint32_t *>(tmp.take(max_pairs * 4));
    uint32_t *uofs = static_cast<uint32_t *>(tmp.take(max_pairs * 4));
    uint32_t *nruns = static_cast<uint32_t *>(tmp.take(16));
    uint64_t *ext = nullptr;
    uint32_t *stage = nullptr;
    if (extend) {
        const size_t keys = std::max(static_cast<size_t>(bmax_cfg) * ecap_i, static_cast<size_t>(link_grid_max) * ecap_l);
        ext = static_cast<uint64_t *>(tmp.take(keys * 8));
        stage = static_cast<uint32_t *>(tmp.take(max_pairs * wmax * 4));
    }
    size_t t1 = 0, t2 = 0, t3 = 0;
    bool ok = pk && pk2 && pv && pv2 && ukey && ucnt && uofs && nruns && dlv && (!extend || (ext && stage));
    ok = ok && hipcub::DeviceRadixSort::SortPairs(nullptr, t1, pk, pk2, pv, pv2, static_cast<int>(max_pairs), 0, 40,
                                                  st) == hipSuccess;
    ok = ok && hipcub::DeviceRunLengthEncode::Encode(nullptr, t2, pk2, ukey, ucnt, nruns, static_cast<int>(max_pairs),
                                                     st) == hipSuccess;
    ok = ok && hipcub::DeviceScan::ExclusiveSum(nullptr, t3, ucnt, uofs, static_cast<int>(max_pairs), st) == hipSuccess;
    const size_t tbytes = std::max(t1, std::max(t2, t3));
    void *temp = ok ? tmp.take(tbytes) : nullptr;
    if (!ok || !temp) {
        (void)hipGetLastError();
        tmp.release();
        al.release();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    ok = hipMemsetAsync(vec, 0, vec_bytes, st) == hipSuccess;
    ok = ok && upload_rows(vec, rf, vectors, dim, n, st);
    ok = ok && hipMemsetAsync(adj0, 0xFF, static_cast<size_t>(n) * pr->Mmax0 * 4, st) == hipSuccess;
    if (rows) ok = ok && hipMemsetAsync(adjU, 0xFF, static_cast<size_t>(rows) * pr->Mmax * 4, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(duoff, uoff.data(), static_cast<size_t>(n) * 4, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(dlv, lv.data(), n, hipMemcpyHostToDevice, st) == hipSuccess;

    DevIndex ix{};
    ix.vec = vec;
    ix.adj0 = adj0;
    ix.uoff = duoff;
    ix.adjU = adjU;
    ix.n = n;
    ix.dim = dim;
    ix.dv4 = (dim + 3) / 4;
    ix.stride4 = rf / 4;
    ix.Mmax = pr->Mmax;
    ix.Mmax0 = pr->Mmax0;
    ix.metric = static_cast<uint32_t>(metric);

    BuildArgs ba{};
    ba.levels = dlv;
    ba.M = M;
    ba.efC = efC;
    ba.wpow2 = 64;
    while (ba.wpow2 < efC) ba.wpow2 <<= 1;
    {
        uint32_t lg = 10;
        while (lg < 12 && (1u << lg) < 8u * efC) ++lg;
        ba.ht_slots = 1u << lg;
    }
    ba.keep_pruned = pr->keep_pruned;
    ba.simple = pr->select_simple;
    ba.extend = extend;
    ba.ext = ext;
    ba.ecap = ecap_i;
    ba.pair_key = pk;
    ba.pair_val = pv;
    LinkArgs la{};
    la.key = ukey;
    la.count = ucnt;
    la.offset = uofs;
    la.val = pv2;
    la.n_runs = nruns;
    la.wpow2 = link_wpow2;
    la.keep_pruned = pr->keep_pruned;
    la.simple = pr->select_simple;
    la.extend = extend;
    la.ext = ext;
    la.ecap = ecap_l;
    la.stage = stage;
    la.stage_w = wmax;

    uint32_t entry = 0, top = lv[0];
    uint32_t s = 1;
    while (ok && s < n) {
        uint32_t b = s / pr->batch_div;
        if (b < 1) b = 1;
        if (b > bmax_cfg) b = bmax_cfg;
        uint32_t e = s + b < n ? s + b : n;
        bool alone = false;
        for (uint32_t j = s; j < e; ++j)
            if (lv[j] > top) {
                if (j == s) {
                    e = s + 1;
                    alone = true;
                } else {
                    e = j;
                }
                break;
            }
        ba.first = s;
        ba.end = e;
        ba.entry = entry;
        ba.top = top;
        ba.upper_base = rows_before[s];
        const size_t npairs = (static_cast<size_t>(e - s) + (rows_before[e] - rows_before[s])) * M;
        ok = with_kernels<BuildKernels>(ix, [&](auto k) { return k.insert(ix, ba, st); }) == hipSuccess;
        ok = ok && hipcub::DeviceRadixSort::SortPairs(temp, t1, pk, pk2, pv, pv2, static_cast<int>(npairs), 0, 40,
                                                      st) == hipSuccess;
        ok = ok && hipcub::DeviceRunLengthEncode::Encode(temp, t2, pk2, ukey, ucnt, nruns, static_cast<int>(npairs),
                                                         st) == hipSuccess;
        ok = ok && hipcub::DeviceScan::ExclusiveSum(temp, t3, ucnt, uofs, static_cast<int>(npairs), st) == hipSuccess;
        const uint32_t grid = static_cast<uint32_t>(std::min<size_t>(npairs, link_grid_max));
        ok = ok && with_kernels<BuildKernels>(ix, [&](auto k) { return k.link(ix, la, grid, st); }) == hipSuccess;
        if (alone && lv[s] > top) {
            entry = s;
            top = lv[s];
        }
        s = e;
    }
    ix.entry = entry;
    ix.max_level = top;
    ix.cell_level = cell_level_of(lv.data(), n, top);
    ix.uid = next_index_uid();
    ok = ok && launch_row_norms(ix, xnorm, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    tmp.release();
    if (!ok) {
        (void)hipGetLastError();
        al.release();
        return HNSW_ERR_DEVICE;
    }
    hnsw_index *h = new hnsw_index();
    h->ix = ix;
    h->xnorm = xnorm;
    h->M = M;
    (void)hipGetDevice(&h->device);
    h->bytes = index_bytes;
    h->allocations = al.got;
    h->levels.assign(lv.begin(), lv.end());
    h->n_upper_rows = rows;
    *out = h;
    return HNSW_OK;
}

hnsw_status hnsw_select_heuristic(const hnsw_index *index, const uint32_t *base, const uint32_t *cand, uint32_t nb,
                                  uint32_t nc, uint32_t Mk, int keep_pruned, int extend, int lc, uint32_t *out,
                                  void *stream) {
    using namespace hnsw;
    if (!index || Mk == 0 || Mk > 64 || nc == 0 || nc > 1024) return HNSW_ERR_INVALID_ARG;
    if (nb == 0) return HNSW_OK;
    if (!is_device_ptr(base) || !is_device_ptr(cand) || !is_device_ptr(out)) return HNSW_ERR_INVALID_ARG;
    const DevIndex &ix = index->ix;
    if (lc < 0 || static_cast<uint32_t>(lc) > ix.max_level) return HNSW_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // ids are checked on the host: every one in range, and with extend every
    // candidate a member of layer lc (its list there is read)
    std::vector<uint32_t> hb(nb), hc(static_cast<size_t>(nb) * nc);
    if (hipMemcpyAsync(hb.data(), base, hb.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hc.data(), cand, hc.size() * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    for (uint32_t b : hb)
        if (b >= ix.n) return HNSW_ERR_INVALID_ARG;
    for (uint32_t c : hc) {
        if (c == kNoLink) continue;
        if (c >= ix.n) return HNSW_ERR_INVALID_ARG;
        if (extend && index->levels[c] < static_cast<uint32_t>(lc)) return HNSW_ERR_INVALID_ARG;
    }
    uint32_t wpow2 = 64;
    while (wpow2 < nc) wpow2 <<= 1;
    uint32_t ecap = 0;
    uint64_t *ext = nullptr;
    if (extend) {
        const uint32_t width = lc ? ix.Mmax : ix.Mmax0;
        ecap = 64;
        while (ecap < static_cast<uint64_t>(nc) * (width + 1)) ecap <<= 1;
        if (hipMalloc(&ext, static_cast<size_t>(nb) * ecap * 8) != hipSuccess) {
            (void)hipGetLastError();
            return HNSW_ERR_OUT_OF_MEMORY;
        }
    }
    const bool ok = with_kernels<BuildKernels>(ix, [&](auto k) {
                        return k.select(ix, base, cand, nb, nc, Mk, wpow2, keep_pruned, extend, lc, ext, ecap, out, st);
                    }) == hipSuccess &&
                    (!ext || hipStreamSynchronize(st) == hipSuccess);
    if (ext) device_free(ext);
    if (!ok) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

}  // extern "C"
