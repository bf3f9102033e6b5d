// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/hnsw_gpu.h"

namespace hnsw {

constexpr uint32_t kNoLink = 0xFFFFFFFFu;

// Device-resident index as the kernels see it.
struct DevIndex {
    const float *vec;      // [n + 1][stride4 * 4] fp32, rows zero padded; row n is all zero
    const uint32_t *adj0;  // [n][Mmax0] layer-0 lists, kNoLink padded
    const int32_t *uoff;   // [n] row of layer 1 in adjU, -1 for level 0
    const uint32_t *adjU;  // [rows][Mmax] lists of layers >= 1
    const uint16_t *vbf16; // [n + 1][bf16_stride16 * 8] BF16 copy or null; row n all zero
    const uint8_t *vfp8;   // [n + 1][fp8_stride16 * 16] FP8-E4M3 copy or null; row n all zero
    const uint8_t *vu8;    // [n + 1][u8_stride16 * 16] 8-bit integer copy or null; row n all zero
    uint32_t bf16_stride16;  // 16-byte pieces per BF16 row
    uint32_t fp8_stride16;   // 16-byte pieces per FP8 row (values, scale, padding)
    uint32_t fp8_pieces;     // pieces of an FP8 row that hold values
    const uint8_t *fp8_scale;   // fp32 scale of FP8 row i at fp8_scale + i * fp8_scale_stride (row n: 0)
    uint32_t fp8_scale_stride;  // row bytes (scale in the row's padding) or 4 (an array after the rows)
    uint32_t u8_stride16;    // 16-byte pieces per 8-bit row (values, padding)
    uint32_t u8_pieces;      // pieces of an 8-bit row that hold values
    uint32_t u8_exact;       // every coordinate is an integer in [0, 255]: the copy equals the fp32 store
    uint32_t n, dim, dv4, stride4;
    uint32_t Mmax, Mmax0, entry, max_level, metric;
    uint32_t cell_level;  // layer whose greedy result groups a batch's queries on the XCDs (cell_level_of)
    uint32_t uid;  // identifies the index among those uploaded by this process (host bookkeeping only)
};

// The learned stop rule's network as the search kernel reads it: BF16
// weights (W1[64][24], W2[64][64], W3[2][64]) and fp32 biases.
constexpr int kMlpIn = 24, kMlpHid = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpOut * kMlpHid + kMlpOut;
struct DevMlp {
    const uint16_t *w1, *w2, *w3;
    const float *b1, *b2, *b3;
    float tau;        // stop when output 0 exceeds tau
    int jmax;         // most halvings of ef at the first checkpoint
    uint32_t period;  // layer-0 expansions between checkpoints
    uint32_t max_ckpt;
};

// One batched search launch.
struct SearchArgs {
    const float *queries;  // [nq][dim]
    uint32_t nq, k, ef;    // ef already raised to k
    int32_t *ids;          // [nq][k]
    float *dists;          // [nq][k]
    uint32_t *counters;    // [nq][4] or null
    uint32_t wcap;         // capacity of W in LDS, multiple of 64, >= ef
    uint32_t wslots;       // LDS slots reserved for W: wcap, or the power of two >= wcap for the stores that sort W
    uint32_t ht_slots;     // visited-table slots, >= 256 (probe steps reach 128 slots and wrap once)
    int mode;              // hnsw_mode
    bool replace;          // low-precision stores: a full visited table replaces an old id (as fp32 always does)
    DevMlp mlp;            // learned stop rule (mode HNSW_MODE_LEARNED)
    float *ckpt_trace;     // learned mode: [nq][max_ckpt][26] features + outputs per checkpoint, or null
    // Scheduled launches (descents first, then layer 0 in a chosen order, see
    // search_kernels.h): workspace of the batch, or null for the one-kernel path.
    uint64_t *sched_start;   // [nq] key of each query's layer-0 entry
    uint32_t *sched_up;      // [nq][2] distance evaluations and expansions above layer 0
    uint32_t *sched_order;   // [nq] query of each layer-0 wave
    uint32_t *sched_cell;    // [nq] node each query's descent reached on layer ix.cell_level
    int sched;               // 0: one kernel; 1: scheduled when the batch exceeds the resident waves; 2: always
    bool no_alloc;           // the caller cannot allocate: workspace from the static scratch array, no timing events
};

// Vector tile shape for a dimension: G lanes share one vector, each lane
// holding F float4 pieces of it (G * F * 4 >= dim).
struct TileShape {
    int G, F;
};
TileShape tile_for(int kind, uint32_t dim);

// Perceptron training kernels.
hipError_t launch_mlp_forward(const float *P, const float *X, uint32_t n, float *out, hipStream_t stream);
uint32_t mlp_grad_waves(uint32_t n);
hipError_t launch_mlp_grad(const float *P, const float *X, const float *Y, uint32_t n, float lambda, float *grad,
                           float *loss, float *scratch, hipStream_t stream);
hipError_t launch_adam(float *P, const float *G, float *M, float *V, uint32_t np, float lr, float b1, float b2,
                       float eps, uint32_t step, hipStream_t stream);

// Quantisation of the fp32 store into the low-precision copies.
hipError_t launch_quantize_bf16(const DevIndex &ix, uint16_t *out, hipStream_t stream);
hipError_t launch_quantize_fp8(const DevIndex &ix, uint8_t *out, uint8_t *scale, hipStream_t stream);
// 8-bit integer copy: code = x rounded to the nearest integer (ties to even),
// clamped to [0, 255]; *inexact (device) is set when some code differs from x.
hipError_t launch_quantize_u8(const DevIndex &ix, uint8_t *out, uint32_t *inexact, hipStream_t stream);

// LDS per wave of a search kernel; `learned` adds the stop rule's buffers.
size_t search_lds_bytes(const SearchArgs &a, bool learned);
// Form of a batch larger than the resident waves (true: the scheduled
// launches).  Per (index, mode, ef, batch-size octave), after one untimed
// call of each form, it times two calls of each (alternating) with events
// read back without blocking, then keeps the faster;
// until then it answers true.  *ev_start / *ev_end, when set, are to be
// recorded on the stream around the batch's launches.  With a.no_alloc it
// only reads a decision already made (creating no record and no event) and
// otherwise answers true.  Called with the workspace mutex held.
bool tuned_form(const DevIndex &ix, const SearchArgs &a, hipStream_t stream, hipEvent_t *ev_start,
                hipEvent_t *ev_end);
// Drops the timing records of an index that is being freed.
void forget_index(uint32_t uid);
// Next index identifier (never 0).
uint32_t next_index_uid();
// The highest layer >= 1 that holds at least kCellMin nodes (1 if none does,
// 0 for a single-layer graph): its nodes split the space into cells that are
// few enough to group a batch's queries and many enough to spread over the XCDs.
constexpr uint32_t kCellMin = 256;
uint32_t cell_level_of(const uint8_t *levels, uint32_t n, uint32_t max_level);

// Visited-table slots for a batch search: what the kernel's LDS share at its
// target occupancy leaves, at least 1024 (the learned kernels 64 fewer).
uint32_t visited_slots(const SearchArgs &a, bool learned);

// Brute-force K-NN (MFMA scan + fp64 rerank).
hipError_t launch_row_norms(const DevIndex &ix, float *out, hipStream_t stream);
uint32_t bf_candidates(uint32_t k);
void bf_plan(const DevIndex &ix, uint32_t nq, uint32_t k, uint32_t *nchunks, uint32_t *chunk);
hipError_t launch_bruteforce(const DevIndex &ix, const float *Q, uint32_t nq, uint32_t k, const float *xnorm,
                             uint64_t *partial, uint32_t nchunks, uint32_t chunk, int32_t *ids, double *d,
                             hipStream_t stream);
hipError_t launch_search(const DevIndex &ix, const SearchArgs &a, hipStream_t stream);
// The same for indices with a vector store above 2 GiB (64-bit addressed gathers).
hipError_t launch_search_wide(const DevIndex &ix, const SearchArgs &a, hipStream_t stream);
// True when every vector store of the index fits the buffered gathers.
bool stores_buffered(const DevIndex &ix);

}  // namespace hnsw

// Opaque handles of the C ABI.
struct hnsw_mlp {
    hnsw::DevMlp net;
    void *mem;
};

struct hnsw_index {
    hnsw::DevIndex ix;
    float *xnorm;  // [n] squared norms of the vectors (brute-force ranking)
    uint32_t M;
    int device;
    uint64_t bytes;
    std::vector<void *> allocations;
    std::vector<uint8_t> levels;  // [n] host copy of the element levels
    uint64_t n_upper_rows;        // rows of adjU
};

namespace hnsw {
// Copies n host rows of dim floats into device rows of rf floats (rf >= dim;
// the padding must already be zero): one copy when the rows are not padded,
// else through pinned staging buffers of packed rows.  A strided copy from
// pageable memory moves one row per transfer and took 9 s for 1M x 96.
bool upload_rows(float *dst, uint32_t rf, const float *src, uint32_t dim, uint32_t n, hipStream_t st);
bool device_count_ok();
bool is_device_ptr(const void *p);
uint64_t mem_cap();

// Frees while persistent server kernels are resident.  hipFree and
// hipHostFree wait for the whole device to go idle, which a resident server
// kernel does only once it is stopped: a free issued then (for example by a
// garbage-collected index) would block its thread until the server's budget
// ran out.  Frees requested while any server runs are therefore held and
// released when the last server has stopped.
void device_free(void *p);
void host_free(void *p);
void server_started();
void server_stopped();
}  // namespace hnsw
