/*
 * hnsw_gpu.h -- C ABI of the MI355X (gfx950) Hierarchical NSW query path.
 *
 * The library answers the K-ANNS problem of Malkov & Yashunin,
 * arXiv:1603.09320, Sec. 1: given a distance, a stored set of n vectors and a
 * query q, return the K stored elements nearest to q.  The search is
 * K-NN-SEARCH (Alg. 5): a greedy descent with ef = 1 through layers L..1,
 * then SEARCH-LAYER (Alg. 2) on layer 0 with ef candidates, returning the K
 * nearest elements of the final list W.
 *
 * Conventions shared by every entry point
 *   - Status codes only; nothing is thrown across the ABI.  Arguments are
 *     validated on the host before anything is enqueued.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Search entry points only enqueue work on it and never synchronise.
 *   - "device" buffers must be device memory of the current HIP device
 *     (e.g. PyTorch tensors); host pointers are rejected with
 *     HNSW_ERR_INVALID_ARG.  The caller owns them and keeps them alive until
 *     the enqueued work has completed.
 *   - Ids are 32-bit.  Output rows are sorted ascending by (distance, id);
 *     rows with fewer than k reachable elements are padded with id -1 and
 *     distance +inf.
 *   - Distances: HNSW_L2SQ is the squared Euclidean distance, HNSW_IP is
 *     1 - <q, x> (cosine distance for unit vectors, Sec. 5.2).  Each distance
 *     is accumulated in double precision and rounded once to float; every
 *     ordering decision compares (float distance, id) keys.
 *   - An index is immutable after upload and may be searched concurrently
 *     from several streams.
 */
#ifndef HNSW_GPU_H
#define HNSW_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hnsw_index hnsw_index; /* opaque, device resident */

typedef enum {
    HNSW_OK = 0,
    HNSW_ERR_INVALID_ARG = 1,   /* null/host pointer, bad size, malformed graph     */
    HNSW_ERR_OUT_OF_MEMORY = 2, /* device allocation failed                          */
    HNSW_ERR_DEVICE = 3,        /* no device, launch or runtime failure              */
    HNSW_ERR_UNSUPPORTED = 4,   /* a size beyond the kernels' limits (dim, ef, deg)  */
    HNSW_ERR_FORMAT = 5,        /* inconsistent graph description                    */
    HNSW_ERR_BUSY = 6           /* serving: no free request slot, submit again later */
} hnsw_status;

typedef enum { HNSW_L2SQ = 0, HNSW_IP = 1 } hnsw_metric;

/* Limits of this build. */
#define HNSW_EF_MAX 1024u   /* largest ef (after ef := max(ef, k))               */
#define HNSW_DIM_MAX 256u   /* largest vector dimension                          */
#define HNSW_DEG_MAX 64u    /* largest Mmax and Mmax0                            */

/*
 * Host-side description of a multilayer graph (Sec. 3, Alg. 1), in the packed
 * form produced by graph construction:
 *   vectors    [n][dim] fp32, row major.
 *   levels     [n] u8: the level l of each element (Alg. 1), <= max_level.
 *   adj0       [n][Mmax0] u32: layer-0 neighbour lists, unused slots
 *              0xFFFFFFFF (4-byte links, Sec. 4.2.3).
 *   upper_off  [n] i32: row of the element's layer-1 list in adjU, -1 for
 *              level-0 elements; the rows of layers 1..level are consecutive.
 *   adjU       [n_upper_rows][Mmax] u32: lists of layers >= 1, padded.
 *   entry_point / max_level: the enter point and top layer L (Alg. 5).
 */
typedef struct {
    uint32_t n, dim;
    uint32_t metric; /* hnsw_metric */
    uint32_t M, Mmax, Mmax0;
    uint32_t max_level, entry_point;
    const float *vectors;
    const uint8_t *levels;
    const uint32_t *adj0;
    const int32_t *upper_off;
    const uint32_t *adjU;
    uint64_t n_upper_rows;
} hnsw_graph_desc;

/*
 * Copy a graph to the current device and return an index handle.
 * All arrays of `g` are host memory, read only during the call (which
 * synchronises `stream` before returning); the caller may free them after.
 * Every link is checked to lie in [0, n) (or be the 0xFFFFFFFF pad), every
 * upper_off row range to lie inside adjU, and the entry point to sit on the
 * top level; a violation returns HNSW_ERR_FORMAT and allocates nothing.
 * Device layout: vectors padded to rows of a multiple of 64 bytes (16 bytes
 * for dim <= 4), adj0/upper_off/adjU copied as given.
 */
hnsw_status hnsw_index_upload(const hnsw_graph_desc *g, void *stream, hnsw_index **out);

/* Release the index and its device memory (NULL is ignored).  The caller
 * must ensure no enqueued search still reads it. */
void hnsw_index_free(hnsw_index *index);

/* Read back index properties: out[0..7] = n, dim, metric, M, Mmax, Mmax0,
 * max_level, entry_point; out[8] = device bytes held; out[9] = rows of the
 * upper layers (n_upper_rows). */
hnsw_status hnsw_index_info(const hnsw_index *index, uint64_t out[10]);

/*
 * Copy the graph of an index back to the host in the packed form of
 * hnsw_graph_desc (host buffers, synchronous): levels [n], adj0 [n][Mmax0],
 * upper_off [n], adjU [n_upper_rows][Mmax] (may be NULL when there are none).
 * Sizes from hnsw_index_info.  For graphs built on the device, so that they
 * can be saved, inspected or searched elsewhere.
 */
hnsw_status hnsw_index_export(const hnsw_index *index, uint8_t *levels, uint32_t *adj0, int32_t *upper_off,
                              uint32_t *adjU);

/*
 * Graph construction on the device: INSERT (Alg. 1) of elements 0..n-1 in id
 * order, in batches that run with few synchronisation points (Sec. 4.1 notes
 * that construction parallelises; the batch schedule below makes the result
 * deterministic).  Every element of a batch searches the graph as it stood
 * before the batch: greedy descent (ef = 1) above its level l, then for each
 * layer lc = min(L, l)..0 SEARCH-LAYER (Alg. 2) with efC candidates entered
 * from all of the previous layer's W, and SELECT-NEIGHBORS-HEURISTIC (Alg. 4)
 * for M links.  The reverse links are then merged per receiving element: a
 * list over Mmax (Mmax0 on layer 0) is selected again by the heuristic from
 * its element over its links and all new ones.  Element 0 becomes the enter
 * point with no links; an element above the current top layer is inserted
 * alone and becomes the enter point.  With batch_div >= n every batch holds
 * one element and the graph is that of the sequential INSERT.
 * extend_candidates (Alg. 4 extendCandidates) adds to each selection's
 * candidates their neighbours on the layer (the base element excepted).  The
 * extensions of the merge step read the lists as they stood before the
 * batch's links, so with one element per batch a merge whose candidates
 * include another list changed by the same element may differ from the
 * sequential INSERT, which merges the receiving lists one after another.
 * Levels: l = floor(-ln(U) * mL), U = (r + 1) * 2^-53 with r the top 53 bits
 * of splitmix64(seed XOR i).
 *   vectors   host fp32 [n][dim] (copied; the caller may free it after).
 * The call synchronises `stream`; it allocates the index (as
 * hnsw_index_upload) and a temporary workspace of about
 * (batch_max + upper rows of a batch) * M * 48 bytes, freed before it returns;
 * extend_candidates adds up to 512 MiB for the extended lists (batches are cut
 * to fit) and (batch_max + upper rows of a batch) * M * max(Mmax, Mmax0) * 4
 * bytes for the merged lists.
 */
typedef struct {
    uint32_t M;          /* links of a new element on each layer (Alg. 1)        */
    uint32_t Mmax;       /* list cap on layers >= 1                               */
    uint32_t Mmax0;      /* list cap on layer 0                                   */
    uint32_t efC;        /* efConstruction (raised to M), <= HNSW_EF_MAX           */
    double mL;           /* level normalisation, e.g. 1 / ln(M)                    */
    uint64_t seed;       /* level draw                                             */
    int keep_pruned;     /* Alg. 4 keepPrunedConnections                           */
    uint32_t batch_div;  /* a batch holds at most (elements inserted) / batch_div  */
    uint32_t batch_max;  /* and at most this many elements (0: 65,536)             */
    int select_simple;   /* 1: SELECT-NEIGHBORS-SIMPLE (Alg. 3, the M nearest)      */
                         /* instead of the heuristic                               */
    int extend_candidates; /* Alg. 4 extendCandidates (ignored with select_simple) */
} hnsw_build_params;
hnsw_status hnsw_index_build(const float *vectors, uint32_t n, uint32_t dim, int metric,
                             const hnsw_build_params *params, void *stream, hnsw_index **out);

/*
 * The device's SELECT-NEIGHBORS-HEURISTIC (Alg. 4) on explicit candidate
 * lists, as graph construction runs it: for base element base[i] of the index
 * and candidates cand[i][0..nc) (element ids; 0xFFFFFFFF entries are
 * skipped), the distances to the base are computed, candidates are taken in
 * (distance, id) order and kept while their distance to the base is smaller
 * than their distance to every element kept before; keep_pruned fills up to
 * Mk with the discarded ones, nearest first.  extend (extendCandidates) first
 * adds every neighbour on layer lc of a candidate, except the base, to the
 * candidates (each element once).  out[i][Mk] receives the kept ids in that
 * order, 0xFFFFFFFF padded.  All pointers device memory; nc <= 1024,
 * Mk <= 64, 0 <= lc <= the index's top layer.  The ids are copied to the host
 * and checked (HNSW_ERR_INVALID_ARG for an id >= n, or, with extend, a
 * candidate whose level is below lc); the call synchronises `stream`.  With
 * extend it allocates nb * 8 * (a power of two >= nc * (list width + 1)) bytes
 * for the call.
 */
hnsw_status hnsw_select_heuristic(const hnsw_index *index, const uint32_t *base, const uint32_t *cand, uint32_t nb,
                                  uint32_t nc, uint32_t Mk, int keep_pruned, int extend, int lc, uint32_t *out,
                                  void *stream);

/*
 * Batched K-NN-SEARCH (Alg. 5), one query per wavefront.
 *   queries   device fp32 [n][dim] row major (the index's dim).
 *   n         number of queries; 0 is a successful no-op.
 *   k         neighbours per query, 1 <= k <= HNSW_EF_MAX.
 *   ef        size of the dynamic list W (Alg. 2); raised to k when smaller;
 *             above HNSW_EF_MAX returns HNSW_ERR_UNSUPPORTED.
 *   ids_out   device i32 [n][k];  dists_out  device fp32 [n][k].
 * A batch of more than 256 queries uses a device workspace of 24 bytes per
 * query (at least 1 MiB), one per (device, stream), allocated on first use,
 * grown to the largest batch seen on that stream and kept until the process
 * ends.  A batch larger than the waves the GPU holds at once can run as three
 * launches on `stream` (every descent, an ordering step, then layer 0 with the
 * queries whose descent ended farthest started first, and queries whose
 * descents passed through the same upper-layer node run together on one XCD);
 * results and counters are those of the one-launch form.  Which form is faster depends on the data
 * (per-query cost spread), so for each (index, mode, ef, batch-size octave)
 * the library times two calls of each form, reading events back without
 * blocking, and then keeps the faster; until then it uses the three launches.
 * Calls on one stream from several threads are serialised while their
 * launches are enqueued.  If the workspace cannot be allocated the batch runs
 * as one launch.
 */
hnsw_status hnsw_search_batch(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k, uint32_t ef,
                              int32_t *ids_out, float *dists_out, void *stream);

/* Search modes of hnsw_search_batch_ex. */
typedef enum {
    HNSW_MODE_PLAIN = 0, /* fp32 vectors, as hnsw_search_batch                       */
    HNSW_MODE_BF16 = 1,  /* traverse the BF16 copy, then exact fp32 rerank of W       */
    HNSW_MODE_FP8 = 2,   /* traverse the FP8-E4M3 copy (per-vector scale), then rerank */
    HNSW_MODE_LEARNED = 3, /* fp32 traversal with the learned early-termination net   */
    HNSW_MODE_U8 = 4       /* traverse the 8-bit integer copy, then rerank (none when exact) */
} hnsw_mode;

/*
 * hnsw_search_batch with a mode and optional per-query counters.
 *   mode       hnsw_mode; BF16/FP8 need hnsw_index_add_lowp first.  In
 *              those modes the descent and the layer-0 search score the
 *              low-precision copy (s * x in double, fp64 accumulation), and
 *              every element of the final W is then re-scored from the fp32
 *              vectors; the output is the K nearest by that exact distance.
 *   mlp        for HNSW_MODE_LEARNED: a network from hnsw_mlp_create (NULL
 *              otherwise); a NULL net in learned mode runs the plain search.
 *              Learned mode needs k <= 64.
 *   counters   NULL or device u32 [n][4]: distance evaluations (all layers),
 *              expansions (all layers), distance evaluations on layer 0,
 *              expansions on layer 0.
 */
hnsw_status hnsw_search_batch_ex(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k, uint32_t ef,
                                 int mode, const void *mlp, int32_t *ids_out, float *dists_out, uint32_t *counters,
                                 void *stream);

/*
 * hnsw_search_batch_ex for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels, results and counters, but the scheduled form's workspace (24 bytes
 * per query) is a static device array of the library, sized for
 * HNSW_NOALLOC_MAX_QUERIES queries (6 MiB), which every device the library
 * runs on holds until the process ends; no device or host memory is
 * allocated and no timing event is created (the form is the one
 * hnsw_search_batch_ex has already measured for this index, mode, ef and
 * batch size, else the scheduled one).
 *   n > HNSW_NOALLOC_MAX_QUERIES -> HNSW_ERR_UNSUPPORTED (nothing enqueued).
 * All calls on one device share that array: calls that overlap on a device
 * (other streams, other threads) race and must be serialised by the caller;
 * calls on one stream are ordered by the stream.  Its contents are fully
 * rewritten by each call before being read, so nothing needs clearing.
 */
#define HNSW_NOALLOC_MAX_QUERIES 262144u
hnsw_status hnsw_search_batch_noalloc(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                      uint32_t ef, int mode, const void *mlp, int32_t *ids_out, float *dists_out,
                                      uint32_t *counters, void *stream);

/*
 * Exact K-NN by brute force over the index's vectors (the problem statement
 * of Sec. 1; the "BF time" column of Table 1), the ground truth for recall.
 * A fp32 matrix-core contraction ranks every stored vector by
 * ||x||^2 - 2<q,x> (L2) or -<q,x> (IP) and keeps the best
 * max(64, 2k)-ish candidates per query; those are re-scored exactly in fp64.
 *   queries    device fp32 [n][dim].
 *   k          1 <= k <= HNSW_BF_K_MAX.
 *   ids_out    device i32 [n][k]; dists_out device f64 [n][k]: exact distances,
 *              rows sorted by (distance, id), padded with (-1, +inf) when k > index n.
 * Allocates stream-ordered scratch of n * chunks * candidates * 8 bytes on
 * `stream` and frees it in stream order.
 */
#define HNSW_BF_K_MAX 128u
hnsw_status hnsw_bruteforce_knn(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                int32_t *ids_out, double *dists_out, void *stream);

/*
 * Measurement aid, not part of the search path: streams `bytes` of device
 * memory at `buf` with 16-byte loads, `blocks` workgroups of 256 threads in a
 * grid-stride loop, and writes the XOR of every 32-bit word each block read to
 * out[block] (device, `blocks` words), so that no load is dropped.  Its time
 * gives the attainable read bandwidth against which the search's algorithmic
 * bytes are also reported.  buf 16-byte aligned, bytes a multiple of 16,
 * 1 <= blocks <= 65,536.  Asynchronous on `stream`.
 */
hnsw_status hnsw_read_probe(const void *buf, uint64_t bytes, uint32_t *out, uint32_t blocks, void *stream);

/*
 * Add a low-precision copy of the vector store for HNSW_MODE_BF16 /
 * HNSW_MODE_FP8 / HNSW_MODE_U8 searches (quantised on the device from the
 * fp32 rows; the call synchronises `stream`).  BF16: round to nearest even.
 * FP8: OCP E4M3 with a per-vector fp32 scale s = max_j |x_j| / 448 (1 for an
 * all-zero row); code = nearest E4M3 value of x_j / s, ties to even,
 * saturating at 448.  U8 (integer-valued data such as SIFT, whose paper
 * build used integer distances, Sec. 5.4): code = x_j rounded to the nearest
 * integer, ties to even, clamped to [0, 255]; when every code equals its
 * coordinate the copy is exact and U8 searches skip the re-rank (their
 * distances are already the fp32 ones).  A second call for a kind already
 * present is a no-op.
 */
hnsw_status hnsw_index_add_lowp(hnsw_index *index, int kind, void *stream);

/*
 * Layout and contents of a low-precision copy: layout[0] = bytes per row,
 * layout[1] = 16-byte pieces holding values, layout[2] = for FP8 the byte
 * offset in host_out of the row scales (n * layout[0]); 0 for BF16; for U8,
 * 1 when the copy is exact, else 0.  host_out (optional) receives the n rows,
 * [n][layout[0]] bytes, and for FP8 then the n fp32 row scales (synchronous
 * copy).
 */
hnsw_status hnsw_index_read_lowp(const hnsw_index *index, int kind, void *host_out, uint64_t layout[3]);

/*
 * The learned stop rule (an addition to the paper's search; its own stop
 * test, Alg. 2, remains in force).  A 24-64-64-2 perceptron scores a feature
 * vector of the layer-0 search state every `period` expansions (at most
 * `max_ckpt` times per query): output 0 > tau ends the search; output 1, at
 * the first checkpoint, halves ef j = clamp(floor(0.5 - out1), 0, jmax)
 * times.  Inference uses BF16 weights and activations with float
 * accumulation in a fixed order, so results are reproducible bit for bit.
 *
 * Parameter layout (fp32, HNSW_MLP_PARAMS values): W1[64][24], b1[64],
 * W2[64][64], b2[64], W3[2][64], b3[2].
 */
#define HNSW_MLP_PARAMS 5890u
typedef struct hnsw_mlp hnsw_mlp;

/* Build an inference net from host fp32 parameters (weights rounded to BF16,
 * nearest even).  NaN/huge parameters or period == 0 -> HNSW_ERR_INVALID_ARG. */
hnsw_status hnsw_mlp_create(const float *params, float tau, int jmax, uint32_t period, uint32_t max_ckpt,
                            hnsw_mlp **out);
void hnsw_mlp_free(hnsw_mlp *mlp);

/*
 * hnsw_search_batch_ex in HNSW_MODE_LEARNED that also records, for each
 * query and checkpoint, the 24 features and the two network outputs:
 * trace_out is device fp32 [n][max_ckpt][26] (rows of checkpoints not
 * reached are left untouched).  For inspecting and testing the stop rule.
 */
hnsw_status hnsw_search_learned_trace(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                      uint32_t ef, const hnsw_mlp *mlp, int32_t *ids_out, float *dists_out,
                                      uint32_t *counters, float *trace_out, void *stream);

/* FP32 training kernels (all pointers device memory, enqueued on `stream`):
 *   forward: out[n][2] = perceptron(x[n][24]) with parameters `params`.
 *   grad:    gradient (HNSW_MLP_PARAMS values) and mean loss of
 *            L = (1/n) sum_s [ c_s * BCE(z0_s, y0_s) + lambda * m_s * (z1_s - y1_s)^2 ]
 *            for labels y[n][4] = (y0, c, y1, m); stream-ordered scratch of
 *            about n/64 * HNSW_MLP_PARAMS floats.
 *   adam:    one Adam step (bias-corrected, step >= 1) on params with moments m, v. */
hnsw_status hnsw_mlp_forward(const float *params, const float *x, uint32_t n, float *out, void *stream);
hnsw_status hnsw_mlp_grad(const float *params, const float *x, const float *y, uint32_t n, float lambda, float *grad,
                          float *loss, void *stream);
hnsw_status hnsw_mlp_adam(float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                          float eps, uint32_t step, void *stream);

/*
 * Continuous-batching server over one index: a persistent kernel whose waves
 * take requests in submission order, each with its own k, ef and mode, while
 * new requests keep arriving; a wave that finishes one request takes the next
 * without waiting for the others (requests overlap on the device).
 *   slots     ring size = most requests in flight (their outputs live in
 *             pinned host memory: the output budget).
 *   waves     persistent wavefronts (each reserves LDS for ef_max).
 *   ef_max    largest ef (after ef := max(ef, k)) a request may use;
 *   k_max     largest k; larger requests are refused (HNSW_ERR_UNSUPPORTED).
 *   mlp       net for HNSW_MODE_LEARNED requests (NULL: those run plain).
 *             Modes served: PLAIN, LEARNED, and BF16 / FP8 when the index
 *             held that copy (hnsw_index_add_lowp) when the server started
 *             (else HNSW_ERR_INVALID_ARG at submission).  Each kind is a
 *             search inlined into the serving kernel, which sets how many of
 *             its waves a SIMD holds: four with plain and learned only, two
 *             with BF16, one with FP8 (256 registers).
 *   budget_s  wall-clock seconds after which every wave exits even without a
 *             stop (a bound on the kernel's lifetime).
 * The server runs on a stream of its own.  Results are bit-identical to
 * hnsw_search_batch_ex with the same (query, k, ef, mode).  An index whose
 * fp32 or low-precision vector store exceeds 2 GiB is refused
 * (HNSW_ERR_UNSUPPORTED): the serving kernel gathers with 32-bit offsets.
 * While a server runs, device and pinned-host frees requested through this
 * library (index, net, other servers) are held until the last server stops:
 * hipFree would wait for the resident server kernel.
 */
typedef struct hnsw_server hnsw_server;
hnsw_status hnsw_server_start(const hnsw_index *index, const hnsw_mlp *mlp, uint32_t slots, uint32_t waves,
                              uint32_t ef_max, uint32_t k_max, double budget_s, hnsw_server **out);
/* Admit one request (host query [dim]); HNSW_ERR_BUSY while its slot is still
 * occupied (backpressure).  *ticket identifies it for hnsw_server_poll. */
hnsw_status hnsw_server_submit(hnsw_server *srv, const float *query, uint32_t k, uint32_t ef, int mode,
                               uint64_t *ticket);
/* Non-blocking: *done = 1 and the k results copied (host buffers) once the
 * request has completed; its slot is then free again. */
hnsw_status hnsw_server_poll(hnsw_server *srv, uint64_t ticket, int32_t *ids, float *dists, int *done);
/* Stop the kernel (waits for every wave to exit) and release the server. */
hnsw_status hnsw_server_stop(hnsw_server *srv);

/*
 * Open-loop replay of a request schedule against one or more servers (a
 * native driver for serving measurements): request i arrives at
 * arrival_s[i] seconds (non-decreasing) and goes to servers[server_of[i]]
 * with query row qidx[i] of queries[server_of[i]] ([nq][dim] host), k[i],
 * ef[i], mode[i].  It is submitted as soon as it has arrived and its slot is
 * free, and polled until done.  Outputs (host): ids/dists [n][out_stride]
 * (both NULL to discard results), t_submit/t_done seconds since the start.  HNSW_ERR_DEVICE if not every
 * request completed within timeout_s.
 */
hnsw_status hnsw_serve_replay(hnsw_server *const *servers, uint32_t n_servers, const float *const *queries,
                              uint64_t n, const double *arrival_s, const uint32_t *server_of, const uint32_t *qidx,
                              const uint32_t *k, const uint32_t *ef, const int32_t *mode, uint32_t out_stride,
                              int32_t *ids, float *dists, double *t_submit, double *t_done, double timeout_s);

/* Human-readable name of a status code (static storage). */
const char *hnsw_status_str(hnsw_status s);

#ifdef __cplusplus
}
#endif

#endif /* HNSW_GPU_H */
