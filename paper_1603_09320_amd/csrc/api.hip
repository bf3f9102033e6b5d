// Host runtime of the C ABI declared in include/hnsw_gpu.h.
//
// Everything here is argument checking, device memory management and kernel
// launches; all arithmetic of the search runs in the kernels.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"


namespace hnsw {

namespace {
std::mutex g_free_mu;
int g_servers = 0;                            // resident server kernels
std::vector<std::pair<void *, bool>> g_held;  // (pointer, host memory) held while servers run
}  // namespace

void device_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_free_mu);
    if (g_servers > 0) {
        g_held.emplace_back(p, false);
        return;
    }
    (void)hipFree(p);
}

void host_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_free_mu);
    if (g_servers > 0) {
        g_held.emplace_back(p, true);
        return;
    }
    (void)hipHostFree(p);
}

void server_started() {
    std::lock_guard<std::mutex> lock(g_free_mu);
    ++g_servers;
}

void server_stopped() {
    std::vector<std::pair<void *, bool>> release;
    {
        std::lock_guard<std::mutex> lock(g_free_mu);
        if (--g_servers == 0) release.swap(g_held);
    }
    for (const auto &h : release) {
        if (h.second) (void)hipHostFree(h.first);
        else (void)hipFree(h.first);
    }
}

bool upload_rows(float *dst, uint32_t rf, const float *src, uint32_t dim, uint32_t n, hipStream_t st) {
    if (rf == dim) {
        if (hipMemcpyAsync(dst, src, static_cast<size_t>(n) * dim * 4, hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return true;
    }
    // two pinned staging buffers of packed rows, alternated so that packing
    // the next chunk overlaps the copy of the previous one
    const size_t chunk_rows = std::max<size_t>(1, (size_t{16} << 20) / (static_cast<size_t>(rf) * 4));
    float *stage[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b) {
        void *p = nullptr;
        ok = hipHostMalloc(&p, chunk_rows * rf * 4, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&done[b], hipEventDisableTiming) == hipSuccess;
        stage[b] = static_cast<float *>(p);
    }
    for (size_t r0 = 0, k = 0; ok && r0 < n; r0 += chunk_rows, ++k) {
        const int b = static_cast<int>(k & 1);
        if (k >= 2) ok = hipEventSynchronize(done[b]) == hipSuccess;  // the buffer's last copy has finished
        const size_t cnt = std::min<size_t>(chunk_rows, n - r0);
        for (size_t i = 0; i < cnt && ok; ++i) {
            float *d = stage[b] + i * rf;
            memcpy(d, src + (r0 + i) * dim, static_cast<size_t>(dim) * 4);
            memset(d + dim, 0, static_cast<size_t>(rf - dim) * 4);
        }
        ok = ok && hipMemcpyAsync(dst + r0 * rf, stage[b], cnt * rf * 4, hipMemcpyHostToDevice, st) == hipSuccess;
        ok = ok && hipEventRecord(done[b], st) == hipSuccess;
    }
    if (hipStreamSynchronize(st) != hipSuccess) ok = false;
    for (int b = 0; b < 2; ++b) {
        if (done[b]) (void)hipEventDestroy(done[b]);
        if (stage[b]) host_free(stage[b]);
    }
    if (!ok) (void)hipGetLastError();
    return ok;
}

bool device_count_ok() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return n > 0;
}

// True for memory the current device can address as device memory.
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged || at.isManaged;
}

// Optional cap on the bytes an upload may allocate (HNSW_DEVICE_MEM_CAP),
// used to exercise the out-of-memory path from the host.
uint64_t mem_cap() {
    const char *s = getenv("HNSW_DEVICE_MEM_CAP");
    if (!s || !*s) return UINT64_MAX;
    return strtoull(s, nullptr, 10);
}

}  // namespace hnsw

namespace {

using hnsw::device_count_ok;
using hnsw::is_device_ptr;
using hnsw::kNoLink;
using hnsw::mem_cap;

uint32_t row_floats(uint32_t dim) {
    const uint32_t v4 = (dim + 3) / 4;
    if (v4 <= 1) return 4;
    return ((v4 + 3) / 4) * 16;  // rows of a multiple of 64 bytes
}

// Structural checks of a graph description; nothing is touched on the device.
hnsw_status validate_graph(const hnsw_graph_desc *g) {
    if (!g || !g->vectors || !g->levels || !g->adj0 || !g->upper_off) return HNSW_ERR_INVALID_ARG;
    if (g->n == 0 || g->n >= 0x7FFFFFFFu || g->dim == 0) return HNSW_ERR_INVALID_ARG;
    if (g->metric != HNSW_L2SQ && g->metric != HNSW_IP) return HNSW_ERR_INVALID_ARG;
    if (g->dim > HNSW_DIM_MAX || g->Mmax0 > HNSW_DEG_MAX || g->Mmax > HNSW_DEG_MAX) return HNSW_ERR_UNSUPPORTED;
    if (g->Mmax0 == 0 || (g->max_level > 0 && g->Mmax == 0)) return HNSW_ERR_FORMAT;
    if (g->max_level > 255 || g->entry_point >= g->n) return HNSW_ERR_FORMAT;
    if (g->levels[g->entry_point] != g->max_level) return HNSW_ERR_FORMAT;
    if (g->n_upper_rows > 0 && !g->adjU) return HNSW_ERR_INVALID_ARG;
    const uint64_t n = g->n;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t l = g->levels[i];
        if (l > g->max_level) return HNSW_ERR_FORMAT;
        const uint32_t *r0 = g->adj0 + i * g->Mmax0;
        for (uint32_t k = 0; k < g->Mmax0; ++k)
            if (r0[k] != kNoLink && r0[k] >= g->n) return HNSW_ERR_FORMAT;
        const int32_t off = g->upper_off[i];
        if (l == 0) {
            if (off != -1) return HNSW_ERR_FORMAT;
            continue;
        }
        if (off < 0 || static_cast<uint64_t>(off) + l > g->n_upper_rows) return HNSW_ERR_FORMAT;
        for (uint32_t lc = 1; lc <= l; ++lc) {
            const uint32_t *ru = g->adjU + (static_cast<uint64_t>(off) + lc - 1) * g->Mmax;
            for (uint32_t k = 0; k < g->Mmax; ++k) {
                const uint32_t e = ru[k];
                if (e == kNoLink) continue;
                // a link on layer lc must point to a member of layer lc
                if (e >= g->n || g->levels[e] < lc) return HNSW_ERR_FORMAT;
            }
        }
    }
    return HNSW_OK;
}

struct Allocator {
    std::vector<void *> got;
    uint64_t bytes = 0;
    uint64_t cap = mem_cap();
    void *take(size_t sz) {
        if (bytes + sz > cap) return nullptr;
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

const char *hnsw_status_str(hnsw_status s) {
    switch (s) {
        case HNSW_OK: return "ok";
        case HNSW_ERR_INVALID_ARG: return "invalid argument";
        case HNSW_ERR_OUT_OF_MEMORY: return "out of device memory";
        case HNSW_ERR_DEVICE: return "device error";
        case HNSW_ERR_UNSUPPORTED: return "unsupported size";
        case HNSW_ERR_FORMAT: return "malformed graph";
        case HNSW_ERR_BUSY: return "busy";
    }
    return "unknown status";
}

hnsw_status hnsw_index_upload(const hnsw_graph_desc *g, void *stream, hnsw_index **out) {
    if (!out) return HNSW_ERR_INVALID_ARG;
    *out = nullptr;
    const hnsw_status v = validate_graph(g);
    if (v != HNSW_OK) return v;
    if (!device_count_ok()) return HNSW_ERR_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);

    const uint32_t rf = row_floats(g->dim);
    const size_t vec_bytes = (static_cast<size_t>(g->n) + 1) * rf * 4;  // + one zero row
    const size_t adj0_bytes = static_cast<size_t>(g->n) * g->Mmax0 * 4;
    const size_t uoff_bytes = static_cast<size_t>(g->n) * 4;
    const size_t adjU_bytes = static_cast<size_t>(g->n_upper_rows) * g->Mmax * 4;

    Allocator al;
    float *vec = static_cast<float *>(al.take(vec_bytes));
    uint32_t *adj0 = static_cast<uint32_t *>(al.take(adj0_bytes));
    int32_t *uoff = static_cast<int32_t *>(al.take(uoff_bytes));
    uint32_t *adjU = static_cast<uint32_t *>(al.take(adjU_bytes));
    float *xnorm = static_cast<float *>(al.take(static_cast<size_t>(g->n) * 4));
    if (!vec || !adj0 || !uoff || !adjU || !xnorm) {
        al.release();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    bool ok = hipMemsetAsync(vec, 0, vec_bytes, st) == hipSuccess;
    ok = ok && hnsw::upload_rows(vec, rf, g->vectors, g->dim, g->n, st);
    ok = ok && hipMemcpyAsync(adj0, g->adj0, adj0_bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(uoff, g->upper_off, uoff_bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    if (adjU_bytes)
        ok = ok && hipMemcpyAsync(adjU, g->adjU, adjU_bytes, hipMemcpyHostToDevice, st) == hipSuccess;
    hnsw::DevIndex ix{};
    ix.vec = vec;
    ix.adj0 = adj0;
    ix.uoff = uoff;
    ix.adjU = adjU;
    ix.n = g->n;
    ix.dim = g->dim;
    ix.dv4 = (g->dim + 3) / 4;
    ix.stride4 = rf / 4;
    ix.Mmax = g->Mmax;
    ix.Mmax0 = g->Mmax0;
    ix.entry = g->entry_point;
    ix.max_level = g->max_level;
    ix.cell_level = hnsw::cell_level_of(g->levels, g->n, g->max_level);
    ix.metric = g->metric;
    ix.uid = hnsw::next_index_uid();
    ok = ok && hnsw::launch_row_norms(ix, xnorm, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        al.release();
        return HNSW_ERR_DEVICE;
    }
    hnsw_index *h = new hnsw_index();
    h->ix = ix;
    h->xnorm = xnorm;
    h->M = g->M;
    (void)hipGetDevice(&h->device);
    h->bytes = al.bytes;
    h->allocations = al.got;
    h->levels.assign(g->levels, g->levels + g->n);
    h->n_upper_rows = g->n_upper_rows;
    *out = h;
    return HNSW_OK;
}

void hnsw_index_free(hnsw_index *index) {
    if (!index) return;
    hnsw::forget_index(index->ix.uid);
    for (void *p : index->allocations) hnsw::device_free(p);
    delete index;
}

hnsw_status hnsw_index_info(const hnsw_index *index, uint64_t out[10]) {
    if (!index || !out) return HNSW_ERR_INVALID_ARG;
    const hnsw::DevIndex &x = index->ix;
    const uint64_t v[10] = {x.n,         x.dim,   x.metric,     index->M, x.Mmax, x.Mmax0,
                            x.max_level, x.entry, index->bytes, index->n_upper_rows};
    memcpy(out, v, sizeof(v));
    return HNSW_OK;
}

hnsw_status hnsw_index_export(const hnsw_index *index, uint8_t *levels, uint32_t *adj0, int32_t *upper_off,
                              uint32_t *adjU) {
    if (!index || !levels || !adj0 || !upper_off || (index->n_upper_rows && !adjU)) return HNSW_ERR_INVALID_ARG;
    const hnsw::DevIndex &x = index->ix;
    memcpy(levels, index->levels.data(), x.n);
    bool ok = hipMemcpy(adj0, x.adj0, static_cast<size_t>(x.n) * x.Mmax0 * 4, hipMemcpyDeviceToHost) == hipSuccess;
    ok = ok && hipMemcpy(upper_off, x.uoff, static_cast<size_t>(x.n) * 4, hipMemcpyDeviceToHost) == hipSuccess;
    if (index->n_upper_rows)
        ok = ok && hipMemcpy(adjU, x.adjU, static_cast<size_t>(index->n_upper_rows) * x.Mmax * 4,
                             hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

static hnsw_status search_impl(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k, uint32_t ef,
                               int mode, const void *mlp, int32_t *ids_out, float *dists_out, uint32_t *counters,
                               float *trace, void *stream, bool no_alloc = false) {
    if (!index) return HNSW_ERR_INVALID_ARG;
    if (no_alloc && n > HNSW_NOALLOC_MAX_QUERIES) return HNSW_ERR_UNSUPPORTED;
    if (k == 0 || ef == 0) return HNSW_ERR_INVALID_ARG;
    if (mode < HNSW_MODE_PLAIN || mode > HNSW_MODE_U8) return HNSW_ERR_UNSUPPORTED;
    if (mode == HNSW_MODE_BF16 && !index->ix.vbf16) return HNSW_ERR_INVALID_ARG;
    if (mode == HNSW_MODE_FP8 && !index->ix.vfp8) return HNSW_ERR_INVALID_ARG;
    if (mode == HNSW_MODE_U8 && !index->ix.vu8) return HNSW_ERR_INVALID_ARG;
    if (mode == HNSW_MODE_LEARNED && !mlp) mode = HNSW_MODE_PLAIN;  // no net: the plain search
    if (mode == HNSW_MODE_LEARNED && k > 64) return HNSW_ERR_UNSUPPORTED;
    const uint32_t efe = ef < k ? k : ef;
    if (efe > HNSW_EF_MAX) return HNSW_ERR_UNSUPPORTED;
    if (n == 0) return HNSW_OK;
    if (!is_device_ptr(queries) || !is_device_ptr(ids_out) || !is_device_ptr(dists_out)) return HNSW_ERR_INVALID_ARG;
    if (counters && !is_device_ptr(counters)) return HNSW_ERR_INVALID_ARG;
    if (trace && !is_device_ptr(trace)) return HNSW_ERR_INVALID_ARG;

    hnsw::SearchArgs a{};
    a.queries = queries;
    a.nq = n;
    a.k = k;
    a.ef = efe;
    a.ids = ids_out;
    a.dists = dists_out;
    a.counters = counters;
    a.wcap = (efe + 63) & ~63u;
    // W needs wcap slots; the low-precision stores sort W after their re-rank
    // (bitonic, a power of two of slots).  A power of two for every store cost
    // the fp32 search a third of its waves per CU just above ef = 256.  An
    // exact 8-bit copy has no re-rank and keeps wcap.
    a.wslots = a.wcap;
    if (mode == HNSW_MODE_BF16 || mode == HNSW_MODE_FP8 || (mode == HNSW_MODE_U8 && !index->ix.u8_exact)) {
        a.wslots = 64;
        while (a.wslots < a.wcap) a.wslots <<= 1;
    }
    a.mode = mode;
    a.mlp = hnsw::DevMlp{};
    if (mode == HNSW_MODE_LEARNED) a.mlp = static_cast<const hnsw_mlp *>(mlp)->net;
    a.ckpt_trace = mode == HNSW_MODE_LEARNED ? trace : nullptr;
    // low-precision stores: a replacing visited table above ef 64 (below, the
    // forgetting one keeps the merge's fast path for batches that forgot nothing)
    a.replace = (mode == HNSW_MODE_BF16 || mode == HNSW_MODE_FP8 || mode == HNSW_MODE_U8) && efe > 64;
    a.ht_slots = hnsw::visited_slots(a, mode == HNSW_MODE_LEARNED);
    a.no_alloc = no_alloc;
    if (hnsw::launch_search(index->ix, a, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

hnsw_status hnsw_search_batch_ex(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k, uint32_t ef,
                                 int mode, const void *mlp, int32_t *ids_out, float *dists_out, uint32_t *counters,
                                 void *stream) {
    return search_impl(index, queries, n, k, ef, mode, mlp, ids_out, dists_out, counters, nullptr, stream);
}

hnsw_status hnsw_search_batch_noalloc(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                      uint32_t ef, int mode, const void *mlp, int32_t *ids_out, float *dists_out,
                                      uint32_t *counters, void *stream) {
    return search_impl(index, queries, n, k, ef, mode, mlp, ids_out, dists_out, counters, nullptr, stream, true);
}

hnsw_status hnsw_search_learned_trace(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                      uint32_t ef, const hnsw_mlp *mlp, int32_t *ids_out, float *dists_out,
                                      uint32_t *counters, float *trace_out, void *stream) {
    if (!mlp || !trace_out) return HNSW_ERR_INVALID_ARG;
    return search_impl(index, queries, n, k, ef, HNSW_MODE_LEARNED, mlp, ids_out, dists_out, counters, trace_out,
                       stream);
}

hnsw_status hnsw_index_add_lowp(hnsw_index *index, int kind, void *stream) {
    if (!index || (kind != HNSW_MODE_BF16 && kind != HNSW_MODE_FP8 && kind != HNSW_MODE_U8))
        return HNSW_ERR_INVALID_ARG;
    hnsw::DevIndex &ix = index->ix;
    if ((kind == HNSW_MODE_BF16 && ix.vbf16) || (kind == HNSW_MODE_FP8 && ix.vfp8) ||
        (kind == HNSW_MODE_U8 && ix.vu8))
        return HNSW_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hnsw::DevIndex nx = ix;
    size_t bytes;
    if (kind == HNSW_MODE_BF16) {
        nx.bf16_stride16 = ((ix.dim + 7) / 8 + 3) & ~3u;
        bytes = (static_cast<size_t>(ix.n) + 1) * nx.bf16_stride16 * 16;
    } else if (kind == HNSW_MODE_U8) {
        nx.u8_pieces = (ix.dim + 15) / 16;
        nx.u8_stride16 = (nx.u8_pieces + 3) & ~3u;
        bytes = (static_cast<size_t>(ix.n) + 1) * nx.u8_stride16 * 16;
    } else {
        // rows padded to 64 bytes; the scale takes 4 bytes of a row's padding
        // when there are any, else the n + 1 scales follow the rows
        nx.fp8_pieces = (ix.dim + 15) / 16;
        nx.fp8_stride16 = (nx.fp8_pieces + 3) & ~3u;
        const bool in_row = nx.fp8_stride16 > nx.fp8_pieces;
        nx.fp8_scale_stride = in_row ? nx.fp8_stride16 * 16 : 4;
        bytes = (static_cast<size_t>(ix.n) + 1) * (nx.fp8_stride16 * 16 + (in_row ? 0 : 4));
    }
    if (index->bytes + bytes > mem_cap()) return HNSW_ERR_OUT_OF_MEMORY;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    // the last 4 bytes of the (zero) row n carry the inexact flag of the 8-bit copy
    uint32_t *flag = static_cast<uint32_t *>(static_cast<void *>(static_cast<uint8_t *>(p) + bytes - 4));
    bool ok = hipMemsetAsync(p, 0, bytes, st) == hipSuccess;
    if (kind == HNSW_MODE_BF16) ok = ok && hnsw::launch_quantize_bf16(nx, static_cast<uint16_t *>(p), st) == hipSuccess;
    else if (kind == HNSW_MODE_U8) ok = ok && hnsw::launch_quantize_u8(nx, static_cast<uint8_t *>(p), flag, st) == hipSuccess;
    else {
        uint8_t *scale = static_cast<uint8_t *>(p) + (nx.fp8_scale_stride == 4
                                                          ? (static_cast<size_t>(ix.n) + 1) * nx.fp8_stride16 * 16
                                                          : static_cast<size_t>(nx.fp8_pieces) * 16);
        nx.fp8_scale = scale;
        ok = ok && hnsw::launch_quantize_fp8(nx, static_cast<uint8_t *>(p), scale, st) == hipSuccess;
    }
    uint32_t inexact = 0;
    if (kind == HNSW_MODE_U8) {
        ok = ok && hipMemcpyAsync(&inexact, flag, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
        ok = ok && hipMemsetAsync(flag, 0, 4, st) == hipSuccess;  // row n is the all-zero row again
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hnsw::device_free(p);
        return HNSW_ERR_DEVICE;
    }
    if (kind == HNSW_MODE_BF16) {
        ix.vbf16 = static_cast<uint16_t *>(p);
        ix.bf16_stride16 = nx.bf16_stride16;
    } else if (kind == HNSW_MODE_U8) {
        ix.vu8 = static_cast<uint8_t *>(p);
        ix.u8_stride16 = nx.u8_stride16;
        ix.u8_pieces = nx.u8_pieces;
        ix.u8_exact = inexact ? 0u : 1u;
    } else {
        ix.vfp8 = static_cast<uint8_t *>(p);
        ix.fp8_stride16 = nx.fp8_stride16;
        ix.fp8_pieces = nx.fp8_pieces;
        ix.fp8_scale = nx.fp8_scale;
        ix.fp8_scale_stride = nx.fp8_scale_stride;
    }
    index->allocations.push_back(p);
    index->bytes += bytes;
    return HNSW_OK;
}

hnsw_status hnsw_index_read_lowp(const hnsw_index *index, int kind, void *host_out, uint64_t layout[3]) {
    if (!index || !layout) return HNSW_ERR_INVALID_ARG;
    const hnsw::DevIndex &ix = index->ix;
    const void *src = kind == HNSW_MODE_BF16 ? static_cast<const void *>(ix.vbf16)
                      : kind == HNSW_MODE_FP8  ? static_cast<const void *>(ix.vfp8)
                      : kind == HNSW_MODE_U8   ? static_cast<const void *>(ix.vu8)
                                               : nullptr;
    if (!src) return HNSW_ERR_INVALID_ARG;
    const uint64_t row = kind == HNSW_MODE_BF16 ? ix.bf16_stride16 * 16ull
                         : kind == HNSW_MODE_U8 ? ix.u8_stride16 * 16ull
                                                : ix.fp8_stride16 * 16ull;
    layout[0] = row;
    layout[1] = kind == HNSW_MODE_BF16 ? ix.bf16_stride16 : (kind == HNSW_MODE_U8 ? ix.u8_pieces : ix.fp8_pieces);
    layout[2] = kind == HNSW_MODE_FP8 ? row * ix.n : (kind == HNSW_MODE_U8 ? ix.u8_exact : 0);
    if (!host_out) return HNSW_OK;
    bool ok = hipMemcpy(host_out, src, row * ix.n, hipMemcpyDeviceToHost) == hipSuccess;
    if (kind == HNSW_MODE_FP8)
        ok = ok && hipMemcpy2D(static_cast<uint8_t *>(host_out) + row * ix.n, 4, ix.fp8_scale, ix.fp8_scale_stride,
                               4, ix.n, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

hnsw_status hnsw_bruteforce_knn(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k,
                                int32_t *ids_out, double *dists_out, void *stream) {
    if (!index || k == 0) return HNSW_ERR_INVALID_ARG;
    if (k > HNSW_BF_K_MAX) return HNSW_ERR_UNSUPPORTED;
    if (n == 0) return HNSW_OK;
    if (!is_device_ptr(queries) || !is_device_ptr(ids_out) || !is_device_ptr(dists_out)) return HNSW_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t nchunks = 1, chunk = 64;
    hnsw::bf_plan(index->ix, n, k, &nchunks, &chunk);
    const size_t scratch = static_cast<size_t>(n) * nchunks * hnsw::bf_candidates(k) * 8;
    void *partial = nullptr;
    if (hipMallocAsync(&partial, scratch, st) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    const hipError_t e = hnsw::launch_bruteforce(index->ix, queries, n, k, index->xnorm,
                                                 static_cast<uint64_t *>(partial), nchunks, chunk, ids_out,
                                                 dists_out, st);
    (void)hipFreeAsync(partial, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

static uint16_t bf16_rne_host(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

hnsw_status hnsw_mlp_create(const float *params, float tau, int jmax, uint32_t period, uint32_t max_ckpt,
                            hnsw_mlp **out) {
    if (!out) return HNSW_ERR_INVALID_ARG;
    *out = nullptr;
    if (!params || period == 0 || jmax < 0 || jmax > 8) return HNSW_ERR_INVALID_ARG;
    for (int i = 0; i < hnsw::kMlpParams; ++i)
        if (!(params[i] == params[i]) || params[i] > 1e30f || params[i] < -1e30f) return HNSW_ERR_INVALID_ARG;
    if (!device_count_ok()) return HNSW_ERR_DEVICE;
    using namespace hnsw;
    const int nW1 = kMlpHid * kMlpIn, nW2 = kMlpHid * kMlpHid, nW3 = kMlpOut * kMlpHid;
    const int ob1 = nW1, oW2 = ob1 + kMlpHid, ob2 = oW2 + nW2, oW3 = ob2 + kMlpHid, ob3 = oW3 + nW3;
    std::vector<uint16_t> w(nW1 + nW2 + nW3);
    for (int i = 0; i < nW1; ++i) w[i] = bf16_rne_host(params[i]);
    for (int i = 0; i < nW2; ++i) w[nW1 + i] = bf16_rne_host(params[oW2 + i]);
    for (int i = 0; i < nW3; ++i) w[nW1 + nW2 + i] = bf16_rne_host(params[oW3 + i]);
    std::vector<float> b(kMlpHid + kMlpHid + kMlpOut);
    memcpy(b.data(), params + ob1, kMlpHid * 4);
    memcpy(b.data() + kMlpHid, params + ob2, kMlpHid * 4);
    memcpy(b.data() + 2 * kMlpHid, params + ob3, kMlpOut * 4);
    const size_t wbytes = w.size() * 2, bytes = wbytes + b.size() * 4;
    void *mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    if (hipMemcpy(mem, w.data(), wbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(static_cast<uint8_t *>(mem) + wbytes, b.data(), b.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        hnsw::device_free(mem);
        return HNSW_ERR_DEVICE;
    }
    hnsw_mlp *m = new hnsw_mlp();
    m->mem = mem;
    const uint16_t *wd = static_cast<const uint16_t *>(mem);
    const float *bd = reinterpret_cast<const float *>(static_cast<uint8_t *>(mem) + wbytes);
    m->net = DevMlp{wd, wd + nW1, wd + nW1 + nW2, bd, bd + kMlpHid, bd + 2 * kMlpHid, tau, jmax, period, max_ckpt};
    *out = m;
    return HNSW_OK;
}

void hnsw_mlp_free(hnsw_mlp *mlp) {
    if (!mlp) return;
    hnsw::device_free(mlp->mem);
    delete mlp;
}

hnsw_status hnsw_mlp_forward(const float *params, const float *x, uint32_t n, float *out, void *stream) {
    if (n == 0) return HNSW_OK;
    if (!is_device_ptr(params) || !is_device_ptr(x) || !is_device_ptr(out)) return HNSW_ERR_INVALID_ARG;
    if (hnsw::launch_mlp_forward(params, x, n, out, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

hnsw_status hnsw_mlp_grad(const float *params, const float *x, const float *y, uint32_t n, float lambda,
                          float *grad, float *loss, void *stream) {
    if (n == 0) return HNSW_ERR_INVALID_ARG;
    if (!is_device_ptr(params) || !is_device_ptr(x) || !is_device_ptr(y) || !is_device_ptr(grad))
        return HNSW_ERR_INVALID_ARG;
    if (loss && !is_device_ptr(loss)) return HNSW_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t waves = hnsw::mlp_grad_waves(n);
    void *scratch = nullptr;
    if (hipMallocAsync(&scratch, waves * (hnsw::kMlpParams + 1) * 4, st) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    const hipError_t e = hnsw::launch_mlp_grad(params, x, y, n, lambda, grad, loss, static_cast<float *>(scratch), st);
    (void)hipFreeAsync(scratch, st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

hnsw_status hnsw_mlp_adam(float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                          float eps, uint32_t step, void *stream) {
    if (step == 0) return HNSW_ERR_INVALID_ARG;
    if (!is_device_ptr(params) || !is_device_ptr(grad) || !is_device_ptr(m) || !is_device_ptr(v))
        return HNSW_ERR_INVALID_ARG;
    if (hnsw::launch_adam(params, grad, m, v, hnsw::kMlpParams, lr, beta1, beta2, eps, step,
                          static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        return HNSW_ERR_DEVICE;
    }
    return HNSW_OK;
}

hnsw_status hnsw_search_batch(const hnsw_index *index, const float *queries, uint32_t n, uint32_t k, uint32_t ef,
                              int32_t *ids_out, float *dists_out, void *stream) {
    return hnsw_search_batch_ex(index, queries, n, k, ef, HNSW_MODE_PLAIN, nullptr, ids_out, dists_out, nullptr,
                                stream);
}

}  // extern "C"
