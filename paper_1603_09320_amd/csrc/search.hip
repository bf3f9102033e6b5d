// Batched K-NN-SEARCH (Alg. 5 of arXiv:1603.09320) for gfx950: one workgroup
// of one wavefront per query; the search itself is search_one in
// search_device.h (or, for batches larger than the chip holds at once, its
// descent and layer-0 parts as separate launches with the queries reordered
// between them, see search_kernels.h).  This unit holds the buffered-gather
// kernels (stores of at most 2 GiB); search_wide.hip holds those for larger
// stores.
#include <stdlib.h>

#include <atomic>
#include <mutex>

#include "search_kernels.h"

namespace hnsw {

// Lane-group tile for a store: G lanes per vector, F pieces per lane.
// fp32 rows use two pieces per lane up to 128 dimensions; low-precision
// rows (8 or 16 values per piece) use one piece per lane up to 16 pieces.
TileShape tile_for(int kind, uint32_t dim) {
    const uint32_t vpp = kind == kF32 ? 4 : (kind == kBF16 ? 8 : 16);  // FP8 and 8-bit: 16
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
    return static_cast<size_t>(a.wslots) * 8 + 64 * 8 + 64 * 4 + (learned ? 64 * 4 : 0) +
           static_cast<size_t>(a.ht_slots) * 4;
}

// The batch kernels keep six waves per SIMD (five for FP8), at most 24 per
// CU sharing 160 KiB of LDS.  The table takes what is left of a 24th of it,
// rounded down to whole KiB (the share itself, so that no allocation rounding
// can cost a wave), and at least 1,024 slots; a fuller table forgets fewer
// ids (a forgotten id is scored again).  FP8 is sized like the others: a
// table filling a 20th of the LDS (all of it at five waves per SIMD)
// measured 2% slower.  A table that grows with ef costs more waves than it
// saves: on glove_like 1.2M at ef 288 (10,000 queries) 1,024 slots took
// 5.53 ms, 2,048 slots 6.15 ms and 512 slots 5.81 ms (at ef 320, 4,096 slots
// 10.3 ms).  Above ef 64 the low-precision stores' table replaces old ids as
// the fp32 one does (on deep_like 10M at ef 256, BF16 / FP8: 1.54 / 1.67 M
// queries/s with a forgetting table of 2,048 slots, 1.37 / 1.49 M with 1,024
// slots, 1.84 / 1.92 M with a replacing table of 1,024 slots).
// HNSW_VISITED_LOG2 = 8..14 fixes a power of two instead.
uint32_t visited_slots(const SearchArgs &a, bool learned) {
    if (const char *v = getenv("HNSW_VISITED_LOG2")) {
        const long x = strtol(v, nullptr, 10);
        if (x >= 8 && x <= 14) return 1u << x;
    }
    const uint32_t base = 1024;
    const uint32_t share = (160u * 1024u / 24u) & ~1023u;
    SearchArgs t = a;
    t.ht_slots = 0;
    const uint32_t fixed = static_cast<uint32_t>(search_lds_bytes(t, false));
    const uint32_t fit = share > fixed ? ((share - fixed) / 4) & ~63u : 0u;
    const uint32_t slots = fit > base ? fit : base;
    // the learned kernels take their extra buffer out of the table, so that
    // they hold as many waves per CU as the plain ones (the table decides no
    // feature of the stop rule)
    return learned ? slots - static_cast<uint32_t>(search_lds_bytes(t, true) - fixed) / 4 : slots;
}

// The store a search mode traverses (descent and layer 0) fits the buffered
// gathers; a low-precision form's re-rank checks the fp32 store itself.
bool traversal_buffered(const DevIndex &ix, int mode) {
    auto fits = [&](uint32_t stride16) { return (static_cast<uint64_t>(ix.n) + 1) * stride16 * 16 <= kBufferedMaxBytes; };
    switch (mode) {
        case HNSW_MODE_BF16: return fits(ix.bf16_stride16);
        case HNSW_MODE_FP8: return fits(ix.fp8_stride16);
        case HNSW_MODE_U8: return fits(ix.u8_stride16);
        default: return fits(ix.stride4);
    }
}

bool stores_buffered(const DevIndex &ix) {
    auto fits = [&](const void *p, uint32_t stride16) {
        return !p || (static_cast<uint64_t>(ix.n) + 1) * stride16 * 16 <= kBufferedMaxBytes;
    };
    return fits(ix.vec, ix.stride4) && fits(ix.vbf16, ix.bf16_stride16) && fits(ix.vfp8, ix.fp8_stride16) &&
           fits(ix.vu8, ix.u8_stride16);
}

namespace {

// Workspace of the scheduled launches, one per (device, stream): kSchedBytes
// per query (layer-0 entry key, the upper layers' counters, the order, the cell).  It
// grows to the largest batch seen on that stream and is kept until the
// process ends.  Launches on one stream run in order, so a buffer is reused
// only after the previous batch's kernels have read it; the mutex is held
// while a batch's kernels are enqueued, so that batches submitted to one
// stream from several threads do not interleave their launches.
constexpr size_t kSchedBytes = 24;
struct SchedBuf {
    int device;
    hipStream_t stream;
    uint8_t *p;
    size_t cap;
};
std::mutex g_sched_mu;
std::vector<SchedBuf> g_sched;

uint8_t *sched_buffer(hipStream_t stream, size_t need) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    SchedBuf *b = nullptr;
    for (SchedBuf &x : g_sched)
        if (x.device == dev && x.stream == stream) b = &x;
    if (!b) {
        g_sched.push_back(SchedBuf{dev, stream, nullptr, 0});
        b = &g_sched.back();
    }
    if (b->cap < need) {
        if (b->p) device_free(b->p);
        b->p = nullptr;
        b->cap = 0;
        size_t cap = 1u << 20;
        while (cap < need) cap <<= 1;
        void *p = nullptr;
        if (hipMalloc(&p, cap) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        b->p = static_cast<uint8_t *>(p);
        b->cap = cap;
    }
    return b->p;
}

// Tuning records of tuned_form.  The forms give identical results, so the
// choice affects time only; on sift_like the scheduled launches are 4-26%
// faster, on deep_like (short layer-0 searches, tight clusters) 1-8% slower.
// Records are keyed by the index's uid (never reused within the process) and
// dropped when the index is freed; the table holds at most kTuneCap records
// (the oldest decided ones make room).
// Protocol: one untimed call of each form (cold caches, first launches), then
// kTuneRuns timed calls alternating scheduled / one-kernel; the form with the
// smaller total wins.
constexpr int kTuneRuns = 4;
struct FormTune {
    uint32_t index;  // DevIndex::uid
    int device, mode;
    uint32_t ef, octave;
    int phase;          // 0, 1 warm-up calls; 2 .. 2 + kTuneRuns - 1 timed calls; then waiting; kDecided
    bool sched;         // decision (phase kDecided)
    hipEvent_t ev[kTuneRuns][2];
    float ms[kTuneRuns];
};
constexpr int kDecided = 3 + kTuneRuns;
std::vector<FormTune> g_tune;
constexpr size_t kTuneCap = 1024;

bool events_done(hipEvent_t e) { return hipEventQuery(e) == hipSuccess; }

void destroy_events(FormTune &t) {
    for (auto &pair : t.ev)
        for (hipEvent_t &e : pair)
            if (e) (void)hipEventDestroy(e), e = nullptr;
}

std::atomic<uint32_t> g_uid{0};

}  // namespace

uint32_t next_index_uid() {
    uint32_t u = ++g_uid;
    if (u == 0) u = ++g_uid;
    return u;
}

uint32_t cell_level_of(const uint8_t *levels, uint32_t n, uint32_t max_level) {
    if (max_level == 0) return 0;
    std::vector<uint64_t> at(max_level + 2, 0);  // at[l]: nodes of level exactly l
    for (uint32_t i = 0; i < n; ++i) ++at[levels[i] <= max_level ? levels[i] : max_level];
    uint64_t above = 0;  // nodes of level >= l
    for (uint32_t l = max_level; l >= 1; --l) {
        above += at[l];
        if (above >= kCellMin) return l;
    }
    return 1;
}

void forget_index(uint32_t uid) {
    std::lock_guard<std::mutex> lk(g_sched_mu);
    size_t j = 0;
    for (size_t i = 0; i < g_tune.size(); ++i) {
        if (g_tune[i].index == uid) {
            destroy_events(g_tune[i]);
            continue;
        }
        g_tune[j++] = g_tune[i];
    }
    g_tune.resize(j);
}

bool tuned_form(const DevIndex &ix, const SearchArgs &a, hipStream_t stream, hipEvent_t *ev_start,
                hipEvent_t *ev_end) {
    *ev_start = *ev_end = nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return true;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    uint32_t octave = 0;
    while ((a.nq >> octave) > 1u) ++octave;
    FormTune *t = nullptr;
    for (FormTune &x : g_tune)
        if (x.index == ix.uid && x.device == dev && x.mode == a.mode && x.ef == a.ef && x.octave == octave) t = &x;
    if (a.no_alloc) return t && t->phase == kDecided ? t->sched : true;
    if (!t) {
        if (g_tune.size() >= kTuneCap) {
            // make room: drop the older half of the decided records (records
            // still timing hold events that are in flight)
            size_t j = 0, dropped = 0;
            for (size_t i = 0; i < g_tune.size(); ++i) {
                if (g_tune[i].phase == kDecided && dropped < kTuneCap / 2) {
                    ++dropped;
                    continue;
                }
                g_tune[j++] = g_tune[i];
            }
            g_tune.resize(j);
            if (g_tune.size() >= kTuneCap) return true;  // every record is mid-timing: no tuning for this call
        }
        g_tune.push_back(FormTune{ix.uid, dev, a.mode, a.ef, octave, 0, true, {}, {}});
        t = &g_tune.back();
    }
    auto give = [&](int k) {
        if (!t->ev[k][0] && (hipEventCreate(&t->ev[k][0]) != hipSuccess || hipEventCreate(&t->ev[k][1]) != hipSuccess)) {
            (void)hipGetLastError();
            destroy_events(*t);
            t->phase = kDecided;  // no events: keep the scheduled form
            t->sched = true;
            return false;
        }
        *ev_start = t->ev[k][0];
        *ev_end = t->ev[k][1];
        return true;
    };
    if (t->phase == kDecided) return t->sched;
    if (t->phase < 2) return t->phase++ == 0;  // untimed: scheduled, then one-kernel
    if (t->phase < 2 + kTuneRuns) {
        const int k = t->phase - 2;
        const bool sched = (k & 1) == 0;
        if (!give(k)) return true;
        ++t->phase;
        return sched;
    }
    // every timed call enqueued: decide once they have all ended (the events
    // are queried, never waited for); until then the scheduled form
    for (int k = 0; k < kTuneRuns; ++k)
        if (!events_done(t->ev[k][1])) return true;
    float tot[2] = {0.f, 0.f};
    bool ok = true;
    for (int k = 0; k < kTuneRuns; ++k) {
        ok = ok && hipEventElapsedTime(&t->ms[k], t->ev[k][0], t->ev[k][1]) == hipSuccess;
        tot[k & 1] += t->ms[k];
    }
    if (!ok) (void)hipGetLastError();
    t->sched = !ok || tot[0] <= tot[1];
    destroy_events(*t);
    t->phase = kDecided;
    return t->sched;
}

// Workspace of the allocation-free entry point (hnsw_search_batch_noalloc):
// the scheduled launches' kSchedBytes per query for up to
// HNSW_NOALLOC_MAX_QUERIES queries, held by every device the library runs on
// until the process ends.  Its device address is taken once per device
// (hipGetSymbolAddress, with that device current); host code passes only that
// address to kernels.  Every element is written by the descent and order
// kernels before it is read, so nothing needs clearing between calls; calls
// that overlap on one device share it and race.
constexpr size_t kNoAllocScratchBytes = static_cast<size_t>(HNSW_NOALLOC_MAX_QUERIES) * kSchedBytes;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (null on failure).
uint8_t *noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<uint8_t *>(ptr);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

// HNSW_WIDE_GATHERS=1 sends every launch through the 64-bit addressed kernels
// (they are otherwise taken only when the traversed store is above 2 GiB), so that tests can
// check them on small indices.  HNSW_SCHEDULE=0 keeps every batch in one
// kernel, HNSW_SCHEDULE=2 schedules every batch (both for tests); by default
// a batch is scheduled when it holds more queries than waves resident at once.
hipError_t launch_search(const DevIndex &ix, const SearchArgs &a0, hipStream_t stream) {
    const char *w = getenv("HNSW_WIDE_GATHERS");
    const bool force_wide = w && w[0] == '1';
    const char *sv = getenv("HNSW_SCHEDULE");
    SearchArgs a = a0;
    a.sched = !sv ? 1 : (sv[0] == '0' ? 0 : (sv[0] == '2' ? 2 : 1));
    a.sched_start = nullptr;
    a.sched_up = nullptr;
    a.sched_order = nullptr;
    a.sched_cell = nullptr;
    std::unique_lock<std::mutex> lk(g_sched_mu, std::defer_lock);
    if (a.sched == 2 || (a.sched == 1 && a.nq > 256)) {
        lk.lock();
        const size_t n = a.nq;
        uint8_t *p;
        if (a.no_alloc) {
            if (n * kSchedBytes > kNoAllocScratchBytes) return hipErrorInvalidValue;
            p = noalloc_scratch();
            if (!p) return hipErrorInvalidSymbol;
        } else {
            p = sched_buffer(stream, n * kSchedBytes);
        }
        if (p) {
            a.sched_start = reinterpret_cast<uint64_t *>(p);
            a.sched_up = reinterpret_cast<uint32_t *>(p + n * 8);
            a.sched_order = reinterpret_cast<uint32_t *>(p + n * 16);
            a.sched_cell = reinterpret_cast<uint32_t *>(p + n * 20);
        } else {
            a.sched = 0;
        }
    }
    if (traversal_buffered(ix, a.mode) && !force_wide) return launch_search_stores<true>(ix, a, stream);
    return launch_search_wide(ix, a, stream);
}

}  // namespace hnsw
