// Continuous-batching serving loop: a persistent kernel whose waves take
// request tickets in order and answer each request with the same search
// (search_one) as the batch path, while the host keeps admitting new
// requests into a ring of slots in fine-grained host memory.
//
// Protocol per ring slot (ServeReq, host memory):
//   host:  writes the query and (k, ef, mode, ticket), then state = 1 (release)
//   wave:  took ticket t from a device counter; waits until slot t % slots has
//          state == 1 and ticket == t (acquire, system scope); searches; writes
//          ids/dists into the slot's output rows; state = 2 (release, system)
//   host:  sees state == 2 (acquire), copies the results, state = 0 (free)
// A slot is reused only after its previous request was consumed, so at most
// `slots` requests are in flight (the output budget).  Every wave reserves
// LDS for ef_max (the LDS budget): a request with ef > ef_max or k > k_max is
// refused at submission.  Waves exit when the host raises the stop flag, or
// unconditionally when their wall-clock budget runs out, so the grid always
// drains.
#include <string.h>

#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "search_device.h"

namespace hnsw {

struct ServeReq {
    uint32_t state;  // 0 free, 1 submitted, 2 done
    uint32_t ticket;
    uint32_t k, ef;
    int32_t mode;
    uint32_t pad[3];
};

struct ServeArgs {
    ServeReq *ring;        // [slots], host memory
    const float *qbuf;     // [slots][dim], host memory
    int32_t *out_ids;      // [slots][kmax], host memory
    float *out_d;          // [slots][kmax], host memory
    uint32_t *counters;    // [slots][4], host memory
    uint32_t *next_ticket; // device memory
    const uint32_t *stop;  // host memory
    uint32_t slots, kmax;
    uint64_t budget_ticks; // wall-clock ticks each wave may live
};

namespace {

// Polling reads of host memory: relaxed system-scope loads go to memory
// without invalidating the caches (an acquire load would invalidate the L2 on
// every poll, for every idle wave); one acquire fence follows a successful poll.
__device__ __forceinline__ uint32_t load_sys(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ uint64_t load_sys64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Every value that steers control flow below is wave-uniform by construction
// (kernel arguments, readfirstlane of loaded request fields, ballots): the
// compiler then keeps the wave converged through the request loop.  With
// per-lane copies of k/ef/mode it may treat the loop as divergent and let
// lanes leave it at different times, which defers the completion flag of a
// served request until the others exit.
// LOWP: the low-precision copies this server's kernel can traverse (bit 0
// BF16, bit 1 FP8).  Each kind's search is inlined into the request loop with
// the lane-group shape the batch kernels use for that store (G, F for fp32;
// GB, FB for BF16; G8, F8 for FP8), and a server instantiates only the kinds
// its index holds: the registers are those of the widest kind inlined.
template <int G, int F, int GB, int FB, int G8, int F8, int METRIC, int LOWP>
__global__ __launch_bounds__(64) void serve_kernel(DevIndex ix, SearchArgs a, ServeArgs sv) {
    extern __shared__ __align__(16) uint8_t smem[];
    const WaveLds s = carve<true>(smem, a);
    const int lane = lane_id();
    const uint64_t t_end = wall_clock64() + sv.budget_ticks;
    bool quit = false;
    while (!quit) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(sv.next_ticket, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        const uint32_t slot = t % sv.slots;
        ServeReq *r = sv.ring + slot;
        int naps = 1;
        for (;;) {
            // state (low word) and ticket (high word) in one read; every lane
            // reads the same words and the wave takes lane 0's copy
            const uint64_t w = load_sys64(reinterpret_cast<const uint64_t *>(r));
            const uint32_t ready = __builtin_amdgcn_readfirstlane(
                static_cast<uint32_t>(static_cast<uint32_t>(w) == 1u && static_cast<uint32_t>(w >> 32) == t));
            if (ready) break;
            const uint32_t stop = __builtin_amdgcn_readfirstlane(load_sys(sv.stop));
            if (stop || wall_clock64() > t_end) {
                quit = true;
                break;
            }
            // Back-off doubles up to 256 sleeps of 2,048 cycles (about 0.2 ms):
            // every idle wave's poll is a read over the host link, and with
            // over a thousand idle waves a short back-off floods it and slows
            // the requests in flight (p50 7 ms against 0.7 ms at 50k req/s).
            for (int z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(32);
            naps = naps < 256 ? naps * 2 : 256;
        }
        if (quit) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the request's fields were written before state = 1
        Job job;
        job.q = sv.qbuf + static_cast<size_t>(slot) * ix.dim;
        job.k = __builtin_amdgcn_readfirstlane(load_sys(&r->k));
        job.ef = __builtin_amdgcn_readfirstlane(load_sys(&r->ef));
        const int mode = static_cast<int>(
            __builtin_amdgcn_readfirstlane(load_sys(reinterpret_cast<const uint32_t *>(&r->mode))));
        job.ids = sv.out_ids + static_cast<size_t>(slot) * sv.kmax;
        job.dists = sv.out_d + static_cast<size_t>(slot) * sv.kmax;
        job.counters = sv.counters + static_cast<size_t>(slot) * 4;
        job.trace = nullptr;
        if ((LOWP & 1) && mode == HNSW_MODE_BF16 && ix.vbf16)
            search_one<GB, FB, METRIC, kBF16, false, true>(ix, a, job, s);
        else if ((LOWP & 2) && mode == HNSW_MODE_FP8 && ix.vfp8)
            search_one<G8, F8, METRIC, kFP8, false, true>(ix, a, job, s);
        else if (mode == HNSW_MODE_LEARNED && a.mlp.w1)
            search_one<G, F, METRIC, kF32, true, true>(ix, a, job, s);
        else
            search_one<G, F, METRIC, kF32, false, true>(ix, a, job, s);
        // every lane's result stores are visible system-wide before the flag;
        // all lanes store the same value
        __hip_atomic_store(&r->state, 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int G, int F, int GB, int FB, int G8, int F8, int LOWP>
hipError_t launch_serve_gfl(const DevIndex &ix, const SearchArgs &a, const ServeArgs &sv, uint32_t waves,
                            hipStream_t st) {
    const size_t lds = search_lds_bytes(a, true);
    if (ix.metric == HNSW_IP)
        hipLaunchKernelGGL((serve_kernel<G, F, GB, FB, G8, F8, HNSW_IP, LOWP>), dim3(waves), dim3(64), lds, st, ix,
                           a, sv);
    else
        hipLaunchKernelGGL((serve_kernel<G, F, GB, FB, G8, F8, HNSW_L2SQ, LOWP>), dim3(waves), dim3(64), lds, st,
                           ix, a, sv);
    return hipGetLastError();
}

template <int G, int F, int GB, int FB, int G8, int F8>
hipError_t launch_serve_gf(const DevIndex &ix, const SearchArgs &a, const ServeArgs &sv, uint32_t waves,
                           hipStream_t st) {
    switch ((ix.vbf16 ? 1 : 0) | (ix.vfp8 ? 2 : 0)) {
        case 0: return launch_serve_gfl<G, F, GB, FB, G8, F8, 0>(ix, a, sv, waves, st);
        case 1: return launch_serve_gfl<G, F, GB, FB, G8, F8, 1>(ix, a, sv, waves, st);
        case 2: return launch_serve_gfl<G, F, GB, FB, G8, F8, 2>(ix, a, sv, waves, st);
        default: return launch_serve_gfl<G, F, GB, FB, G8, F8, 3>(ix, a, sv, waves, st);
    }
}

}  // namespace

hipError_t launch_serve(const DevIndex &ix, const SearchArgs &a, const ServeArgs &sv, uint32_t waves,
                        hipStream_t st) {
    // The fp32 shape of the dimension selects the kernel; within each fp32
    // shape's range of dimensions the BF16 and FP8 shapes below hold every
    // coordinate (8 and 16 values per piece), as the batch kernels' shapes do.
    const TileShape t = tile_for(kF32, ix.dim);
    switch (t.G * 16 + t.F) {
        case 1 * 16 + 1: return launch_serve_gf<1, 1, 1, 1, 1, 1>(ix, a, sv, waves, st);     // d <= 4
        case 2 * 16 + 2: return launch_serve_gf<2, 2, 2, 1, 1, 1>(ix, a, sv, waves, st);     // d <= 16
        case 4 * 16 + 2: return launch_serve_gf<4, 2, 4, 1, 2, 1>(ix, a, sv, waves, st);     // d <= 32
        case 8 * 16 + 2: return launch_serve_gf<8, 2, 8, 1, 4, 1>(ix, a, sv, waves, st);     // d <= 64
        case 16 * 16 + 2: return launch_serve_gf<16, 2, 16, 1, 8, 1>(ix, a, sv, waves, st);  // d <= 128
        default: return launch_serve_gf<16, 4, 16, 2, 16, 1>(ix, a, sv, waves, st);          // d <= 256
    }
}

}  // namespace hnsw

// ------------------------------------------------------------ host runtime

namespace hnsw {
hipError_t launch_serve(const DevIndex &ix, const SearchArgs &a, const ServeArgs &sv, uint32_t waves,
                        hipStream_t st);
}

struct hnsw_server {
    const hnsw_index *index;
    hnsw::SearchArgs a;
    hnsw::ServeArgs sv;        // pointers as the device sees them
    hnsw::ServeReq *ring;      // host views
    float *qbuf;
    int32_t *oids;
    float *od;
    uint32_t *cnt;
    uint32_t *stop;
    uint32_t *next_ticket_dev;
    hipStream_t stream;
    uint64_t next_ticket;
    uint32_t slots, kmax, efmax, dim;
    int lowp;  // copies the kernel traverses (bit 0 BF16, bit 1 FP8), fixed at start
    bool have_mlp;
    double budget_s;
};

namespace {

template <typename T>
T *host_alloc(size_t count, std::vector<void *> &got) {
    void *p = nullptr;
    if (hipHostMalloc(&p, count * sizeof(T) + 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    memset(p, 0, count * sizeof(T) + 64);
    got.push_back(p);
    return static_cast<T *>(p);
}

template <typename T>
T *dev_view(T *host) {
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return static_cast<T *>(d);
}

// Releases a server whose kernel is not (or no longer) resident; frees go
// through the holding path, since other servers may still be running.
void free_server(hnsw_server *s) {
    hnsw::host_free(s->ring);
    hnsw::host_free(s->qbuf);
    hnsw::host_free(s->oids);
    hnsw::host_free(s->od);
    hnsw::host_free(s->cnt);
    hnsw::host_free(s->stop);
    hnsw::device_free(s->next_ticket_dev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

hnsw_status hnsw_server_start(const hnsw_index *index, const hnsw_mlp *mlp, uint32_t slots, uint32_t waves,
                              uint32_t ef_max, uint32_t k_max, double budget_s, hnsw_server **out) {
    if (!out) return HNSW_ERR_INVALID_ARG;
    *out = nullptr;
    if (!index || slots == 0 || slots > (1u << 20) || waves == 0 || waves > 65536 || k_max == 0 ||
        k_max > ef_max || !(budget_s > 0.0) || budget_s > 3600.0)
        return HNSW_ERR_INVALID_ARG;
    if (ef_max > HNSW_EF_MAX) return HNSW_ERR_UNSUPPORTED;
    // the serving kernel gathers with 32-bit buffer offsets only
    if (!hnsw::stores_buffered(index->ix)) return HNSW_ERR_UNSUPPORTED;
    if (!hnsw::device_count_ok()) return HNSW_ERR_DEVICE;
    hnsw_server *s = new hnsw_server();
    memset(static_cast<void *>(s), 0, sizeof(*s));
    s->index = index;
    s->slots = slots;
    s->kmax = k_max;
    s->efmax = ef_max;
    s->dim = index->ix.dim;
    s->have_mlp = mlp != nullptr;
    s->lowp = (index->ix.vbf16 ? 1 : 0) | (index->ix.vfp8 ? 2 : 0);
    s->budget_s = budget_s;
    std::vector<void *> got;
    s->ring = host_alloc<hnsw::ServeReq>(slots, got);
    s->qbuf = host_alloc<float>(static_cast<size_t>(slots) * s->dim, got);
    s->oids = host_alloc<int32_t>(static_cast<size_t>(slots) * k_max, got);
    s->od = host_alloc<float>(static_cast<size_t>(slots) * k_max, got);
    s->cnt = host_alloc<uint32_t>(static_cast<size_t>(slots) * 4, got);
    s->stop = host_alloc<uint32_t>(1, got);
    bool ok = s->ring && s->qbuf && s->oids && s->od && s->cnt && s->stop;
    ok = ok && hipMalloc(&s->next_ticket_dev, 4) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
    // zeroed on the server's own stream, so the kernel launched next on that
    // stream sees 0 (a null-stream memset is not ordered with it)
    ok = ok && hipMemsetAsync(s->next_ticket_dev, 0, 4, s->stream) == hipSuccess;
    int dev = 0, khz = 0;
    ok = ok && hipGetDevice(&dev) == hipSuccess &&
         hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0;
    if (!ok) {
        (void)hipGetLastError();
        free_server(s);
        return HNSW_ERR_OUT_OF_MEMORY;
    }
    hnsw::ServeArgs &sv = s->sv;
    sv.ring = dev_view(s->ring);
    sv.qbuf = dev_view(s->qbuf);
    sv.out_ids = dev_view(s->oids);
    sv.out_d = dev_view(s->od);
    sv.counters = dev_view(s->cnt);
    sv.stop = dev_view(s->stop);
    sv.next_ticket = s->next_ticket_dev;
    sv.slots = slots;
    sv.kmax = k_max;
    sv.budget_ticks = static_cast<uint64_t>(budget_s * 1000.0 * khz);
    if (!sv.ring || !sv.qbuf || !sv.out_ids || !sv.out_d || !sv.counters || !sv.stop) {
        free_server(s);
        return HNSW_ERR_DEVICE;
    }
    hnsw::SearchArgs &a = s->a;
    a = hnsw::SearchArgs{};
    a.wcap = (ef_max + 63) & ~63u;
    a.wslots = 64;
    while (a.wslots < a.wcap) a.wslots <<= 1;
    uint32_t lg = 10;
    while (lg < 11 && (1u << lg) < 8u * ef_max) ++lg;
    a.ht_slots = 1u << lg;
    a.mode = HNSW_MODE_PLAIN;
    a.mlp = mlp ? mlp->net : hnsw::DevMlp{};
    if (hnsw::launch_serve(index->ix, a, sv, waves, s->stream) != hipSuccess) {
        (void)hipGetLastError();
        free_server(s);
        return HNSW_ERR_DEVICE;
    }
    hnsw::server_started();
    *out = s;
    return HNSW_OK;
}

hnsw_status hnsw_server_submit(hnsw_server *srv, const float *query, uint32_t k, uint32_t ef, int mode,
                               uint64_t *ticket) {
    if (!srv || !query || !ticket || k == 0) return HNSW_ERR_INVALID_ARG;
    if (mode < HNSW_MODE_PLAIN || mode > HNSW_MODE_LEARNED) return HNSW_ERR_INVALID_ARG;
    const uint32_t efe = ef < k ? k : ef;
    if (k > srv->kmax || efe > srv->efmax) return HNSW_ERR_UNSUPPORTED;
    const hnsw::DevIndex &ix = srv->index->ix;
    if (mode == HNSW_MODE_BF16 && !(srv->lowp & 1)) return HNSW_ERR_INVALID_ARG;
    if (mode == HNSW_MODE_FP8 && !(srv->lowp & 2)) return HNSW_ERR_INVALID_ARG;
    if (mode == HNSW_MODE_LEARNED && (!srv->have_mlp || k > 64)) return HNSW_ERR_UNSUPPORTED;
    const uint32_t slot = static_cast<uint32_t>(srv->next_ticket % srv->slots);
    hnsw::ServeReq *r = srv->ring + slot;
    if (__atomic_load_n(&r->state, __ATOMIC_ACQUIRE) != 0u) return HNSW_ERR_BUSY;
    memcpy(srv->qbuf + static_cast<size_t>(slot) * srv->dim, query, static_cast<size_t>(srv->dim) * 4);
    r->k = k;
    r->ef = efe;
    r->mode = mode;
    r->ticket = static_cast<uint32_t>(srv->next_ticket);
    __atomic_store_n(&r->state, 1u, __ATOMIC_RELEASE);
    *ticket = srv->next_ticket++;
    return HNSW_OK;
}

hnsw_status hnsw_server_poll(hnsw_server *srv, uint64_t ticket, int32_t *ids, float *dists, int *done) {
    if (!srv || !done) return HNSW_ERR_INVALID_ARG;
    *done = 0;
    if (ticket >= srv->next_ticket || ticket + srv->slots < srv->next_ticket) return HNSW_ERR_INVALID_ARG;
    const uint32_t slot = static_cast<uint32_t>(ticket % srv->slots);
    hnsw::ServeReq *r = srv->ring + slot;
    if (__atomic_load_n(&r->state, __ATOMIC_ACQUIRE) != 2u || r->ticket != static_cast<uint32_t>(ticket))
        return HNSW_OK;
    const uint32_t k = r->k;
    if (ids) memcpy(ids, srv->oids + static_cast<size_t>(slot) * srv->kmax, k * 4);
    if (dists) memcpy(dists, srv->od + static_cast<size_t>(slot) * srv->kmax, k * 4);
    __atomic_store_n(&r->state, 0u, __ATOMIC_RELEASE);
    *done = 1;
    return HNSW_OK;
}

hnsw_status hnsw_server_stop(hnsw_server *srv) {
    if (!srv) return HNSW_ERR_INVALID_ARG;
    __atomic_store_n(srv->stop, 1u, __ATOMIC_RELEASE);
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t q = hipStreamQuery(srv->stream);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) {
            (void)hipGetLastError();
            return HNSW_ERR_DEVICE;  // the kernel failed: memory is kept (it may still be referenced)
        }
        if (seconds_since(t0) > srv->budget_s + 10.0) return HNSW_ERR_DEVICE;
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
    free_server(srv);
    hnsw::server_stopped();
    return HNSW_OK;
}

hnsw_status hnsw_serve_replay(hnsw_server *const *servers, uint32_t n_servers, const float *const *queries,
                              uint64_t n, const double *arrival_s, const uint32_t *server_of, const uint32_t *qidx,
                              const uint32_t *k, const uint32_t *ef, const int32_t *mode, uint32_t out_stride,
                              int32_t *ids, float *dists, double *t_submit, double *t_done, double timeout_s) {
    if (!servers || !queries || !arrival_s || !server_of || !qidx || !k || !ef || !mode || !t_submit || !t_done ||
        n_servers == 0 || (!ids) != (!dists))
        return HNSW_ERR_INVALID_ARG;
    for (uint64_t i = 0; i < n; ++i) {
        if (server_of[i] >= n_servers || !servers[server_of[i]] || (ids && k[i] > out_stride))
            return HNSW_ERR_INVALID_ARG;
        if (i && arrival_s[i] < arrival_s[i - 1]) return HNSW_ERR_INVALID_ARG;
    }
    std::vector<uint64_t> ticket(n, 0);
    std::vector<uint64_t> inflight;
    inflight.reserve(1 << 16);
    uint64_t next = 0, done_count = 0;
    const auto t0 = std::chrono::steady_clock::now();
    while (done_count < n) {
        const double now = seconds_since(t0);
        if (now > timeout_s) return HNSW_ERR_DEVICE;
        while (next < n && arrival_s[next] <= now) {
            hnsw_server *s = servers[server_of[next]];
            const float *q = queries[server_of[next]] + static_cast<size_t>(qidx[next]) * s->dim;
            const hnsw_status st = hnsw_server_submit(s, q, k[next], ef[next], mode[next], &ticket[next]);
            if (st == HNSW_ERR_BUSY) break;  // backpressure: keep polling, then retry
            if (st != HNSW_OK) return st;
            t_submit[next] = seconds_since(t0);
            inflight.push_back(next++);
        }
        for (size_t j = 0; j < inflight.size();) {
            const uint64_t i = inflight[j];
            int d = 0;
            const hnsw_status st = hnsw_server_poll(servers[server_of[i]], ticket[i],
                                                    ids ? ids + i * out_stride : nullptr,
                                                    dists ? dists + i * out_stride : nullptr, &d);
            if (st != HNSW_OK) return st;
            if (d) {
                t_done[i] = seconds_since(t0);
                ++done_count;
                inflight[j] = inflight.back();
                inflight.pop_back();
            } else {
                ++j;
            }
        }
    }
    return HNSW_OK;
}

}  // extern "C"
