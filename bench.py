"""Benchmark of batched HNSW K-NN-SEARCH on one MI355X.

Workload (default): the 1M x 128 SIFT-like Gaussian mixture (1,000 centres,
sigma 20, integer coordinates 0..255), graph built by the oracle's INSERT
with M = 16, Mmax0 = 32, efConstruction = 200; 10,000 seeded queries, K = 10.
A step is one batched search call over all 10,000 queries.  A batch larger
than the waves resident at once runs as three launches on one stream
(descent_kernel, order_kernel, layer0_kernel: every descent first, then
layer 0 with the queries whose descent ended farthest started first); the
HIP events bracket the whole call.

For every form of the search (plain fp32 traversal, BF16 and FP8-E4M3
traversal with an exact fp32 re-rank, and the learned early-termination
search where a trained net is given) the ef sweep picks the smallest swept
ef whose mean tie-aware recall@10 against exact brute force reaches 0.95;
that ef is timed.  `value` is the plain form's throughput; every form is
reported under `forms`.  Recall ground truth comes from the library's exact
brute-force kernel (checked against the oracle's brute force by the tests).
Printed: one JSON line.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload sift_like]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (graph file, base vectors, queries, K)
    "sift_like": ("graphs/sift_like_1M.bin", 1_000_000, 10_000, 10),
    "glove_like": ("graphs/glove_like_1200k.bin", 1_200_000, 10_000, 10),
    "deep_like": ("graphs/deep_like_1M.bin", 1_000_000, 10_000, 10),
    "uniform4": ("graphs/uniform4_1M.bin", 1_000_000, 10_000, 10),
}
EF_SWEEP = [10, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128, 160, 192, 256, 320, 384, 512, 640, 800]
# points of the recall / throughput curve (the workload's ef range, 10..800)
CURVE_EFS = [10, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 800]
HBM_PEAK_GBS = 8000.0
METRIC = "QPS at recall@10≥0.95, plain vs learned/low-precision; HBM GB/s"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("search.hip", "search_kernels.h", "search_device.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1603_09320_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


RECALL_SLACK = 1e-9


def recall(ids, X, Q, gt_d64, metric=0):
    """Tie-aware recall@K: an id counts when its fp64 distance is <= the true
    K-th.  The two fp64 sums (here and in the brute force) may add the same
    terms in different orders, which moves them by ~1e-16 relative; a slack of
    1e-9 relative keeps the true K-th neighbour from being counted as a miss
    (fp32 inputs cannot separate distances that close)."""
    K = ids.shape[1]
    out = []
    for s in range(0, len(ids), 10000):  # bounded memory for large batches
        i = ids[s:s + 10000]
        x = X[np.clip(i, 0, None)].astype(np.float64)
        q = Q[s:s + 10000, None, :].astype(np.float64)
        d = ((x - q) ** 2).sum(-1) if metric == 0 else 1.0 - (x * q).sum(-1)
        d[i < 0] = np.inf
        dk = gt_d64[s:s + 10000, K - 1:K]
        out.append((d <= dk + RECALL_SLACK * np.abs(dk) + 1e-12).sum(1) / K)
    return np.concatenate(out)


def row_bytes(mode: int, dim: int) -> int:
    """Bytes of one vector as the traversal reads it (values only, plus the FP8 scale)."""
    return {0: 4 * dim, 1: 2 * dim, 2: dim + 4, 3: 4 * dim, 4: dim}[mode]


def algorithmic_bytes(cnt, graph, K, mode, ef, includes_rerank, reranks=None):
    """Bytes the method must move per step: one adjacency row per expansion
    (layer 0: 4*Mmax0, upper layers: 4*Mmax), one vector per distance
    evaluation, the query and the K results; the low-precision forms add one
    fp32 row per re-ranked element of W.  ``cnt`` rows: distance evaluations
    (all layers), expansions (all layers), distance evaluations on layer 0,
    expansions on layer 0 -- the oracle's counts (exact visited sets) or the
    GPU's (which also count ids scored again after the visited table forgot
    them, descent neighbours scored again on each hop and, with
    ``includes_rerank``, the re-ranked elements)."""
    c = cnt.astype(np.int64)
    dim = graph["dim"]
    exp_u = c[:, 1] - c[:, 3]
    if reranks is None:
        reranks = mode in (1, 2, 4)
    rer = np.minimum(ef, graph["n"]) if reranks else 0
    trav = c[:, 0] - (rer if includes_rerank else 0)
    per_q = (c[:, 3] * 4 * graph["Mmax0"] + exp_u * 4 * graph["Mmax"] + trav * row_bytes(mode, dim)
             + rer * 4 * dim + 4 * dim + 8 * K)
    return int(per_q.sum())


def load_traffic(kernel_hash: str, workload: str, ef: int):
    """HBM bytes per launch measured by rocprofv3 counters, if taken on this exact kernel."""
    p = os.path.join(ROOT, "profiles", f"search_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        t = json.load(open(p))
    except Exception:
        return None
    if t.get("kernel_hash") != kernel_hash or int(t.get("ef", -1)) != ef:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(G, Q, K, ef, seconds=10.0):
    """The oracle's K-NN-SEARCH on the host over bounded query samples: one
    thread (the paper's regime) and every core the process may use."""
    out = {}
    for leg, threads in (("one_thread", 1), ("all_cores", host_cores())):
        n = min(len(Q), 32 * threads)
        t0 = time.time()
        G.search(Q[:n], K, ef, nthreads=threads)
        dt = time.time() - t0
        n2 = int(min(len(Q), max(n, n * seconds / max(dt, 1e-3) * 0.5)))
        if n2 > n:
            t0 = time.time()
            G.search(Q[:n2], K, ef, nthreads=threads)
            dt, n = time.time() - t0, n2
        out[leg] = {"value": round(n / dt, 2), "cores": threads, "queries": n, "seconds": round(dt, 2)}
        log(f"[bench] oracle {leg}: {out[leg]}")
    a = out["all_cores"]
    return {"value": a["value"], "unit": "queries/s", "cores": a["cores"], "kind": "oracle",
            "sample": f"first {a['queries']} of {len(Q)} queries, K={K}, ef={ef}, same graph; one thread: "
                      f"{out['one_thread']['value']} queries/s over the first {out['one_thread']['queries']}",
            "one_thread": out["one_thread"]["value"], "cpu_model": cpu_model()}


def oracle_counts(G, X, Q, K, ef, mode, mlp_file=None):
    """The oracle's per-query work counters at the same graph, queries and ef
    (untimed; the exact visited set of Alg. 2): plain search, the
    low-precision mirror, or the learned search with the same net."""
    import oracle

    threads = host_cores()
    if mode == 3:
        z = np.load(mlp_file)
        r = G.search_learned(Q, K, ef, net=oracle.bf16_net(z["params"]), tau=float(z["tau"]), jmax=int(z["jmax"]),
                             T=int(z["period"]), max_ckpt=int(z["max_ckpt"]), nthreads=threads)
        return r["counters"]
    if mode in (1, 2, 4):
        _, dec, sc = {1: oracle.quantize_bf16, 2: oracle.quantize_fp8, 4: oracle.quantize_u8}[mode](X)
        G.set_lowp(dec, sc)
    try:
        _, _, cnt = G.search(Q, K, ef, nthreads=threads, counters=True)
    finally:
        G.set_lowp(None, None)
    return cnt


class Runner:
    def __init__(self, index, q, X, Q, K, gt_d64, metric, stream, mlp=None):
        self.index, self.q, self.X, self.Q, self.K = index, q, X, Q, K
        self.gt, self.metric, self.stream, self.mlp = gt_d64, metric, stream, mlp

    def search(self, ef, mode, out=None, counters=False):
        return self.index.search(self.q, self.K, ef, mode=mode, mlp=self.mlp if mode == 3 else None,
                                 counters=counters, out=out)

    def sweep(self, mode, efs, target):
        import torch

        curve = []
        for ef in efs:
            ids, _ = self.search(ef, mode)
            torch.cuda.synchronize()
            r = float(recall(ids.cpu().numpy(), self.X, self.Q, self.gt, self.metric).mean())
            curve.append({"ef": ef, "recall": round(r, 5)})
            log(f"[bench] mode={mode} ef={ef} recall@{self.K}={r:.4f}")
            if r >= target:
                return ef, r, curve
        return curve[-1]["ef"], curve[-1]["recall"], curve

    def time(self, ef, mode, steps, warmup):
        import torch

        n = self.q.shape[0]
        dev = self.q.device
        ids = torch.empty((n, self.K), dtype=torch.int32, device=dev)
        dists = torch.empty((n, self.K), dtype=torch.float32, device=dev)
        # the library picks a batch's launch form by timing both on the first
        # calls of each (index, mode, ef, batch size) (one untimed call and two
        # timed calls of each form); these calls, each waited for, let it
        # decide before the warm-up and the timed steps
        for _ in range(8):
            self.search(ef, mode, out=(ids, dists))
            torch.cuda.synchronize()
        for _ in range(warmup):
            self.search(ef, mode, out=(ids, dists))
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for s, e in evs:
            s.record(self.stream)
            self.search(ef, mode, out=(ids, dists))
            e.record(self.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall * 1000.0 / steps, float(np.mean([s.elapsed_time(e) for s, e in evs]))


# Each server's persistent grid must stay resident next to the other's: the
# main index's kernel (plain, learned, BF16 and FP8 inlined) holds two waves
# per SIMD by its registers, and at ef_max = 512 a wave reserves 13.3 KB of
# LDS; 512 + 1024 waves fit together.
def serve_bench(hnsw, index, Q, mlp, rates=(50_000, 100_000, 200_000, 500_000), duration_s=2.5, warmup_s=0.5,
                seed=7):
    """Continuous-batching serving: an open-loop Poisson replay over two live
    servers, the main index (plain, learned when a net is loaded, BF16 and
    FP8 requests) and a 1M x 4 uniform index (built by the oracle, file
    graphs/uniform4_1M.bin; plain and BF16); per request K in {1, 10, 100}, ef
    uniform in [K, 512].  Each rate runs duration_s of arrivals; the
    statistics cover the requests that arrive after warmup_s (the steady
    state): p50/p99 latency (arrival to completion), completed requests per
    second, and the occupancy of the request slots (requests in flight between
    submission and completion: mean, p99 and peak, against the 4,096 slots of
    each server)."""
    import synthdata

    upath = os.path.join(ROOT, WORKLOADS["uniform4"][0])
    if not os.path.exists(upath):
        log(f"[serve] missing {upath}: serving measured over the main index alone")
        g4 = None
    else:
        g4 = hnsw.graphfile.read(upath)
    idx4 = hnsw.Index(g4, synthdata.base("uniform4", g4["n"])) if g4 else None
    Q4 = synthdata.queries("uniform4", 10_000) if g4 else None
    index.add_lowp(hnsw.MODE_BF16)
    index.add_lowp(hnsw.MODE_FP8)
    if idx4 is not None:
        idx4.add_lowp(hnsw.MODE_BF16)
    out = []
    rng = np.random.default_rng(seed)
    slots = 4096
    for rate in rates:
        # 512 waves for the main index (its kernel inlines every kind), 1024
        # for the uniform4 one: both grids are resident together
        servers = [hnsw.Server(index, mlp=mlp, slots=slots, waves=512, ef_max=512, k_max=100, budget_s=120.0)]
        if idx4 is not None:
            servers.append(hnsw.Server(idx4, mlp=None, slots=slots, waves=1024, ef_max=512, k_max=100,
                                       budget_s=120.0))
        n_req = int(rate * duration_s)
        try:
            arrival = np.cumsum(rng.exponential(1.0 / rate, n_req))
            server_of = rng.integers(0, len(servers), n_req).astype(np.uint32)
            qidx = rng.integers(0, len(Q), n_req).astype(np.uint32)
            k = rng.choice([1, 10, 100], n_req).astype(np.uint32)
            ef = rng.integers(k.astype(np.int64), 513).astype(np.uint32)
            modes = [0, 1, 2, 3] if mlp is not None else [0, 1, 2]
            mode = rng.choice(modes, n_req).astype(np.int32)
            mode[(mode == 3) & ((k > 64) | (server_of == 1))] = 0
            mode[(mode == 2) & (server_of == 1)] = 1
            qs = [Q] + ([Q4] if idx4 is not None else [])
            r = hnsw.replay(servers, qs, arrival, server_of, qidx, k, ef, mode, keep_results=False,
                            timeout_s=60.0)
        finally:
            for sv in servers:
                sv.stop()
        steady = arrival >= warmup_s
        lat = (r["t_done"][steady] - arrival[steady]) * 1e3
        ns = int(steady.sum())
        span = float(r["t_done"][steady].max() - arrival[steady][0])
        # requests in flight at each submission and completion instant (of the steady window)
        ev = np.concatenate([np.stack([r["t_submit"], np.ones(n_req)], 1), np.stack([r["t_done"], -np.ones(n_req)], 1)])
        ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]
        inflight = np.cumsum(ev[:, 1])[ev[:, 0] >= warmup_s]
        row = {"offered_rps": rate, "requests": n_req, "steady_requests": ns, "steady_s": round(duration_s - warmup_s, 2),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3), "completed_rps": round(ns / span, 1),
               "in_flight_mean": round(float(np.mean(inflight)), 1),
               "in_flight_p99": round(float(np.percentile(inflight, 99)), 1),
               "in_flight_max": int(inflight.max()), "slots": slots * len(servers)}
        log(f"[serve] {row}")
        out.append(row)
    if idx4 is not None:
        idx4.close()
    return {"indices": ["main index", "uniform4 1M x 4"] if idx4 is not None else ["main index"],
            "requests": "K in {1,10,100}, ef uniform in [K,512], modes plain/bf16/fp8 (main index), plain/bf16 "
                        "(uniform4)" + ("/learned (K<=64, main index)" if mlp is not None else ""),
            "rates": out}


def read_probe_bench(hnsw, gib=4, steps=10, warmup=3):
    """The attainable HBM read bandwidth: the library's streaming-read probe
    (16-byte loads, grid-stride) over `gib` GiB, timed with events (median of
    `steps`), at the best of several grid sizes."""
    import torch

    buf = torch.ones(gib << 28, dtype=torch.float32, device="cuda")
    nbytes = buf.numel() * 4
    stream = torch.cuda.current_stream()
    best = None
    for blocks in (2048, 8192, 16384, 32768, 65536):
        for _ in range(warmup):
            hnsw.read_probe(buf, blocks)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            hnsw.read_probe(buf, blocks)
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        gbs = nbytes / (ms / 1e3) / 1e9
        log(f"[probe] {blocks} blocks: {ms:.3f} ms, {gbs:.1f} GB/s")
        if best is None or gbs > best["GBs"]:
            best = {"GBs": round(gbs, 1), "blocks": blocks, "bytes": nbytes, "ms": round(ms, 4)}
    del buf
    return best


def learned_glove_bench(hnsw, steps=10, warmup=2, target=0.95, batches=(10_000, 100_000)):
    """The learned stop rule on glove_like 1.2M x 100 (inner product) with the
    net trained and calibrated for it: plain and learned are each timed at the
    smallest ef of a grid of step 16 that reaches recall@10 >= 0.95.  Two
    batch sizes: the 10,000 test queries in one call, and 100,000 queries of
    the same law in one call (a batch long enough that its last, longest
    searches are a small part of it).  recall_histogram[j]: the queries that
    found j of their K nearest."""
    import torch

    import synthdata

    path, n, nq0, K = WORKLOADS["glove_like"]
    gpath = os.path.join(ROOT, path)
    mpath = os.path.join(ROOT, "paper_1603_09320_amd", "nets", "glove_like.mlp.npz")
    if not (os.path.exists(gpath) and os.path.exists(mpath)):
        log("[glove] graph or net missing: skipped")
        return None
    g = hnsw.graphfile.read(gpath)
    X = synthdata.base("glove_like", g["n"])
    index = hnsw.Index(g, X)
    mlp = hnsw.Mlp.load(mpath)
    out = {"workload": f"glove_like {g['n']}x{g['dim']} inner product, K={K}", "target_recall": target,
           "net": {"tau": mlp.tau, "jmax": mlp.jmax, "period": mlp.period, "max_ckpt": mlp.max_ckpt}}
    for nq in batches:
        Q = synthdata.queries("glove_like", nq)
        q = torch.from_numpy(Q).cuda()
        _, gt = hnsw.bruteforce(index, q, K)
        torch.cuda.synchronize()
        run = Runner(index, q, X, Q, K, gt.cpu().numpy(), g["metric"], torch.cuda.current_stream(), mlp)
        efs = list(range(192, 513, 16))
        res = {"queries": nq}
        for form, mode in (("plain", 0), ("learned", 3)):
            ef, rec, _ = run.sweep(mode, efs, target)
            ids, _, cnt = run.search(ef, mode, counters=True)
            torch.cuda.synchronize()
            c = cnt.cpu().numpy().astype(np.float64)
            # per-query recall@K: how many queries found 0, 1, ..., K of their K nearest
            per_q = recall(ids.cpu().numpy(), X, Q, gt.cpu().numpy(), g["metric"])
            hist = np.bincount(np.rint(per_q * K).astype(np.int64), minlength=K + 1)
            ms, kern_ms = run.time(ef, mode, steps, warmup)
            res[form] = {"ef": ef, "recall": round(rec, 5), "qps": round(nq / (ms / 1000.0), 1),
                         "ms_per_batch": round(ms, 4), "kernel_ms": round(kern_ms, 4),
                         "layer0_expansions_per_query": round(float(c[:, 3].mean()), 2),
                         "distance_evals_per_query": round(float(c[:, 0].mean()), 1),
                         "recall_histogram": [int(v) for v in hist]}
            log(f"[glove] {nq} queries, {form}: {res[form]}")
        res["learned_vs_plain_qps"] = round(res["learned"]["qps"] / res["plain"]["qps"], 4)
        out[f"batch_{nq}"] = res
        del q
    mlp.close()
    index.close()
    return out


def deep10m_bench(hnsw, steps=10, warmup=2, n=10_000_000, nq=10_000, K=10, efs=(64, 128, 256)):
    """Low-precision traversal at its own size: 10M x 96 from the deep_like law
    (10,000 centres N(0, I), x = c + 0.5 g), graph built on the GPU by the
    library's batched INSERT (M = 24, Mmax0 = 48, efConstruction = 200); K =
    10, ef in {64, 128, 256}; fp32 traversal against BF16 and FP8-E4M3
    traversal with an exact fp32 re-rank; recall@10 against the exact brute
    force (fp64 re-rank of a matrix-core scan)."""
    import torch

    import synthdata

    t0 = time.time()
    X = synthdata.base("deep_like", n)
    Q = synthdata.queries("deep_like", nq)
    gen_s = time.time() - t0
    t0 = time.time()
    index = hnsw.Index.build(X, M=24, efC=200, seed=4003)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    info = index.info()
    log(f"[deep10m] generated in {gen_s:.1f} s, built in {build_s:.1f} s: L={info['max_level']}")
    q = torch.from_numpy(Q).cuda()
    stream = torch.cuda.current_stream()
    bs, be = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bs.record(stream)
    _, gt = hnsw.bruteforce(index, q, K)
    be.record(stream)
    torch.cuda.synchronize()
    bf_ms = bs.elapsed_time(be)
    gt = gt.cpu().numpy()
    run = Runner(index, q, X, Q, K, gt, 0, stream)
    graph = {"dim": 96, "n": n, "Mmax0": info["Mmax0"], "Mmax": info["Mmax"]}
    rows = {}
    for form, mode in (("plain", 0), ("bf16", 1), ("fp8", 2)):
        if mode:
            index.add_lowp(mode)
        for ef in efs:
            ids, _, cnt = run.search(ef, mode, counters=True)
            torch.cuda.synchronize()
            rec = float(recall(ids.cpu().numpy(), X, Q, gt).mean())
            ms, kern_ms = run.time(ef, mode, steps, warmup)
            alg = algorithmic_bytes(cnt.cpu().numpy().astype(np.uint32), graph, K, mode, ef, includes_rerank=True)
            r = {"recall": round(rec, 5), "qps": round(nq / (ms / 1000.0), 1), "ms_per_step": round(ms, 4),
                 "kernel_ms": round(kern_ms, 4), "gpu_count_GBs": round(alg / (kern_ms / 1000.0) / 1e9, 1)}
            if mode:
                r["recall_loss_vs_fp32"] = round(rows[f"plain_ef{ef}"]["recall"] - rec, 5)
                r["qps_vs_fp32"] = round(r["qps"] / rows[f"plain_ef{ef}"]["qps"], 4)
            rows[f"{form}_ef{ef}"] = r
            log(f"[deep10m] {form} ef={ef}: {r}")
    index.close()
    return {"workload": f"deep_like {n}x96 (10,000 centres, spread 0.5), {nq} queries, K={K}; graph built on the "
                        f"GPU: M=24, Mmax0=48, efConstruction=200",
            "build_s": round(build_s, 2), "bruteforce_ms": round(bf_ms, 1),
            "counts": "gpu (the oracle does not search device-built graphs)", "results": rows}


def _ef_for_recall(idx, q, X, Q, gt, K, target, efs, steps=5):
    """Smallest ef of the grid whose recall@K reaches the target, with its
    batch time (ms, mean of `steps` event-timed calls) and work counters."""
    import torch

    stream = torch.cuda.current_stream()
    run = Runner(idx, q, X, Q, K, gt, 0, stream)
    last = None
    for ef in efs:
        ids, _, cnt = run.search(ef, 0, counters=True)
        torch.cuda.synchronize()
        r = float(recall(ids.cpu().numpy(), X, Q, gt).mean())
        last = (ef, r, cnt)
        if r >= target:
            break
    ef, r, cnt = last
    _, kern = run.time(ef, 0, steps, 2)
    c = cnt.cpu().numpy().astype(np.float64)
    return {"ef": ef, "recall": round(r, 4), "ms_per_batch": round(kern, 4),
            "us_per_query": round(kern * 1000.0 / len(Q), 4), "dist_evals": round(float(c[:, 0].mean()), 1),
            "reached": bool(r >= target)}


def paper_experiments(hnsw, which=None):
    """The paper's synthetic-data experiments (Sec. 4.1, Figs. 3, 6, 7, 11 and
    the distance-count scaling of Sec. 5.1), on graphs built by the library on
    the GPU; query time per query of a 10,000-query batch at the smallest ef
    reaching the recall target.
      fig3: query time vs mL on random d = 4 vectors (10M), M = 6, with the
            heuristic (Alg. 4) and with the M nearest (Alg. 3), at recall 0.95
            and 0.99;
      fig6: query time vs Mmax0 on the 1M sift_like set (M = 16), at recall
            0.95 and 0.99;
      fig7: Alg. 3 against Alg. 4, and Alg. 4 with extendCandidates, on 1M
            d = 10 vectors, uniform and from 100 isolated clusters, at recall
            0.9, 0.95 and 0.99;
      fig11: the ef needed for recall 0.9 / 0.99 (10-NN) vs the set size, d = 4;
      distance evaluations per query against recall (10M, d = 4) and, at
      recall 0.95, against the set size (d = 8, 100k to 10M).
    which: names of the experiments to run (fig3, fig6, fig7, fig11, scaling);
    all when None."""
    import torch

    import synthdata

    efs = [10, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512, 640, 800, 1024]
    out = {}

    def setup(workload, n, nq=10000, K=10):
        X = synthdata.base(workload, n)
        Q = synthdata.queries(workload, nq)
        return X, Q

    def gt_of(idx, q, K):
        _, gt = hnsw.bruteforce(idx, q, K)
        torch.cuda.synchronize()
        return gt.cpu().numpy()

    def want(name):
        return which is None or name in which

    # Fig. 3: mL on 10M random d=4
    if want("fig3"):
        fig3(hnsw, setup, gt_of, out)
    if want("fig6"):
        fig6(hnsw, setup, gt_of, efs, out)
    if want("fig7"):
        fig7(hnsw, setup, gt_of, efs, out)
    if want("fig11"):
        fig11(hnsw, setup, gt_of, out)
    if want("scaling"):
        scaling_d8(hnsw, setup, gt_of, out)
    return out


def fig3(hnsw, setup, gt_of, out):
    import math

    import torch

    X, Q = setup("uniform4", 10_000_000)
    q = torch.from_numpy(Q).cuda()
    rows = []
    gt = None
    for heur in (True, False):
        for mL in (0.0, 0.2, 0.4, 1.0 / math.log(6), 0.8, 1.2):
            t0 = time.time()
            idx = hnsw.Index.build(X, M=6, Mmax0=12, efC=100, mL=mL, seed=5003, heuristic=heur)
            torch.cuda.synchronize()
            bt = time.time() - t0
            if gt is None:
                gt = gt_of(idx, q, 10)
            for target in (0.95, 0.99):
                r = _ef_for_recall(idx, q, X, Q, gt, 10, target, list(range(10, 65, 2)))
                r.update(mL=round(mL, 4), selection="heuristic" if heur else "simple", build_s=round(bt, 2),
                         layers=idx.info()["max_level"] + 1, target=target)
                log(f"[fig3] {r}")
                rows.append(r)
            idx.close()
    out["fig3_mL_uniform4_10M"] = {"M": 6, "Mmax0": 12, "efC": 100, "K": 10, "rows": rows}


def fig6(hnsw, setup, gt_of, efs, out):
    import torch

    X, Q = setup("sift_like", 1_000_000)
    q = torch.from_numpy(Q).cuda()
    rows = []
    gt = None
    for m0 in (16, 24, 32, 48, 64):
        idx = hnsw.Index.build(X, M=16, Mmax0=m0, efC=200, seed=2003)
        if gt is None:
            gt = gt_of(idx, q, 10)
        for target in (0.95, 0.99):
            r = _ef_for_recall(idx, q, X, Q, gt, 10, target, efs)
            r.update(Mmax0=m0, target=target)
            log(f"[fig6] {r}")
            rows.append(r)
        idx.close()
    out["fig6_Mmax0_sift_like_1M"] = {"M": 16, "efC": 200, "K": 10, "rows": rows}


def fig7(hnsw, setup, gt_of, efs, out):
    """Neighbour selection on clustered and uniform d = 10: the M nearest
    (Alg. 3), the heuristic (Alg. 4), and the heuristic with extendCandidates."""
    import torch

    rows = []
    for wl in ("uniform10", "clustered10"):
        X, Q = setup(wl, 1_000_000)
        q = torch.from_numpy(Q).cuda()
        gt = None
        for sel in ("heuristic", "simple", "heuristic+extend"):
            t0 = time.time()
            idx = hnsw.Index.build(X, M=8, efC=100, seed=6003, heuristic=sel != "simple",
                                   extend=sel == "heuristic+extend")
            torch.cuda.synchronize()
            bt = time.time() - t0
            if gt is None:
                gt = gt_of(idx, q, 10)
            for target in (0.9, 0.95, 0.99):
                r = _ef_for_recall(idx, q, X, Q, gt, 10, target, efs)
                r.update(data=wl, selection=sel, build_s=round(bt, 2), target=target)
                log(f"[fig7] {r}")
                rows.append(r)
            idx.close()
    out["fig7_selection_d10_1M"] = {"M": 8, "Mmax0": 16, "efC": 100, "K": 10, "rows": rows}


def fig11(hnsw, setup, gt_of, out):
    import torch

    # Fig. 11: ef needed for a fixed recall vs N, d=4
    rows = []
    for n in (10_000, 100_000, 1_000_000, 10_000_000):
        X, Q = setup("uniform4", n)
        q = torch.from_numpy(Q).cuda()
        idx = hnsw.Index.build(X, M=6, Mmax0=12, efC=100, seed=5003)
        gt = gt_of(idx, q, 10)
        for target in (0.9, 0.99):
            r = _ef_for_recall(idx, q, X, Q, gt, 10, target, list(range(10, 401, 2)), steps=3)
            r.update(n=n, target=target)
            log(f"[fig11] {r}")
            rows.append(r)
        if n == 10_000_000:
            # distance evaluations against recall on the largest set (Sec. 5.1)
            curve = []
            run = Runner(idx, q, X, Q, 10, gt, 0, torch.cuda.current_stream())
            for ef in (10, 12, 16, 20, 24, 32, 48, 64, 96, 128):
                ids, _, cnt = run.search(ef, 0, counters=True)
                torch.cuda.synchronize()
                curve.append({"ef": ef, "recall": round(float(recall(ids.cpu().numpy(), X, Q, gt).mean()), 4),
                              "dist_evals": round(float(cnt.cpu().numpy()[:, 0].astype(np.float64).mean()), 1)})
            log(f"[dist-vs-recall] {curve}")
            out["dist_evals_vs_recall_uniform4_10M"] = {"M": 6, "Mmax0": 12, "efC": 100, "K": 10, "curve": curve}
        idx.close()
    out["fig11_ef_vs_n_uniform4"] = {"M": 6, "Mmax0": 12, "efC": 100, "K": 10, "rows": rows}


def scaling_d8(hnsw, setup, gt_of, out):
    import torch

    # distance evaluations at recall 0.95 against the set size, d = 8 (Sec. 5.1)
    rows = []
    for n in (100_000, 1_000_000, 10_000_000):
        X, Q = setup("uniform8", n)
        q = torch.from_numpy(Q).cuda()
        idx = hnsw.Index.build(X, M=8, Mmax0=16, efC=100, seed=8003)
        gt = gt_of(idx, q, 10)
        r = _ef_for_recall(idx, q, X, Q, gt, 10, 0.95, list(range(10, 201, 2)), steps=3)
        r.update(n=n, layers=idx.info()["max_level"] + 1)
        log(f"[scaling-d8] {r}")
        rows.append(r)
        idx.close()
    out["dist_evals_vs_n_uniform8"] = {"M": 8, "Mmax0": 16, "efC": 100, "K": 10, "target": 0.95, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sift_like", choices=sorted(WORKLOADS))
    ap.add_argument("--ef", type=int, default=0, help="time this ef for every form instead of sweeping")
    ap.add_argument("--forms", default="plain,bf16,fp8,u8,learned",
                    help="comma list of plain,bf16,fp8,u8,learned (learned needs a trained net file)")
    ap.add_argument("--target-recall", type=float, default=0.95)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle legs (host timing and the oracle's work counts)")
    ap.add_argument("--no-k1", action="store_true", help="skip the K = 1 measurement")
    ap.add_argument("--no-curve", action="store_true",
                    help="skip the recall / throughput curve over ef 10..800 (skipped with --ef too)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-glove", action="store_true", help="skip the learned-rule measurement on glove_like")
    ap.add_argument("--no-deep10m", action="store_true",
                    help="skip the 10M x 96 low-precision measurement (graph built on the GPU)")
    ap.add_argument("--paper-experiments", action="store_true",
                    help="run the paper's synthetic-data experiments (Figs. 3, 6, 7, 11) instead; prints their JSON")
    ap.add_argument("--experiments", default="",
                    help="with --paper-experiments: comma list of fig3,fig6,fig7,fig11,scaling (default all)")
    ap.add_argument("--copy-probe-bytes", type=int, default=0,
                    help="also run a plain device-to-device copy of this size (counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the path shards by queries over replicated indices; not built here)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1603_09320_amd as hnsw
    import synthdata

    if a.paper_experiments:
        torch.cuda.set_device(0)
        which = set(a.experiments.split(",")) if a.experiments else None
        print(json.dumps({"paper_experiments": paper_experiments(hnsw, which)}), flush=True)
        return
    path, n, nq, K = WORKLOADS[a.workload]
    gpath = os.path.join(ROOT, path)
    if not os.path.exists(gpath):
        log(f"missing graph file {gpath}: build it with  python -m oracle.build_graph {a.workload} --n {n}")
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    graph = hnsw.graphfile.read(gpath)
    X = synthdata.base(a.workload, graph["n"])
    Q = synthdata.queries(a.workload, nq)
    log(f"[bench] {a.workload}: n={graph['n']} dim={graph['dim']} nq={nq} K={K} L={graph['max_level']}")
    index = hnsw.Index(graph, X)
    q = torch.from_numpy(Q).to(dev)
    stream = torch.cuda.current_stream()

    # exact ground truth on the GPU (matrix-core scan + fp64 rerank), timed
    hnsw.bruteforce(index, q[:64], K)
    torch.cuda.synchronize()
    bs, be = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    bs.record(stream)
    _, gt_d = hnsw.bruteforce(index, q, K)
    be.record(stream)
    torch.cuda.synchronize()
    bf_ms = bs.elapsed_time(be)
    gt_d64 = gt_d.cpu().numpy()
    log(f"[bench] brute-force ground truth: {nq} queries in {bf_ms:.1f} ms")

    mlp = None
    mpath = os.path.join(ROOT, "paper_1603_09320_amd", "nets", f"{a.workload}.mlp.npz")
    forms = [f for f in a.forms.split(",") if f]
    if "learned" in forms:
        if os.path.exists(mpath) and hasattr(hnsw, "Mlp"):
            mlp = hnsw.Mlp.load(mpath)
        else:
            forms.remove("learned")
    run = Runner(index, q, X, Q, K, gt_d64, graph["metric"], stream, mlp)
    mode_of = {"plain": 0, "bf16": 1, "fp8": 2, "learned": 3, "u8": 4}
    results = {}
    gpu_cnt = {}
    rerank_of = {0: False, 1: True, 2: True, 3: False, 4: True}
    for form in forms:
        mode = mode_of[form]
        if mode in (1, 2, 4):
            index.add_lowp(mode)
        if mode == 4:
            rerank_of[4] = not index.read_lowp(4)[1]  # an exact 8-bit copy needs no re-rank
        if a.ef:
            ids, _ = run.search(a.ef, mode)
            torch.cuda.synchronize()
            ef, rec = a.ef, float(recall(ids.cpu().numpy(), X, Q, gt_d64, graph["metric"]).mean())
            curve = [{"ef": ef, "recall": round(rec, 5)}]
        else:
            ef, rec, curve = run.sweep(mode, EF_SWEEP, a.target_recall)
        _, _, cnt = run.search(ef, mode, counters=True)
        torch.cuda.synchronize()
        cnt = cnt.cpu().numpy().astype(np.uint32)
        gpu_cnt[form] = cnt
        ms, kern_ms = run.time(ef, mode, a.steps, a.warmup)
        alg = algorithmic_bytes(cnt, graph, K, mode, ef, includes_rerank=True, reranks=rerank_of[mode])
        c = cnt.astype(np.float64)
        results[form] = {"ef": ef, "recall": round(rec, 5), "qps": round(nq / (ms / 1000.0), 1),
                         "ms_per_step": round(ms, 4), "kernel_ms": round(kern_ms, 4),
                         "gpu_count_bytes_per_step": alg,
                         "gpu_count_GBs": round(alg / (kern_ms / 1000.0) / 1e9, 1),
                         "gpu_dist_evals_per_query": round(float(c[:, 0].mean()), 2),
                         "expansions_per_query": round(float(c[:, 1].mean()), 2),
                         "layer0_expansions_per_query": round(float(c[:, 3].mean()), 2),
                         "sweep": curve}
        if form == "plain":
            # both launch forms forced, to show which one the library picked
            fm = {}
            for name, val in (("one_kernel", "0"), ("scheduled", "2")):
                os.environ["HNSW_SCHEDULE"] = val
                try:
                    fm[name] = round(run.time(ef, mode, max(5, a.steps // 2), a.warmup)[1], 4)
                finally:
                    del os.environ["HNSW_SCHEDULE"]
            fm["chosen"] = min(("one_kernel", "scheduled"), key=lambda k: abs(fm[k] - kern_ms))
            results[form]["launch_forms_kernel_ms"] = fm
        log(f"[bench] {form}: {results[form]}")

    # the K = 1 half of the workload: plain fp32, recall@1 against the exact nearest neighbour
    k1 = None
    if not a.no_k1 and "plain" in forms:
        run1 = Runner(index, q, X, Q, 1, gt_d64[:, :1], graph["metric"], stream)
        ef1, rec1, curve1 = run1.sweep(0, EF_SWEEP, a.target_recall)
        ms1, kern1 = run1.time(ef1, 0, a.steps, a.warmup)
        k1 = {"ef": ef1, "recall_at_1": round(rec1, 5), "qps": round(nq / (ms1 / 1000.0), 1),
              "ms_per_step": round(ms1, 4), "kernel_ms": round(kern1, 4), "sweep": curve1}
        log(f"[bench] plain K=1: {k1}")

    # the recall / throughput trade-off over ef 10..800, plain fp32 and the 8-bit
    # copy (not with --ef, which times one ef only)
    curves = None
    if not a.no_curve and not a.ef:
        curves = {}
        for form in [f for f in ("plain", "u8") if f in forms]:
            pts = []
            for ef in CURVE_EFS:
                ids, _ = run.search(ef, mode_of[form])
                torch.cuda.synchronize()
                r = float(recall(ids.cpu().numpy(), X, Q, gt_d64, graph["metric"]).mean())
                ms, kern = run.time(ef, mode_of[form], 5, 1)
                pts.append({"ef": ef, "recall": round(r, 5), "qps": round(nq / (ms / 1000.0), 1),
                            "kernel_ms": round(kern, 4)})
            curves[form] = pts
            log(f"[bench] curve {form}: {pts}")

    if a.copy_probe_bytes:
        src = torch.ones(a.copy_probe_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {a.copy_probe_bytes} bytes read and written, twice")
        del src, dst

    serving = None
    if not a.no_serve:
        serving = serve_bench(hnsw, index, Q, mlp)
    glove = None
    if not a.no_glove and a.workload == "sift_like":
        glove = learned_glove_bench(hnsw)
    deep = None
    if not a.no_deep10m and a.workload == "sift_like":
        deep = deep10m_bench(hnsw)

    head = results.get("plain") or next(iter(results.values()))
    cpu = None
    counts = "gpu"
    if not a.no_cpu_baseline:
        import oracle

        G = oracle.Graph.from_packed(X, graph)
        cpu = cpu_baseline(G, Q, K, head["ef"])
        log(f"[bench] cpu baseline: {cpu}")
        # algorithmic bytes from the oracle's counts (exact visited sets) at each form's ef
        for form, r in results.items():
            oc = oracle_counts(G, X, Q, K, r["ef"], mode_of[form], mpath if form == "learned" else None)
            alg = algorithmic_bytes(oc, graph, K, mode_of[form], r["ef"], includes_rerank=False,
                                    reranks=rerank_of[mode_of[form]])
            oc = oc.astype(np.float64)
            r["bytes_per_step"] = alg
            r["algorithmic_GBs"] = round(alg / (r["kernel_ms"] / 1000.0) / 1e9, 1)
            r["dist_evals_per_query"] = round(float(oc[:, 0].mean()), 2)
            r["oracle_expansions_equal"] = bool(np.array_equal(oc[:, 1], gpu_cnt[form][:, 1].astype(np.float64)))
            log(f"[bench] {form}: oracle counts {r['dist_evals_per_query']} distance evaluations per query, "
                f"{r['algorithmic_GBs']} GB/s algorithmic")
        counts = "oracle"
        del G
    if counts == "gpu":
        for r in results.values():
            r["bytes_per_step"] = r["gpu_count_bytes_per_step"]
            r["algorithmic_GBs"] = r["gpu_count_GBs"]
    khash = kernel_source_hash()
    achieved = head["algorithmic_GBs"]
    # the attainable read bandwidth (not with --ef, which times one ef only)
    probe = None if a.ef else read_probe_bench(hnsw)
    traffic = load_traffic(khash, a.workload, head["ef"])
    out = {
        "metric": METRIC,
        "value": head["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload} {graph['n']}x{graph['dim']}, {nq} queries, K={K}, plain fp32 "
                               f"traversal at the smallest swept ef with recall@{K}>=0.95",
                   "ef": head["ef"], "recall": head["recall"], "M": graph["M"], "Mmax0": graph["Mmax0"],
                   "efConstruction": graph["efC"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_kind": "L2-to-fabric bytes per call (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a "
                                     "plain copy); they include hits in the Infinity Cache (MALL)",
                     "kernel": ("search call: descent_kernel + order_kernel + layer0_kernel (one stream, "
                                "event-timed together)"
                                if head.get("launch_forms_kernel_ms", {}).get("chosen", "scheduled") == "scheduled"
                                else "search call: search_kernel (one launch, event-timed)"),
                     "kernel_ms": head["kernel_ms"],
                     "algorithmic_bytes_per_launch": head["bytes_per_step"], "counts": counts,
                     "kernel_hash": khash,
                     "attainable_read": probe,
                     # algorithmic bytes include hits in L2 and the Infinity Cache, so this can exceed 1
                     "frac_of_attainable_read": round(achieved / probe["GBs"], 4) if probe else None,
                     # the counted L2-to-fabric bytes over the same time, against the same probe
                     "traffic_GBs": round(traffic / (head["kernel_ms"] / 1e3) / 1e9, 1) if traffic else None,
                     "traffic_frac_of_attainable_read": (round(traffic / (head["kernel_ms"] / 1e3) / 1e9 / probe["GBs"], 4)
                                                         if traffic and probe else None)},
        "forms": results,
        "plain_k1": k1,
        "recall_qps_curve": curves,
        "bruteforce": {"ms": round(bf_ms, 3), "queries": nq,
                       "tflops": round(2.0 * nq * graph["n"] * graph["dim"] / (bf_ms / 1000.0) / 1e12, 2)},
        "cpu_baseline": cpu,
        "serving": serving,
        "learned_glove_like": glove,
        "lowp_deep_10m": deep,
    }
    print(json.dumps(out), flush=True)
    index.close()


if __name__ == "__main__":
    main()
