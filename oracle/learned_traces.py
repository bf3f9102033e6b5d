"""Training traces for the learned stop rule, from the oracle's K-NN-SEARCH.

TEST INFRASTRUCTURE: the oracle searches seeded training queries (a seed
disjoint from the evaluation queries) on the oracle-built graph with ef = ef_cap
and records, every `period` layer-0 expansions, the 24 checkpoint features and
the top-K list.  Labels per sampled checkpoint (y0, c, y1, m):
  y0 = 1 when the top-K set at the checkpoint already equals the final top-K set
       of the full search (stopping there loses nothing), else 0; c = 1;
  y1 = -j* at the first checkpoint (m = 1), where j* is the largest number of
       halvings of ef_cap (at most jmax) for which a plain search returns the same
       top-K set as ef_cap (and so do all fewer halvings); m = 0 elsewhere.

    python -m oracle.learned_traces glove_like --nq 100000 --ef 512 --out graphs/glove_like.traces.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthdata  # noqa: E402
from oracle.build_graph import graph_path  # noqa: E402

N_OF = {"glove_like": 1200000, "sift_like": 1000000, "deep_like": 1000000, "uniform4": 1000000}


def make(workload, nq, ef, K=10, period=8, max_ckpt=64, jmax=5, per_query=7, threads=None, seed=0, log=print):
    threads = threads or os.cpu_count() or 1
    p = oracle.load_graph(graph_path(workload, N_OF[workload]))
    X = synthdata.base(workload, p["n"])
    G = oracle.Graph.from_packed(X, p)
    Q = synthdata.queries(workload, nq, train=True)
    t0 = time.time()
    r = G.search_learned(Q, K, ef, T=period, max_ckpt=max_ckpt, trace=True, nthreads=threads)
    log(f"[traces] traced search of {nq} queries at ef={ef}: {time.time() - t0:.0f}s")
    final = [set(row) for row in r["ids"]]
    same = np.ones(nq, dtype=bool)
    jstar = np.zeros(nq, dtype=np.int32)
    for j in range(1, jmax + 1):
        e = max(K, ef >> j)
        ids, _ = G.search(Q, K, e, nthreads=threads)
        same &= np.array([set(ids[i]) == final[i] for i in range(nq)])
        jstar[same] = j
    log(f"[traces] ef sweep done: {time.time() - t0:.0f}s; mean j* {jstar.mean():.2f}")
    rng = np.random.default_rng(seed)
    feats, labels = [], []
    for i in range(nq):
        n_ck = int(r["info"][i, 0])
        if n_ck == 0:
            continue
        picks = [0]
        if n_ck > 1:
            picks += list(rng.choice(np.arange(1, n_ck), size=min(per_query - 1, n_ck - 1), replace=False))
        for k in picks:
            y0 = float(set(r["topk"][i, k]) == final[i])
            feats.append(r["feat"][i, k])
            labels.append((y0, 1.0, -float(jstar[i]) if k == 0 else 0.0, 1.0 if k == 0 else 0.0))
    F = np.asarray(feats, dtype=np.float32)
    Y = np.asarray(labels, dtype=np.float32)
    log(f"[traces] {len(F)} samples, stop-positive fraction {Y[:, 0].mean():.3f}")
    return F, Y, dict(workload=workload, nq=nq, ef=ef, K=K, period=period, max_ckpt=max_ckpt, jmax=jmax)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(N_OF))
    ap.add_argument("--nq", type=int, default=100000)
    ap.add_argument("--ef", type=int, default=512)
    ap.add_argument("--out", required=True)
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--period", type=int, default=8, help="layer-0 expansions between checkpoints")
    ap.add_argument("--max-ckpt", type=int, default=64)
    a = ap.parse_args()
    F, Y, meta = make(a.workload, a.nq, a.ef, period=a.period, max_ckpt=a.max_ckpt, threads=a.threads)
    np.savez(a.out, feats=F, labels=Y, **meta)
    print(f"[traces] wrote {a.out}", flush=True)
