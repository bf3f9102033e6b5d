"""Exact K-NN ground truth of a workload, computed by the oracle's brute force.

TEST INFRASTRUCTURE: writes ``graphs/<workload>_<n>.gt.npz`` holding, for the
first ``nq`` seeded queries, the ids of the K nearest base vectors in
(fp64 distance, id) order and their fp64 distances (Sec. 1's problem
statement).  The benchmark reads this file (it never runs the oracle) and the
tests check the GPU brute-force kernel against it.

    python -m oracle.ground_truth sift_like --n 1000000 --nq 10000 --k 100
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
from oracle.build_graph import PARAMS, graph_path  # noqa: E402


def gt_path(workload: str, n: int) -> str:
    return graph_path(workload, n)[:-4] + ".gt.npz"


def compute(workload: str, n: int, nq: int, k: int, threads: int) -> str:
    metric = PARAMS[workload][0]
    X = synthdata.base(workload, n)
    Q = synthdata.queries(workload, nq)
    t0 = time.time()
    ids, d64 = oracle.bruteforce(X, Q, k, metric=metric, nthreads=threads)
    out = gt_path(workload, n)
    np.savez(out, ids=ids, d64=d64, nq=nq, k=k, n=n)
    print(f"[{workload}] ground truth {nq} x {k} in {time.time() - t0:.0f}s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(PARAMS))
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--nq", type=int, default=10000)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    compute(a.workload, a.n, a.nq, a.k, a.threads)
