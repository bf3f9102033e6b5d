"""Build an HNSW graph with the oracle's INSERT (Alg. 1) and write it to a graph file.

TEST INFRASTRUCTURE: the graphs the GPU path searches come from here, so that
every graph (an input of the parity tests and of the benchmark) is produced by
the oracle and never by the GPU code under test.

    python -m oracle.build_graph sift_like --n 1000000 --out graphs/sift_like_1M.bin

Construction parameters per workload (M, Mmax0, efC; Mmax = M and
mL = 1/ln M throughout, Alg. 4 heuristic with both flags false):
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthdata  # noqa: E402

# workload -> (metric, M, Mmax0, efC, level seed)
PARAMS = {
    "uniform16": (oracle.L2, 16, 32, 100, 1003),
    "sift_like": (oracle.L2, 16, 32, 200, 2003),
    "glove_like": (oracle.IP, 16, 32, 200, 3004),
    "deep_like": (oracle.L2, 24, 48, 200, 4003),
    "uniform4": (oracle.L2, 16, 32, 200, 5003),
}


def graph_path(workload: str, n: int) -> str:
    tag = f"{n // 1000000}M" if n % 1000000 == 0 else (f"{n // 1000}k" if n % 1000 == 0 else str(n))
    return os.path.join(ROOT, "graphs", f"{workload}_{tag}.bin")


def build(workload: str, n: int, out: str | None = None, verbose: bool = True) -> str:
    metric, M, Mmax0, efC, seed = PARAMS[workload]
    out = out or graph_path(workload, n)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    X = synthdata.base(workload, n)
    t0 = time.time()

    def progress(a, b):
        if verbose:
            print(f"[{workload}] inserted {a}/{b}  {time.time() - t0:.0f}s", flush=True)

    g = oracle.Graph.build(X, progress=progress, chunk=max(1000, n // 100), metric=metric, M=M, Mmax=M,
                           Mmax0=Mmax0, efC=efC, mL=1.0 / math.log(M), seed=seed)
    oracle.save_graph(out, g)
    if verbose:
        print(f"[{workload}] wrote {out} in {time.time() - t0:.0f}s", flush=True)
    return out


def ensure(workload: str, n: int) -> str:
    """Path of the graph file, building it first if it is not there."""
    p = graph_path(workload, n)
    if not os.path.exists(p):
        build(workload, n, p, verbose=False)
    return p


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(PARAMS))
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    build(a.workload, a.n, a.out)
