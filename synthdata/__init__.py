"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no part of the search method: it only draws base and query
vectors.  Both the CPU oracle's tests and the GPU path's tests and benchmark
take their inputs from here, so that the two sides see identical bytes.

Workloads (stand-ins for the paper's datasets, which are not available):

* ``uniform16``   -- 10,000 x 16 i.i.d. U[0,1) fp32 base, 1,000 queries.  Stand-in
  for the random hypercube sets of Sec. 5.1 / Table 1 ("Random vectors").
* ``sift_like``   -- 1,000,000 x 128 Gaussian mixture, 1,000 centres U[0,255]^128,
  sigma 20, rounded half-to-even and clamped to the integers 0..255, stored fp32;
  10,000 queries from the same mixture.  Stand-in for SIFT 1M (Table 1).
* ``glove_like``  -- 1,200,000 x 100 unit vectors from 2,000 clusters with
  Zipf(1.1) sizes, x = normalise(mu + 0.6 (s * g) / 10) with a decaying spread
  profile s_j proportional to j^-0.25 (j = 1..100, mean square 1), so that the
  within-cluster spread is concentrated in fewer directions than an isotropic
  one; inner-product metric.  Stand-in for GloVe 1.2M angular (Table 1).
* ``deep_like``   -- d=96 Gaussian mixture with 10,000 centres N(0, I) and spread
  0.5.  Stand-in for DEEP (Table 1).
* ``uniform4``    -- 1,000,000 x 4 U[0,1).  Stand-in for the d=4 random sets
  (Sec. 4.1, Table 1).
* ``uniform8``    -- d=8 U[0,1): the random set of the paper's scaling of the
  distance count with the set size (Sec. 5.1).
* ``uniform10`` / ``clustered10`` -- d=10 random vectors, U[0,1) or drawn from
  100 isolated clusters (centres U[0,1)^10, each point a centre plus 0.02 g),
  the two data sets of the paper's comparison of neighbour selection methods
  (Sec. 4.1).

Every array is float32, C-contiguous, shape [n][d].  Generation is chunked
with fixed chunk sizes and separate PCG64 streams per purpose, so the bytes
depend only on (workload, seed, n) and never on available memory.
"""
from __future__ import annotations

import numpy as np

CHUNK = 65536

# Seeds per workload: (mixture/centres, base, queries, train queries).
SEEDS = {
    "uniform16": dict(base=1001, queries=1002, train=1004),
    "sift_like": dict(mix=2000, base=2001, queries=2002, train=2004),
    "glove_like": dict(mix=3000, base=3001, queries=3002, train=3003),
    "deep_like": dict(mix=4000, base=4001, queries=4002, train=4004),
    "uniform4": dict(base=5001, queries=5002, train=5004),
    "uniform10": dict(base=6001, queries=6002, train=6004),
    "uniform8": dict(base=8001, queries=8002, train=8004),
    "clustered10": dict(mix=7000, base=7001, queries=7002, train=7004),
}

DIMS = {"uniform16": 16, "sift_like": 128, "glove_like": 100, "deep_like": 96, "uniform4": 4, "uniform10": 10,
        "clustered10": 10, "uniform8": 8}
METRIC = {"uniform16": "l2", "sift_like": "l2", "glove_like": "ip", "deep_like": "l2", "uniform4": "l2",
          "uniform10": "l2", "clustered10": "l2", "uniform8": "l2"}


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def _uniform(n: int, d: int, seed: int) -> np.ndarray:
    g = _rng(seed, 0)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        out[s:e] = g.random((e - s, d), dtype=np.float64).astype(np.float32)
    return out


def _sift_centres(seed: int) -> np.ndarray:
    return _rng(seed, 0).uniform(0.0, 255.0, size=(1000, 128))


def _sift_points(n: int, seed: int, centres: np.ndarray) -> np.ndarray:
    ga, gn = _rng(seed, 1), _rng(seed, 2)
    out = np.empty((n, 128), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        j = ga.integers(0, centres.shape[0], size=e - s)
        x = centres[j] + 20.0 * gn.standard_normal((e - s, 128))
        out[s:e] = np.clip(np.rint(x), 0.0, 255.0).astype(np.float32)
    return out


def _glove_mixture(seed: int):
    g = _rng(seed, 0)
    mu = g.standard_normal((2000, 100))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    w = np.arange(1, 2001, dtype=np.float64) ** -1.1
    return mu, w / w.sum()


GLOVE_SPREAD_DECAY = 0.25


def _glove_profile() -> np.ndarray:
    """Per-coordinate spread s_j = c * j^-0.25, scaled to mean square 1."""
    s = np.arange(1, 101, dtype=np.float64) ** -GLOVE_SPREAD_DECAY
    return s * np.sqrt(100.0 / np.sum(s * s))


def _glove_points(n: int, seed: int, mix, sigma: float = 0.6) -> np.ndarray:
    mu, w = mix
    ga, gn = _rng(seed, 1), _rng(seed, 2)
    counts = ga.multinomial(n, w)
    labels = np.repeat(np.arange(len(w)), counts)
    ga.shuffle(labels)
    prof = _glove_profile()
    out = np.empty((n, 100), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        x = mu[labels[s:e]] + sigma * (gn.standard_normal((e - s, 100)) * prof) / 10.0
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = x.astype(np.float32)
    return out


def _deep_centres(seed: int) -> np.ndarray:
    return _rng(seed, 0).standard_normal((10000, 96))


def _deep_points(n: int, seed: int, centres: np.ndarray) -> np.ndarray:
    ga, gn = _rng(seed, 1), _rng(seed, 2)
    out = np.empty((n, 96), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        j = ga.integers(0, centres.shape[0], size=e - s)
        out[s:e] = (centres[j] + 0.5 * gn.standard_normal((e - s, 96))).astype(np.float32)
    return out


def _clustered_points(n: int, seed: int, mix_seed: int) -> np.ndarray:
    centres = _rng(mix_seed, 0).random((100, 10))
    ga, gn = _rng(seed, 1), _rng(seed, 2)
    out = np.empty((n, 10), dtype=np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        j = ga.integers(0, 100, size=e - s)
        out[s:e] = (centres[j] + 0.02 * gn.standard_normal((e - s, 10))).astype(np.float32)
    return out


def base(workload: str, n: int) -> np.ndarray:
    """The first ``n`` base vectors of ``workload`` (prefix-stable in n only per CHUNK)."""
    sd = SEEDS[workload]
    if workload == "uniform16":
        return _uniform(n, 16, sd["base"])
    if workload == "uniform4":
        return _uniform(n, 4, sd["base"])
    if workload == "uniform10":
        return _uniform(n, 10, sd["base"])
    if workload == "uniform8":
        return _uniform(n, 8, sd["base"])
    if workload == "clustered10":
        return _clustered_points(n, sd["base"], sd["mix"])
    if workload == "sift_like":
        return _sift_points(n, sd["base"], _sift_centres(sd["mix"]))
    if workload == "glove_like":
        return _glove_points(n, sd["base"], _glove_mixture(sd["mix"]))
    if workload == "deep_like":
        return _deep_points(n, sd["base"], _deep_centres(sd["mix"]))
    raise KeyError(workload)


def queries(workload: str, n: int, train: bool = False) -> np.ndarray:
    """``n`` query vectors drawn from the same law as the base set.

    ``train=True`` selects a disjoint seed used for training traces.
    """
    sd = SEEDS[workload]
    seed = sd["train"] if train else sd["queries"]
    if workload == "uniform16":
        return _uniform(n, 16, seed)
    if workload == "uniform4":
        return _uniform(n, 4, seed)
    if workload == "uniform10":
        return _uniform(n, 10, seed)
    if workload == "uniform8":
        return _uniform(n, 8, seed)
    if workload == "clustered10":
        return _clustered_points(n, seed, sd["mix"])
    if workload == "sift_like":
        return _sift_points(n, seed, _sift_centres(sd["mix"]))
    if workload == "glove_like":
        return _glove_points(n, seed, _glove_mixture(sd["mix"]))
    if workload == "deep_like":
        return _deep_points(n, seed, _deep_centres(sd["mix"]))
    raise KeyError(workload)


def random_graph(n: int, degree: int, seed: int, dim: int = 4, tie_grid: int = 0, repeat_frac: float = 0.0):
    """A random directed graph plus points, for equivalence checks on tiny inputs.

    Returns ``(X, adj)`` where ``adj`` is uint32 [n][degree] padded with
    0xFFFFFFFF.  With ``tie_grid > 0`` the coordinates are integers in
    [0, tie_grid), which makes equal distances (ties) common.  With
    ``repeat_frac > 0`` about that fraction of each list's later links are
    overwritten by copies of earlier links of the same list (a list naming one
    element twice), drawn from a stream of their own.
    """
    g = _rng(seed, 7)
    if tie_grid:
        X = g.integers(0, tie_grid, size=(n, dim)).astype(np.float32)
    else:
        X = g.random((n, dim), dtype=np.float64).astype(np.float32)
    adj = np.full((n, degree), 0xFFFFFFFF, dtype=np.uint32)
    for i in range(n):
        k = int(g.integers(1, degree + 1))
        nb = g.choice(n - 1, size=min(k, n - 1), replace=False)
        nb = np.where(nb >= i, nb + 1, nb)
        adj[i, : len(nb)] = nb
    if repeat_frac > 0:
        gr = _rng(seed, 8)
        for i in range(n):
            k = int((adj[i] != 0xFFFFFFFF).sum())
            for j in range(1, k):
                if gr.random() < repeat_frac:
                    adj[i, j] = adj[i, int(gr.integers(0, j))]
    return X, adj
