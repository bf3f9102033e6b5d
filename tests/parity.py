"""The per-query parity rule between the GPU path and the oracle.

For each query: if the id rows are equal, every distance must agree within
1e-5 relative (denominator max(|d_oracle|, tau)); if they differ, the query
is tie-exempt only when at every differing rank the exact (fp64) distances of
the two competing ids differ by at most 1e-6 relative.  Anything else fails.
"""
from __future__ import annotations

import numpy as np

import oracle

REL_DIST = 1e-5
REL_TIE = 1e-6


def compare(gpu_ids, gpu_d, or_ids, or_d, X, Q, metric, tau=None):
    gpu_ids = np.asarray(gpu_ids)
    gpu_d = np.asarray(gpu_d, dtype=np.float64)
    or_ids = np.asarray(or_ids)
    or_d = np.asarray(or_d, dtype=np.float64)
    if tau is None:
        # 1e-3 of the median distance (L2); on tie-heavy grids most returned
        # distances can be exactly 0 (duplicates of the query), so the median
        # is taken over the positive ones
        pos = np.abs(or_d[np.isfinite(or_d) & (or_d != 0)])
        tau = 1.0 if metric == oracle.IP else 1e-3 * (float(np.median(pos)) if pos.size else 1.0)
    res = dict(n=len(gpu_ids), equal=0, exempt=0, fail=0, failed=[], max_rel=0.0)
    for i in range(len(gpu_ids)):
        if np.array_equal(gpu_ids[i], or_ids[i]):
            a, b = gpu_d[i], or_d[i]
            fin = np.isfinite(b)
            if not np.array_equal(np.isfinite(a), fin):
                res["fail"] += 1
                res["failed"].append(i)
                continue
            rel = np.abs(a[fin] - b[fin]) / np.maximum(np.abs(b[fin]), tau)
            m = float(rel.max()) if rel.size else 0.0
            res["max_rel"] = max(res["max_rel"], m)
            if m <= REL_DIST:
                res["equal"] += 1
            else:
                res["fail"] += 1
                res["failed"].append(i)
            continue
        diff = np.flatnonzero(gpu_ids[i] != or_ids[i])
        pair = np.stack([gpu_ids[i][diff], or_ids[i][diff]])
        if (pair < 0).any():
            res["fail"] += 1
            res["failed"].append(i)
            continue
        d = oracle.pair_dist(X, np.repeat(Q[i:i + 1], 2, axis=0), pair, metric)
        rel = np.abs(d[0] - d[1]) / np.maximum(np.abs(d[1]), tau)
        if (rel <= REL_TIE).all():
            res["exempt"] += 1
        else:
            res["fail"] += 1
            res["failed"].append(i)
    return res


def recall_at_k(ids, X, Q, gt_d64, metric):
    """Tie-aware recall: a returned id counts if its fp64 distance <= the true
    K-th, within 1e-9 relative (the ground truth may sum the same terms in
    another order)."""
    d = oracle.pair_dist(X, Q, np.asarray(ids, dtype=np.int32), metric)
    K = gt_d64.shape[1]
    dk = gt_d64[:, -1:]
    return np.sum(d <= dk + 1e-9 * np.abs(dk) + 1e-12, axis=1) / K
