"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Each test names the passage it checks.  None of them re-derives the oracle's
own formula: they compare against closed forms, brute force on tiny inputs,
special cases the paper states, hand-traced examples, or a differently
structured model of the same algorithm.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synthdata

# ------------------------------------------------------------------ helpers


def l2_64(X, q):
    d = X.astype(np.float64) - q.astype(np.float64)
    return np.einsum("ij,ij->i", d, d)


def layer_lists(p, lc):
    """Neighbour lists of layer lc from the packed form: dict id -> list."""
    out = {}
    if lc == 0:
        for i in range(p["n"]):
            row = p["adj0"][i]
            out[i] = [int(v) for v in row if v != 0xFFFFFFFF]
        return out
    for i in range(p["n"]):
        if p["levels"][i] >= lc:
            row = p["adjU"][p["upper_off"][i] + lc - 1]
            out[i] = [int(v) for v in row if v != 0xFFFFFFFF]
    return out


@pytest.fixture(scope="module")
def g0():
    X = synthdata.base("uniform16", 10000)
    return oracle.Graph.build(X, M=16, efC=100, seed=1003)


# ------------------------------------------------------------ P2: levels


def test_level_law_chi_square():
    """Alg. 1's level l = floor(-ln U * mL) with mL = 1/ln M has P(l = k) = (1 - 1/M) M^-k.

    Closed form: P(l >= k) = P(U <= exp(-k/mL)) = M^-k.  (Eq. (1)'s E[l+1] = mL + 1
    ignores the floor; the exact mean is 1/(M-1).)
    """
    M, n = 16, 1_000_000
    lv = oracle.levels(2003, n, 1.0 / math.log(M))
    counts = np.bincount(lv, minlength=8).astype(np.float64)
    p = np.array([(1 - 1 / M) * M ** -k for k in range(4)] + [M ** -4])
    obs = np.array(list(counts[:4]) + [counts[4:].sum()])
    exp = p * n
    chi2 = float(np.sum((obs - exp) ** 2 / exp))
    assert chi2 < 18.47, (obs, exp, chi2)  # chi-square(4 dof) 99.9% quantile
    assert abs(lv.mean() - 1 / (M - 1)) < 5 * math.sqrt(0.07 / n) + 1e-3


def test_level_law_other_M_and_mL_zero():
    M, n = 4, 400_000
    lv = oracle.levels(7, n, 1.0 / math.log(M))
    for k in range(4):
        frac = np.mean(lv >= k)
        assert abs(frac - M ** -k) < 5 * math.sqrt(M ** -k / n) + 1e-9
    # mL = 0: a single layer (Sec. 4.1)
    assert np.all(oracle.levels(7, 1000, 0.0) == 0)


# --------------------------------------------------- P3: graph invariants


def test_graph_invariants(g0):
    """Degrees bounded by Mmax / Mmax0 (Alg. 1 shrink), no self loops or duplicates,
    links on layer lc join members of layer lc, entry point on the top level."""
    p = g0.packed()
    lv = p["levels"]
    assert p["max_level"] == lv.max()
    ep = p["entry_point"]
    assert lv[ep] == lv.max()
    # the entry point is the first element that reached the top level (Alg. 1, last lines)
    assert ep == int(np.flatnonzero(lv == lv.max())[0])
    for lc in range(p["max_level"] + 1):
        lists = layer_lists(p, lc)
        cap = p["Mmax0"] if lc == 0 else p["Mmax"]
        for i, nb in lists.items():
            assert len(nb) <= cap
            assert i not in nb
            assert len(set(nb)) == len(nb)
            assert all(lv[e] >= lc for e in nb)
            if len(lists) > 1:  # a layer with two or more members has no isolated element
                assert len(nb) >= 1
    # P9: packed link bytes = n*Mmax0*4 + rows*Mmax*4, rows = sum of levels
    assert p["rows"] == int(lv.astype(np.int64).sum())
    assert p["adj0"].nbytes + p["adjU"].nbytes == p["n"] * p["Mmax0"] * 4 + p["rows"] * p["Mmax"] * 4


def test_graph_file_roundtrip(g0, tmp_path):
    p = g0.packed()
    path = str(tmp_path / "g.bin")
    oracle.save_graph(path, p)
    q = oracle.load_graph(path)
    for k in ("levels", "adj0", "upper_off", "adjU"):
        assert np.array_equal(p[k], q[k])
    for k in ("n", "dim", "M", "Mmax", "Mmax0", "max_level", "entry_point", "rows"):
        assert p[k] == q[k]
    raw = bytearray(open(path, "rb").read())
    raw[200] ^= 1
    open(path, "wb").write(bytes(raw))
    with pytest.raises(ValueError):
        oracle.load_graph(path)


# ---------------------------------- P1: exhaustive search equals brute force


@pytest.mark.parametrize("n,dim,metric", [(600, 8, oracle.L2), (1500, 3, oracle.L2), (800, 12, oracle.IP)])
def test_search_with_ef_ge_n_is_exact(n, dim, metric):
    """With ef >= N no element is ever evicted from W (Alg. 2), so a connected
    layer 0 is explored completely and Alg. 5 returns the exact K-NN (Sec. 1)."""
    g = np.random.default_rng(n)
    X = g.random((n, dim)).astype(np.float32)
    Q = g.random((60, dim)).astype(np.float32)
    if metric == oracle.IP:
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    G = oracle.Graph.build(X, metric=metric, M=6, efC=40, seed=5)
    p = G.packed()
    # layer 0 reachable from the entry point (BFS over the directed lists)
    lists = layer_lists(p, 0)
    seen = {p["entry_point"]}
    todo = [p["entry_point"]]
    while todo:
        v = todo.pop()
        for e in lists[v]:
            if e not in seen:
                seen.add(e)
                todo.append(e)
    assert len(seen) == n
    K = 10
    ids, ds = G.search(Q, K, ef=n)
    # brute force in the same key order: fp32-rounded distance, then id
    for qi in range(len(Q)):
        if metric == oracle.L2:
            d = l2_64(X, Q[qi])
        else:
            d = 1.0 - X.astype(np.float64) @ Q[qi].astype(np.float64)
        d32 = d.astype(np.float32)
        order = np.lexsort((np.arange(n), d32))[:K]
        assert np.array_equal(ids[qi], order), qi
        assert np.array_equal(ds[qi], d32[order])


def test_bruteforce_on_a_grid():
    """Brute force on the integer grid {0..9}^2: the 5 nearest of grid point (4,4)
    are itself (0), then its 4 axis neighbours (1), in id order."""
    xs = np.array([(i, j) for i in range(10) for j in range(10)], dtype=np.float32)
    q = np.array([[4.0, 4.0]], dtype=np.float32)
    ids, d = oracle.bruteforce(xs, q, 9)
    assert ids[0, 0] == 44 and d[0, 0] == 0.0
    assert list(ids[0, 1:5]) == [34, 43, 45, 54] and np.all(d[0, 1:5] == 1.0)
    assert sorted(ids[0, 5:9]) == [33, 35, 53, 55] and np.all(d[0, 5:9] == 2.0)


# ---------------------------------------------- P4 / P5: Alg. 4 special cases


def _flat_graph(X, metric=oracle.L2):
    n = X.shape[0]
    packed = dict(metric=metric, M=4, Mmax=4, Mmax0=8, entry_point=0, max_level=0,
                  levels=np.zeros(n, np.uint8), adj0=np.full((n, 8), 0xFFFFFFFF, np.uint32),
                  adjU=np.zeros((0, 4), np.uint32))
    return oracle.Graph.from_packed(X, packed)


def test_heuristic_1d_gives_delaunay_neighbours():
    """Sec. 3: on 1-D data the heuristic returns the exact Delaunay neighbours,
    i.e. the predecessor and successor of the base element."""
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(3, 60))
        x = rng.permutation(rng.choice(100000, size=n, replace=False)).astype(np.float32)[:, None]
        G = _flat_graph(x)
        b = int(rng.integers(0, n))
        cand = [i for i in range(n) if i != b]
        sel = set(int(v) for v in G.select_heuristic(b, cand, M=n))
        order = np.argsort(x[:, 0])
        pos = int(np.flatnonzero(order == b)[0])
        expect = set()
        if pos > 0:
            expect.add(int(order[pos - 1]))
        if pos < n - 1:
            expect.add(int(order[pos + 1]))
        assert sel == expect, (trial, sel, expect)


def test_heuristic_contains_relative_neighbourhood_graph():
    """Sec. 3: with enough candidates the heuristic keeps every relative
    neighbourhood graph edge of the base element."""
    rng = np.random.default_rng(12)
    for trial in range(100):
        n, d = int(rng.integers(5, 120)), int(rng.integers(2, 6))
        X = rng.random((n, d)).astype(np.float32)
        G = _flat_graph(X)
        b = int(rng.integers(0, n))
        cand = [i for i in range(n) if i != b]
        sel = set(int(v) for v in G.select_heuristic(b, cand, M=n))
        D = np.sqrt(((X[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1))
        for p in cand:
            # RNG edge (b, p): no r with max(d(b,r), d(p,r)) < d(b,p)
            others = [r for r in range(n) if r not in (b, p)]
            if all(max(D[b, r], D[p, r]) >= D[b, p] for r in others):
                assert p in sel, (trial, p)


def test_heuristic_flags():
    """Alg. 4's keepPrunedConnections tops R up to M from the discarded queue,
    nearest first (extendCandidates: the two tests after this one)."""
    x = np.array([[0.0], [1.0], [2.0], [3.0], [-1.0], [10.0]], dtype=np.float32)
    G = _flat_graph(x)
    # base 0: candidates 1,2,3 on one side -> only 1 kept (2 and 3 are closer to 1)
    assert list(G.select_heuristic(0, [1, 2, 3], M=3)) == [1]
    assert list(G.select_heuristic(0, [1, 2, 3], M=3, keep_pruned=True)) == [1, 2, 3]
    assert list(G.select_heuristic(0, [3, 2, 1, 4], M=2)) == [1, 4]


def _linked_graph(X, lists, width=8):
    """One-layer graph whose layer-0 lists are given (dict id -> ids)."""
    n = X.shape[0]
    adj0 = np.full((n, width), 0xFFFFFFFF, np.uint32)
    for i, lst in lists.items():
        adj0[i, :len(lst)] = lst
    packed = dict(metric=oracle.L2, M=4, Mmax=4, Mmax0=width, entry_point=0, max_level=0,
                  levels=np.zeros(n, np.uint8), adj0=adj0, adjU=np.zeros((0, 4), np.uint32))
    return oracle.Graph.from_packed(X, packed)


def test_heuristic_extend_candidates_worked_example():
    """Alg. 4 extendCandidates on 1-D points, worked by hand.  Points 0..5 at
    0, 1, 2, 3, -1, 10; lists 3: {2, 5}, 2: {1, 3}, 4: {0, 1}, 5: {3}.
    Base 0, candidates {3}: the extension adds 2 and 5; taken in distance
    order 2 (2), 3 (3), 5 (10), 2 is kept and both others are nearer to 2 than
    to the base, so R = [2] (plain: [3]); keepPrunedConnections tops up with
    3 and 5.  Candidates {3, 4}: the extension adds 2, 5 (from 3) and 1 (from
    4; the base itself is not added); 1 and 4 tie at distance 1 and go in id
    order, both kept (4 is 2 away from 1), so R = [1, 4] (plain: [4, 3])."""
    x = np.array([[0.0], [1.0], [2.0], [3.0], [-1.0], [10.0]], dtype=np.float32)
    G = _linked_graph(x, {3: [2, 5], 2: [1, 3], 4: [0, 1], 5: [3]})
    assert list(G.select_heuristic(0, [3], M=2)) == [3]
    assert list(G.select_heuristic(0, [3], M=2, extend=True)) == [2]
    assert list(G.select_heuristic(0, [3], M=3, extend=True, keep_pruned=True)) == [2, 3, 5]
    assert list(G.select_heuristic(0, [3, 4], M=2)) == [4, 3]
    assert list(G.select_heuristic(0, [3, 4], M=2, extend=True)) == [1, 4]
    assert list(G.select_heuristic(0, [3, 4], M=4, extend=True)) == [1, 4]
    assert list(G.select_heuristic(0, [3, 4], M=5, extend=True, keep_pruned=True)) == [1, 4, 2, 3, 5]


def _extended_selection_model(X, lists, base, cand, M, keep_pruned):
    """Alg. 4 with extendCandidates written out from its definition: the
    candidates plus every listed neighbour of a candidate, the base excepted,
    each element once; visited nearest first ((distance, id) order); an
    element is kept when it is nearer to the base than to every element kept
    so far; the discarded ones top R up, nearest first, under keepPruned."""
    def d(a, b):
        return np.float32(((X[a].astype(np.float64) - X[b].astype(np.float64)) ** 2).sum())
    W = list(dict.fromkeys(list(cand) + [e for c in cand for e in lists.get(c, []) if e != base]))
    W.sort(key=lambda e: (d(e, base), e))
    R, Wd = [], []
    for e in W:
        if len(R) >= M:
            break
        if all(d(e, base) < d(e, r) for r in R):
            R.append(e)
        else:
            Wd.append(e)
    if keep_pruned:
        R += Wd[:M - len(R)]
    return R


def test_heuristic_extend_candidates_matches_model():
    """The oracle's extended selection equals the model above on random small
    graphs with integer coordinates (exact distances, so ties are real ties and
    both sides order them by id)."""
    rng = np.random.default_rng(21)
    for trial in range(300):
        n, dim = int(rng.integers(6, 40)), int(rng.integers(1, 4))
        X = rng.integers(0, 6, size=(n, dim)).astype(np.float32)
        lists = {i: [int(v) for v in rng.choice(np.setdiff1d(np.arange(n), [i]), int(rng.integers(0, 6)),
                                                replace=False)] for i in range(n)}
        G = _linked_graph(X, lists)
        base = int(rng.integers(0, n))
        cand = [int(v) for v in rng.choice(np.setdiff1d(np.arange(n), [base]), int(rng.integers(1, min(8, n - 1))),
                                           replace=False)]
        M = int(rng.integers(1, 8))
        keep = bool(rng.integers(0, 2))
        got = [int(v) for v in G.select_heuristic(base, cand, M=M, extend=True, keep_pruned=keep)]
        assert got == _extended_selection_model(X, lists, base, cand, M, keep), (trial, got)


# ------------------------------------------------- P6: k-NN graph special case


def test_mL_zero_simple_selection_gives_knn_graph():
    """Sec. 4.1: mL = 0, Mmax0 = M and Alg. 3 produce a (directed) k-NN graph.

    With efC >= N every search of the insertion finds the exact M-NN among the
    earlier elements, so element i ends with the M nearest (to i) of
    S_i = M-NN(i, earlier) united with the later elements that linked to i.
    """
    rng = np.random.default_rng(21)
    n, d, M = 150, 2, 12
    X = rng.random((n, d)).astype(np.float32)
    G = oracle.Graph.build(X, M=M, Mmax=M, Mmax0=M, efC=n, mL=0.0, seed=1, heuristic=False)
    p = G.packed()
    assert p["max_level"] == 0
    D = ((X[:, None, :].astype(np.float64) - X[None, :, :]) ** 2).sum(-1).astype(np.float32)

    def knn(i, pool):
        pool = np.array(sorted(pool))
        order = np.lexsort((pool, D[i, pool]))
        return [int(v) for v in pool[order[:M]]]

    first = {i: knn(i, range(i)) for i in range(1, n)}
    lists = layer_lists(p, 0)
    for i in range(n):
        S = set(first.get(i, [])) | {j for j in range(i + 1, n) if i in first[j]}
        assert sorted(lists[i]) == sorted(knn(i, S)) if S else lists[i] == [], i


# --------------------------------------------------- P8: hand-traced example


def _golden(name):
    """key -> list of values from a tests/golden text fixture."""
    out = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.split("#")[0].split()
        if line:
            out[line[0]] = line[1:]
    return out


def test_search_layer_hand_trace():
    """Alg. 2 on a path graph of points x_i = i (1-D): the hand trace stored
    in tests/golden/search_layer_path_trace.txt (query 6.4, enter point 0,
    ef = 2: the beam walks right and stops with W = {6, 7})."""
    gd = _golden("search_layer_path_trace.txt")
    n = int(gd["points"][0])
    x = np.arange(n, dtype=np.float32)[:, None]
    adj = np.full((n, 8), 0xFFFFFFFF, np.uint32)
    for i in range(n):
        nb = [j for j in (i - 1, i + 1) if 0 <= j < n]
        adj[i, : len(nb)] = nb
    packed = dict(metric=oracle.L2, M=4, Mmax=4, Mmax0=8, entry_point=0, max_level=0,
                  levels=np.zeros(n, np.uint8), adj0=adj, adjU=np.zeros((0, 4), np.uint32))
    G = oracle.Graph.from_packed(x, packed)
    ids, ds, ndist = G.search_layer(np.array([float(gd["query"][0])], np.float32), [int(gd["enter"][0])],
                                    ef=int(gd["ef"][0]), lc=0)
    assert list(ids) == [int(v) for v in gd["result_ids"]]
    assert np.allclose(ds, [float(v) for v in gd["result_dists"]], rtol=1e-6)
    assert ndist == int(gd["distance_evaluations"][0])  # 0 (entry) + 1..8 once each; 9 never seen


# ---------------------------------------------- P7 / P8: search equivalences


def _model_beam(X, adj, q, ep, ef, lossy=0.0, rng=None):
    """The beam form the GPU kernel uses (an independent model, not the oracle):
    W is one sorted list of at most ef keys with an 'expanded' flag; the
    nearest unexpanded entry is expanded; its unvisited neighbours are scored
    together and W <- top-ef(W united with them); duplicates are dropped.
    ``lossy`` forgets visited marks at random (false negatives only)."""
    def key(i):
        d = float(np.float32(((X[i].astype(np.float64) - q.astype(np.float64)) ** 2).sum()))
        return (d, i)

    visited = {ep}
    W = [(key(ep), False)]
    while True:
        un = [k for k, (kk, done) in enumerate(W) if not done]
        if not un:
            break
        c = un[0]
        W[c] = (W[c][0], True)
        cid = W[c][0][1]
        fresh = []
        for e in adj[cid]:
            if e == 0xFFFFFFFF:
                continue
            e = int(e)
            if e in visited:
                continue
            if not (lossy and rng.random() < lossy):
                visited.add(e)
            fresh.append(key(e))
        have = {k for k, _ in W}
        merged = W + [(k, False) for k in fresh if k not in have]
        merged = list({k: (k, f) for k, f in sorted(merged, key=lambda t: (t[0], not t[1]))}.values())
        merged.sort(key=lambda t: t[0])
        W = merged[:ef]
    return [k[1] for k, _ in W]


@pytest.mark.parametrize("lossy", [0.0, 0.3])
def test_literal_search_layer_equals_beam_model(lossy):
    """A3/A4: the literal two-heap Alg. 2 and the bounded sorted-beam form with
    batch neighbourhood merges (and a lossy visited set plus de-duplication)
    return the same W, on random graphs with many distance ties."""
    rng = np.random.default_rng(31 + int(lossy * 10))
    for trial in range(300):
        n = int(rng.integers(5, 80))
        X, adj = synthdata.random_graph(n, 6, seed=trial, dim=2, tie_grid=4)
        packed = dict(metric=oracle.L2, M=3, Mmax=3, Mmax0=6, entry_point=0, max_level=0,
                      levels=np.zeros(n, np.uint8), adj0=adj, adjU=np.zeros((0, 3), np.uint32))
        G = oracle.Graph.from_packed(X, packed)
        q = rng.integers(0, 4, size=2).astype(np.float32)
        ep = int(rng.integers(0, n))
        ef = int(rng.integers(1, 12))
        ids, _, _ = G.search_layer(q, [ep], ef=ef, lc=0)
        model = _model_beam(X, adj, q, ep, ef, lossy=lossy, rng=rng)
        assert list(ids) == model, (trial, list(ids), model)


def test_ef1_is_greedy_descent():
    """A3c: SEARCH-LAYER with ef = 1 equals 'move to the (dist, id)-smallest of
    the current element and its neighbours until no move'."""
    rng = np.random.default_rng(41)
    for trial in range(300):
        n = int(rng.integers(3, 60))
        X, adj = synthdata.random_graph(n, 5, seed=1000 + trial, dim=2, tie_grid=5)
        packed = dict(metric=oracle.L2, M=3, Mmax=3, Mmax0=5, entry_point=0, max_level=0,
                      levels=np.zeros(n, np.uint8), adj0=adj, adjU=np.zeros((0, 3), np.uint32))
        G = oracle.Graph.from_packed(X, packed)
        q = rng.integers(0, 5, size=2).astype(np.float32)
        cur = int(rng.integers(0, n))
        ids, _, _ = G.search_layer(q, [cur], ef=1, lc=0)

        def key(i):
            return (float(np.float32(((X[i].astype(np.float64) - q) ** 2).sum())), i)

        while True:
            best = min([cur] + [int(e) for e in adj[cur] if e != 0xFFFFFFFF], key=key)
            if best == cur:
                break
            cur = best
        assert list(ids) == [cur], trial


# ------------------------------------------------------ P9: memory model


def test_memory_model_against_paper_range():
    """Sec. 4.2.3: link memory per element is (Mmax0 + mL*Mmax) * 4 bytes, which
    the paper puts at about 60-450 bytes for M in [6, 48].  With the level law's
    floor the exact expectation is (Mmax0 + Mmax/(M-1)) * 4; the oracle's packed
    graph must match that, and the paper's own formula must span its range."""
    gd = _golden("memory_per_element.txt")
    m_lo, m_hi = int(gd["m_low"][0]), int(gd["m_high"][0])
    b_lo, b_hi = float(gd["bytes_low"][0]), float(gd["bytes_high"][0])
    # the paper's formula with Mmax0 = 2M, Mmax = M, mL = 1/ln M
    lo = (2 * m_lo + m_lo / math.log(m_lo)) * 4
    hi = (2 * m_hi + m_hi / math.log(m_hi)) * 4
    assert abs(lo - b_lo) / b_lo < 0.1 and abs(hi - b_hi) / b_hi < 0.05
    M, n = 16, 1_000_000
    lv = oracle.levels(99, n, 1 / math.log(M))
    per = (2 * M * n + M * lv.astype(np.int64).sum()) * 4 / n
    assert abs(per - (2 * M + M / (M - 1)) * 4) < 0.5
