"""GPU parity of the plain K-NN-SEARCH path against the oracle, through the C ABI.

Every graph is built by the oracle; the GPU and the oracle search the same
graph with the same seeded queries, and the per-query parity rule of
``tests/parity.py`` is applied.  The distance accumulation on both sides is
fp64 rounded once to fp32, so ids are expected to agree exactly
(zero tie exemptions) and distances bit for bit.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import synthdata
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hnsw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_09320_amd as h

    h.lib()
    return h


def _index(h, G, X):
    return h.Index(G.packed(), X)


@pytest.fixture(scope="module")
def cfg0():
    X = synthdata.base("uniform16", 10000)
    Q = synthdata.queries("uniform16", 1000)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    return X, Q, G


def _run_parity(h, G, X, Q, K, ef, metric=oracle.L2, counters=True):
    idx = _index(h, G, X)
    q = torch.from_numpy(Q).cuda()
    ids, ds, cnt = idx.search(q, K, ef, counters=True)
    torch.cuda.synchronize()
    ids, ds, cnt = ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)
    oi, od, oc = G.search(Q, K, ef, nthreads=8, counters=True)
    r = parity.compare(ids, ds, oi, od, X, Q, metric)
    _log(f"parity K={K} ef={ef}: {r['equal']} equal, {r['exempt']} tie-exempt, {r['fail']} fail, "
         f"max rel {r['max_rel']:.2e}")
    assert r["fail"] == 0, r["failed"][:10]
    assert r["exempt"] == 0
    # identical W evolution: identical expansion counts; the visited table may
    # forget, so the GPU scores at least as many elements as the oracle
    assert np.array_equal(cnt[:, 3], oc[:, 3].astype(np.uint32))
    assert np.array_equal(cnt[:, 1], oc[:, 1].astype(np.uint32))
    assert (cnt[:, 2] >= oc[:, 2].astype(np.uint32)).all()
    return ids, ds, cnt, oc


@pytest.mark.parametrize("ef", [10, 50, 200])
def test_parity_uniform16(hnsw, cfg0, ef):
    _log(f"case uniform16 10k x 16, K=10 ef={ef}")
    X, Q, G = cfg0
    ids, ds, cnt, oc = _run_parity(hnsw, G, X, Q, 10, ef)
    assert np.array_equal(ds, G.search(Q, 10, ef, nthreads=8)[1])


@pytest.mark.parametrize("K,ef", [(1, 1), (1, 10), (10, 1), (64, 64), (100, 300), (200, 1024), (1024, 1)])
def test_parity_k_ef_edges(hnsw, cfg0, K, ef):
    _log(f"case uniform16 K={K} ef={ef}")
    X, Q, G = cfg0
    _run_parity(hnsw, G, X, Q[:300], K, ef)


@pytest.mark.parametrize("dim", [1, 3, 5, 8, 17, 33, 64, 100, 130, 256])
def test_parity_dims(hnsw, dim):
    """Every lane-group tile shape, with dimensions that leave a ragged tail."""
    _log(f"case random dim={dim}")
    rng = np.random.default_rng(dim)
    X = rng.random((3000, dim)).astype(np.float32)
    Q = rng.random((200, dim)).astype(np.float32)
    G = oracle.Graph.build(X, M=8, efC=60, seed=7)
    _run_parity(hnsw, G, X, Q, 10, 40)


@pytest.mark.parametrize("dim", [3, 17, 100, 130])
def test_parity_wide_gathers(hnsw, monkeypatch, dim):
    """The 64-bit addressed kernels (taken for vector stores above 2 GiB),
    forced on small indices: same results as the oracle."""
    _log(f"case wide gathers dim={dim}")
    monkeypatch.setenv("HNSW_WIDE_GATHERS", "1")
    rng = np.random.default_rng(100 + dim)
    X = rng.random((3000, dim)).astype(np.float32)
    Q = rng.random((200, dim)).astype(np.float32)
    G = oracle.Graph.build(X, M=8, efC=60, seed=7)
    _run_parity(hnsw, G, X, Q, 10, 40)


@pytest.mark.parametrize("K,ef", [(10, 50), (1, 1), (64, 200), (200, 1024)])
def test_parity_scheduled_launches(hnsw, cfg0, monkeypatch, K, ef):
    """The scheduled form (every descent first, then layer 0 with the queries
    reordered), forced on a small batch: the oracle's results and counters,
    and the one-kernel path's outputs bit for bit."""
    _log(f"case scheduled launches K={K} ef={ef}")
    X, Q, G = cfg0
    monkeypatch.setenv("HNSW_SCHEDULE", "2")
    ids, ds, cnt, _ = _run_parity(hnsw, G, X, Q, K, ef)
    monkeypatch.setenv("HNSW_SCHEDULE", "0")
    idx = _index(hnsw, G, X)
    i1, d1, c1 = idx.search(torch.from_numpy(Q).cuda(), K, ef, counters=True)
    torch.cuda.synchronize()
    assert np.array_equal(ids, i1.cpu().numpy()) and np.array_equal(ds, d1.cpu().numpy())
    assert np.array_equal(cnt, c1.cpu().numpy().astype(np.uint32))


@pytest.mark.parametrize("nq", [1, 2, 3, 257, 4097, 20000])
def test_scheduled_batch_sizes_and_wide_ip(hnsw, monkeypatch, nq):
    """Scheduled launches: tiny batches, sizes around the order kernel's
    1024-query tiles, and a batch spanning two of its 16,384-query rounds;
    inner product, through the 64-bit addressed kernels."""
    _log(f"case scheduled nq={nq} IP wide")
    monkeypatch.setenv("HNSW_SCHEDULE", "2")
    monkeypatch.setenv("HNSW_WIDE_GATHERS", "1")
    rng = np.random.default_rng(nq)
    X = rng.normal(size=(4000, 24)).astype(np.float32)
    Q = rng.normal(size=(nq, 24)).astype(np.float32)
    G = oracle.Graph.build(X, metric=oracle.IP, M=8, efC=40, seed=5)
    _run_parity(hnsw, G, X, Q, 10, 32, metric=oracle.IP)


def test_scheduled_concurrent_threads_and_streams(hnsw, cfg0, monkeypatch):
    """Scheduled launches submitted by four host threads, two per stream: each
    stream has its own workspace (grown while other batches run, by a 60,000-
    query batch), and batches sharing a stream never interleave their three
    launches.  Every result equals the serial one."""
    import threading

    _log("case scheduled launches from threads and streams")
    monkeypatch.setenv("HNSW_SCHEDULE", "2")
    X, Q, G = cfg0
    idx = _index(hnsw, G, X)
    q = torch.from_numpy(Q).cuda()
    ref_i, ref_d = idx.search(q, 10, 50)
    torch.cuda.synchronize()
    ref_i, ref_d = ref_i.cpu().numpy(), ref_d.cpu().numpy()
    big = q.repeat(60, 1).contiguous()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results, errors = {}, []

    def worker(j, stream):
        try:
            outs = []
            for r in range(6):
                qq = big if (j, r) in ((1, 2), (2, 3)) else q[:[1000, 300, 700][r % 3]]
                with torch.cuda.stream(stream):
                    ids, ds = idx.search(qq, 10, 50, stream=stream)
                outs.append((ids, ds))
            stream.synchronize()
            results[j] = [(i.cpu().numpy(), d.cpu().numpy()) for i, d in outs]
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(j, streams[j % 2])) for j in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    assert sorted(results) == [0, 1, 2, 3]
    for j, outs in results.items():
        for ids, ds in outs:
            n = ids.shape[0]
            reps = max(1, n // len(Q))
            ei = np.tile(ref_i, (reps, 1))[:n] if n > len(Q) else ref_i[:n]
            ed = np.tile(ref_d, (reps, 1))[:n] if n > len(Q) else ref_d[:n]
            assert np.array_equal(ids, ei) and np.array_equal(ds, ed), (j, n)


def test_default_form_choice_repeated_calls(hnsw, cfg0, monkeypatch):
    """A batch above the resident capacity with the default form choice: the
    first calls time the scheduled and the one-kernel forms (events read back
    later, without blocking), later ones use the faster.  Every call, with or
    without a synchronisation before the next, returns the same results, and
    those equal the oracle's on a sample."""
    _log("case default form choice, repeated 12,000-query calls")
    monkeypatch.delenv("HNSW_SCHEDULE", raising=False)
    X, _, G = cfg0
    Q = synthdata.queries("uniform16", 12000)
    idx = _index(hnsw, G, X)
    q = torch.from_numpy(Q).cuda()
    outs = []
    for r in range(8):
        ids, ds = idx.search(q, 10, 50)
        if r % 3 == 2:
            torch.cuda.synchronize()
        outs.append((ids, ds))
    torch.cuda.synchronize()
    first_i, first_d = outs[0][0].cpu().numpy(), outs[0][1].cpu().numpy()
    for ids, ds in outs[1:]:
        assert np.array_equal(ids.cpu().numpy(), first_i) and np.array_equal(ds.cpu().numpy(), first_d)
    sample = np.random.default_rng(5).choice(len(Q), size=200, replace=False)
    oi, od = G.search(Q[sample], 10, 50, nthreads=8)
    r = parity.compare(first_i[sample], first_d[sample], oi, od, X, Q[sample], oracle.L2)
    assert r["fail"] == 0 and r["exempt"] == 0


@pytest.mark.parametrize("ef", [10, 64])
def test_parity_ties_and_duplicates(hnsw, ef):
    """Integer grid coordinates: most distances tie, and many points are exact
    duplicates of others; every decision falls to the id order of the key."""
    _log(f"case ties and duplicates ef={ef}")
    rng = np.random.default_rng(5)
    X = rng.integers(0, 6, size=(3000, 4)).astype(np.float32)
    Q = rng.integers(0, 6, size=(300, 4)).astype(np.float32)
    G = oracle.Graph.build(X, M=8, efC=40, seed=11)
    _run_parity(hnsw, G, X, Q, 10, ef)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_parity_random_graphs_with_ties(hnsw, seed):
    """Arbitrary single-layer graphs (random out-lists of 1..16 links) on
    points of a small integer grid, uploaded as they are: the search follows
    the graph it is given, not one with HNSW's structure."""
    _log(f"case random graph seed={seed}")
    X, adj = synthdata.random_graph(2000, 16, seed, dim=3, tie_grid=5)
    n = len(X)
    packed = dict(metric=oracle.L2, M=8, Mmax=8, Mmax0=16, entry_point=0, max_level=0,
                  levels=np.zeros(n, np.uint8), adj0=adj, upper_off=np.full(n, -1, np.int32),
                  adjU=np.zeros((0, 8), np.uint32))
    G = oracle.Graph.from_packed(X, packed)
    Q = np.random.default_rng(seed).integers(0, 5, size=(200, 3)).astype(np.float32)
    for ef in (5, 40):
        _run_parity(hnsw, G, X, Q, 10, ef)


def test_parity_inner_product(hnsw):
    _log("case glove_like 20k x 100 IP")
    X = synthdata.base("glove_like", 20000)
    Q = synthdata.queries("glove_like", 300)
    G = oracle.Graph.build(X, metric=oracle.IP, M=16, efC=100, seed=3004)
    for ef in (10, 100, 400):
        _run_parity(hnsw, G, X, Q, 10, ef, metric=oracle.IP)


def test_parity_sift_like_subset(hnsw):
    _log("case sift_like 30k x 128")
    X = synthdata.base("sift_like", 30000)
    Q = synthdata.queries("sift_like", 300)
    G = oracle.Graph.build(X, M=16, efC=200, seed=2003)
    for K, ef in ((1, 10), (10, 10), (10, 64), (10, 256), (10, 800)):
        _run_parity(hnsw, G, X, Q, K, ef)


def test_tiny_graphs_and_padding(hnsw):
    """n = 1 (entry point only, no links) and n < K: rows are padded with (-1, +inf)."""
    for n in (1, 2, 7):
        _log(f"case tiny n={n}")
        X = np.arange(n * 4, dtype=np.float32).reshape(n, 4)
        G = oracle.Graph.build(X, M=4, efC=10, seed=1)
        Q = np.array([[1.0, 2.0, 3.0, 4.0], [100.0, 0.0, 0.0, 0.0]], dtype=np.float32)
        ids, ds, _, _ = _run_parity(hnsw, G, X, Q, 10, 20)
        assert (ids[:, n:] == -1).all() and np.isinf(ds[:, n:]).all()
        assert sorted(ids[0, :n]) == list(range(n))


def test_empty_batch_and_errors(hnsw, cfg0):
    X, Q, G = cfg0
    idx = _index(hnsw, G, X)
    q = torch.from_numpy(Q[:4]).cuda()
    ids, ds = idx.search(q[:0], 10, 10)
    assert ids.shape == (0, 10)
    with pytest.raises(hnsw.HnswError) as e:
        idx.search(q, 10, 2000)
    assert e.value.code == 4
    with pytest.raises(hnsw.HnswError) as e:
        idx.search(q, 0, 10)
    assert e.value.code == 1
    # host pointers are rejected
    import ctypes as C

    hq = np.ascontiguousarray(Q[:4])
    hi = np.empty((4, 10), np.int32)
    hd = np.empty((4, 10), np.float32)
    code = hnsw.lib().hnsw_search_batch(idx.handle, hq.ctypes.data_as(C.c_void_p), 4, 10, 10,
                                        hi.ctypes.data_as(C.c_void_p), hd.ctypes.data_as(C.c_void_p), None)
    assert code == 1


def test_plain_entry_point_and_determinism(hnsw, cfg0):
    X, Q, G = cfg0
    idx = _index(hnsw, G, X)
    q = torch.from_numpy(Q).cuda()
    a = hnsw.search_batch(idx, q, 10, 50)
    b = idx.search(q, 10, 50)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c = idx.search(q, 10, 50, stream=s)
    torch.cuda.synchronize()
    for x, y in ((a, b), (a, c)):
        assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])


FULL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "graphs", "sift_like_1M.bin")


@pytest.mark.skipif(not os.path.exists(FULL), reason="1M sift_like graph file not built")
def test_parity_sift_like_full_size_sampled(hnsw):
    """The 1M x 128 workload in the benchmark's launch shape: all 10,000 queries
    on the GPU, a sample checked against the oracle on the same graph."""
    _log("case sift_like 1M x 128 full size, sampled")
    p = hnsw.graphfile.read(FULL)
    X = synthdata.base("sift_like", p["n"])
    Q = synthdata.queries("sift_like", 10000)
    idx = hnsw.Index(p, X)
    G = oracle.Graph.from_packed(X, p)
    q = torch.from_numpy(Q).cuda()
    sample = np.random.default_rng(0).choice(10000, size=150, replace=False)
    for K, ef in ((10, 56), (10, 64), (10, 256), (1, 32)):
        ids, ds, cnt = idx.search(q, K, ef, counters=True)
        torch.cuda.synchronize()
        ids, ds = ids.cpu().numpy(), ds.cpu().numpy()
        oi, od, oc = G.search(Q[sample], K, ef, nthreads=8, counters=True)
        r = parity.compare(ids[sample], ds[sample], oi, od, X, Q[sample], oracle.L2)
        _log(f"full-size K={K} ef={ef}: {r}")
        assert r["fail"] == 0 and r["exempt"] == 0
        # properties over every query: valid distinct ids, sorted keys, exact distances
        assert ((ids >= 0) & (ids < p["n"])).all()
        assert all(len(set(row)) == K for row in ids)
        assert (np.diff(ds, axis=1) >= 0).all()
        d64 = oracle.pair_dist(X, Q, ids)
        assert np.array_equal(d64.astype(np.float32), ds)



def test_scheduled_order_full_size_two_rounds(hnsw, monkeypatch):
    """The scheduled form on the 1M x 128 graph with 20,000 queries: the order
    kernel's two 16,384-query rounds, queries grouped by the layer-3 node their
    descent reached and dealt to the XCDs; outputs and counters equal the
    one-kernel form's bit for bit, on every call (the order of queries that
    share a bin follows the order of their atomics and may change)."""
    _log("case sift_like 1M x 128, 20,000 queries, scheduled against one kernel")
    p = hnsw.graphfile.read(FULL)
    X = synthdata.base("sift_like", p["n"])
    Q = synthdata.queries("sift_like", 20000)
    idx = hnsw.Index(p, X)
    q = torch.from_numpy(Q).cuda()
    out = {}
    for form in ("2", "0", "2b"):
        monkeypatch.setenv("HNSW_SCHEDULE", form[0])
        ids, ds, cnt = idx.search(q, 10, 56, counters=True)
        torch.cuda.synchronize()
        out[form] = (ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy())
    for other in ("0", "2b"):
        for a, b in zip(out["2"], out[other]):
            assert np.array_equal(a, b), other
    assert ((out["2"][0] >= 0) & (out["2"][0] < p["n"])).all()
    idx.close()

def test_read_probe_reads_every_word(hnsw):
    """The bandwidth probe folds every 32-bit word it reads: the XOR of its
    per-block words equals the XOR of the buffer, for grids smaller and larger
    than the buffer's 16-byte words (tail loop and unrolled loop)."""
    rng = np.random.default_rng(5)
    for words16 in (1, 37, 4096, 100_003):
        h = rng.integers(0, 2**32, size=words16 * 4, dtype=np.uint64).astype(np.uint32)
        buf = torch.from_numpy(h.view(np.int32)).cuda()
        want = int(np.bitwise_xor.reduce(h))
        for blocks in (1, 3, 64, 1024):
            out = hnsw.read_probe(buf, blocks).cpu().numpy().view(np.uint32)
            assert int(np.bitwise_xor.reduce(out)) == want, (words16, blocks)
    with pytest.raises(hnsw.HnswError):
        hnsw.read_probe(torch.zeros(3, dtype=torch.int32).cuda())  # 12 bytes: not a multiple of 16
