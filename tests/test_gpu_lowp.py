"""Low-precision traversal (BF16 / FP8-E4M3 with per-vector scale) plus an
exact fp32 re-rank, on the GPU through the C ABI, against the oracle."""
import os

import numpy as np
import pytest

import oracle
import synthdata
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hnsw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_09320_amd as h

    h.lib()
    return h


def _special_rows(dim):
    rows = [np.zeros(dim), np.full(dim, 1e-30), np.linspace(-3, 3, dim), np.full(dim, -7.0)]
    r = np.linspace(-448.0, 448.0, dim)
    r[::3] *= 1e-3
    rows.append(r)
    rows.append(np.geomspace(1e-6, 1e6, dim) * np.where(np.arange(dim) % 2, 1, -1))
    return np.array(rows, dtype=np.float32)


@pytest.mark.parametrize("workload,n", [("deep_like", 20000), ("sift_like", 5000), ("glove_like", 5000)])
def test_quantized_codes_match_oracle(hnsw, workload, n):
    print(f"case quantize {workload} n={n}", flush=True)
    X = synthdata.base(workload, n)
    X = np.concatenate([X, _special_rows(X.shape[1])])
    idx = hnsw.Index(dict(n=len(X), dim=X.shape[1], metric=0, M=4, Mmax=4, Mmax0=4, max_level=0, entry_point=0,
                          levels=np.zeros(len(X), np.uint8), adj0=np.full((len(X), 4), 0xFFFFFFFF, np.uint32),
                          upper_off=np.full(len(X), -1, np.int32), adjU=np.zeros((0, 4), np.uint32)), X)
    idx.add_lowp(hnsw.MODE_BF16)
    idx.add_lowp(hnsw.MODE_FP8)
    gb, _ = idx.read_lowp(hnsw.MODE_BF16)
    ob, _, _ = oracle.quantize_bf16(X)
    assert np.array_equal(gb, ob)
    g8, gs = idx.read_lowp(hnsw.MODE_FP8)
    o8, _, osc = oracle.quantize_fp8(X)
    assert np.array_equal(gs, osc)
    assert np.array_equal(g8, o8)
    idx.add_lowp(hnsw.MODE_U8)
    gu, exact = idx.read_lowp(hnsw.MODE_U8)
    ou = oracle.quantize_u8(X)[0]
    assert np.array_equal(gu, ou)
    assert exact == bool(np.array_equal(ou.astype(np.float32), X))


QUANT = {1: oracle.quantize_bf16, 2: oracle.quantize_fp8, 4: oracle.quantize_u8}


def _lowp_parity(hnsw, X, Q, G, K, ef, kind, metric):
    p = G.packed()
    idx = hnsw.Index(p, X)
    idx.add_lowp(kind)
    ids, ds, cnt = idx.search(torch.from_numpy(Q).cuda(), K, ef, mode=kind, counters=True)
    torch.cuda.synchronize()
    ids, ds, cnt = ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)
    codes, dec, sc = QUANT[kind](X)
    G.set_lowp(dec, sc)
    oi, od, oc = G.search(Q, K, ef, nthreads=8, counters=True)
    G.set_lowp(None, None)
    r = parity.compare(ids, ds, oi, od, X, Q, metric)
    print(f"lowp kind={kind} K={K} ef={ef}: {r['equal']} equal, {r['exempt']} exempt, {r['fail']} fail", flush=True)
    assert r["fail"] == 0 and r["exempt"] == 0
    assert np.array_equal(cnt[:, 3], oc[:, 3].astype(np.uint32))
    return ids, ds


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_lowp_parity_deep_like(hnsw, kind):
    print(f"case lowp deep_like 20k x 96 kind={kind}", flush=True)
    X = synthdata.base("deep_like", 20000)
    Q = synthdata.queries("deep_like", 300)
    G = oracle.Graph.build(X, M=24, efC=100, seed=4003)
    for ef in (10, 64, 256):
        _lowp_parity(hnsw, X, Q, G, 10, ef, kind, oracle.L2)


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_lowp_parity_inner_product_and_dims(hnsw, kind):
    print(f"case lowp glove_like 8k x 100 IP kind={kind}", flush=True)
    X = synthdata.base("glove_like", 8000)
    Q = synthdata.queries("glove_like", 200)
    G = oracle.Graph.build(X, metric=oracle.IP, M=16, efC=80, seed=3004)
    _lowp_parity(hnsw, X, Q, G, 10, 100, kind, oracle.IP)
    for dim in (3, 17, 40, 130, 256):
        rng = np.random.default_rng(dim)
        X = rng.normal(size=(2500, dim)).astype(np.float32)
        Q = rng.normal(size=(100, dim)).astype(np.float32)
        G = oracle.Graph.build(X, M=8, efC=40, seed=2)
        _lowp_parity(hnsw, X, Q, G, 10, 50, kind, oracle.L2)


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_lowp_parity_wide_gathers(hnsw, monkeypatch, kind):
    """Low-precision traversal and re-rank through the 64-bit addressed
    kernels (taken for stores above 2 GiB), forced on a small index."""
    print(f"case lowp wide gathers kind={kind}", flush=True)
    monkeypatch.setenv("HNSW_WIDE_GATHERS", "1")
    X = synthdata.base("deep_like", 6000)
    Q = synthdata.queries("deep_like", 150)
    G = oracle.Graph.build(X, M=16, efC=60, seed=4004)
    _lowp_parity(hnsw, X, Q, G, 10, 64, kind, oracle.L2)


def test_bf16_equals_fp32_on_integer_data(hnsw):
    """Integer coordinates are exact in BF16: the BF16 search returns exactly the fp32 search's output."""
    X = synthdata.base("sift_like", 30000)
    Q = synthdata.queries("sift_like", 500)
    G = oracle.Graph.build(X, M=16, efC=200, seed=2003)
    idx = hnsw.Index(G.packed(), X)
    idx.add_lowp(hnsw.MODE_BF16)
    q = torch.from_numpy(Q).cuda()
    for ef in (10, 64, 300):
        a = idx.search(q, 10, ef)
        b = idx.search(q, 10, ef, mode=hnsw.MODE_BF16)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_u8_store_exact_on_integer_data(hnsw):
    """SIFT-like coordinates are integers in [0, 255]: the 8-bit copy is exact
    (codes equal the oracle's), its search skips the re-rank, and returns the
    fp32 search's ids and distances bit for bit, with the same expansions (the
    distance counts may differ: the fp32 store's visited table replaces old
    ids when full, the low-precision ones forget the new id); a store with
    other values is flagged inexact."""
    X = synthdata.base("sift_like", 30000)
    Q = synthdata.queries("sift_like", 500)
    G = oracle.Graph.build(X, M=16, efC=200, seed=2003)
    idx = hnsw.Index(G.packed(), X)
    idx.add_lowp(hnsw.MODE_U8)
    codes, exact = idx.read_lowp(hnsw.MODE_U8)
    assert exact and np.array_equal(codes, oracle.quantize_u8(X)[0])
    q = torch.from_numpy(Q).cuda()
    for K, ef in ((10, 10), (10, 64), (1, 32), (100, 300)):
        a = idx.search(q, K, ef, counters=True)
        b = idx.search(q, K, ef, mode=hnsw.MODE_U8, counters=True)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), (K, ef)
        assert torch.equal(a[2][:, 1], b[2][:, 1]) and torch.equal(a[2][:, 3], b[2][:, 3]), (K, ef)
    Y = synthdata.base("deep_like", 3000)
    idy = hnsw.Index(oracle.Graph.build(Y, M=8, efC=20, seed=1).packed(), Y)
    idy.add_lowp(hnsw.MODE_U8)
    cy, ey = idy.read_lowp(hnsw.MODE_U8)
    assert not ey and np.array_equal(cy, oracle.quantize_u8(Y)[0])


def test_lowp_requires_copy(hnsw):
    X = synthdata.base("uniform16", 500)
    G = oracle.Graph.build(X, M=8, efC=20, seed=1)
    idx = hnsw.Index(G.packed(), X)
    with pytest.raises(hnsw.HnswError) as e:
        idx.search(torch.from_numpy(X[:3]).cuda(), 5, 10, mode=hnsw.MODE_FP8)
    assert e.value.code == 1


@pytest.mark.parametrize("kind", [1, 2, 4])
def test_lowp_parity_scheduled(hnsw, monkeypatch, kind):
    """Low-precision traversal and re-rank in the scheduled form (descents
    first, layer 0 reordered), forced on a small batch."""
    print(f"case lowp scheduled kind={kind}", flush=True)
    monkeypatch.setenv("HNSW_SCHEDULE", "2")
    X = synthdata.base("deep_like", 6000)
    Q = synthdata.queries("deep_like", 700)
    G = oracle.Graph.build(X, M=16, efC=60, seed=4005)
    for ef in (10, 64):
        _lowp_parity(hnsw, X, Q, G, 10, ef, kind, oracle.L2)


FULL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "graphs", "sift_like_1M.bin")


@pytest.mark.skipif(not os.path.exists(FULL), reason="1M sift_like graph file not built")
@pytest.mark.parametrize("kind", [1, 2, 4])
def test_lowp_full_size_sampled(hnsw, kind):
    """The 1M x 128 workload in the benchmark's launch shape (all 10,000
    queries, K = 10, ef = 56 as timed): a sample against the oracle's
    low-precision mirror on the same graph."""
    print(f"case lowp sift_like 1M full size kind={kind}", flush=True)
    p = hnsw.graphfile.read(FULL)
    X = synthdata.base("sift_like", p["n"])
    Q = synthdata.queries("sift_like", 10000)
    idx = hnsw.Index(p, X)
    idx.add_lowp(kind)
    G = oracle.Graph.from_packed(X, p)
    _, dec, sc = QUANT[kind](X)
    G.set_lowp(dec, sc)
    sample = np.random.default_rng(1).choice(10000, size=150, replace=False)
    for K, ef in ((10, 56), (10, 128)):
        ids, ds = idx.search(torch.from_numpy(Q).cuda(), K, ef, mode=kind)
        torch.cuda.synchronize()
        ids, ds = ids.cpu().numpy(), ds.cpu().numpy()
        oi, od = G.search(Q[sample], K, ef, nthreads=8)
        r = parity.compare(ids[sample], ds[sample], oi, od, X, Q[sample], oracle.L2)
        print(f"  K={K} ef={ef}: {r['equal']} equal, {r['exempt']} exempt, {r['fail']} fail", flush=True)
        assert r["fail"] == 0 and r["exempt"] == 0
        # every query: distinct ids, sorted, and the distances are the exact fp32 ones (re-rank)
        assert all(len(set(row)) == K for row in ids)
        assert (np.diff(ds, axis=1) >= 0).all()
        assert np.array_equal(oracle.pair_dist(X, Q, ids).astype(np.float32), ds)
    G.set_lowp(None, None)
