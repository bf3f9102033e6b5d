"""GPU brute-force K-NN (matrix-core scan + fp64 rerank) against the oracle's
brute force, the plain definition of the problem (Sec. 1)."""
import os
import sys

import numpy as np
import pytest

import oracle
import synthdata

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hnsw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_09320_amd as h

    h.lib()
    return h


def _flat(X, metric):
    n = X.shape[0]
    return dict(n=n, dim=X.shape[1], metric=metric, M=4, Mmax=4, Mmax0=4, max_level=0, entry_point=0,
                levels=np.zeros(n, np.uint8), adj0=np.full((n, 4), 0xFFFFFFFF, np.uint32),
                upper_off=np.full(n, -1, np.int32), adjU=np.zeros((0, 4), np.uint32))


def _check(hnsw, X, Q, k, metric, exact_d=True):
    print(f"case bruteforce n={X.shape[0]} d={X.shape[1]} nq={Q.shape[0]} k={k} metric={metric}", flush=True)
    idx = hnsw.Index(_flat(X, metric), X)
    ids, d = hnsw.bruteforce(idx, torch.from_numpy(Q).cuda(), k)
    torch.cuda.synchronize()
    ids, d = ids.cpu().numpy(), d.cpu().numpy()
    oi, od = oracle.bruteforce(X, Q, k, metric=metric, nthreads=8)
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(d), fin)
    rel = np.abs(d[fin] - od[fin]) / np.maximum(np.abs(od[fin]), 1e-30)
    assert rel.max(initial=0) <= (0 if exact_d else 1e-12)
    mism = np.flatnonzero((ids != oi).any(axis=1))
    for i in mism:
        # only exchanges between elements at equal fp64 distance are allowed
        a = oracle.pair_dist(X, Q[i:i + 1], ids[i:i + 1], metric)[0]
        b = oracle.pair_dist(X, Q[i:i + 1], oi[i:i + 1], metric)[0]
        assert np.allclose(a, b, rtol=1e-12, atol=0), i
    return ids, d


def test_bruteforce_uniform16(hnsw):
    X = synthdata.base("uniform16", 10000)
    Q = synthdata.queries("uniform16", 500)
    _check(hnsw, X, Q, 10, oracle.L2, exact_d=False)


def test_bruteforce_integer_data_exact(hnsw):
    """SIFT-like integer coordinates: every fp32 partial sum is an exact integer,
    so ids and distances must equal the oracle's exactly."""
    X = synthdata.base("sift_like", 40000)
    Q = synthdata.queries("sift_like", 300)
    ids, d = _check(hnsw, X, Q, 100, oracle.L2)
    oi, od = oracle.bruteforce(X, Q, 100, nthreads=8)
    assert np.array_equal(ids, oi)


@pytest.mark.parametrize("k", [1, 33, 64, 128])
def test_bruteforce_inner_product_and_k(hnsw, k):
    X = synthdata.base("glove_like", 15000)
    Q = synthdata.queries("glove_like", 200)
    _check(hnsw, X, Q, k, oracle.IP, exact_d=False)


@pytest.mark.parametrize("n,dim", [(5, 3), (63, 17), (100, 130), (2000, 256)])
def test_bruteforce_ragged_and_padding(hnsw, n, dim):
    rng = np.random.default_rng(n + dim)
    X = rng.random((n, dim)).astype(np.float32)
    Q = rng.random((37, dim)).astype(np.float32)
    k = 10
    ids, d = _check(hnsw, X, Q, k, oracle.L2, exact_d=False)
    if n < k:
        assert (ids[:, n:] == -1).all() and np.isinf(d[:, n:]).all()


GT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "graphs", "sift_like_1M.gt.npz")


@pytest.mark.skipif(not os.path.exists(GT), reason="oracle ground truth file for sift_like 1M not built")
def test_bruteforce_full_size_against_oracle_file(hnsw):
    """1M x 128, all 10,000 queries, against the oracle's stored brute force."""
    print("case bruteforce sift_like 1M full size", flush=True)
    gt = np.load(GT)
    X = synthdata.base("sift_like", 1000000)
    Q = synthdata.queries("sift_like", 10000)
    idx = hnsw.Index(_flat(X, oracle.L2), X)
    ids, d = hnsw.bruteforce(idx, torch.from_numpy(Q).cuda(), 100)
    torch.cuda.synchronize()
    assert np.array_equal(ids.cpu().numpy(), gt["ids"][:, :100])
    assert np.array_equal(d.cpu().numpy(), gt["d64"][:, :100])
