"""The visited table under pressure, on the GPU through the C ABI, against the
oracle's exact visited set (Alg. 2).

The table may forget an id (it is then scored again) but never reports an
unseen one as visited; de-duplication against W (and among the keys of one
neighbourhood) keeps W free of repeats, so results must equal the oracle's.
These tests force a table of 256 slots (``HNSW_VISITED_LOG2=8``), far below
what the searches visit, for every store and the learned rule, in both launch
forms, up to ef = 1024; and they search graphs whose adjacency rows list one
element twice, where both copies are forgotten together.
"""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import mlp_ref
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


@pytest.fixture(scope="module")
def cfg():
    X = synthdata.base("uniform16", 10000)
    Q = synthdata.queries("uniform16", 300)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    return X, Q, G


def _mirror(hnsw, G, X, mode):
    if mode in (hnsw.MODE_BF16, hnsw.MODE_FP8):
        _, dec, sc = (oracle.quantize_bf16 if mode == hnsw.MODE_BF16 else oracle.quantize_fp8)(X)
        G.set_lowp(dec, sc)
    else:
        G.set_lowp(None, None)


def _check(hnsw, G, X, Q, idx, K, ef, mode, metric=oracle.L2, net=None, tau=0.0):
    q = torch.from_numpy(Q).cuda()
    mlp = hnsw.Mlp(net, tau=tau, jmax=0) if mode == hnsw.MODE_LEARNED else None
    ids, ds, cnt = idx.search(q, K, ef, mode=mode, mlp=mlp, counters=True)
    torch.cuda.synchronize()
    ids, ds, cnt = ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)
    if mode == hnsw.MODE_LEARNED:
        ro = G.search_learned(Q, K, ef, net=oracle.bf16_net(net), tau=tau, jmax=0, nthreads=8)
        oi, od, oc = ro["ids"], ro["dists"], ro["counters"]
    else:
        _mirror(hnsw, G, X, mode)
        oi, od, oc = G.search(Q, K, ef, nthreads=8, counters=True)
        G.set_lowp(None, None)
    r = parity.compare(ids, ds, oi, od, X, Q, metric)
    extra = float(cnt[:, 2].astype(np.float64).sum() / max(1.0, oc[:, 2].astype(np.float64).sum()))
    print(f"  mode={mode} K={K} ef={ef}: {r['equal']} equal, {r['exempt']} exempt, {r['fail']} fail; "
          f"layer-0 distance evaluations x{extra:.3f} of the exact set", flush=True)
    assert r["fail"] == 0 and r["exempt"] == 0, r["failed"][:10]
    assert np.array_equal(cnt[:, 3], oc[:, 3].astype(np.uint32))
    assert (cnt[:, 2] >= oc[:, 2].astype(np.uint32)).all()
    # no id twice in a row of the output
    for row in ids:
        v = row[row >= 0]
        assert len(np.unique(v)) == len(v)
    return extra


@pytest.mark.parametrize("sched", ["0", "2"])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_tiny_visited_table_all_modes(hnsw, cfg, monkeypatch, mode, sched):
    print(f"case visited table 256 slots mode={mode} sched={sched}", flush=True)
    monkeypatch.setenv("HNSW_VISITED_LOG2", "8")
    monkeypatch.setenv("HNSW_SCHEDULE", sched)
    X, Q, G = cfg
    idx = hnsw.Index(G.packed(), X)
    if mode in (1, 2):
        idx.add_lowp(mode)
    net = mlp_ref.init(5) if mode == 3 else None
    extras = []
    for K, ef in ((10, 64), (10, 256), (50, 1024)):
        # the learned rule with a threshold that never stops: every checkpoint
        # still runs, with the forgetting table underneath
        extras.append(_check(hnsw, G, X, Q, idx, K, ef, mode, net=net, tau=1e30))
    assert max(extras) > 1.05  # the table did forget


@pytest.mark.parametrize("sched", ["0", "2"])
@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("seed", [1, 2])
def test_repeated_links_with_forgetting(hnsw, monkeypatch, mode, sched, seed):
    """Rows that list one element two or more times, on a tie-heavy integer
    grid, with a table too small for the graph: both copies of a repeated id
    are forgotten in the same expansion, scored, and only one may enter W."""
    print(f"case repeated links seed={seed} mode={mode} sched={sched}", flush=True)
    monkeypatch.setenv("HNSW_VISITED_LOG2", "8")
    monkeypatch.setenv("HNSW_SCHEDULE", sched)
    X, adj = synthdata.random_graph(2000, 32, seed, dim=3, tie_grid=5, repeat_frac=0.3)
    rows_with_repeats = sum(len(set(r[r != 0xFFFFFFFF])) < (r != 0xFFFFFFFF).sum() for r in adj)
    assert rows_with_repeats > 1000
    n = len(X)
    packed = dict(metric=oracle.L2, M=16, Mmax=16, Mmax0=32, entry_point=0, max_level=0,
                  levels=np.zeros(n, np.uint8), adj0=adj, upper_off=np.full(n, -1, np.int32),
                  adjU=np.zeros((0, 16), np.uint32))
    G = oracle.Graph.from_packed(X, packed)
    Q = np.random.default_rng(seed).integers(0, 5, size=(300, 3)).astype(np.float32)
    idx = hnsw.Index(G.packed(), X)
    if mode in (1, 2):
        idx.add_lowp(mode)
    for K, ef in ((10, 5), (10, 40), (10, 200), (64, 1024)):
        _check(hnsw, G, X, Q, idx, K, ef, mode)
