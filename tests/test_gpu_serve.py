"""Continuous-batching serving loop on the GPU: every request's result equals
the oracle's search with the same (query, k, ef, mode) -- the plain search,
the low-precision mirror for BF16 and FP8, the learned search with the same
net -- and the standalone batch search, alone and in a mixed Poisson stream
over two indices; admission backpressure and refusals."""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import mlp_ref

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
def setup(hnsw):
    out = {}
    for name, n in (("uniform16", 10000), ("sift_like", 20000)):
        X = synthdata.base(name, n)
        Q = synthdata.queries(name, 400)
        G = oracle.Graph.build(X, M=16, efC=100, seed=3)
        idx = hnsw.Index(G.packed(), X)
        idx.add_lowp(hnsw.MODE_BF16)
        idx.add_lowp(hnsw.MODE_FP8)
        params = mlp_ref.init(7)
        net = hnsw.Mlp(params, tau=1.0, jmax=2)
        out[name] = (X, Q, idx, net)
        ORACLE[name] = (G, oracle.bf16_net(params), 1.0, 2)
    return out


ORACLE = {}


def _oracle_one(hnsw, name, X, q, k, ef, mode):
    """The oracle's answer to one request (ids, float distances)."""
    G, wnet, tau, jmax = ORACLE[name]
    q = np.ascontiguousarray(q.reshape(1, -1), dtype=np.float32)
    if mode == hnsw.MODE_LEARNED:
        r = G.search_learned(q, k, ef, net=wnet, tau=tau, jmax=jmax)
        return r["ids"][0], r["dists"][0]
    if mode in (hnsw.MODE_BF16, hnsw.MODE_FP8):
        key = (name, mode)
        if key not in _MIRRORS:
            _MIRRORS[key] = (oracle.quantize_bf16 if mode == hnsw.MODE_BF16 else oracle.quantize_fp8)(X)[1:]
        G.set_lowp(*_MIRRORS[key])
        try:
            i, d = G.search(q, k, ef)
        finally:
            G.set_lowp(None, None)
        return i[0], d[0]
    i, d = G.search(q, k, ef)
    return i[0], d[0]


_MIRRORS = {}


def _wait(srv, ticket, k, deadline):
    import time

    while True:
        r = srv.poll(ticket, k)
        if r is not None:
            return r
        assert time.time() < deadline, f"request {ticket} not served in time"


def _standalone(hnsw, idx, net, Q, k, ef, mode):
    ids, ds = idx.search(torch.from_numpy(np.ascontiguousarray(Q)).cuda(), k, ef, mode=mode,
                         mlp=net if mode == hnsw.MODE_LEARNED else None)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), ds.cpu().numpy()


def test_submit_poll_equals_batch(hnsw, setup):
    print("case serve submit/poll uniform16", flush=True)
    X, Q, idx, net = setup["uniform16"]
    import time

    srv = hnsw.Server(idx, mlp=net, slots=64, waves=64, ef_max=256, k_max=64, budget_s=30.0)
    deadline = time.time() + 20.0
    try:
        rng = np.random.default_rng(0)
        reqs = []
        # the first request alone, then a stream
        t0 = srv.submit(Q[0], 10, 32, hnsw.MODE_PLAIN)
        first = _wait(srv, t0, 10, deadline)
        for i in range(200):
            k = int(rng.choice([1, 10, 64]))
            ef = int(rng.integers(k, 257))
            mode = int(rng.choice([hnsw.MODE_PLAIN, hnsw.MODE_BF16, hnsw.MODE_FP8, hnsw.MODE_LEARNED]))
            while True:
                try:
                    t = srv.submit(Q[i], k, ef, mode)
                    break
                except hnsw.HnswError as e:
                    assert e.code == 6
                    assert time.time() < deadline, "no slot freed in time"
                    for r in reqs:
                        if r[-1] is None:
                            r[-1] = srv.poll(r[0], r[2])
            reqs.append([t, i, k, ef, mode, None])
        for r in reqs:
            if r[-1] is None:
                r[-1] = _wait(srv, r[0], r[2], deadline)
    finally:
        srv.stop()
    ids, _ = _standalone(hnsw, idx, None, Q[:1], 10, 32, hnsw.MODE_PLAIN)
    assert np.array_equal(first[0], ids[0])
    for t, i, k, ef, mode, res in reqs:
        ids, ds = _standalone(hnsw, idx, net, Q[i:i + 1], k, ef, mode)
        assert np.array_equal(res[0], ids[0]) and np.array_equal(res[1], ds[0]), (i, k, ef, mode)
        oi, od = _oracle_one(hnsw, "uniform16", X, Q[i], k, ef, mode)
        assert np.array_equal(res[0], oi) and np.array_equal(res[1], od), ("oracle", i, k, ef, mode)


def test_backpressure_and_refusals(hnsw, setup):
    X, Q, idx, net = setup["uniform16"]
    srv = hnsw.Server(idx, mlp=None, slots=8, waves=2, ef_max=64, k_max=10, budget_s=30.0)
    try:
        with pytest.raises(hnsw.HnswError) as e:
            srv.submit(Q[0], 10, 100)
        assert e.value.code == 4  # ef above ef_max
        with pytest.raises(hnsw.HnswError) as e:
            srv.submit(Q[0], 11, 20)
        assert e.value.code == 4  # k above k_max
        with pytest.raises(hnsw.HnswError) as e:
            srv.submit(Q[0], 10, 20, hnsw.MODE_U8)  # the serving kernel runs plain, learned, BF16 and FP8
        assert e.value.code == 1
        tickets = [srv.submit(Q[i], 10, 32) for i in range(8)]
        with pytest.raises(hnsw.HnswError) as e:
            srv.submit(Q[8], 10, 32)
        assert e.value.code == 6  # all slots occupied until results are taken
        import time

        deadline = time.time() + 20.0
        got = {t: _wait(srv, t, 10, deadline) for t in tickets}
        srv.submit(Q[8], 10, 32)  # a slot is free again
    finally:
        srv.stop()
    ids, ds = _standalone(hnsw, idx, None, Q[:8], 10, 32, hnsw.MODE_PLAIN)
    for j, t in enumerate(tickets):
        assert np.array_equal(got[t][0], ids[j])


def test_mixed_poisson_stream_two_indices(hnsw, setup):
    """Requests arriving while others run (Poisson, two indices, mixed k/ef/mode):
    each result is the standalone result."""
    print("case serve replay two indices", flush=True)
    names = ["uniform16", "sift_like"]
    servers = [hnsw.Server(setup[nm][2], mlp=setup[nm][3], slots=512, waves=256, ef_max=512, k_max=100,
                           budget_s=60.0) for nm in names]
    try:
        rng = np.random.default_rng(42)
        n = 4000
        arrival = np.cumsum(rng.exponential(1.0 / 50000.0, n))
        server_of = rng.integers(0, 2, n).astype(np.uint32)
        qidx = rng.integers(0, 400, n).astype(np.uint32)
        k = rng.choice([1, 10, 100], n).astype(np.uint32)
        ef = np.array([rng.integers(kk, 513) for kk in k], dtype=np.uint32)
        mode = rng.choice([hnsw.MODE_PLAIN, hnsw.MODE_BF16, hnsw.MODE_FP8, hnsw.MODE_LEARNED], n).astype(np.int32)
        mode[(k > 64) & (mode == hnsw.MODE_LEARNED)] = hnsw.MODE_PLAIN
        r = hnsw.replay(servers, [setup[nm][1] for nm in names], arrival, server_of, qidx, k, ef, mode,
                        out_stride=100, timeout_s=30.0)
    finally:
        for s in servers:
            s.stop()
    lat = r["t_done"] - arrival
    print(f"  p50 {np.percentile(lat, 50) * 1e3:.3f} ms  p99 {np.percentile(lat, 99) * 1e3:.3f} ms", flush=True)
    assert (lat > 0).all()
    # group identical (server, k, ef, mode) requests for the standalone check
    for s_i, nm in enumerate(names):
        X, Q, idx, net = setup[nm]
        for i in np.flatnonzero(server_of == s_i)[:600]:
            ids, ds = _standalone(hnsw, idx, net, Q[qidx[i]:qidx[i] + 1], int(k[i]), int(ef[i]), int(mode[i]))
            assert np.array_equal(r["ids"][i, :k[i]], ids[0]), (nm, i)
            assert np.array_equal(r["dists"][i, :k[i]], ds[0]), (nm, i)
        # every served request of this index against the oracle
        for i in np.flatnonzero(server_of == s_i):
            oi, od = _oracle_one(hnsw, nm, X, Q[qidx[i]], int(k[i]), int(ef[i]), int(mode[i]))
            assert np.array_equal(r["ids"][i, :k[i]], oi), ("oracle", nm, i, int(k[i]), int(ef[i]), int(mode[i]))
            assert np.array_equal(r["dists"][i, :k[i]], od), ("oracle", nm, i)


def test_free_while_serving_returns_at_once(hnsw, setup):
    """Releasing an index (or net) while a server kernel is resident must not
    wait for the device to go idle: the library holds such frees until the
    last server stops.  The server's short budget bounds the test."""
    import time

    X, Q, idx, net = setup["uniform16"]
    srv = hnsw.Server(idx, mlp=None, slots=8, waves=4, ef_max=64, k_max=10, budget_s=8.0)
    try:
        G = oracle.Graph.build(X[:500], M=8, efC=20, seed=1)
        extra = hnsw.Index(G.packed(), X[:500])
        extra_net = hnsw.Mlp(mlp_ref.init(3), tau=0.0, jmax=0)
        t0 = time.time()
        extra.close()
        del extra_net
        dt = time.time() - t0
        assert dt < 2.0, f"free blocked for {dt:.1f} s while a server ran"
        t = srv.submit(Q[0], 10, 32)
        assert _wait(srv, t, 10, time.time() + 5.0) is not None
    finally:
        srv.stop()
