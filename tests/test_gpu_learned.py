"""The learned stop rule on the GPU: perceptron training kernels against the
fp64 reference (gradient check), and the learned search against the
oracle's learned search with the same network."""
import os

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


def _batch(n, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, 24)).astype(np.float32)
    Y = np.stack([g.integers(0, 2, n), g.uniform(0.5, 2.0, n), g.normal(size=n), g.integers(0, 2, n)],
                 axis=1).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("n", [1, 63, 1000, 4099])
def test_mlp_forward_and_gradient_match_fp64(hnsw, n):
    print(f"case mlp grad n={n}", flush=True)
    p = mlp_ref.init(n)
    X, Y = _batch(n, n + 1)
    P, Xd, Yd = (torch.from_numpy(a).cuda() for a in (p, X, Y))
    z = hnsw.mlp_forward(P, Xd).cpu().numpy().astype(np.float64)
    zr, _ = mlp_ref.forward(p.astype(np.float64), X)
    assert np.abs(z - zr).max() <= 1e-5 * max(1.0, np.abs(zr).max())
    g, loss = hnsw.mlp_grad(P, Xd, Yd, lam=0.7)
    lr, gr = mlp_ref.loss_and_grad(p.astype(np.float64), X, Y, lam=0.7)
    g = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    assert abs(float(loss.cpu()) - lr) <= 1e-5 * max(1.0, abs(lr))


def test_adam_step_matches_reference(hnsw):
    p = mlp_ref.init(1)
    g = np.random.default_rng(2).normal(size=p.size).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    P, G, Md, Vd = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in (1, 2, 3):
        hnsw.mlp_adam(P, G, Md, Vd, 1e-3, step)
        pr, mr, vr = mlp_ref.adam_step(pr, g.astype(np.float64), mr, vr, 1e-3, step)
    assert np.allclose(P.cpu().numpy(), pr, rtol=1e-5, atol=1e-7)


def _net_with_spread_stops(G, Q, K, ef, seed):
    """A random net (weights already BF16 values) whose stop threshold sits
    inside the spread of its logits."""
    net = oracle.bf16_net(mlp_ref.init(seed))
    r = G.search_learned(Q, K, ef, trace=True, nthreads=8)
    feats = np.concatenate([r["feat"][i, :r["info"][i, 0]] for i in range(len(Q))])
    out = oracle.mlp_forward_bf16(net, feats)
    tau = float(np.quantile(out[:, 0], 0.8))
    # centre output 1 around -1.5 so the first checkpoint halves ef 0..3 times
    net[-1] = np.float32(net[-1] - np.median(out[:, 1]) - 1.5)
    return net, tau


@pytest.mark.parametrize("workload,metric,n", [("uniform16", oracle.L2, 10000), ("glove_like", oracle.IP, 20000)])
def test_checkpoint_features_and_outputs_equal_oracle(hnsw, workload, metric, n):
    """With a threshold that never stops, every checkpoint's 24 features and both
    network outputs equal the oracle's bit for bit."""
    print(f"case learned features {workload}", flush=True)
    X = synthdata.base(workload, n)
    Q = synthdata.queries(workload, 300)
    G = oracle.Graph.build(X, metric=metric, M=16, efC=100, seed=7)
    net = mlp_ref.init(5)
    r = G.search_learned(Q, 10, 200, trace=True, nthreads=8)
    mlp = hnsw.Mlp(net, tau=1e30, jmax=0)
    net = oracle.bf16_net(net)
    idx = hnsw.Index(G.packed(), X)
    ids, ds, cnt, tr = idx.search_learned_trace(torch.from_numpy(Q).cuda(), 10, 200, mlp)
    torch.cuda.synchronize()
    tr = tr.cpu().numpy()
    assert np.array_equal(ids.cpu().numpy(), r["ids"])
    for i in range(len(Q)):
        k = int(r["info"][i, 0])
        assert np.isnan(tr[i, k:]).all() and not np.isnan(tr[i, :k]).any(), i
        bad = np.argwhere(tr[i, :k, :24] != r["feat"][i, :k])
        assert bad.size == 0, (i, bad[:5], tr[i, bad[0][0], bad[0][1]], r["feat"][i, bad[0][0], bad[0][1]])
        out = oracle.mlp_forward_bf16(net, r["feat"][i, :k])
        assert np.array_equal(tr[i, :k, 24:], out), i


@pytest.mark.parametrize("workload,metric,n,dim_ef,sched", [("uniform16", oracle.L2, 10000, 200, "1"),
                                                            ("glove_like", oracle.IP, 20000, 256, "1"),
                                                            ("sift_like", oracle.L2, 20000, 128, "1"),
                                                            ("sift_like", oracle.L2, 20000, 128, "2")])
def test_learned_search_parity(hnsw, monkeypatch, workload, metric, n, dim_ef, sched):
    """sched "2" forces the scheduled form (descents first, layer 0 reordered)."""
    print(f"case learned parity {workload} n={n} sched={sched}", flush=True)
    monkeypatch.setenv("HNSW_SCHEDULE", sched)
    X = synthdata.base(workload, n)
    Q = synthdata.queries(workload, 400)
    G = oracle.Graph.build(X, metric=metric, M=16, efC=100, seed=7)
    K, ef = 10, dim_ef
    net, tau = _net_with_spread_stops(G, Q, K, ef, seed=11)
    for jmax in (0, 3):
        ro = G.search_learned(Q, K, ef, net=net, tau=tau, jmax=jmax, nthreads=8)
        stopped = (ro["info"][:, 1] > 0).mean()
        mlp = hnsw.Mlp(net, tau=tau, jmax=jmax)
        idx = hnsw.Index(G.packed(), X)
        ids, ds, cnt = idx.search(torch.from_numpy(Q).cuda(), K, ef, mode=hnsw.MODE_LEARNED, mlp=mlp,
                                  counters=True)
        torch.cuda.synchronize()
        ids, ds, cnt = ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)
        print(f"  jmax={jmax}: oracle stopped {stopped:.2f} of queries, efs {np.unique(ro['info'][:, 2])}",
              flush=True)
        assert 0.05 < stopped < 0.95
        assert np.array_equal(ids, ro["ids"]) and np.array_equal(ds, ro["dists"])
        assert np.array_equal(cnt[:, 3], ro["counters"][:, 3].astype(np.uint32))


def test_learned_mode_without_net_is_plain(hnsw):
    X = synthdata.base("uniform16", 5000)
    Q = synthdata.queries("uniform16", 100)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    idx = hnsw.Index(G.packed(), X)
    q = torch.from_numpy(Q).cuda()
    a = idx.search(q, 10, 64)
    b = idx.search(q, 10, 64, mode=hnsw.MODE_LEARNED, mlp=None)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    with pytest.raises(hnsw.HnswError):
        hnsw.Mlp(np.full(hnsw.MLP_PARAMS, np.nan, np.float32))


GLOVE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "graphs", "glove_like_1200k.bin")
NET = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1603_09320_amd", "nets",
                   "glove_like.mlp.npz")


GLOVE_GT = GLOVE[:-4] + ".gt.npz"


@pytest.mark.skipif(not (os.path.exists(GLOVE) and os.path.exists(NET) and os.path.exists(GLOVE_GT)),
                    reason="glove_like graph, net or oracle ground truth file not built")
def test_trained_net_gain_on_glove_like(hnsw):
    """What the trained network gains over the method without it, on the
    1.2M x 100 inner-product workload with its calibrated (ef, tau): the plain
    search at that ef, and the plain search at every smaller swept ef that
    reaches at least the learned recall, do more layer-0 expansions."""
    print("case learned gain glove_like 1.2M", flush=True)
    p = hnsw.graphfile.read(GLOVE)
    X = synthdata.base("glove_like", p["n"])
    Q = synthdata.queries("glove_like", 10000)[:4000]
    idx = hnsw.Index(p, X)
    q = torch.from_numpy(Q).cuda()
    gt = np.load(GLOVE_GT)["d64"][:4000, :10]
    net = hnsw.Mlp.load(NET)
    ef = int(np.load(NET)["ef"])

    def run(ef_, mode, mlp=None):
        ids, _, cnt = idx.search(q, 10, ef_, mode=mode, mlp=mlp, counters=True)
        torch.cuda.synchronize()
        ids, cnt = ids.cpu().numpy(), cnt.cpu().numpy().astype(np.float64)
        x = X[np.clip(ids, 0, None)].astype(np.float64)
        d = 1.0 - (x * Q[:, None, :].astype(np.float64)).sum(-1)
        dk = gt[:, 9:10]
        return float(((d <= dk + 1e-9 * np.abs(dk) + 1e-12).sum(1) / 10).mean()), float(cnt[:, 3].mean())

    rec_l, exp_l = run(ef, hnsw.MODE_LEARNED, net)
    rec_p, exp_p = run(ef, hnsw.MODE_PLAIN)
    print(f"  learned ef={ef} tau={net.tau}: recall {rec_l:.4f}, {exp_l:.1f} layer-0 expansions", flush=True)
    print(f"  plain   ef={ef}: recall {rec_p:.4f}, {exp_p:.1f}", flush=True)
    assert rec_l >= rec_p - 0.01
    assert exp_l <= 0.9 * exp_p
    # the plain search needs more work than the learned one to reach the learned recall
    for e in range(32, ef + 1, 32):
        r, x_ = run(e, hnsw.MODE_PLAIN)
        print(f"  plain   ef={e}: recall {r:.4f}, {x_:.1f}", flush=True)
        if r >= rec_l:
            assert x_ > exp_l


FULL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "graphs", "sift_like_1M.bin")
SIFT_NET = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1603_09320_amd",
                        "nets", "sift_like.mlp.npz")


@pytest.mark.skipif(not (os.path.exists(FULL) and os.path.exists(SIFT_NET)), reason="1M sift_like graph or net missing")
def test_learned_full_size_sampled(hnsw):
    """The trained sift_like net on the 1M x 128 workload at its calibrated ef,
    all 10,000 queries in the benchmark's launch shape: a sample against the
    oracle's learned search with the same (BF16) net."""
    print("case learned sift_like 1M full size", flush=True)
    p = hnsw.graphfile.read(FULL)
    X = synthdata.base("sift_like", p["n"])
    Q = synthdata.queries("sift_like", 10000)
    idx = hnsw.Index(p, X)
    z = np.load(SIFT_NET)
    mlp = hnsw.Mlp.load(SIFT_NET)
    ef = int(z["ef"])
    ids, ds, cnt = idx.search(torch.from_numpy(Q).cuda(), 10, ef, mode=hnsw.MODE_LEARNED, mlp=mlp, counters=True)
    torch.cuda.synchronize()
    ids, ds, cnt = ids.cpu().numpy(), ds.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)
    G = oracle.Graph.from_packed(X, p)
    sample = np.random.default_rng(2).choice(10000, size=150, replace=False)
    ro = G.search_learned(Q[sample], 10, ef, net=oracle.bf16_net(z["params"]), tau=float(z["tau"]),
                          jmax=int(z["jmax"]), T=int(z["period"]), max_ckpt=int(z["max_ckpt"]), nthreads=8)
    stopped = float((ro["info"][:, 1] > 0).mean())
    print(f"  ef={ef}: oracle stopped {stopped:.2f} of the sample", flush=True)
    assert np.array_equal(ids[sample], ro["ids"]) and np.array_equal(ds[sample], ro["dists"])
    assert np.array_equal(cnt[sample, 3], ro["counters"][:, 3].astype(np.uint32))
