"""Pins of the fp64 perceptron reference and of the learned stop rule's oracle."""
import os

import numpy as np

import oracle
import synthdata
from oracle import mlp_ref


def _batch(n, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, mlp_ref.IN))
    Y = np.stack([g.integers(0, 2, n), g.uniform(0.5, 2.0, n), g.normal(size=n), g.integers(0, 2, n)], axis=1)
    return X, Y


def test_backprop_matches_central_differences():
    """P12: the fp64 backward pass equals central finite differences of the objective."""
    p = mlp_ref.init(3).astype(np.float64)
    X, Y = _batch(40, 4)
    loss, g = mlp_ref.loss_and_grad(p, X, Y, lam=0.7)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(mlp_ref.NPARAMS, 300, replace=False), np.arange(mlp_ref.NPARAMS - 130,
                                                                                    mlp_ref.NPARAMS)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (mlp_ref.loss_and_grad(p + e, X, Y, 0.7)[0] - mlp_ref.loss_and_grad(p - e, X, Y, 0.7)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g[i])


def test_loss_special_cases():
    """With all weights zero the logits are the biases: BCE(0, y) = log 2 for every sample."""
    p = np.zeros(mlp_ref.NPARAMS)
    X, Y = _batch(10, 1)
    Y[:, 1] = 1.0
    Y[:, 3] = 0.0
    loss, g = mlp_ref.loss_and_grad(p, X, Y)
    assert abs(loss - np.log(2.0)) < 1e-15


def _int_net(seed, w2_per_row=4):
    """Integer parameters small enough that every value of the forward pass is
    an integer below 256 before the output layer (exact in BF16): weights in
    {-1, 0, 1}, a sparse and non-symmetric W2 (at most ``w2_per_row`` nonzeros
    per row), biases in [-2, 2]."""
    g = np.random.default_rng(seed)
    d = {"W1": g.integers(-1, 2, (mlp_ref.HID, mlp_ref.IN)), "b1": g.integers(-2, 3, mlp_ref.HID),
         "W2": np.zeros((mlp_ref.HID, mlp_ref.HID)), "b2": g.integers(-2, 3, mlp_ref.HID),
         "W3": g.integers(-1, 2, (mlp_ref.OUT, mlp_ref.HID)), "b3": g.integers(-2, 3, mlp_ref.OUT)}
    for o in range(mlp_ref.HID):
        cols = g.choice(mlp_ref.HID, size=w2_per_row, replace=False)
        d["W2"][o, cols] = g.choice([-1.0, 1.0], size=w2_per_row)
    assert not np.array_equal(d["W2"], d["W2"].T)
    return {k: np.asarray(v, dtype=np.float64) for k, v in d.items()}


def test_oracle_network_arithmetic_is_bf16_exact():
    """The oracle's stop-rule network rounds inputs and hidden values to BF16 and
    accumulates in float.  With integer inputs in [-2, 2] and the integer net of
    ``_int_net`` every hidden value is an integer below 256 and every sum is
    exact, so the network must equal the integer forward pass exactly -- with a
    non-symmetric W2, so a transposed weight matrix (or a swapped layer) fails."""
    for seed in range(4):
        d = _int_net(seed)
        net = mlp_ref.pack(d).astype(np.float32)
        F = np.random.default_rng(100 + seed).integers(-2, 3, (200, mlp_ref.IN)).astype(np.float64)
        h1 = np.maximum(F @ d["W1"].T + d["b1"], 0)
        h2 = np.maximum(h1 @ d["W2"].T + d["b2"], 0)
        z = h2 @ d["W3"].T + d["b3"]
        assert np.abs(h1).max() < 256 and np.abs(h2).max() < 256, "fixture must stay BF16-exact"
        assert (h1 > 0).mean() > 0.3 and (h2 > 0).mean() > 0.2 and np.unique(z).size > 10, "fixture too trivial"
        out = oracle.mlp_forward_bf16(net, F.astype(np.float32))
        assert np.array_equal(out, z.astype(np.float32)), seed
        # the transposed W2 gives a different answer on this fixture
        zt = np.maximum(h1 @ d["W2"] + d["b2"], 0) @ d["W3"].T + d["b3"]
        assert not np.array_equal(zt, z)


def test_oracle_network_within_bf16_bound_of_fp64_reference():
    """On random He-initialised nets (weights already BF16 values) and normal
    inputs, the BF16/float network differs from the fp64 reference forward of
    the same parameters by no more than the propagated rounding bound: each
    BF16 rounding of an input or a hidden value moves it by at most 2^-9 of its
    size, each float sum by at most 2^-23 per term."""
    u, e = 2.0 ** -9, 64 * 2.0 ** -23
    for seed in range(5):
        net = oracle.bf16_net(mlp_ref.init(seed))
        d = mlp_ref.unpack(net)
        F = np.random.default_rng(seed).normal(size=(300, mlp_ref.IN)) * 3
        out = oracle.mlp_forward_bf16(net, F.astype(np.float32)).astype(np.float64)
        z, (X, a1, h1, a2, h2) = mlp_ref.forward(net.astype(np.float64), F.astype(np.float32))
        # first-order bound on the deviation of each layer's values
        aW1, aW2, aW3 = np.abs(d["W1"]), np.abs(d["W2"]), np.abs(d["W3"])
        dx = u * np.abs(X)
        dh1 = dx @ aW1.T + e * (np.abs(X) @ aW1.T + np.abs(d["b1"]))
        dh1 = dh1 + u * (np.abs(h1) + dh1)
        dh2 = dh1 @ aW2.T + e * ((np.abs(h1) + dh1) @ aW2.T + np.abs(d["b2"]))
        dh2 = dh2 + u * (np.abs(h2) + dh2)
        dz = dh2 @ aW3.T + e * ((np.abs(h2) + dh2) @ aW3.T + np.abs(d["b3"]))
        err = np.abs(out - z)
        assert (err <= 1.01 * dz + 1e-30).all(), float((err / dz).max())
        assert (err > 0).any()  # the rounding is really applied


def _features_golden():
    out = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "checkpoint_features.txt")):
        line = line.split("#")[0].split()
        if line:
            out[line[0]] = line[1:]
    return out


def _quot(s):
    a, b = s.split("/")
    return np.float32(a) / np.float32(b)


def _one_layer(X, rows, deg):
    n = len(X)
    adj = np.full((n, deg), 0xFFFFFFFF, np.uint32)
    for i, nb in rows.items():
        adj[i, :len(nb)] = nb
    return dict(metric=oracle.L2, M=deg, Mmax=deg, Mmax0=deg, entry_point=0, max_level=0,
                levels=np.zeros(n, np.uint8), adj0=adj, adjU=np.zeros((0, deg), np.uint32))


def test_checkpoint_features_hand_worked():
    """The 24 checkpoint features of the learned stop rule on two hand-built
    one-layer graphs, against the values worked out by hand in
    tests/golden/checkpoint_features.txt (a path walked by a beam of 4, and a
    branching graph where the next element to expand sits at rank 1 of W and
    only one top-K id is new at the second checkpoint)."""
    gd = _features_golden()
    n = int(gd["path.points"][0])
    Xp = np.arange(n, dtype=np.float32)[:, None]
    rows = {i: [j for j in (i - 1, i + 1) if 0 <= j < n] for i in range(n)}
    xb = np.array([float(v) for v in gd["branch.x"]], np.float32)[:, None]
    brows = {}
    for item in gd["branch.links"]:
        a, b = item.split(":")
        brows[int(a)] = [int(v) for v in b.split(",")]
    for name, X, packed in (("path", Xp, _one_layer(Xp, rows, 2)), ("branch", xb, _one_layer(xb, brows, 4))):
        G = oracle.Graph.from_packed(X, packed)
        q = np.array([[float(gd[f"{name}.query"][0])]], np.float32)
        K, ef, T = int(gd[f"{name}.K"][0]), int(gd[f"{name}.ef"][0]), int(gd[f"{name}.T"][0])
        r = G.search_learned(q, K, ef, T=T, max_ckpt=2, trace=True)
        assert r["info"][0, 0] == 2, name
        for ck in (1, 2):
            want = np.array([_quot(v) for v in gd[f"{name}.ckpt{ck}"]], np.float32)
            got = r["feat"][0, ck - 1]
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, (name, ck, bad, got[bad], want[bad])


def test_learned_search_without_net_is_plain_and_traces_are_consistent():
    X = synthdata.base("uniform16", 6000)
    Q = synthdata.queries("uniform16", 60)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    r = G.search_learned(Q, 10, 120, trace=True)
    ids, ds = G.search(Q, 10, 120)
    assert np.array_equal(r["ids"], ids) and np.array_equal(r["dists"], ds)
    n_ck = r["info"][:, 0]
    exp0 = r["counters"][:, 3].astype(np.int64)
    assert np.array_equal(n_ck, np.minimum(exp0 // 8, 64))
    # the last recorded top-K list is the final top-K when the search ends right after it
    for i in range(len(Q)):
        k = n_ck[i]
        assert k > 0 and (r["feat"][i, :k, 23] == 1.0).all()
        assert (r["feat"][i, :k, 0] > 0).all()
        if exp0[i] == 8 * k:
            assert set(r["topk"][i, k - 1]) == set(ids[i])


def test_stop_rule_with_a_constant_net():
    """A net whose stop logit is the bias alone: bias > tau stops at the first
    checkpoint (8 expansions); bias < tau never stops."""
    X = synthdata.base("uniform16", 6000)
    Q = synthdata.queries("uniform16", 40)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    net = np.zeros(mlp_ref.NPARAMS, dtype=np.float32)
    net[-2] = 1.0  # b3[0]
    r = G.search_learned(Q, 10, 200, net=net, tau=0.5)
    assert (r["info"][:, 1] == 1).all() and (r["counters"][:, 3] == 8).all()
    r = G.search_learned(Q, 10, 200, net=net, tau=2.0)
    ids, _ = G.search(Q, 10, 200)
    assert (r["info"][:, 1] == 0).all() and np.array_equal(r["ids"], ids)
    # ef halving: out1 = b3[1] = -2.6 -> floor(3.1) = 3 halvings of 200 -> 25
    net[-2], net[-1] = -1.0, -2.6
    r = G.search_learned(Q, 10, 200, net=net, tau=0.0, jmax=5)
    assert (r["info"][:, 2] == 25).all()
    small, _, cs = G.search(Q, 10, 25, counters=True)
    assert (r["info"][:, 1] == 0).all()
    # the first 8 expansions are the same with ef 200 and 25 (nothing ranked
    # below 25th can be expanded before 25 others), so once W is cut to its 25
    # nearest the search is the plain one with ef 25
    assert (cs[:, 3] > 8).all()
    assert np.array_equal(r["ids"], small)
