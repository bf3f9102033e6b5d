"""Pins of the fp64 perceptron reference and of the learned stop rule's oracle."""
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


def test_oracle_network_arithmetic_is_bf16_exact():
    """The oracle's stop-rule network rounds inputs and hidden values to BF16 and
    accumulates in float; on inputs, weights and biases that are small integers
    every step is exact, so it equals the integer computation."""
    g = np.random.default_rng(0)
    p = mlp_ref.init(0)
    d = mlp_ref.unpack(p)
    for k in d:
        d[k] = g.integers(-3, 4, d[k].shape).astype(np.float64)
    net = mlp_ref.pack(d).astype(np.float32)
    F = g.integers(-4, 5, (50, mlp_ref.IN)).astype(np.float32)
    out = oracle.mlp_forward_bf16(net, F)
    h1 = np.maximum(F @ d["W1"].T + d["b1"], 0)
    h2 = np.maximum(h1 @ d["W2"].T + d["b2"], 0)
    z = h2 @ d["W3"].T + d["b3"]
    assert np.all(np.abs(z) < 2 ** 24)
    # hidden values may exceed 8 bits: compare against the same BF16 rounding of the integers
    ok = (np.abs(h1) < 256).all() and (np.abs(h2) < 256).all()
    if ok:
        assert np.array_equal(out, z.astype(np.float32))


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
    small, _ = G.search(Q, 10, 25)
    assert (r["info"][:, 1] == 0).all()
