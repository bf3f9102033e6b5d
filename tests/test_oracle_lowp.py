"""Pins of the oracle's low-precision store (BF16 / OCP FP8-E4M3 with per-vector
scale) and of K-NN-SEARCH over it with an fp32 re-rank of the final W."""
import numpy as np
import pytest

import oracle
import synthdata

# Values fixed by the OCP 8-bit floating point specification (E4M3: bias 7,
# 3 mantissa bits, no infinities, S.1111.111 = NaN, max 448).
E4M3_KNOWN = {
    0x00: 0.0, 0x01: 2.0 ** -9, 0x07: 7 * 2.0 ** -9, 0x08: 2.0 ** -6, 0x38: 1.0, 0x39: 1.125, 0x3F: 1.875,
    0x40: 2.0, 0x77: 240.0, 0x78: 256.0, 0x7E: 448.0, 0xB8: -1.0, 0xFE: -448.0,
}


def test_e4m3_known_codes():
    for code, v in E4M3_KNOWN.items():
        assert oracle.e4m3_value(code) == v, hex(code)
    assert np.isnan(oracle.e4m3_value(0x7F)) and np.isnan(oracle.e4m3_value(0xFF))


def test_e4m3_codes_strictly_increase_and_round_trip():
    vals = [oracle.e4m3_value(c) for c in range(0x7F)]
    assert all(a < b for a, b in zip(vals, vals[1:]))
    assert len(set(vals)) == 127
    for c in range(0x7F):
        assert oracle.e4m3_rne(vals[c]) == c
        if c:
            assert oracle.e4m3_rne(-vals[c]) == 0x80 | c


def test_e4m3_round_to_nearest_even_and_saturation():
    vals = [oracle.e4m3_value(c) for c in range(0x7F)]
    for c in range(0x7E):
        mid = (vals[c] + vals[c + 1]) / 2  # exactly representable in float here
        even = c if c % 2 == 0 else c + 1
        assert oracle.e4m3_rne(np.float32(mid)) == even, hex(c)
        below = np.nextafter(np.float32(mid), np.float32(0))
        above = np.nextafter(np.float32(mid), np.float32(1e9))
        assert oracle.e4m3_rne(below) == c and oracle.e4m3_rne(above) == c + 1
    assert oracle.e4m3_rne(-0.0) == 0x80 and oracle.e4m3_rne(0.0) == 0x00  # the sign of zero is kept
    for x in (448.0, 449.0, 464.0, 1e6):
        assert oracle.e4m3_rne(x) == 0x7E and oracle.e4m3_rne(-x) == 0xFE


def test_bf16_rounding():
    # 1 + 2^-8 is the midpoint of 1 and 1 + 2^-7: ties to even (1.0); 1 + 3*2^-8 ties up to 1 + 2^-6
    assert oracle.bf16_rne(1.0) == 0x3F80
    assert oracle.bf16_rne(1.00390625) == 0x3F80
    assert oracle.bf16_rne(1.01171875) == 0x3F82
    assert oracle.bf16_rne(-2.0) == 0xC000
    # integers 0..255 need at most 8 significant bits: exact in bf16
    X = np.arange(256, dtype=np.float32)[:, None]
    codes, dec, sc = oracle.quantize_bf16(X)
    assert np.array_equal(dec, X) and (sc == 1).all()


def test_fp8_scale_maps_the_largest_magnitude_to_448():
    X = synthdata.base("deep_like", 2000)
    codes, dec, sc = oracle.quantize_fp8(X)
    mx = np.abs(X).max(axis=1)
    assert np.array_equal(sc, (mx / np.float32(448.0)).astype(np.float32))
    top = codes[np.arange(len(X)), np.abs(X).argmax(axis=1)] & 0x7F
    assert (top == 0x7E).all()
    # relative error of the per-vector scaled code: at most half a unit in the last place of
    # E4M3 (2^-4 relative for normals) plus the subnormal spacing
    err = np.abs(dec * sc[:, None] - X)
    assert (err <= np.abs(X) * 2.0 ** -4 + sc[:, None] * 2.0 ** -10 + 1e-12).all()


def test_bf16_traversal_equals_fp32_on_integer_data():
    """Integer coordinates 0..255 are exact in BF16, so traversal over the BF16
    copy is the fp32 traversal, and the re-rank leaves the same results."""
    X = synthdata.base("sift_like", 8000)
    Q = synthdata.queries("sift_like", 100)
    G = oracle.Graph.build(X, M=16, efC=100, seed=2003)
    ref = G.search(Q, 10, 64)
    codes, dec, sc = oracle.quantize_bf16(X)
    G.set_lowp(dec, sc)
    low = G.search(Q, 10, 64)
    assert np.array_equal(ref[0], low[0]) and np.array_equal(ref[1], low[1])


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_lowp_search_with_ef_ge_n_reranks_to_the_exact_answer(kind):
    """ef >= N keeps every reachable element in W; re-ranking W with the fp32
    vectors then returns the exact K-NN whatever the traversal precision."""
    rng = np.random.default_rng(5)
    X = rng.normal(size=(700, 24)).astype(np.float32)
    Q = rng.normal(size=(40, 24)).astype(np.float32)
    G = oracle.Graph.build(X, M=6, efC=40, seed=9)
    codes, dec, sc = (oracle.quantize_bf16 if kind == "bf16" else oracle.quantize_fp8)(X)
    G.set_lowp(dec, sc)
    ids, ds = G.search(Q, 10, 700)
    bi, bd = oracle.bruteforce(X, Q, 10, by_f32=True)
    assert np.array_equal(ids, bi)
    assert np.array_equal(ds, bd.astype(np.float32))
