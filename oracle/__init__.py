"""Python handle on the CPU oracle (``hnsw_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU product path.  It shares no
code with the GPU library; the two meet only in the seeded inputs of
``synthdata`` and in the graph file format written here (read by the product
with its own reader).

Graph file format (little endian), written by :func:`save_graph`:

    magic  b"HNSWGRF1"
    header 16 x u32: version=1, n, dim, metric (0 L2, 1 IP), M, Mmax, Mmax0,
           efC, max_level, entry_point, heuristic, extend, keep_pruned, 0, 0, 0
           then f64 mL, u64 level_seed, u64 n_upper_rows
    levels      u8  [n]            (zero padded to a multiple of 8 bytes)
    adj0        u32 [n][Mmax0]     0xFFFFFFFF marks an unused slot
    upper_off   i32 [n]            row of layer 1 in adjU, -1 for level 0
                                   (zero padded to a multiple of 8 bytes)
    adjU        u32 [rows][Mmax]   an element's rows for layers 1..level are
                                   consecutive
    checksum    u64                sum of u64 words w_i * (2i+1) mod 2^64 over
                                   every preceding byte (zero padded)
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hnsw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhnsw_oracle.so")
_lib = None

L2, IP = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB_PATH)
        vp, u32, u64, i32, f64 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_double
        L.or_levels.argtypes = [u64, u32, f64, vp]
        L.or_create.restype = vp
        L.or_create.argtypes = [vp, u32, u32, u32, u32, u32, u32, u32, f64, u64, i32, i32, i32]
        L.or_insert_range.restype = u32
        L.or_insert_range.argtypes = [vp, u32, u32]
        L.or_free.argtypes = [vp]
        L.or_search.argtypes = [vp, vp, u32, u32, u32, vp, vp, vp, i32]
        L.or_search_layer.restype = u32
        L.or_search_layer.argtypes = [vp, vp, vp, u32, u32, i32, vp, vp, vp]
        L.or_select_heuristic.restype = u32
        L.or_select_heuristic.argtypes = [vp, u32, vp, u32, u32, i32, i32, i32, vp]
        L.or_bruteforce.argtypes = [vp, u32, u32, u32, vp, u32, u32, i32, vp, vp, i32]
        L.or_pair_dist.argtypes = [vp, u32, u32, vp, vp, u64, u32, vp]
        L.or_info.argtypes = [vp, vp]
        L.or_export.argtypes = [vp, vp, vp, vp, vp]
        L.or_import.restype = vp
        L.or_import.argtypes = [vp, u32, u32, u32, u32, u32, u32, C.c_int64, i32, vp, vp, vp]
        L.or_set_vectors.argtypes = [vp, vp]
        L.or_set_lowp.argtypes = [vp, vp, vp]
        L.or_quantize_bf16.argtypes = [vp, u64, u32, vp, vp]
        L.or_quantize_fp8.argtypes = [vp, u64, u32, vp, vp, vp]
        L.or_e4m3_value.restype = C.c_float
        L.or_e4m3_value.argtypes = [C.c_uint8]
        L.or_e4m3_rne.restype = C.c_uint8
        L.or_e4m3_rne.argtypes = [C.c_float]
        L.or_bf16_rne.restype = C.c_uint16
        L.or_bf16_rne.argtypes = [C.c_float]
        L.or_search_learned.argtypes = [vp, vp, u32, u32, u32, i32, i32, vp, C.c_float, i32, vp, vp, vp, vp, vp,
                                        vp, i32]
        L.or_mlp_forward.argtypes = [vp, vp, u32, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def levels(seed: int, n: int, mL: float) -> np.ndarray:
    """Levels of Alg. 1 for elements 0..n-1 (counter-based, so prefix-stable)."""
    out = np.empty(n, dtype=np.uint8)
    lib().or_levels(seed, n, mL, _p(out))
    return out


class Graph:
    """An HNSW multilayer graph held by the oracle.

    Built by INSERT (Alg. 1) over ``X`` in id order, or imported from the
    packed form.  ``X`` (float32 [n][dim]) is kept alive by this object.
    """

    def __init__(self, handle, X: np.ndarray, params: dict):
        self._h = handle
        self.X = X
        self.params = params

    # -- construction ------------------------------------------------------
    @classmethod
    def create(cls, X, metric=L2, M=16, Mmax=None, Mmax0=None, efC=100, mL=None, seed=1,
               heuristic=True, extend=False, keep_pruned=False):
        X = np.ascontiguousarray(X, dtype=np.float32)
        n, dim = X.shape
        Mmax = M if Mmax is None else Mmax
        Mmax0 = 2 * M if Mmax0 is None else Mmax0
        mL = 1.0 / math.log(M) if mL is None else mL
        h = lib().or_create(_p(X), n, dim, metric, M, Mmax, Mmax0, efC, mL, seed,
                            int(heuristic), int(extend), int(keep_pruned))
        params = dict(metric=metric, M=M, Mmax=Mmax, Mmax0=Mmax0, efC=efC, mL=mL, seed=seed,
                      heuristic=int(heuristic), extend=int(extend), keep_pruned=int(keep_pruned))
        return cls(h, X, params)

    def insert_range(self, start: int, end: int) -> int:
        r = lib().or_insert_range(self._h, start, end)
        if r == 0xFFFFFFFF:
            raise ValueError("insert_range must continue from the last inserted id")
        return r

    @classmethod
    def build(cls, X, progress=None, chunk=20000, **kw):
        g = cls.create(X, **kw)
        n = g.X.shape[0]
        for s in range(0, n, chunk):
            g.insert_range(s, min(n, s + chunk))
            if progress:
                progress(min(n, s + chunk), n)
        return g

    @classmethod
    def from_packed(cls, X, packed: dict):
        X = np.ascontiguousarray(X, dtype=np.float32)
        lv = np.ascontiguousarray(packed["levels"], dtype=np.uint8)
        a0 = np.ascontiguousarray(packed["adj0"], dtype=np.uint32)
        aU = np.ascontiguousarray(packed["adjU"], dtype=np.uint32)
        if aU.size == 0:
            aU = np.zeros((1, packed["Mmax"]), dtype=np.uint32)
        n, dim = X.shape
        h = lib().or_import(_p(X), n, dim, packed["metric"], packed["M"], packed["Mmax"], packed["Mmax0"],
                            int(packed["entry_point"]), int(packed["max_level"]), _p(lv), _p(a0), _p(aU))
        g = cls(h, X, {k: packed[k] for k in ("metric", "M", "Mmax", "Mmax0")})
        g._keep = (lv, a0, aU)
        return g

    def __del__(self):
        if getattr(self, "_h", None):
            lib().or_free(self._h)
            self._h = None

    # -- queries -------------------------------------------------------------
    def info(self) -> dict:
        out = np.zeros(12, dtype=np.uint64)
        lib().or_info(self._h, _p(out))
        keys = ["n", "dim", "metric", "M", "Mmax", "Mmax0", "efC", "max_level", "entry_point", "rows",
                "n_inserted", "seed"]
        return {k: int(v) for k, v in zip(keys, out)}

    def packed(self) -> dict:
        """The packed adjacency arrays (see the module docstring)."""
        inf = self.info()
        n, rows = inf["n"], inf["rows"]
        lv = np.empty(n, dtype=np.uint8)
        a0 = np.empty((n, inf["Mmax0"]), dtype=np.uint32)
        uo = np.empty(n, dtype=np.int32)
        aU = np.empty((max(rows, 1), inf["Mmax"]), dtype=np.uint32)
        lib().or_export(self._h, _p(lv), _p(a0), _p(uo), _p(aU))
        d = dict(inf)
        d.update(levels=lv, adj0=a0, upper_off=uo, adjU=aU[:rows])
        for k in ("mL", "heuristic", "extend", "keep_pruned"):
            d[k] = self.params.get(k, 0)
        return d

    def search(self, Q, K: int, ef: int, nthreads: int = 1, counters: bool = False):
        """K-NN-SEARCH (Alg. 5) for every row of Q; returns (ids int32, dists fp32[, counters])."""
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        nq = Q.shape[0]
        ids = np.empty((nq, K), dtype=np.int32)
        ds = np.empty((nq, K), dtype=np.float32)
        cnt = np.zeros((nq, 4), dtype=np.uint64) if counters else None
        lib().or_search(self._h, _p(Q), nq, K, ef, _p(ids), _p(ds), _p(cnt) if counters else None, nthreads)
        return (ids, ds, cnt) if counters else (ids, ds)

    def search_layer(self, q, ep, ef: int, lc: int):
        """One SEARCH-LAYER (Alg. 2) call; returns (ids, dists) sorted and the distance count."""
        q = np.ascontiguousarray(q, dtype=np.float32)
        ep = np.ascontiguousarray(ep, dtype=np.uint32)
        cap = max(ef, len(ep))
        ids = np.empty(cap, dtype=np.int32)
        ds = np.empty(cap, dtype=np.float32)
        nd = np.zeros(1, dtype=np.uint64)
        m = lib().or_search_layer(self._h, _p(q), _p(ep), len(ep), ef, lc, _p(ids), _p(ds), _p(nd))
        return ids[:m], ds[:m], int(nd[0])

    def search_learned(self, Q, K: int, ef: int, net=None, tau: float = 0.0, jmax: int = 0, T: int = 8,
                       max_ckpt: int = 64, trace: bool = False, nthreads: int = 1):
        """K-NN-SEARCH with the learned stop rule (``net``: flat float32 parameters,
        weights already BF16 values) or, with ``net=None``, the plain search
        with a trace of checkpoint features and top-K lists.

        Returns dict(ids, dists, counters, info[, feat, topk]); info[i] =
        (checkpoints reached, checkpoint where the rule stopped or 0, ef at the end).
        """
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        nq = Q.shape[0]
        ids = np.empty((nq, K), dtype=np.int32)
        ds = np.empty((nq, K), dtype=np.float32)
        cnt = np.zeros((nq, 4), dtype=np.uint64)
        info = np.zeros((nq, 3), dtype=np.int32)
        feat = np.zeros((nq, max_ckpt, MLP_IN), dtype=np.float32) if trace else None
        topk = np.full((nq, max_ckpt, K), -1, dtype=np.int32) if trace else None
        w = None if net is None else np.ascontiguousarray(net, dtype=np.float32)
        if w is not None:
            assert w.size == MLP_PARAMS
        lib().or_search_learned(self._h, _p(Q), nq, K, ef, T, max_ckpt, _p(w) if w is not None else None,
                                float(tau), jmax, _p(ids), _p(ds), _p(cnt), _p(feat) if trace else None,
                                _p(topk) if trace else None, _p(info), nthreads)
        out = dict(ids=ids, dists=ds, counters=cnt, info=info)
        if trace:
            out.update(feat=feat, topk=topk)
        return out

    def set_lowp(self, decoded, scale):
        """Traverse over a low-precision copy (decoded values, per-vector scales) and
        re-rank the final W with the fp32 vectors; ``None`` restores the plain search."""
        if decoded is None:
            lib().or_set_lowp(self._h, None, None)
            self._lowp = None
            return
        dq = np.ascontiguousarray(decoded, dtype=np.float32)
        sc = np.ascontiguousarray(scale, dtype=np.float32)
        assert dq.shape == self.X.shape and sc.shape == (self.X.shape[0],)
        self._lowp = (dq, sc)
        lib().or_set_lowp(self._h, _p(dq), _p(sc))

    def select_heuristic(self, base_id: int, cand, M: int, lc: int = 0, extend=False, keep_pruned=False):
        cand = np.ascontiguousarray(cand, dtype=np.uint32)
        out = np.empty(max(M, 1) + len(cand), dtype=np.uint32)
        m = lib().or_select_heuristic(self._h, base_id, _p(cand), len(cand), M, lc, int(extend),
                                      int(keep_pruned), _p(out))
        return out[:m]


MLP_IN, MLP_HID, MLP_OUT = 24, 64, 2
MLP_PARAMS = MLP_HID * MLP_IN + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_OUT * MLP_HID + MLP_OUT


def bf16_net(params):
    """The inference form of fp32 parameters: weights rounded to BF16 (nearest
    even, by the oracle's own rounding), biases kept in float."""
    p = np.array(params, dtype=np.float32, copy=True)
    nW1, nW2, nW3 = MLP_HID * MLP_IN, MLP_HID * MLP_HID, MLP_OUT * MLP_HID
    for lo, n in ((0, nW1), (nW1 + MLP_HID, nW2), (nW1 + MLP_HID + nW2 + MLP_HID, nW3)):
        _, dec, _ = quantize_bf16(p[lo:lo + n].reshape(1, -1))
        p[lo:lo + n] = dec.ravel()
    return p


def mlp_forward_bf16(net, feat):
    """The stop-rule perceptron exactly as the search applies it (BF16 inputs and
    hidden values, float accumulation in input order)."""
    w = np.ascontiguousarray(net, dtype=np.float32)
    f = np.ascontiguousarray(feat, dtype=np.float32).reshape(-1, MLP_IN)
    out = np.empty((f.shape[0], MLP_OUT), dtype=np.float32)
    lib().or_mlp_forward(_p(w), _p(f), f.shape[0], _p(out))
    return out


def quantize_bf16(X):
    """fp32 -> bf16 codes (round to nearest even) and their exact float values."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    codes = np.empty(X.shape, dtype=np.uint16)
    dec = np.empty(X.shape, dtype=np.float32)
    lib().or_quantize_bf16(_p(X), X.shape[0], X.shape[1], _p(codes), _p(dec))
    return codes, dec, np.ones(X.shape[0], dtype=np.float32)


def quantize_fp8(X):
    """fp32 -> per-vector scaled FP8-E4M3 codes, scales, and the codes' exact float values."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    codes = np.empty(X.shape, dtype=np.uint8)
    dec = np.empty(X.shape, dtype=np.float32)
    sc = np.empty(X.shape[0], dtype=np.float32)
    lib().or_quantize_fp8(_p(X), X.shape[0], X.shape[1], _p(codes), _p(sc), _p(dec))
    return codes, dec, sc


def quantize_u8(X):
    """fp32 -> 8-bit integer codes (the integer store of Sec. 5.4's SIFT build):
    the nearest integer (ties to even), clamped to [0, 255]; returns codes, their
    float values and unit scales."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    codes = np.clip(np.rint(X), 0, 255).astype(np.uint8)
    return codes, codes.astype(np.float32), np.ones(X.shape[0], dtype=np.float32)


def e4m3_value(code: int) -> float:
    return float(lib().or_e4m3_value(code))


def e4m3_rne(x: float) -> int:
    return int(lib().or_e4m3_rne(x))


def bf16_rne(x: float) -> int:
    return int(lib().or_bf16_rne(x))


def bruteforce(X, Q, K: int, metric=L2, by_f32=False, nthreads: int = 1):
    """Exact K-NN by all distances (fp64); returns (ids int32 [nq][K], d64 [nq][K])."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    nq = Q.shape[0]
    ids = np.empty((nq, K), dtype=np.int32)
    d64 = np.empty((nq, K), dtype=np.float64)
    lib().or_bruteforce(_p(X), X.shape[0], X.shape[1], metric, _p(Q), nq, K, int(by_f32), _p(ids), _p(d64),
                        nthreads)
    return ids, d64


def pair_dist(X, Q, ids, metric=L2):
    """fp64 distance between query row i and each id in ids[i] (-1 gives +inf)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    out = np.empty(ids.shape, dtype=np.float64)
    per = ids.shape[1] if ids.ndim == 2 else 1
    lib().or_pair_dist(_p(X), X.shape[1], metric, _p(Q), _p(ids), ids.size, per, _p(out))
    return out


# --------------------------------------------------------------- graph files
MAGIC = b"HNSWGRF1"


def _checksum(buf: bytes) -> int:
    """Integrity word: sum over little-endian u64 words w_i (zero padded) of w_i * (2i + 1), mod 2^64."""
    a = np.frombuffer(buf, dtype=np.uint8)
    pad = (-len(a)) % 8
    if pad:
        a = np.concatenate([a, np.zeros(pad, dtype=np.uint8)])
    w = a.view(np.uint64)
    total = np.uint64(0)
    with np.errstate(over="ignore"):
        for s in range(0, len(w), 1 << 22):
            blk = w[s:s + (1 << 22)]
            k = np.arange(s, s + len(blk), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
            total = total + np.sum(blk * k, dtype=np.uint64)
    return int(total)


def save_graph(path: str, g: "Graph | dict"):
    p = g.packed() if isinstance(g, Graph) else g
    n, rows = p["n"], p["rows"]
    hdr = np.array([1, n, p["dim"], p["metric"], p["M"], p["Mmax"], p["Mmax0"], p.get("efC", 0),
                    p["max_level"], p["entry_point"], p.get("heuristic", 1), p.get("extend", 0),
                    p.get("keep_pruned", 0), 0, 0, 0], dtype=np.uint32)
    tail = np.array([p.get("mL", 0.0)], dtype=np.float64).tobytes() + \
        np.array([p.get("seed", 0), rows], dtype=np.uint64).tobytes()
    lv = np.asarray(p["levels"], dtype=np.uint8).tobytes()
    lv += b"\0" * ((-len(lv)) % 8)
    uo = np.asarray(p["upper_off"], dtype=np.int32).tobytes()
    uo += b"\0" * ((-len(uo)) % 8)
    chunks = [MAGIC, hdr.tobytes(), tail, lv, np.ascontiguousarray(p["adj0"], dtype=np.uint32).tobytes(), uo,
              np.ascontiguousarray(p["adjU"], dtype=np.uint32).tobytes()]
    body = b"".join(chunks)
    cs = _checksum(body)
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        f.write(body)
        f.write(np.array([cs], dtype=np.uint64).tobytes())
    os.replace(tmp, path)


def load_graph(path: str) -> dict:
    raw = np.fromfile(path, dtype=np.uint8)
    if raw[:8].tobytes() != MAGIC:
        raise ValueError("not a graph file")
    hdr = raw[8:72].view(np.uint32)
    mL = float(raw[72:80].view(np.float64)[0])
    seed, rows = (int(v) for v in raw[80:96].view(np.uint64))
    n, dim, metric, M, Mmax, Mmax0, efC, max_level, entry = (int(v) for v in hdr[1:10])
    off = 96
    lv = raw[off:off + n].copy()
    off += n + ((-n) % 8)
    a0 = raw[off:off + 4 * n * Mmax0].view(np.uint32).reshape(n, Mmax0).copy()
    off += 4 * n * Mmax0
    uo = raw[off:off + 4 * n].view(np.int32).copy()
    off += 4 * n + ((-4 * n) % 8)
    aU = raw[off:off + 4 * rows * Mmax].view(np.uint32).reshape(rows, Mmax).copy()
    off += 4 * rows * Mmax
    cs = int(raw[off:off + 8].view(np.uint64)[0])
    if cs != _checksum(raw[:off].tobytes()):
        raise ValueError("graph file checksum mismatch")
    return dict(n=n, dim=dim, metric=metric, M=M, Mmax=Mmax, Mmax0=Mmax0, efC=efC, max_level=max_level,
                entry_point=entry, heuristic=int(hdr[10]), extend=int(hdr[11]), keep_pruned=int(hdr[12]),
                mL=mL, seed=seed, rows=rows, levels=lv, adj0=a0, upper_off=uo, adjU=aU)

