"""Python binding of the gfx950 HNSW query library (``libhnsw_gpu.so``).

Argument marshalling only: tensors are passed to the C ABI of
``include/hnsw_gpu.h`` as raw device pointers on the current torch stream;
every step of the search runs in the library's HIP kernels.  There is no CPU
fallback: if the library is missing the import of :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import graphfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhnsw_gpu.so")

HNSW_L2SQ, HNSW_IP = 0, 1
MODE_PLAIN, MODE_BF16, MODE_FP8, MODE_LEARNED, MODE_U8 = 0, 1, 2, 3, 4
EF_MAX, DIM_MAX, DEG_MAX = 1024, 256, 64
NOALLOC_MAX_QUERIES = 262144

STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "device error", 4: "unsupported size",
          5: "malformed graph", 6: "busy"}


class HnswError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn}: {STATUS.get(code, code)} ({code})")
        self.code = code


class GraphDesc(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("dim", C.c_uint32), ("metric", C.c_uint32),
        ("M", C.c_uint32), ("Mmax", C.c_uint32), ("Mmax0", C.c_uint32),
        ("max_level", C.c_uint32), ("entry_point", C.c_uint32),
        ("vectors", C.c_void_p), ("levels", C.c_void_p), ("adj0", C.c_void_p),
        ("upper_off", C.c_void_p), ("adjU", C.c_void_p), ("n_upper_rows", C.c_uint64),
    ]


class BuildParams(C.Structure):
    _fields_ = [
        ("M", C.c_uint32), ("Mmax", C.c_uint32), ("Mmax0", C.c_uint32), ("efC", C.c_uint32),
        ("mL", C.c_double), ("seed", C.c_uint64), ("keep_pruned", C.c_int),
        ("batch_div", C.c_uint32), ("batch_max", C.c_uint32), ("select_simple", C.c_int),
        ("extend_candidates", C.c_int),
    ]


# name -> (restype, argtypes); the exported symbols of include/hnsw_gpu.h
_vp, _u32, _u64, _i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
SIGNATURES = {
    "hnsw_status_str": (C.c_char_p, [C.c_int]),
    "hnsw_index_upload": (C.c_int, [C.POINTER(GraphDesc), _vp, C.POINTER(_vp)]),
    "hnsw_index_free": (None, [_vp]),
    "hnsw_index_info": (C.c_int, [_vp, _vp]),
    "hnsw_index_export": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "hnsw_index_build": (C.c_int, [_vp, _u32, _u32, _i32, C.POINTER(BuildParams), _vp, C.POINTER(_vp)]),
    "hnsw_select_heuristic": (C.c_int, [_vp, _vp, _vp, _u32, _u32, _u32, _i32, _i32, _i32, _vp, _vp]),
    "hnsw_search_batch": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp]),
    "hnsw_search_batch_ex": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "hnsw_search_batch_noalloc": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "hnsw_bruteforce_knn": (C.c_int, [_vp, _vp, _u32, _u32, _vp, _vp, _vp]),
    "hnsw_read_probe": (C.c_int, [_vp, _u64, _vp, _u32, _vp]),
    "hnsw_index_add_lowp": (C.c_int, [_vp, _i32, _vp]),
    "hnsw_index_read_lowp": (C.c_int, [_vp, _i32, _vp, _vp]),
    "hnsw_search_learned_trace": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "hnsw_server_start": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _u32, C.c_double, C.POINTER(_vp)]),
    "hnsw_server_submit": (C.c_int, [_vp, _vp, _u32, _u32, _i32, C.POINTER(_u64)]),
    "hnsw_server_poll": (C.c_int, [_vp, _u64, _vp, _vp, C.POINTER(_i32)]),
    "hnsw_server_stop": (C.c_int, [_vp]),
    "hnsw_serve_replay": (C.c_int, [_vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                    C.c_double]),
    "hnsw_mlp_create": (C.c_int, [_vp, C.c_float, _i32, _u32, _u32, C.POINTER(_vp)]),
    "hnsw_mlp_free": (None, [_vp]),
    "hnsw_mlp_forward": (C.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "hnsw_mlp_grad": (C.c_int, [_vp, _vp, _vp, _u32, C.c_float, _vp, _vp, _vp]),
    "hnsw_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, C.c_float, C.c_float, C.c_float, C.c_float, _u32, _vp]),
}

MLP_PARAMS = 5890

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1603_09320_amd.build_ext.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, code: int):
    if code != 0:
        raise HnswError(fn, code)


def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _np(a):
    return a.ctypes.data_as(C.c_void_p)


class Index:
    """A graph uploaded to the current GPU (an ``hnsw_index``)."""

    def __init__(self, graph: dict, vectors: np.ndarray, stream=None):
        X = np.ascontiguousarray(vectors, dtype=np.float32)
        if X.shape != (graph["n"], graph["dim"]):
            raise ValueError(f"vectors {X.shape} do not match graph ({graph['n']}, {graph['dim']})")
        self._arrays = [X, np.ascontiguousarray(graph["levels"], dtype=np.uint8),
                        np.ascontiguousarray(graph["adj0"], dtype=np.uint32),
                        np.ascontiguousarray(graph["upper_off"], dtype=np.int32),
                        np.ascontiguousarray(graph["adjU"], dtype=np.uint32)]
        X, lv, a0, uo, aU = self._arrays
        d = GraphDesc(graph["n"], graph["dim"], graph["metric"], graph["M"], graph["Mmax"], graph["Mmax0"],
                      graph["max_level"], graph["entry_point"], _np(X).value, _np(lv).value, _np(a0).value,
                      _np(uo).value, _np(aU).value if aU.size else None, aU.shape[0] if aU.size else 0)
        h = C.c_void_p()
        _check("hnsw_index_upload", lib().hnsw_index_upload(C.byref(d), _stream_ptr(stream), C.byref(h)))
        self._h = h
        self._arrays = None
        self.n, self.dim, self.metric = graph["n"], graph["dim"], graph["metric"]

    @classmethod
    def from_file(cls, path: str, vectors: np.ndarray, stream=None) -> "Index":
        return cls(graphfile.read(path), vectors, stream)

    @classmethod
    def build(cls, vectors: np.ndarray, metric: int = HNSW_L2SQ, M: int = 16, Mmax=None, Mmax0=None, efC: int = 200,
              mL=None, seed: int = 1, keep_pruned: bool = False, batch_div: int = 16, batch_max: int = 65536,
              heuristic: bool = True, extend: bool = False, stream=None) -> "Index":
        """Graph construction on the GPU (``hnsw_index_build``): INSERT in batches of at
        most 1/batch_div of the elements inserted so far (batch_max at most).  extend:
        Alg. 4's extendCandidates."""
        import math

        X = np.ascontiguousarray(vectors, dtype=np.float32)
        n, dim = X.shape
        p = BuildParams(M, M if Mmax is None else Mmax, 2 * M if Mmax0 is None else Mmax0, efC,
                        1.0 / math.log(M) if mL is None else mL, seed, int(keep_pruned), batch_div, batch_max,
                        int(not heuristic), int(extend))
        h = C.c_void_p()
        _check("hnsw_index_build", lib().hnsw_index_build(_np(X), n, dim, metric, C.byref(p), _stream_ptr(stream),
                                                          C.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self._arrays = None
        self.n, self.dim, self.metric = n, dim, metric
        return self

    def export(self) -> dict:
        """The graph in packed form (``hnsw_index_export``), keys as the graph files use."""
        inf = self.info()
        n, rows = inf["n"], inf["rows"]
        lv = np.empty(n, dtype=np.uint8)
        a0 = np.empty((n, inf["Mmax0"]), dtype=np.uint32)
        uo = np.empty(n, dtype=np.int32)
        aU = np.empty((max(rows, 1), inf["Mmax"]), dtype=np.uint32)
        _check("hnsw_index_export", lib().hnsw_index_export(self._h, _np(lv), _np(a0), _np(uo), _np(aU)))
        d = dict(inf)
        d.update(levels=lv, adj0=a0, upper_off=uo, adjU=aU[:rows])
        return d

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = np.zeros(10, dtype=np.uint64)
        _check("hnsw_index_info", lib().hnsw_index_info(self._h, _np(out)))
        keys = ["n", "dim", "metric", "M", "Mmax", "Mmax0", "max_level", "entry_point", "device_bytes", "rows"]
        return {k: int(v) for k, v in zip(keys, out)}

    def search_learned_trace(self, queries, k: int, ef: int, mlp, stream=None):
        """Learned search that also returns per-checkpoint features and outputs
        (float32 [n][max_ckpt][26], NaN where a checkpoint was not reached)."""
        import torch

        q = queries.contiguous()
        n = q.shape[0]
        ids = torch.empty((n, k), dtype=torch.int32, device=q.device)
        dists = torch.empty((n, k), dtype=torch.float32, device=q.device)
        cnt = torch.zeros((n, 4), dtype=torch.int32, device=q.device)
        tr = torch.full((n, mlp.max_ckpt, 26), float("nan"), dtype=torch.float32, device=q.device)
        _check("hnsw_search_learned_trace", lib().hnsw_search_learned_trace(
            self._h, _dptr(q), n, k, ef, mlp.handle, _dptr(ids), _dptr(dists), _dptr(cnt), _dptr(tr),
            _stream_ptr(stream)))
        return ids, dists, cnt, tr

    def add_lowp(self, kind: int, stream=None):
        """Quantise the store on the device (``MODE_BF16``, ``MODE_FP8`` or ``MODE_U8``)."""
        _check("hnsw_index_add_lowp", lib().hnsw_index_add_lowp(self._h, kind, _stream_ptr(stream)))

    def read_lowp(self, kind: int):
        """(codes, scales): the device copy as numpy (BF16 uint16 [n][dim];
        FP8 uint8 [n][dim] and fp32 scales [n]; U8 uint8 [n][dim] and
        whether the copy is exact)."""
        lay = np.zeros(3, dtype=np.uint64)
        _check("hnsw_index_read_lowp", lib().hnsw_index_read_lowp(self._h, kind, None, _np(lay)))
        row = int(lay[0])
        extra = 4 * self.n if kind == MODE_FP8 else 0  # FP8: the row scales follow the rows
        buf = np.empty(self.n * row + extra, dtype=np.uint8)
        _check("hnsw_index_read_lowp", lib().hnsw_index_read_lowp(self._h, kind, _np(buf), _np(lay)))
        raw = buf[:self.n * row].reshape(self.n, row)
        if kind == MODE_BF16:
            return raw.view(np.uint16)[:, :self.dim].copy(), np.ones(self.n, np.float32)
        if kind == MODE_U8:
            return raw[:, :self.dim].copy(), bool(lay[2])
        off = int(lay[2])
        return raw[:, :self.dim].copy(), buf[off:off + extra].copy().view(np.float32)

    def close(self):
        if getattr(self, "_h", None):
            lib().hnsw_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search(self, queries, k: int, ef: int, mode: int = MODE_PLAIN, mlp=None, counters: bool = False,
               out=None, stream=None, no_alloc: bool = False):
        """K-NN-SEARCH (Alg. 5) of every row of ``queries`` (a float32 CUDA tensor [n][dim]).

        Returns (ids int32 [n][k], dists float32 [n][k]) and, with ``counters``,
        a uint32-valued int32 tensor [n][4] of work counters.  ``out`` may give
        preallocated (ids, dists[, counters]) tensors.  ``no_alloc`` calls
        ``hnsw_search_batch_noalloc`` (the library allocates nothing; with
        ``out`` given, neither does this method).
        """
        import torch

        if queries.dtype != torch.float32 or not queries.is_cuda or queries.dim() != 2:
            raise ValueError("queries must be a float32 CUDA tensor [n][dim]")
        if queries.shape[1] != self.dim:
            raise ValueError(f"queries have dim {queries.shape[1]}, index has {self.dim}")
        q = queries.contiguous()
        n = q.shape[0]
        if out is None:
            ids = torch.empty((n, k), dtype=torch.int32, device=q.device)
            dists = torch.empty((n, k), dtype=torch.float32, device=q.device)
            cnt = torch.zeros((n, 4), dtype=torch.int32, device=q.device) if counters else None
        else:
            ids, dists = out[0], out[1]
            cnt = out[2] if counters else None
        mlp_ptr = C.c_void_p(mlp.handle.value) if mlp is not None else None
        fn = "hnsw_search_batch_noalloc" if no_alloc else "hnsw_search_batch_ex"
        code = getattr(lib(), fn)(self._h, _dptr(q), n, k, ef, mode, mlp_ptr, _dptr(ids), _dptr(dists),
                                  _dptr(cnt) if cnt is not None else None, _stream_ptr(stream))
        _check(fn, code)
        return (ids, dists, cnt) if counters else (ids, dists)


class Mlp:
    """An inference net of the learned stop rule (``hnsw_mlp``).

    ``params``: fp32 [MLP_PARAMS] (W1[64][24], b1, W2[64][64], b2, W3[2][64], b3);
    ``tau``: stop threshold on output 0; ``jmax``: most ef halvings at the first
    checkpoint; ``period``/``max_ckpt``: checkpoint spacing and count.
    """

    def __init__(self, params, tau=0.0, jmax=0, period=8, max_ckpt=64):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters, got {p.size}")
        h = C.c_void_p()
        _check("hnsw_mlp_create", lib().hnsw_mlp_create(_np(p), float(tau), int(jmax), int(period), int(max_ckpt),
                                                        C.byref(h)))
        self._h = h
        self.params, self.tau, self.jmax, self.period, self.max_ckpt = p, tau, jmax, period, max_ckpt

    @property
    def handle(self):
        return self._h

    def save(self, path: str):
        np.savez(path, params=self.params, tau=self.tau, jmax=self.jmax, period=self.period, max_ckpt=self.max_ckpt)

    @classmethod
    def load(cls, path: str) -> "Mlp":
        z = np.load(path)
        return cls(z["params"], float(z["tau"]), int(z["jmax"]), int(z["period"]), int(z["max_ckpt"]))

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            lib().hnsw_mlp_free(h)

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: module globals may already be gone
            pass


def mlp_forward(params, x, stream=None):
    """FP32 forward of the perceptron: out [n][2] for device tensors params [MLP_PARAMS], x [n][24]."""
    import torch

    out = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
    _check("hnsw_mlp_forward", lib().hnsw_mlp_forward(_dptr(params), _dptr(x), x.shape[0], _dptr(out),
                                                      _stream_ptr(stream)))
    return out


def mlp_grad(params, x, y, lam=1.0, stream=None):
    """Gradient [MLP_PARAMS] and mean loss of the training objective (device tensors)."""
    import torch

    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check("hnsw_mlp_grad", lib().hnsw_mlp_grad(_dptr(params), _dptr(x), _dptr(y), x.shape[0], float(lam), _dptr(g),
                                                _dptr(loss), _stream_ptr(stream)))
    return g, loss


def mlp_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check("hnsw_mlp_adam", lib().hnsw_mlp_adam(_dptr(params), _dptr(grad), _dptr(m), _dptr(v), float(lr),
                                                float(beta1), float(beta2), float(eps), int(step),
                                                _stream_ptr(stream)))


class Server:
    """A continuous-batching server over one index (``hnsw_server``)."""

    def __init__(self, index: Index, mlp=None, slots=1024, waves=1024, ef_max=512, k_max=100, budget_s=60.0):
        h = C.c_void_p()
        _check("hnsw_server_start", lib().hnsw_server_start(index.handle, mlp.handle if mlp is not None else None,
                                                            slots, waves, ef_max, k_max, float(budget_s),
                                                            C.byref(h)))
        self._h, self.index, self.mlp, self.k_max = h, index, mlp, k_max

    @property
    def handle(self):
        return self._h

    def submit(self, query, k: int, ef: int, mode: int = MODE_PLAIN) -> int:
        q = np.ascontiguousarray(query, dtype=np.float32)
        t = C.c_uint64()
        _check("hnsw_server_submit", lib().hnsw_server_submit(self._h, _np(q), k, ef, mode, C.byref(t)))
        return t.value

    def poll(self, ticket: int, k: int):
        ids = np.empty(k, dtype=np.int32)
        ds = np.empty(k, dtype=np.float32)
        d = C.c_int32()
        _check("hnsw_server_poll", lib().hnsw_server_poll(self._h, ticket, _np(ids), _np(ds), C.byref(d)))
        return (ids, ds) if d.value else None

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check("hnsw_server_stop", lib().hnsw_server_stop(h))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def replay(servers, queries, arrival_s, server_of, qidx, k, ef, mode, out_stride=None, keep_results=True,
           timeout_s=60.0):
    """Open-loop replay of a request schedule (``hnsw_serve_replay``).

    ``queries``: one host float32 [nq][dim] array per server.  Returns dict of
    t_submit/t_done (seconds from the start) and, with ``keep_results``,
    ids/dists [n][out_stride].
    """
    n = len(arrival_s)
    out_stride = out_stride or int(np.max(k))
    qs = [np.ascontiguousarray(q, dtype=np.float32) for q in queries]
    srv = (C.c_void_p * len(servers))(*[s.handle.value for s in servers])
    qp = (C.c_void_p * len(qs))(*[q.ctypes.data for q in qs])
    arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
    so, qi = np.ascontiguousarray(server_of, np.uint32), np.ascontiguousarray(qidx, np.uint32)
    kk, ee, mm = np.ascontiguousarray(k, np.uint32), np.ascontiguousarray(ef, np.uint32), np.ascontiguousarray(
        mode, np.int32)
    ids = np.full((n, out_stride) if keep_results else (1, 1), -1, dtype=np.int32)
    ds = np.full(ids.shape, np.inf, dtype=np.float32)
    ts = np.zeros(n, dtype=np.float64)
    td = np.zeros(n, dtype=np.float64)
    code = lib().hnsw_serve_replay(srv, len(servers), qp, n, _np(arr), _np(so), _np(qi), _np(kk), _np(ee), _np(mm),
                                   out_stride if keep_results else 0, _np(ids) if keep_results else None,
                                   _np(ds) if keep_results else None, _np(ts), _np(td), float(timeout_s))
    _check("hnsw_serve_replay", code)
    out = dict(t_submit=ts, t_done=td)
    if keep_results:
        out.update(ids=ids, dists=ds)
    return out


def read_probe(buf, blocks: int = 2048, stream=None):
    """``hnsw_read_probe`` over a CUDA tensor (16-byte aligned, size a multiple of 16 bytes);
    returns the per-block XOR words, int32 [blocks] on the device."""
    import torch

    out = torch.empty(blocks, dtype=torch.int32, device=buf.device)
    _check("hnsw_read_probe", lib().hnsw_read_probe(_dptr(buf), buf.numel() * buf.element_size(), _dptr(out), blocks,
                                                    _stream_ptr(stream)))
    return out


def bruteforce(index: Index, queries, k: int, stream=None):
    """Exact K-NN (``hnsw_bruteforce_knn``): (ids int32 [n][k], fp64 distances [n][k])."""
    import torch

    n = queries.shape[0]
    ids = torch.empty((n, k), dtype=torch.int32, device=queries.device)
    d = torch.empty((n, k), dtype=torch.float64, device=queries.device)
    q = queries.contiguous()
    _check("hnsw_bruteforce_knn", lib().hnsw_bruteforce_knn(index.handle, _dptr(q), n, k, _dptr(ids), _dptr(d),
                                                            _stream_ptr(stream)))
    return ids, d


def select_heuristic(index: Index, base, cand, Mk: int, keep_pruned: bool = False, extend: bool = False, lc: int = 0,
                     stream=None):
    """The device's SELECT-NEIGHBORS-HEURISTIC on explicit lists (``hnsw_select_heuristic``):
    base int32 [nb], cand int32 [nb][nc] (-1 skipped) CUDA tensors; returns int32 [nb][Mk], -1 padded.
    extend: extendCandidates over the candidates' lists on layer lc."""
    import torch

    b = base.to(torch.int32).contiguous()
    c = cand.to(torch.int32).contiguous()
    out = torch.empty((b.shape[0], Mk), dtype=torch.int32, device=b.device)
    _check("hnsw_select_heuristic", lib().hnsw_select_heuristic(index.handle, _dptr(b), _dptr(c), b.shape[0],
                                                                c.shape[1], Mk, int(keep_pruned), int(extend),
                                                                int(lc), _dptr(out), _stream_ptr(stream)))
    return out


def search_batch(index: Index, queries, k: int, ef: int, stream=None):
    """The plain ``hnsw_search_batch`` entry point."""
    import torch

    n = queries.shape[0]
    ids = torch.empty((n, k), dtype=torch.int32, device=queries.device)
    dists = torch.empty((n, k), dtype=torch.float32, device=queries.device)
    _check("hnsw_search_batch", lib().hnsw_search_batch(index.handle, _dptr(queries), n, k, ef, _dptr(ids),
                                                        _dptr(dists), _stream_ptr(stream)))
    return ids, dists
