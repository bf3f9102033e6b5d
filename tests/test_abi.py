"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/*.h, and rejects malformed input before
touching a device."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

import oracle
import synthdata

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hnsw():
    import paper_1603_09320_amd as h

    if not os.path.exists(h.LIB_PATH):
        from paper_1603_09320_amd import build_ext

        build_ext.build()
    h.lib()
    return h


def declared_functions():
    names = set()
    for path in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(hnsw_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported(hnsw):
    names = declared_functions()
    assert "hnsw_search_batch" in names and "hnsw_index_upload" in names
    raw = C.CDLL(hnsw.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) <= set(hnsw.SIGNATURES), set(names) - set(hnsw.SIGNATURES)


def test_status_strings(hnsw):
    for code, text in hnsw.STATUS.items():
        assert hnsw.lib().hnsw_status_str(code).decode() == text


def _desc(hnsw, p, X):
    keep = [np.ascontiguousarray(X, np.float32), np.ascontiguousarray(p["levels"], np.uint8),
            np.ascontiguousarray(p["adj0"], np.uint32), np.ascontiguousarray(p["upper_off"], np.int32),
            np.ascontiguousarray(p["adjU"], np.uint32)]
    ptr = [a.ctypes.data if a.size else None for a in keep]
    d = hnsw.GraphDesc(p["n"], p["dim"], p["metric"], p["M"], p["Mmax"], p["Mmax0"], p["max_level"],
                       p["entry_point"], ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], keep[4].shape[0])
    return d, keep


def _upload(hnsw, d):
    h = C.c_void_p()
    return hnsw.lib().hnsw_index_upload(C.byref(d), None, C.byref(h)), h


@pytest.fixture(scope="module")
def small():
    X = synthdata.base("uniform16", 2000)
    return X, oracle.Graph.build(X, M=8, efC=40, seed=3).packed()


def test_malformed_graphs_rejected_on_host(hnsw, small):
    X, p = small
    bad = []
    q = dict(p, adj0=p["adj0"].copy()); q["adj0"][5, 0] = p["n"]; bad.append((q, 5))          # link out of range
    q = dict(p, entry_point=p["n"]); bad.append((q, 5))                                         # entry out of range
    lv = p["levels"].copy(); z = int(np.flatnonzero(lv == 0)[0])
    q = dict(p, entry_point=z); bad.append((q, 5))                                              # entry not on top level
    if p["rows"]:
        q = dict(p, adjU=p["adjU"].copy())
        q["adjU"][0, 0] = z                                                                     # level-0 element on layer 1
        bad.append((q, 5))
        uo = p["upper_off"].copy(); uo[int(np.flatnonzero(lv > 0)[0])] = p["rows"]
        bad.append((dict(p, upper_off=uo), 5))                                                  # row range outside adjU
    bad.append((dict(p, dim=300), 4))                                                            # dim above the limit
    bad.append((dict(p, metric=7), 1))
    for q, want in bad:
        Xq = X if q["dim"] == X.shape[1] else np.zeros((p["n"], q["dim"]), np.float32)
        d, keep = _desc(hnsw, q, Xq)
        code, h = _upload(hnsw, d)
        assert code == want, (code, want)
        assert not h.value


def test_null_arguments(hnsw):
    L = hnsw.lib()
    assert L.hnsw_search_batch(None, None, 1, 1, 1, None, None, None) == 1
    assert L.hnsw_index_upload(None, None, None) == 1
    L.hnsw_index_free(None)
    assert L.hnsw_index_info(None, None) == 1


def test_no_device_reports_device_error(hnsw, small):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    X, p = small
    d, keep = _desc(hnsw, p, X)
    code, h = _upload(hnsw, d)
    assert code == 3 and not h.value


def test_product_reader_matches_oracle_writer(hnsw, small, tmp_path):
    X, p = small
    path = str(tmp_path / "g.bin")
    oracle.save_graph(path, p)
    r = hnsw.graphfile.read(path)
    for k in ("levels", "adj0", "upper_off", "adjU"):
        assert np.array_equal(np.asarray(r[k]), p[k])
    for k in ("n", "dim", "metric", "M", "Mmax", "Mmax0", "max_level", "entry_point", "rows"):
        assert r[k] == p[k]
