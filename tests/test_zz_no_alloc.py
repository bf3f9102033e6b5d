"""The allocation-free search entry point (hnsw_search_batch_noalloc) against
hnsw_search_batch_ex, through the C ABI: two calls in a row, the second with
a smaller batch, in the scheduled form (whose workspace is the library's
static scratch array) and in the default form choice; every output and
counter bit-identical.  Sizes above the scratch array's limit are refused
before anything is enqueued."""
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


@pytest.fixture(scope="module")
def cfg(hnsw):
    X = synthdata.base("uniform16", 10000)
    G = oracle.Graph.build(X, M=16, efC=100, seed=1003)
    idx = hnsw.Index(G.packed(), X)
    idx.add_lowp(hnsw.MODE_FP8)
    Q = synthdata.queries("uniform16", 6000)
    return idx, torch.from_numpy(Q).cuda()


def _outs(n, k, dev):
    return (torch.full((n, k), -7, dtype=torch.int32, device=dev), torch.full((n, k), -7.0, device=dev),
            torch.full((n, 4), -7, dtype=torch.int32, device=dev))


@pytest.mark.parametrize("sched", ["2", None])
@pytest.mark.parametrize("mode", [0, 2])
def test_noalloc_equals_search_batch_ex(hnsw, cfg, monkeypatch, sched, mode):
    print(f"case no-alloc search sched={sched} mode={mode}", flush=True)
    if sched is None:
        monkeypatch.delenv("HNSW_SCHEDULE", raising=False)
    else:
        monkeypatch.setenv("HNSW_SCHEDULE", sched)
    idx, q = cfg
    for n, k, ef in ((6000, 10, 64), (1500, 16, 40)):
        qq = q[:n]
        ref = idx.search(qq, k, ef, mode=mode, counters=True)
        out = _outs(n, k, q.device)
        got = idx.search(qq, k, ef, mode=mode, counters=True, out=out, no_alloc=True)
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(a, b), (n, k, ef)


def test_noalloc_refuses_oversized_batch(hnsw, cfg):
    idx, q = cfg
    n = hnsw.NOALLOC_MAX_QUERIES + 1
    big = q[:1].expand(n, q.shape[1]).contiguous()
    out = _outs(n, 1, q.device)
    with pytest.raises(hnsw.HnswError) as e:
        idx.search(big, 1, 8, out=out, counters=True, no_alloc=True)
    assert e.value.code == 4
    torch.cuda.synchronize()
    assert (out[0] == -7).all()  # nothing was enqueued
