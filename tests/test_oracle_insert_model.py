"""INSERT (Alg. 1) on several layers, pinned by a second, differently built
model of the paper's construction: plain Python lists and sets in place of
the oracle's heaps and packed rows, written from Algs. 1, 2 and 4 and the
readings the oracle takes (ties broken by (distance, id); a new element links
to M neighbours on every layer; a list over its cap is re-selected by the
heuristic from its element, new link included; all of W is the next layer's
entry set; strict keep test of the heuristic).  On 2-4 layer graphs of 300
elements the two must produce the same neighbour set for every element on
every layer.  An INSERT that handed only the nearest element of W down, kept
the first M candidates, or skipped the greedy phase above the element's
level would build a different graph."""
import math

import numpy as np
import pytest

import oracle


class Model:
    def __init__(self, X, levels, M, Mmax, Mmax0, efC):
        self.X = np.asarray(X, dtype=np.float64)
        self.lv = [int(v) for v in levels]
        self.M, self.Mmax, self.Mmax0, self.efC = M, Mmax, Mmax0, efC
        self.links = {}  # (layer, element) -> list of ids
        self.entry = None
        self.top = -1

    def d(self, a, b):
        v = self.X[a] - self.X[b]
        return np.float32(float(np.dot(v, v)))  # fp64 sum rounded once to float

    def dq(self, x, b):
        v = x - self.X[b]
        return np.float32(float(np.dot(v, v)))

    def search(self, x, entries, ef, lc):
        """Alg. 2 with sorted Python lists: returns W sorted by (distance, id)."""
        seen = set(entries)
        cand = sorted((self.dq(x, e), e) for e in seen)
        found = list(cand)
        while cand:
            c = cand.pop(0)
            if c > found[-1]:
                break
            for e in self.links.get((lc, c[1]), []):
                if e in seen:
                    continue
                seen.add(e)
                k = (self.dq(x, e), e)
                if len(found) < ef or k < found[-1]:
                    cand.append(k)
                    cand.sort()
                    found.append(k)
                    found.sort()
                    if len(found) > ef:
                        found.pop()
        return found

    def heuristic(self, base_key, cand_ids, m):
        """Alg. 4 (both flags off): candidates by increasing (distance, id)
        to the base; keep one while it is strictly nearer to the base than to
        every element already kept."""
        out = []
        for dist, e in sorted((base_key(e), e) for e in cand_ids):
            if len(out) == m:
                break
            if all(dist < self.d(e, r) for r in out):
                out.append(e)
        return out

    def insert(self, q):
        x = self.X[q]
        l = self.lv[q]
        if self.entry is None:
            self.entry, self.top = q, l
            return
        ep = [self.entry]
        for lc in range(self.top, l, -1):
            ep = [self.search(x, ep, 1, lc)[0][1]]
        for lc in range(min(self.top, l), -1, -1):
            W = self.search(x, ep, self.efC, lc)
            nb = self.heuristic(lambda e: self.dq(x, e), [e for _, e in W], self.M)
            self.links[(lc, q)] = list(nb)
            cap = self.Mmax0 if lc == 0 else self.Mmax
            for e in nb:
                lst = self.links.setdefault((lc, e), [])
                lst.append(q)
                if len(lst) > cap:
                    self.links[(lc, e)] = self.heuristic(lambda r, e=e: self.d(e, r), lst, cap)
            ep = [e for _, e in W]
        if l > self.top:
            self.entry, self.top = q, l


def _oracle_lists(p):
    n = p["n"]
    out = {}
    for i in range(n):
        out[(0, i)] = sorted(int(v) for v in p["adj0"][i] if v != 0xFFFFFFFF)
        for lc in range(1, int(p["levels"][i]) + 1):
            row = p["adjU"][p["upper_off"][i] + lc - 1]
            out[(lc, i)] = sorted(int(v) for v in row if v != 0xFFFFFFFF)
    return out


@pytest.mark.parametrize("data,seed", [("uniform", 1), ("uniform", 2), ("grid", 3), ("grid", 4)])
def test_insert_matches_list_model_on_several_layers(data, seed):
    n, dim, M, efC = 300, 3, 4, 8
    g = np.random.default_rng(seed)
    if data == "grid":
        X = g.integers(0, 12, size=(n, dim)).astype(np.float32)  # many ties and some duplicates
    else:
        X = g.random((n, dim)).astype(np.float32)
    mL = 1.0 / math.log(M)
    G = oracle.Graph.build(X, M=M, Mmax=M, Mmax0=2 * M, efC=efC, mL=mL, seed=seed)
    p = G.packed()
    assert p["max_level"] >= 2, "fixture should span several layers"
    assert (p["levels"] >= 1).sum() > 40
    model = Model(X, p["levels"], M, M, 2 * M, efC)
    for q in range(n):
        model.insert(q)
    assert model.entry == p["entry_point"] and model.top == p["max_level"]
    want = {k: sorted(v) for k, v in model.links.items()}
    got = _oracle_lists(p)
    for key in got:
        assert got[key] == want.get(key, []), (key, got[key], want.get(key))
    assert set(want) <= set(got)
