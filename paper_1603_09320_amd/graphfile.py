"""Reader of the graph file that graph construction writes.

Layout (little endian):

    magic  b"HNSWGRF1"
    16 x u32: version, n, dim, metric, M, Mmax, Mmax0, efC, max_level,
              entry_point, heuristic, extend, keep_pruned, 3 reserved
    f64 mL, u64 level seed, u64 n_upper_rows
    levels u8 [n]            (zero padded to 8 bytes)
    adj0   u32 [n][Mmax0]    0xFFFFFFFF = unused slot
    upper_off i32 [n]        (zero padded to 8 bytes)
    adjU   u32 [rows][Mmax]
    u64 integrity word: sum over the preceding bytes read as u64 words w_i
        (zero padded) of w_i * (2i + 1), modulo 2^64
"""
from __future__ import annotations

import numpy as np

MAGIC = b"HNSWGRF1"


def _integrity(raw: np.ndarray) -> int:
    pad = (-len(raw)) % 8
    a = raw if not pad else np.concatenate([raw, np.zeros(pad, dtype=np.uint8)])
    w = a.view(np.uint64)
    acc = 0
    step = 1 << 21
    for s in range(0, len(w), step):
        blk = w[s:s + step].astype(np.uint64)
        k = (np.arange(s, s + len(blk), dtype=np.uint64) << np.uint64(1)) | np.uint64(1)
        with np.errstate(over="ignore"):
            acc = (acc + int(np.sum(blk * k, dtype=np.uint64))) & ((1 << 64) - 1)
    return acc


def read(path: str, verify: bool = True) -> dict:
    raw = np.fromfile(path, dtype=np.uint8)
    if len(raw) < 104 or raw[:8].tobytes() != MAGIC:
        raise ValueError(f"{path}: not a graph file")
    h = raw[8:72].view(np.uint32)
    if int(h[0]) != 1:
        raise ValueError(f"{path}: unsupported version {int(h[0])}")
    n, dim, metric, M, Mmax, Mmax0, efC, max_level, entry = (int(v) for v in h[1:10])
    mL = float(raw[72:80].view(np.float64)[0])
    seed, rows = (int(v) for v in raw[80:96].view(np.uint64))
    off = 96
    levels = raw[off:off + n]
    off += n + (-n) % 8
    adj0 = raw[off:off + 4 * n * Mmax0].view(np.uint32).reshape(n, Mmax0)
    off += 4 * n * Mmax0
    upper_off = raw[off:off + 4 * n].view(np.int32)
    off += 4 * n + (-(4 * n)) % 8
    adjU = raw[off:off + 4 * rows * Mmax].view(np.uint32).reshape(rows, Mmax)
    off += 4 * rows * Mmax
    if len(raw) != off + 8:
        raise ValueError(f"{path}: truncated or oversized file")
    if verify and _integrity(raw[:off]) != int(raw[off:off + 8].view(np.uint64)[0]):
        raise ValueError(f"{path}: integrity word mismatch")
    return dict(n=n, dim=dim, metric=metric, M=M, Mmax=Mmax, Mmax0=Mmax0, efC=efC, max_level=max_level,
                entry_point=entry, mL=mL, seed=seed, rows=rows, levels=levels, adj0=adj0, upper_off=upper_off,
                adjU=adjU)
