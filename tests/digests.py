"""Digests for the full-size parity checks: hashing only, no similarity arithmetic.

The CPU oracle cannot run inside a GPU test at full size, so a committed
script (tests/golden/make_fullsize_digests.py) runs it once, on the CPU, and
stores a digest of the generated input and one digest per output row.  The
GPU tests regenerate the same input, check its digest first (so that a
generator that drew something else is reported as such, not as a wrong
result), and then compare every output row.

  input_digest  SHA-256 over the offsets (uint64, little-endian) followed by
                the SHA-256 of every set's IDs (uint64, little-endian, in the
                generated order).  Per-set hashing runs on a thread pool.
  row digest    the first 16 hex digits of SHA-256 over one output row:
                B (int32), then C (int64), then J (binary64 bits), each
                little-endian, over the row's entries in the layout's order
                (the full row, or j >= i for the packed upper layout).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os

import numpy as np

ROW_HEX = 16


def _le(a: np.ndarray, dt: str) -> bytes:
    return np.ascontiguousarray(a, dtype=np.dtype(dt).newbyteorder("<")).tobytes()


def input_digest(ids: np.ndarray, off: np.ndarray, threads: int | None = None) -> str:
    off = np.asarray(off, dtype=np.uint64)
    n = off.size - 1

    def one(i):
        a, b = int(off[i]), int(off[i + 1])
        return hashlib.sha256(memoryview(np.ascontiguousarray(ids[a:b], dtype="<u8")).cast("B")).digest()

    with cf.ThreadPoolExecutor(max_workers=threads or min(16, os.cpu_count() or 1)) as ex:
        per = list(ex.map(one, range(n)))
    h = hashlib.sha256(_le(off, "u8"))
    for d in per:
        h.update(d)
    return h.hexdigest()


def row_digest(B, C, J) -> str:
    h = hashlib.sha256(_le(B, "i4"))
    h.update(_le(C, "i8"))
    h.update(_le(np.asarray(J, dtype=np.float64).view(np.uint64), "u8"))
    return h.hexdigest()[:ROW_HEX]


def upper_row(i: int, n: int) -> slice:
    """Entries of row i (j >= i) in the packed upper layout."""
    s = i * n - i * (i - 1) // 2
    return slice(s, s + n - i)


def row_digests(B, C, J, n: int, upper: bool, threads: int | None = None) -> list:
    """One digest per row of n x n results (full: arrays of n*n entries, row
    major; upper: packed arrays of n(n+1)/2 entries)."""
    B, C, J = (np.asarray(x).reshape(-1) for x in (B, C, J))

    def one(i):
        sl = upper_row(i, n) if upper else slice(i * n, (i + 1) * n)
        return row_digest(B[sl], C[sl], J[sl])

    with cf.ThreadPoolExecutor(max_workers=threads or min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(n)))


def read_golden(path: str) -> dict:
    """Parse a digest file written by make_fullsize_digests.py."""
    out = {"rows": [], "requests": []}
    cur = None
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        if key == "row":
            (cur["rows"] if cur is not None else out["rows"]).append(rest.split()[1])
        elif key == "request":
            f = rest.split()
            cur = {"request": int(f[0]), "nq": int(f[2]), "input": f[4], "q_card_sum": int(f[6]), "rows": []}
            out["requests"].append(cur)
        else:
            out[key] = rest
    return out
