"""TEST INFRASTRUCTURE ONLY: the CPU oracle for exact Jaccard similarity.

A plain C implementation (``oracle.c``) of the definitions in Sec. II-A of the
paper: sets are normalised (sorted, repeats dropped), intersections and unions
are counted in one walk over two sorted lists, and J = |X cap Y| / |X cup Y| in
binary64 with J(empty, empty) = 1.  ``kmers`` writes out the k-mer
definition of Sec. II-B in numpy (base-4 digits, reverse complement).  It
shares no code with the GPU library and is loaded only by the tests, the smoke
check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def _bind(lib):
    P = ctypes.POINTER
    u64p, i64p, i32p, dp = P(ctypes.c_uint64), P(ctypes.c_int64), P(ctypes.c_int32), P(ctypes.c_double)
    lib.oracle_normalize.argtypes = [u64p, u64p, ctypes.c_int32, u64p, u64p]
    lib.oracle_counts.argtypes = [u64p, ctypes.c_uint64, u64p, ctypes.c_uint64, u64p, u64p]
    lib.oracle_counts.restype = None
    lib.oracle_jaccard.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_jaccard.restype = ctypes.c_double
    lib.oracle_pairs.argtypes = [u64p, u64p, ctypes.c_int32, u64p, u64p, ctypes.c_int32, ctypes.c_int64,
                                 i32p, i32p, i64p, i64p, dp]
    lib.oracle_cross.argtypes = [u64p, u64p, ctypes.c_int32, u64p, u64p, ctypes.c_int32, i64p, i64p, dp]
    lib.oracle_threads.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """The oracle library (built on first use).  ``path`` loads another build of it."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _csr(ids, off):
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    off = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    if ids.size == 0:
        ids = np.zeros(1, dtype=np.uint64)[:0]
    return ids, off


def threads(lib=None) -> int:
    return int((lib or load()).oracle_threads())


def normalize(ids, off, lib=None):
    """Each set sorted, repeats dropped: (ids, offsets)."""
    lib = lib or load()
    ids, off = _csr(ids, off)
    n = off.size - 1
    out = np.empty(max(1, ids.size), dtype=np.uint64)
    oo = np.empty(n + 1, dtype=np.uint64)
    rc = lib.oracle_normalize(_p(ids, ctypes.c_uint64), _p(off, ctypes.c_uint64), n,
                              _p(out, ctypes.c_uint64), _p(oo, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("oracle_normalize: bad offsets")
    return out[: int(oo[-1])].copy(), oo


def cross_normalized(qs, qo, xs, xo, lib=None):
    """All pairs of two normalised collections: (inter, union, J), each [nq, nx]."""
    lib = lib or load()
    qs, qo = _csr(qs, qo)
    xs, xo = _csr(xs, xo)
    nq, nx = qo.size - 1, xo.size - 1
    qs1 = qs if qs.size else np.zeros(1, np.uint64)
    xs1 = xs if xs.size else np.zeros(1, np.uint64)
    inter = np.empty((nq, nx), dtype=np.int64)
    uni = np.empty((nq, nx), dtype=np.int64)
    jac = np.empty((nq, nx), dtype=np.float64)
    rc = lib.oracle_cross(_p(qs1, ctypes.c_uint64), _p(qo, ctypes.c_uint64), nq,
                          _p(xs1, ctypes.c_uint64), _p(xo, ctypes.c_uint64), nx,
                          _p(inter, ctypes.c_int64), _p(uni, ctypes.c_int64), _p(jac, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_cross failed")
    return inter, uni, jac


def all_pairs(ids, off, lib=None):
    """Exact all-pairs result of one collection.

    Returns dict with ``inter`` (= B, int64 [n,n]), ``union`` (= C, int64),
    ``J`` (float64) and ``card`` (|X_i|, int64 [n]).
    """
    lib = lib or load()
    s, so = normalize(ids, off, lib)
    inter, uni, jac = cross_normalized(s, so, s, so, lib)
    card = np.diff(so.astype(np.int64))
    return {"inter": inter, "union": uni, "J": jac, "card": card}


def cross(qids, qoff, ids, off, lib=None):
    """Exact query x database result: dict with inter, union, J [nq, n] and q_card, card."""
    lib = lib or load()
    qs, qo = normalize(qids, qoff, lib)
    xs, xo = normalize(ids, off, lib)
    inter, uni, jac = cross_normalized(qs, qo, xs, xo, lib)
    return {"inter": inter, "union": uni, "J": jac,
            "q_card": np.diff(qo.astype(np.int64)), "card": np.diff(xo.astype(np.int64))}


def pairs_normalized(qs, qo, xs, xo, qi, xi, lib=None):
    """Selected pairs (qi[k], xi[k]) of two normalised collections: (inter, union, J)."""
    lib = lib or load()
    qs, qo = _csr(qs, qo)
    xs, xo = _csr(xs, xo)
    qi = np.ascontiguousarray(np.asarray(qi, dtype=np.int32))
    xi = np.ascontiguousarray(np.asarray(xi, dtype=np.int32))
    k = qi.size
    qs1 = qs if qs.size else np.zeros(1, np.uint64)
    xs1 = xs if xs.size else np.zeros(1, np.uint64)
    inter = np.empty(k, dtype=np.int64)
    uni = np.empty(k, dtype=np.int64)
    jac = np.empty(k, dtype=np.float64)
    rc = lib.oracle_pairs(_p(qs1, ctypes.c_uint64), _p(qo, ctypes.c_uint64), qo.size - 1,
                          _p(xs1, ctypes.c_uint64), _p(xo, ctypes.c_uint64), xo.size - 1, k,
                          _p(qi, ctypes.c_int32), _p(xi, ctypes.c_int32),
                          _p(inter, ctypes.c_int64), _p(uni, ctypes.c_int64), _p(jac, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_pairs: index out of range")
    return inter, uni, jac


# ---------------------------------------------------------------------------
# k-mers (Sec. II-B: the length-k substrings of a sequence).  A k-mer's ID is
# its bases (A = 0, C = 1, G = 2, T = 3) read as a base-4 number, first base
# most significant; canonical: the smaller of it and its reverse complement
# (the complement of each base, 3 - x, in reverse order).
def kmers(seq, k: int, canonical: bool = False) -> np.ndarray:
    """IDs of the k-mers of one sequence (uint8 base codes), in position order."""
    x = np.asarray(seq, dtype=np.uint64)
    npos = x.size - k + 1
    if npos <= 0:
        return np.zeros(0, dtype=np.uint64)
    fwd = np.zeros(npos, dtype=np.uint64)
    rev = np.zeros(npos, dtype=np.uint64)
    for j in range(k):  # digit j of the k-mer at position i is base i + j
        fwd = fwd * np.uint64(4) + x[j:j + npos]
        rev = rev * np.uint64(4) + (np.uint64(3) - x[k - 1 - j:k - 1 - j + npos])
    return np.minimum(fwd, rev) if canonical else fwd


def kmer_sets(samples, k: int, canonical: bool = False):
    """CSR (ids, offsets) of every sample's k-mers (sample = list of sequences)."""
    per = [np.concatenate([kmers(s, k, canonical) for s in seqs]) if seqs else np.zeros(0, np.uint64)
           for seqs in samples]
    off = np.zeros(len(per) + 1, dtype=np.uint64)
    np.cumsum([p.size for p in per], out=off[1:])
    return (np.concatenate(per) if per else np.zeros(0, np.uint64)), off
