"""Seeded synthetic set collections (inputs only; no similarity arithmetic).

The C generator in ``synth.c`` draws n sets of hashed 64-bit IDs in CSR form
(``ids``, ``offsets``).  Both the CPU oracle and the GPU path take their inputs
from here; neither shares anything else.

Named workloads stand in for the paper's genome k-mer collections (Sec. V-A2,
datasets not available): sizes, sharing structure, universe width and row
batching follow the five configurations of this project (tiny, paper-like,
precision, batching, serving).  The ``bernoulli_*`` workloads are the paper's
own synthetic indicator matrices (Sec. V-A3, swept over p in Sec. V-C): every entry of
an m x n matrix is 1 with probability p, independently.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Spec(ctypes.Structure):
    _fields_ = [
        ("pool_seed", ctypes.c_uint64),
        ("sample_seed", ctypes.c_uint64),
        ("universe_bits", ctypes.c_uint32),
        ("n", ctypes.c_int32),
        ("size_kind", ctypes.c_int32),
        ("n_pools", ctypes.c_int32),
        ("size_a", ctypes.c_double),
        ("size_b", ctypes.c_double),
        ("size_lo", ctypes.c_double),
        ("size_hi", ctypes.c_double),
        ("share_lo", ctypes.c_double),
        ("share_hi", ctypes.c_double),
        ("dup_rate", ctypes.c_double),
        ("pool_start", ctypes.POINTER(ctypes.c_uint64)),
        ("pool_size", ctypes.POINTER(ctypes.c_uint64)),
        ("density", ctypes.c_double),
        ("rows", ctypes.c_uint64),
    ]


def _bind(lib):
    P = ctypes.POINTER
    lib.synth_offsets.argtypes = [P(_Spec), P(ctypes.c_uint64)]
    lib.synth_plan.argtypes = [P(_Spec), ctypes.c_int32, P(ctypes.c_uint64)]
    lib.synth_fill.argtypes = [P(_Spec), ctypes.c_int32, ctypes.c_int32, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    lib.synth_fill_list.argtypes = [P(_Spec), ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_uint64),
                                    P(ctypes.c_uint64)]
    lib.synth_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    lib.synth_rmat.restype = ctypes.c_int64
    return lib


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def use_library(path: str) -> None:
    """Generate with another build of synth.c from now on (e.g. one built with sanitizers)."""
    global _lib
    _lib = _bind(ctypes.CDLL(path))


@dataclasses.dataclass(frozen=True)
class Spec:
    """Parameters of one synthetic collection."""
    n: int
    universe_bits: int
    size_kind: int            # 0 log-uniform [size_a, size_b]; 1 log-normal(median size_a, sigma size_b) clipped;
                              # 2 Bernoulli: each of `rows` rows in each set with probability `density`
    size_a: float
    size_b: float
    share_lo: float
    share_hi: float
    pool_start: tuple
    pool_size: tuple
    pool_seed: int
    sample_seed: int
    size_lo: float = 0.0
    size_hi: float = 0.0
    dup_rate: float = 0.0
    density: float = 0.0
    rows: int = 0

    def replace(self, **kw) -> "Spec":
        return dataclasses.replace(self, **kw)

    def _c(self):
        ps = (ctypes.c_uint64 * max(1, len(self.pool_start)))(*self.pool_start)
        pz = (ctypes.c_uint64 * max(1, len(self.pool_size)))(*self.pool_size)
        s = _Spec(self.pool_seed & 0xFFFFFFFFFFFFFFFF, self.sample_seed & 0xFFFFFFFFFFFFFFFF,
                  self.universe_bits, self.n, self.size_kind, len(self.pool_size),
                  self.size_a, self.size_b, self.size_lo, self.size_hi,
                  self.share_lo, self.share_hi, self.dup_rate,
                  ctypes.cast(ps, ctypes.POINTER(ctypes.c_uint64)),
                  ctypes.cast(pz, ctypes.POINTER(ctypes.c_uint64)),
                  self.density, self.rows)
        s._keep = (ps, pz)
        return s


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


_offsets_cache: dict = {}


def offsets(spec) -> np.ndarray:
    """CSR offsets (uint64[n+1]).  A Bernoulli set's size is known only by
    drawing it, so those offsets are kept for the last few specs asked for."""
    if isinstance(spec, Graph):
        return spec.off.copy()
    if spec.size_kind == 2 and spec in _offsets_cache:
        return _offsets_cache[spec].copy()
    lib = _load()
    off = np.empty(spec.n + 1, dtype=np.uint64)
    cs = spec._c()
    lib.synth_offsets(ctypes.byref(cs), _u64p(off))
    if spec.size_kind == 2:
        while len(_offsets_cache) >= 4:
            _offsets_cache.pop(next(iter(_offsets_cache)))
        _offsets_cache[spec] = off.copy()
    return off


def plan(spec: Spec, i: int):
    """(size, pool_part, dups, cluster) of sample i."""
    lib = _load()
    out = np.empty(4, dtype=np.uint64)
    cs = spec._c()
    lib.synth_plan(ctypes.byref(cs), i, _u64p(out))
    return int(out[0]), int(out[1]), int(out[2]), int(out[3].astype(np.int64))


def generate(spec, out: Optional[np.ndarray] = None):
    """Whole collection: (ids uint64[N], offsets uint64[n+1])."""
    if isinstance(spec, Graph):
        if out is None:
            return spec.ids.copy(), spec.off.copy()
        out[:spec.ids.size] = spec.ids
        return out[:spec.ids.size], spec.off.copy()
    lib = _load()
    off = offsets(spec)
    total = int(off[-1])
    ids = out if out is not None else np.empty(total, dtype=np.uint64)
    assert ids.dtype == np.uint64 and ids.size >= total and ids.flags.c_contiguous
    cs = spec._c()
    rc = lib.synth_fill(ctypes.byref(cs), 0, spec.n, _u64p(off), _u64p(ids))
    if rc != 0:
        raise RuntimeError("synth_fill failed")
    return ids[:total], off


def generate_samples(spec, idx: Sequence[int]):
    """Only the listed samples, packed in list order: (ids, offsets[len(idx)+1])."""
    if isinstance(spec, Graph):
        idx = np.asarray(idx, dtype=np.int64)
        parts = [spec.ids[int(spec.off[i]):int(spec.off[i + 1])] for i in idx]
        off = np.zeros(idx.size + 1, dtype=np.uint64)
        np.cumsum([x.size for x in parts], out=off[1:])
        return (np.concatenate(parts) if parts else np.zeros(0, np.uint64)), off
    lib = _load()
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    full = offsets(spec)
    sizes = (full[idx.astype(np.int64) + 1] - full[idx.astype(np.int64)]).astype(np.uint64)
    off = np.zeros(idx.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=off[1:])
    ids = np.empty(int(off[-1]), dtype=np.uint64)
    cs = spec._c()
    rc = lib.synth_fill_list(ctypes.byref(cs), idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             _u64p(off), _u64p(ids))
    if rc != 0:
        raise RuntimeError("synth_fill_list failed")
    return ids, off


def rmat_graph(scale: int, edge_factor: int, seed: int = 0, a: float = 0.57, b: float = 0.19, c: float = 0.19):
    """Neighbourhoods N(v), v < 2^scale, of an undirected R-MAT graph (power-law
    degrees; Graph500's quadrant probabilities by default): (ids, offsets), each
    set ascending without repeats, IDs < 2^scale."""
    lib = _load()
    nv = 1 << scale
    off = np.empty(nv + 1, dtype=np.uint64)
    ids = np.empty(2 * edge_factor * nv, dtype=np.uint64)
    total = lib.synth_rmat(scale, edge_factor, (_SEED_BASE + 7 + seed) & 0xFFFFFFFFFFFFFFFF, a, b, c,
                           _u64p(off), _u64p(ids))
    if total < 0:
        raise ValueError("bad R-MAT parameters")
    return ids[:total].copy(), off


class Graph:
    """Neighbourhoods of a generated graph as a set collection (n = 2^scale
    sets, IDs < 2^scale); offsets / generate / generate_samples accept it."""

    def __init__(self, scale: int, edge_factor: int, seed: int = 0):
        self.scale, self.edge_factor, self.seed = scale, edge_factor, seed
        self.ids, self.off = rmat_graph(scale, edge_factor, seed)
        self.n = 1 << scale
        self.universe_bits = scale
        self.size_kind = -1


# Vertex similarity workloads: (scale, edge factor).  All pairs of the 8192
# vertices of a scale-13 graph (within the row-list path's sample limit); a
# scale-20 graph as a query database (link prediction: new vertices' sets
# against every neighbourhood).
GRAPHS = {"graph_s13_ef64": (13, 64), "graph_s20_ef16": (20, 16)}


# ---------------------------------------------------------------------------
# Named workloads.
_SEED_BASE = 0x1911042000


def _nested_pools(count: int, base_log2: float, step: float):
    sizes = tuple(int(round(2.0 ** (base_log2 + c * step))) for c in range(count))
    return tuple(0 for _ in sizes), sizes


def _disjoint_pools(count: int, size: int):
    return tuple(c * size for c in range(count)), tuple(size for _ in range(count))


def bernoulli(p: float, rows_log2: int = 25, n: int = 10000, seed: int = 0) -> Spec:
    """Indicator matrix of 2^rows_log2 rows and n samples, each entry 1 with probability p.

    IDs are the row indices, so the universe is exactly the rows (U = rows_log2)."""
    return Spec(n=n, universe_bits=rows_log2, size_kind=2, size_a=0.0, size_b=0.0, share_lo=0.0, share_hi=0.0,
                pool_start=(), pool_size=(), pool_seed=_SEED_BASE + 6, sample_seed=_SEED_BASE + 106 + seed,
                density=float(p), rows=1 << rows_log2)


# The density sweep: m = 2^25 (the paper's 32M rows), n = 10k, p = 1e-4 .. 1e-2;
# at p = 0.1 the 3.4e10 IDs of m = 2^25 would not fit in HBM next to their
# sort buffers, so that point takes m = 2^22.
BERNOULLI = {"bernoulli_p1e-4": (1e-4, 25), "bernoulli_p1e-3": (1e-3, 25), "bernoulli_p1e-2": (1e-2, 25),
             "bernoulli_p1e-1": (1e-1, 22)}


def workload(name: str):
    """The five configurations (full size), the Bernoulli density sweep and the
    vertex-similarity graphs (a Graph)."""
    if name in GRAPHS:
        return Graph(*GRAPHS[name])
    if name in BERNOULLI:
        p, rl = BERNOULLI[name]
        return bernoulli(p, rl)
    if name == "tiny":
        # n=32, universe 2^24, sizes log-uniform [1e3,1e5], share U[0,0.8] of one 2^16 pool
        return Spec(n=32, universe_bits=24, size_kind=0, size_a=1e3, size_b=1e5,
                    share_lo=0.0, share_hi=0.8, pool_start=(0,), pool_size=(1 << 16,),
                    pool_seed=_SEED_BASE + 1, sample_seed=_SEED_BASE + 101)
    if name == "paperlike":
        # n=1024, universe 2^40, log-normal(median 1e6, sigma 1) clipped [1e4,1e7],
        # 20 nested cluster pools 2^(22 + c/4), share U[0.3,0.9]
        st, sz = _nested_pools(20, 22.0, 0.25)
        return Spec(n=1024, universe_bits=40, size_kind=1, size_a=1e6, size_b=1.0, size_lo=1e4, size_hi=1e7,
                    share_lo=0.3, share_hi=0.9, pool_start=st, pool_size=sz,
                    pool_seed=_SEED_BASE + 2, sample_seed=_SEED_BASE + 102)
    if name == "precision":
        # n=4096, universe 2^32, sizes log-uniform [1e5,1e6], 70% from one 2^22 core pool
        return Spec(n=4096, universe_bits=32, size_kind=0, size_a=1e5, size_b=1e6,
                    share_lo=0.7, share_hi=0.7, pool_start=(0,), pool_size=(1 << 22,),
                    pool_seed=_SEED_BASE + 3, sample_seed=_SEED_BASE + 103)
    if name == "batching":
        # n=10000, universe 2^36, sizes log-uniform [1e3,1e6], 50 disjoint 2^22 pools, share U[0.3,0.9]
        st, sz = _disjoint_pools(50, 1 << 22)
        return Spec(n=10000, universe_bits=36, size_kind=0, size_a=1e3, size_b=1e6,
                    share_lo=0.3, share_hi=0.9, pool_start=st, pool_size=sz,
                    pool_seed=_SEED_BASE + 4, sample_seed=_SEED_BASE + 104)
    if name == "serving_db":
        # n=8192, universe 2^36, sizes log-uniform [1e5,1e6], 64 disjoint 2^22 pools, share U[0.3,0.9]
        st, sz = _disjoint_pools(64, 1 << 22)
        return Spec(n=8192, universe_bits=36, size_kind=0, size_a=1e5, size_b=1e6,
                    share_lo=0.3, share_hi=0.9, pool_start=st, pool_size=sz,
                    pool_seed=_SEED_BASE + 5, sample_seed=_SEED_BASE + 105)
    raise KeyError(name)


def query_spec(db: Spec, request: int, nq: int) -> Spec:
    """Query sets of one serving request: 1e4..1e6 IDs, 0..90% from random DB pools."""
    return Spec(n=nq, universe_bits=db.universe_bits, size_kind=0, size_a=1e4, size_b=1e6,
                share_lo=0.0, share_hi=0.9, pool_start=db.pool_start, pool_size=db.pool_size,
                pool_seed=db.pool_seed, sample_seed=db.sample_seed * 7919 + 1000003 * (request + 1))


# Batch rows (the paper's m~) used with each workload, as log2.
BATCH_BITS = {"tiny": 24, "paperlike": 26, "precision": 32, "batching": 26, "serving_db": 26}
BATCH_BITS.update({name: rl for name, (p, rl) in BERNOULLI.items()})  # one batch of all rows
BATCH_BITS.update({name: sc for name, (sc, ef) in GRAPHS.items()})


def scaled(spec: Spec, n: Optional[int] = None, size_scale: float = 1.0, pool_scale: float = 1.0,
           seed_offset: int = 0, dup_rate: Optional[float] = None) -> Spec:
    """A smaller variant of a workload with the same structure (for tests)."""
    kw = dict(n=spec.n if n is None else n,
              size_a=spec.size_a * size_scale if spec.size_kind == 0 else spec.size_a * size_scale,
              size_b=spec.size_b * size_scale if spec.size_kind == 0 else spec.size_b,
              size_lo=spec.size_lo * size_scale, size_hi=spec.size_hi * size_scale,
              pool_start=tuple(int(math.floor(x * pool_scale)) for x in spec.pool_start),
              pool_size=tuple(max(1, int(math.floor(x * pool_scale))) for x in spec.pool_size),
              sample_seed=spec.sample_seed + seed_offset)
    if dup_rate is not None:
        kw["dup_rate"] = dup_rate
    return spec.replace(**kw)


# ---------------------------------------------------------------------------
# Sequences (inputs of the k-mer front end): base codes A = 0, C = 1, G = 2,
# T = 3, and their 2-bit packed form.
def random_genomes(n: int, length: int, n_refs: int = 4, mutation: float = 0.01, seqs_per_sample: int = 1,
                   seed: int = 0):
    """n samples, each `seqs_per_sample` sequences of about `length` bases: a
    copy of one of n_refs random reference genomes (cut into pieces) with each
    base substituted with probability `mutation`.  Returns a list (per sample)
    of lists of uint8 base-code arrays."""
    rng = np.random.default_rng((_SEED_BASE + 8 + seed) & 0xFFFFFFFF)
    refs = [rng.integers(0, 4, size=length, dtype=np.uint8) for _ in range(n_refs)]
    out = []
    for i in range(n):
        g = refs[int(rng.integers(0, n_refs))].copy()
        hit = rng.choice(length, size=int(rng.binomial(length, mutation)), replace=False)  # substituted bases
        g[hit] = (g[hit] + rng.integers(1, 4, size=hit.size, dtype=np.uint8)) % 4
        cuts = np.sort(rng.choice(np.arange(1, length), size=seqs_per_sample - 1, replace=False)) \
            if seqs_per_sample > 1 else np.zeros(0, np.int64)
        out.append(np.split(g, cuts))
    return out


def pack_2bit(seqs):
    """Sequences (uint8 base codes) -> (words uint64, seq_off uint64[len+1]):
    base b of the concatenation at bits 2 (b mod 32) of word b / 32."""
    lens = np.array([s.size for s in seqs], dtype=np.uint64)
    off = np.zeros(len(seqs) + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    L = int(off[-1])
    nw = max(1, (L + 31) // 32)
    bases = np.zeros(nw * 32, dtype=np.uint8)
    if L:
        bases[:L] = np.concatenate(seqs)
    b = bases.reshape(nw, 32)
    words = np.zeros(nw, dtype=np.uint64)
    for j in range(32):  # base j of each word at bits 2j
        words |= b[:, j].astype(np.uint64) << np.uint64(2 * j)
    return words, off
