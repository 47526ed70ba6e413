"""ctypes binding of libjas (include/jas.h): argument marshalling only.

Every function keeps the C name and order of arguments.  Device buffers are
torch tensors (their ``data_ptr()``), host buffers numpy arrays (with
JAS_HOST_PTRS); ``stream`` is a ``torch.cuda.Stream`` or None for torch's
current stream.  A non-OK status raises :class:`JasError`.  All computation
happens in the HIP library; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libjas.so")

JAS_OK, JAS_EINVAL, JAS_ENOMEM, JAS_EOVERFLOW, JAS_EDEVICE, JAS_EBUSY, JAS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
JAS_HOST_PTRS = 0x1
JAS_KEEP_IDS = 0x2
JAS_UPPER = 0x10
JAS_FORCE_POPCOUNT = 0x20
JAS_FORCE_MFMA = 0x40
JAS_TUNE = 0x80
JAS_ACCUMULATE = 0x100
JAS_CANONICAL = 0x200
JAS_NO_WAIT = 0x400
JAS_QUERY_ONLY = 0x800
JAS_DB_CARD, JAS_DB_WORDS, JAS_DB_LIST_PAIRS, JAS_DB_LIST_PTR, JAS_DB_LIST_SAMPLES, JAS_DB_KEYS = range(6)


def JAS_GRAM_VARIANT(v: int) -> int:
    """jas_gram flag: run MFMA tile variant v (0 <= v < jas_gram_variants())."""
    return (int(v) + 1) << 16

STATUS_NAMES = {0: "JAS_OK", -1: "JAS_EINVAL", -2: "JAS_ENOMEM", -3: "JAS_EOVERFLOW", -4: "JAS_EDEVICE",
                -5: "JAS_EBUSY", -6: "JAS_EUNSUPPORTED"}

# Every symbol include/jas.h declares.
EXPORTS = sorted(["jas_encode", "jas_gram", "jas_finalize", "jas_kmer_offsets", "jas_kmers", "jas_relabel", "jas_gram_variants", "jas_card_limit", "jas_query", "jas_query_noalloc", "jas_query_workspace_bytes",
                  "jas_db_size", "jas_db_stats", "jas_db_part_size", "jas_db_read", "jas_db_free",
                  "jas_plan_create", "jas_plan_encode", "jas_plan_check", "jas_plan_db", "jas_plan_threshold",
                  "jas_plan_tuning", "jas_plan_free", "jas_last_error", "jas_version", "jas_timing_enable",
                  "jas_timing_report", "jas_trim"])


class JasError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class jas_encode_opts(ctypes.Structure):
    _fields_ = [("universe_bits", ctypes.c_uint32), ("batch_bits", ctypes.c_uint32),
                ("dense_min_degree", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("word_bits", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class jas_encode_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in
                ["n_ids", "n_pairs", "n_rows", "n_shared_rows", "n_packed_rows", "n_list_rows", "n_batches",
                 "n_word_rows", "nnz_words", "word_pairs_F", "list_pairs", "device_bytes", "dense_min_degree",
                 "word_bits", "w_rows", "w_stride", "n_list_pairs", "dense_tiles", "word_pairs_W"]]

    def to_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class jas_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libjas.so (building it first if it is not there)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build(force=False)
    if not os.path.exists(path):
        raise ImportError(f"libjas.so not found at {path}; run paper_1911_04200_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, u32, i32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64
    lib.jas_encode.argtypes = [vp, vp, i32, ctypes.POINTER(jas_encode_opts), vp, ctypes.POINTER(vp),
                               ctypes.POINTER(jas_encode_stats)]
    lib.jas_encode.restype = ctypes.c_int
    lib.jas_gram.argtypes = [vp, u32, vp, vp, vp, vp, vp]
    lib.jas_kmer_offsets.restype = i32
    lib.jas_kmer_offsets.argtypes = [vp, ctypes.c_int64, vp, i32, u32, vp]
    lib.jas_kmers.restype = i32
    lib.jas_kmers.argtypes = [vp, vp, ctypes.c_int64, u32, u32, vp, vp]
    lib.jas_relabel.restype = i32
    lib.jas_relabel.argtypes = [vp, u64, u32, vp, vp, ctypes.POINTER(u64), ctypes.POINTER(u32)]
    lib.jas_finalize.restype = i32
    lib.jas_finalize.argtypes = [i32, u32, vp, vp, vp, vp, vp]
    lib.jas_gram.restype = ctypes.c_int
    lib.jas_query.argtypes = [vp, vp, vp, i32, u32, vp, vp, vp, vp, vp]
    lib.jas_query.restype = ctypes.c_int
    lib.jas_query_noalloc.argtypes = [vp, vp, vp, i32, u32, vp, vp, vp, vp, vp]
    lib.jas_query_noalloc.restype = ctypes.c_int
    lib.jas_query_workspace_bytes.argtypes = [vp, i32, u64]
    lib.jas_query_workspace_bytes.restype = u64
    lib.jas_db_size.argtypes = [vp]
    lib.jas_db_size.restype = i32
    lib.jas_card_limit.argtypes = []
    lib.jas_card_limit.restype = u64
    lib.jas_gram_variants.argtypes = []
    lib.jas_gram_variants.restype = i32
    lib.jas_db_stats.argtypes = [vp, ctypes.POINTER(jas_encode_stats)]
    lib.jas_db_stats.restype = ctypes.c_int
    lib.jas_db_part_size.argtypes = [vp, i32]
    lib.jas_db_part_size.restype = u64
    lib.jas_db_read.argtypes = [vp, i32, u64, u64, vp]
    lib.jas_db_read.restype = ctypes.c_int
    lib.jas_plan_create.argtypes = [vp, vp, i32, ctypes.POINTER(jas_encode_opts), ctypes.c_double, vp,
                                    ctypes.POINTER(vp)]
    lib.jas_plan_create.restype = ctypes.c_int
    lib.jas_plan_encode.argtypes = [vp, vp, vp, vp]
    lib.jas_plan_encode.restype = ctypes.c_int
    lib.jas_plan_check.argtypes = [vp, vp, ctypes.POINTER(jas_encode_stats)]
    lib.jas_plan_check.restype = ctypes.c_int
    lib.jas_plan_db.argtypes = [vp]
    lib.jas_plan_db.restype = vp
    lib.jas_plan_threshold.argtypes = [vp]
    lib.jas_plan_threshold.restype = u32
    lib.jas_plan_tuning.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_double), i32]
    lib.jas_plan_tuning.restype = i32
    lib.jas_plan_free.argtypes = [vp]
    lib.jas_plan_free.restype = None
    lib.jas_db_free.argtypes = [vp]
    lib.jas_db_free.restype = None
    lib.jas_last_error.restype = ctypes.c_char_p
    lib.jas_version.restype = ctypes.c_char_p
    lib.jas_trim.argtypes = []
    lib.jas_trim.restype = None
    lib.jas_timing_enable.argtypes = [i32]
    lib.jas_timing_enable.restype = None
    lib.jas_timing_report.argtypes = [ctypes.POINTER(jas_kernel_time), i32]
    lib.jas_timing_report.restype = i32
    _lib = lib
    return lib


def _check(status: int):
    if status != JAS_OK:
        raise JasError(status, load().jas_last_error().decode())


def _ptr(x):
    """Raw address of a torch tensor, numpy array or int (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data if x.size else None
    if hasattr(x, "data_ptr"):
        return x.data_ptr() if x.numel() else None
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Db:
    """Owns a jas_db handle; frees it with jas_db_free."""

    def __init__(self, handle: int):
        self.handle = handle

    @property
    def n(self) -> int:
        return jas_db_size(self)

    def close(self):
        if self.handle:
            load().jas_db_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _h(db):
    return getattr(db, "handle", db)


def jas_encode(ids, offsets, n: int, opts: jas_encode_opts, stream=None):
    """jas_encode: returns (Db, stats dict)."""
    lib = load()
    out = ctypes.c_void_p()
    st = jas_encode_stats()
    s = None if (opts.flags & JAS_HOST_PTRS and stream is None) else _stream(stream)
    _check(lib.jas_encode(_ptr(ids), _ptr(offsets), n, ctypes.byref(opts), s, ctypes.byref(out), ctypes.byref(st)))
    return Db(out.value), st.to_dict()


def jas_gram(db, flags: int, stream, B, card=None, den=None, J=None):
    lib = load()
    s = None if (flags & JAS_HOST_PTRS and stream is None) else _stream(stream)
    _check(lib.jas_gram(_h(db), flags, s, _ptr(B), _ptr(card), _ptr(den), _ptr(J)))


def jas_finalize(n: int, flags: int, stream, B, card, den=None, J=None):
    _check(load().jas_finalize(n, flags, _stream(stream), _ptr(B), _ptr(card), _ptr(den), _ptr(J)))


def jas_kmer_offsets(seq_off: np.ndarray, smp_off: np.ndarray, k: int) -> np.ndarray:
    """Host: the CSR offsets (uint64[n+1]) of the samples' k-mers."""
    seq_off = np.ascontiguousarray(seq_off, dtype=np.uint64)
    smp_off = np.ascontiguousarray(smp_off, dtype=np.uint64)
    out = np.empty(smp_off.size, dtype=np.uint64)
    _check(load().jas_kmer_offsets(seq_off.ctypes.data, seq_off.size - 1, smp_off.ctypes.data, smp_off.size - 1, k,
                                   out.ctypes.data))
    return out


def jas_kmers(seq, seq_off: np.ndarray, k: int, flags: int, stream, ids):
    """Device: the k-mer IDs of every sequence into ids (seq_off on the host)."""
    seq_off = np.ascontiguousarray(seq_off, dtype=np.uint64)
    _check(load().jas_kmers(_ptr(seq), seq_off.ctypes.data, seq_off.size - 1, k, flags, _stream(stream), _ptr(ids)))


def jas_relabel(ids, n_ids: int, universe_bits: int, stream, out):
    """Device IDs -> their ranks among the distinct IDs; returns (D, new universe_bits)."""
    d, u = ctypes.c_uint64(), ctypes.c_uint32()
    _check(load().jas_relabel(_ptr(ids), n_ids, universe_bits, _stream(stream), _ptr(out), ctypes.byref(d),
                              ctypes.byref(u)))
    return int(d.value), int(u.value)


def jas_query(db, q_ids, q_offsets, nq: int, flags: int, stream, B, q_card=None, den=None, J=None):
    lib = load()
    s = None if (flags & JAS_HOST_PTRS and stream is None) else _stream(stream)
    _check(lib.jas_query(_h(db), _ptr(q_ids), _ptr(q_offsets), nq, flags, s, _ptr(B), _ptr(q_card), _ptr(den),
                         _ptr(J)))


def jas_query_noalloc(db, q_ids, q_offsets, nq: int, flags: int, stream, B, q_card=None, den=None, J=None):
    _check(load().jas_query_noalloc(_h(db), _ptr(q_ids), _ptr(q_offsets), nq, flags, _stream(stream), _ptr(B),
                                    _ptr(q_card), _ptr(den), _ptr(J)))


def jas_query_workspace_bytes(db, nq: int, n_q_ids: int) -> int:
    return int(load().jas_query_workspace_bytes(_h(db), nq, n_q_ids))


def jas_db_size(db) -> int:
    return int(load().jas_db_size(_h(db)))


def jas_card_limit() -> int:
    return int(load().jas_card_limit())


def jas_gram_variants() -> int:
    return int(load().jas_gram_variants())


def jas_db_stats(db) -> dict:
    st = jas_encode_stats()
    _check(load().jas_db_stats(_h(db), ctypes.byref(st)))
    return st.to_dict()


class Plan:
    """Owns a jas_plan handle; .db is its (plan-owned) encoded database."""

    def __init__(self, handle: int):
        self.handle = handle

    @property
    def db(self) -> int:
        return int(load().jas_plan_db(self.handle))

    @property
    def threshold(self) -> int:
        return int(load().jas_plan_threshold(self.handle))

    def tuning(self) -> list:
        lib = load()
        k = lib.jas_plan_tuning(self.handle, None, None, 0)
        t = (ctypes.c_uint32 * max(k, 1))()
        ms = (ctypes.c_double * max(k, 1))()
        lib.jas_plan_tuning(self.handle, t, ms, k)
        return [(int(t[i]), float(ms[i])) for i in range(k)]

    def close(self):
        if self.handle:
            load().jas_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def jas_plan_create(ids, offsets, n: int, opts: jas_encode_opts, headroom: float = 0.25, stream=None) -> Plan:
    out = ctypes.c_void_p()
    _check(load().jas_plan_create(_ptr(ids), _ptr(offsets), n, ctypes.byref(opts), float(headroom), _stream(stream),
                                  ctypes.byref(out)))
    return Plan(out.value)


def jas_plan_encode(plan, ids, offsets, stream=None):
    _check(load().jas_plan_encode(_h(plan), _ptr(ids), _ptr(offsets), _stream(stream)))


def jas_plan_check(plan, stream=None) -> dict:
    st = jas_encode_stats()
    _check(load().jas_plan_check(_h(plan), _stream(stream), ctypes.byref(st)))
    return st.to_dict()


_PART_DTYPE = {JAS_DB_CARD: np.int64, JAS_DB_WORDS: np.uint64, JAS_DB_LIST_PAIRS: np.uint32,
               JAS_DB_LIST_PTR: np.uint64, JAS_DB_LIST_SAMPLES: np.uint32, JAS_DB_KEYS: np.uint64}


def jas_db_part_size(db, part: int) -> int:
    return int(load().jas_db_part_size(_h(db), part))


def jas_db_read(db, part: int, first: int = 0, count: int | None = None) -> np.ndarray:
    """Elements [first, first + count) of a db part (all of it by default), as a host array."""
    size = jas_db_part_size(db, part)
    count = size - first if count is None else count
    out = np.empty(max(count, 0), dtype=_PART_DTYPE.get(part, np.uint64))
    _check(load().jas_db_read(_h(db), part, first, count, out.ctypes.data if out.size else None))
    return out


def jas_db_free(db):
    if isinstance(db, Db):
        db.close()
    else:
        load().jas_db_free(db)


def jas_last_error() -> str:
    return load().jas_last_error().decode()


def jas_version() -> str:
    return load().jas_version().decode()


def jas_timing_enable(on: bool = True):
    load().jas_timing_enable(1 if on else 0)


def jas_timing_report(cap: int = 64) -> dict:
    """{kernel name: (launches, total ms)} since the last report; resets the totals."""
    arr = (jas_kernel_time * cap)()
    k = load().jas_timing_report(arr, cap)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(k, cap))}


def jas_trim():
    load().jas_trim()
