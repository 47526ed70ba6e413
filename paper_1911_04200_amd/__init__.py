"""Exact all-pairs Jaccard similarity on AMD MI355X (SimilarityAtScale hot path).

The compute lives in ``libjas.so`` (HIP, gfx950) behind the C ABI of
``include/jas.h``; :mod:`.jas` is its ctypes binding and :mod:`.api` adds
torch-allocating conveniences on top.
"""
from .jas import (JAS_FORCE_MFMA, JAS_FORCE_POPCOUNT, JAS_HOST_PTRS, JAS_KEEP_IDS, JAS_UPPER, Db, JasError,
                  jas_db_free, jas_db_size, jas_db_stats, jas_encode, jas_encode_opts, jas_gram, jas_last_error,
                  jas_query, jas_query_workspace_bytes, jas_version)
from .api import encode, gram, query

__all__ = ["Db", "JasError", "encode", "gram", "query", "jas_encode", "jas_gram", "jas_query", "jas_db_free",
           "jas_db_size", "jas_db_stats", "jas_last_error", "jas_version", "jas_query_workspace_bytes",
           "jas_encode_opts", "JAS_HOST_PTRS", "JAS_KEEP_IDS", "JAS_UPPER", "JAS_FORCE_POPCOUNT", "JAS_FORCE_MFMA"]
