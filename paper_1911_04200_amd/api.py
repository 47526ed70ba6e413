"""Torch-allocating conveniences over the C ABI (outputs are new device tensors)."""
from __future__ import annotations

import torch

from .jas import (JAS_KEEP_IDS, JAS_QUERY_ONLY, JAS_UPPER, jas_encode, jas_encode_opts, jas_gram, jas_query)


def _dev_u64(x, device):
    t = torch.as_tensor(x)
    if t.dtype != torch.uint64:
        t = t.to(torch.int64).view(torch.uint64) if t.dtype == torch.int64 else t.to(torch.uint64)
    return t.to(device).contiguous()


def encode(ids, offsets, universe_bits: int, batch_bits: int = 0, dense_min_degree: int = 0, keep_ids: bool = False,
           hbm_budget_bytes: int = 0, word_bits: int = 64, device="cuda", stream=None, query_only: bool = False):
    """Encode n CSR sets (device tensors, or anything torch.as_tensor accepts).  query_only
    (with keep_ids) keeps only what queries need."""
    ids_t = _dev_u64(ids, device)
    off_t = _dev_u64(offsets, device)
    n = off_t.numel() - 1
    flags = (JAS_KEEP_IDS if keep_ids else 0) | (JAS_QUERY_ONLY if query_only else 0)
    opts = jas_encode_opts(universe_bits, batch_bits, dense_min_degree, flags, hbm_budget_bytes, word_bits)
    return jas_encode(ids_t, off_t, n, opts, stream)


def gram(db, upper: bool = False, want_den: bool = True, want_J: bool = True, flags: int = 0, device="cuda",
         stream=None):
    """All pairs: dict of B (int32), card (int64), den (int64), J (float64)."""
    n = db.n
    length = n * (n + 1) // 2 if upper else n * n
    B = torch.empty(length, dtype=torch.int32, device=device)
    card = torch.empty(n, dtype=torch.int64, device=device)
    den = torch.empty(length, dtype=torch.int64, device=device) if want_den else None
    J = torch.empty(length, dtype=torch.float64, device=device) if want_J else None
    jas_gram(db, flags | (JAS_UPPER if upper else 0), stream, B, card, den, J)
    shape = (length,) if upper else (n, n)
    out = {"B": B.view(shape), "card": card}
    if den is not None:
        out["den"] = den.view(shape)
    if J is not None:
        out["J"] = J.view(shape)
    return out


def query(db, q_ids, q_offsets, device="cuda", stream=None, flags: int = 0):
    """Query sets x database: dict of B, q_card, den, J ([nq, n])."""
    qi = _dev_u64(q_ids, device)
    qo = _dev_u64(q_offsets, device)
    nq = qo.numel() - 1
    n = db.n
    B = torch.empty((nq, n), dtype=torch.int32, device=device)
    qc = torch.empty(nq, dtype=torch.int64, device=device)
    den = torch.empty((nq, n), dtype=torch.int64, device=device)
    J = torch.empty((nq, n), dtype=torch.float64, device=device)
    jas_query(db, qi, qo, nq, flags, stream, B, qc, den, J)
    return {"B": B, "q_card": qc, "den": den, "J": J}
