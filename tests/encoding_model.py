"""A plain host model of the encoded indicator matrix (tests only).

Written from the paper's definitions, with numpy, to check what jas_encode
stores (not how): the nonzeros of A are the distinct (ID, sample) pairs; a
row (ID) is kept if it is nonzero (the filter f of Eq. (5)) and, for the
Gram product, only if it is shared by >= 2 sets (a row of one set adds only
to B_ii = |X_i|); rows shared by >= t sets are bit-packed, the others kept as
row lists (t = dense_min_degree).  Packed rows are cut into batches of m~ =
2^batch_bits IDs (Eq. (3)) and compacted in ID order inside a batch (Eq. (6));
packed row p of a batch is bit p mod b of word row floor(p / b) of that batch
(the bit rule before Eq. (7)), word rows of all batches numbered in batch
order.  The stored array keeps one 64-bit element per (row, column): a word
row itself for b = 64, the low (even word row) or high (odd word row) half
of element row floor(r / 2) for b = 32.  The row lists are the pairs a < b
of each list row's sets as (a << 16) | b.
"""
from __future__ import annotations

import numpy as np


def model(sets_ids: np.ndarray, sets_off: np.ndarray, batch_bits: int, universe_bits: int, word_bits: int,
          dmin: int):
    """Expected encoding of normalised CSR sets (each sorted, no repeats)."""
    n = sets_off.size - 1
    card = np.diff(sets_off.astype(np.int64))
    sample = np.repeat(np.arange(n, dtype=np.int64), card)
    ids = sets_ids.astype(np.uint64)
    order = np.lexsort((sample, ids))  # by ID, then sample
    ids, sample = ids[order], sample[order]
    uid, first, deg = np.unique(ids, return_index=True, return_counts=True)
    shared = deg >= 2
    packed = shared & (deg >= dmin)
    listed = shared & ~packed
    bb = min(batch_bits, universe_bits) if batch_bits else universe_bits
    # packed rows, batch by batch in ID order
    prow = np.flatnonzero(packed)
    pbatch = (uid[prow] >> np.uint64(bb)).astype(np.int64) if prow.size else np.zeros(0, np.int64)
    bvals, bstart, bcount = np.unique(pbatch, return_index=True, return_counts=True)
    p_in_batch = np.arange(prow.size) - np.repeat(bstart, bcount)
    words_per_batch = (bcount + word_bits - 1) // word_bits
    wbase = np.concatenate([[0], np.cumsum(words_per_batch)]).astype(np.int64)
    word_row = np.repeat(wbase[:-1], bcount) + p_in_batch // word_bits
    bit = p_in_batch % word_bits
    h = int(wbase[-1])
    if word_bits == 64:
        w_rows, erow, ebit = h, word_row, bit
    else:
        w_rows, erow, ebit = (h + 1) // 2, word_row // 2, bit + 32 * (word_row % 2)
    stride = ((max(n, 1) + 127) // 128) * 128
    W = np.zeros((w_rows, stride), dtype=np.uint64)
    rdeg = deg[prow]
    er = np.repeat(erow, rdeg)
    eb = np.repeat(ebit, rdeg).astype(np.uint64)
    cols = np.concatenate([sample[first[r]:first[r] + deg[r]] for r in prow]) if prow.size else np.zeros(0, np.int64)
    np.bitwise_or.at(W, (er, cols), np.left_shift(np.uint64(1), eb))
    # row lists: pairs a < b of each list row, as (a << 16) | b
    pairs = []
    for r in np.flatnonzero(listed):
        s = sample[first[r]:first[r] + deg[r]]
        a, b = np.triu_indices(s.size, 1)
        pairs.append((s[a].astype(np.uint32) << np.uint32(16)) | s[b].astype(np.uint32))
    pairs = np.concatenate(pairs) if pairs else np.zeros(0, np.uint32)
    sbits = (n - 1).bit_length() if n > 1 else 0  # ceil(log2 n)
    keys = (ids << np.uint64(sbits)) | sample.astype(np.uint64)
    nz_halves = [(W & np.uint64(0xFFFFFFFF)) != 0, (W >> np.uint64(32)) != 0] if word_bits == 32 else [W != 0]
    z_rows = np.concatenate([z.sum(axis=1) for z in nz_halves]) if w_rows else np.zeros(0, np.int64)
    return {
        "card": card, "W": W, "w_rows": w_rows, "stride": stride, "list_pairs": pairs, "keys": keys,
        "packed_ids": uid[prow], "packed_erow": erow, "packed_ebit": ebit,
        "stats": {"n_pairs": int(ids.size), "n_rows": int(uid.size), "n_shared_rows": int(shared.sum()),
                  "n_packed_rows": int(packed.sum()), "n_list_rows": int(listed.sum()),
                  "n_batches": int(bvals.size), "n_word_rows": h, "nnz_words": int(z_rows.sum()),
                  "word_pairs_F": int((z_rows * (z_rows + 1) // 2).sum()),
                  "list_pairs": int(pairs.size)},
    }


def decode_packed(W: np.ndarray, n: int, packed_ids, packed_erow, packed_ebit):
    """Per sample, the IDs of its packed rows read back from the stored words."""
    table = {(int(e), int(b)): int(i) for i, e, b in zip(packed_ids, packed_erow, packed_ebit)}
    out = [[] for _ in range(n)]
    rows, cols = np.nonzero(W[:, :n])
    for e, c in zip(rows, cols):
        w = int(W[e, c])
        while w:
            b = (w & -w).bit_length() - 1
            out[c].append(table[(int(e), b)])
            w &= w - 1
    return [np.array(sorted(x), dtype=np.uint64) for x in out]
