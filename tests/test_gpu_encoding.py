"""The stored encoding against a host model of its definition (round trip).

jas_db_read returns what jas_encode stored; tests/encoding_model.py builds
the same arrays on the host from the oracle's normalised sets by the paper's
definitions (filter, batches, compaction, bit rule; Eqs. (3), (5), (6)).
Every stored word, list pair, key and counter must match; the words decoded
back through the model's row table must give each set's packed IDs; and the
word width b (32 or 64, Sec. III-B) must leave B unchanged.
"""
import numpy as np
import pytest

import encoding_model
import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1911_04200_amd import jas as cabi  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


CASES = {
    "paperlike": lambda: (synth.scaled(synth.workload("paperlike"), n=200, size_scale=0.004, pool_scale=0.004,
                                       dup_rate=0.01), 26),
    "batching": lambda: (synth.scaled(synth.workload("batching"), n=300, size_scale=0.003, pool_scale=0.002), 20),
    "bernoulli": lambda: (synth.bernoulli(0.05, rows_log2=12, n=130, seed=3), 8),
    "tiny_n1": lambda: (synth.scaled(synth.workload("tiny"), n=1, size_scale=0.05), 24),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("word_bits", [32, 64])
@pytest.mark.parametrize("dmin", [2, 5, 0])
def test_stored_encoding_matches_the_model(case, word_bits, dmin):
    spec, bb = CASES[case]()
    ids, off = synth.generate(spec)
    n = off.size - 1
    opts = cabi.jas_encode_opts(spec.universe_bits, bb, dmin, cabi.JAS_KEEP_IDS, 0, word_bits)
    db, st = cabi.jas_encode(dev(ids), dev(off), n, opts, None)
    torch.cuda.synchronize()
    s, so = oracle.normalize(ids, off)
    m = encoding_model.model(s, so, bb, spec.universe_bits, word_bits, int(st["dense_min_degree"]))
    assert st["word_bits"] == word_bits and st["w_rows"] == m["w_rows"] and st["w_stride"] == m["stride"]
    t = (n + 127) // 128  # the packed Gram's work units: (stored word row, 128-column tile pair)
    assert st["dense_tiles"] == m["w_rows"] * (t * (t + 1) // 2)
    assert st["word_pairs_W"] == st["dense_tiles"] * 128 * 128
    if word_bits == 64:  # whole tiles run, zero words included (F counts b-bit words)
        assert st["word_pairs_W"] >= st["word_pairs_F"]
    for k, v in m["stats"].items():
        assert st[k] == v, f"stats[{k}] = {st[k]}, model {v}"
    assert np.array_equal(cabi.jas_db_read(db, cabi.JAS_DB_CARD), m["card"])
    W = cabi.jas_db_read(db, cabi.JAS_DB_WORDS).reshape(m["w_rows"], m["stride"])
    bad = np.argwhere(W != m["W"])
    assert bad.size == 0, f"stored words differ at (row, column) {bad[:5].tolist()}"
    keys = cabi.jas_db_read(db, cabi.JAS_DB_KEYS)
    assert np.array_equal(keys, m["keys"])
    pairs = cabi.jas_db_read(db, cabi.JAS_DB_LIST_PAIRS)
    assert st["n_list_pairs"] == pairs.size
    if pairs.size:
        assert np.all(np.diff((pairs >> np.uint32(16)).astype(np.int64)) >= 0), "pairs not ordered by a"
    assert np.array_equal(np.sort(pairs), np.sort(m["list_pairs"]))
    # decoded words: each set's packed rows
    dec = encoding_model.decode_packed(W, n, m["packed_ids"], m["packed_erow"], m["packed_ebit"])
    packed = set(m["packed_ids"].tolist())
    for i in range(n):
        want = np.array(sorted(x for x in s[int(so[i]):int(so[i + 1])].tolist() if x in packed), dtype=np.uint64)
        assert np.array_equal(dec[i], want), f"set {i}: decoded packed IDs differ"
    db.close()


@pytest.mark.parametrize("case", ["paperlike", "batching", "bernoulli"])
def test_word_width_leaves_B_unchanged(case):
    spec, bb = CASES[case]()
    ids, off = synth.generate(spec)
    n = off.size - 1
    ref = oracle.all_pairs(ids, off)
    outs = {}
    for word_bits in (32, 64):
        opts = cabi.jas_encode_opts(spec.universe_bits, bb, 2, 0, 0, word_bits)
        db, st = cabi.jas_encode(dev(ids), dev(off), n, opts, None)
        for flags in (0, cabi.JAS_FORCE_POPCOUNT):
            B = torch.empty(n * n, dtype=torch.int32, device="cuda")
            J = torch.empty(n * n, dtype=torch.float64, device="cuda")
            cabi.jas_gram(db, flags, None, B, None, None, J)
            torch.cuda.synchronize()
            outs[(word_bits, flags)] = (B.cpu().numpy().reshape(n, n), J.cpu().numpy().reshape(n, n))
        db.close()
    for (wb, flags), (B, J) in outs.items():
        assert np.array_equal(B, ref["inter"]), f"b = {wb}, flags {flags}"
        assert np.array_equal(J.view(np.uint64), ref["J"].view(np.uint64)), f"b = {wb}, flags {flags}"
