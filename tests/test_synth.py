"""The input generator: determinism, shape and sharing structure (no GPU)."""
import numpy as np

import synth


def test_deterministic_and_subset_regeneration():
    s = synth.scaled(synth.workload("batching"), n=40, size_scale=0.01, pool_scale=0.01)
    a, ao = synth.generate(s)
    b, bo = synth.generate(s)
    assert np.array_equal(a, b) and np.array_equal(ao, bo)
    idx = [7, 3, 39]
    c, co = synth.generate_samples(s, idx)
    for k, i in enumerate(idx):
        assert np.array_equal(c[int(co[k]):int(co[k + 1])], a[int(ao[i]):int(ao[i + 1])])


def test_universe_and_sizes():
    for name in ["tiny", "paperlike", "precision", "batching", "serving_db"]:
        s = synth.workload(name)
        off = synth.offsets(s)
        sizes = np.diff(off.astype(np.int64))
        assert sizes.size == s.n
        if s.size_kind == 0:
            assert sizes.min() >= round(s.size_a) and sizes.max() <= round(s.size_b)
        else:
            assert sizes.min() >= s.size_lo and sizes.max() <= s.size_hi
    s = synth.workload("tiny")
    ids, off = synth.generate(s)
    assert ids.max() < (1 << 24)


def test_pool_part_is_distinct_and_from_the_pool():
    s = synth.scaled(synth.workload("tiny"), n=16)
    ids, off = synth.generate(s)
    pool_ids = None
    for i in range(s.n):
        size, k, dups, c = synth.plan(s, i)
        x = ids[int(off[i]):int(off[i]) + k]
        assert np.unique(x).size == k
    # the pool has 2^16 IDs: the union of all pool parts stays inside it
    allpool = np.concatenate([ids[int(off[i]):int(off[i]) + synth.plan(s, i)[1]] for i in range(s.n)])
    assert np.unique(allpool).size <= (1 << 16)


def test_duplicates_injected():
    s = synth.scaled(synth.workload("tiny"), n=4, dup_rate=0.05)
    ids, off = synth.generate(s)
    for i in range(4):
        x = ids[int(off[i]):int(off[i + 1])]
        size, k, dups, c = synth.plan(s, i)
        assert x.size == size + dups and dups > 0
        assert np.unique(x).size <= size
