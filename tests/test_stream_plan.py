"""Host side of the streamed product: the part slices and their gather (no GPU)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synth
from paper_1911_04200_amd import stream


def test_parts_cut_every_set_at_the_id_ranges():
    spec = synth.bernoulli(0.01, rows_log2=14, n=37, seed=4)
    ids, off = synth.generate(spec)
    for pb in (0, 1, 3, 14):
        bounds = stream.plan_parts(ids, off, 14, pb)
        assert bounds.shape == ((1 << pb) + 1, 37)
        assert np.array_equal(bounds[0], off[:-1]) and np.array_equal(bounds[-1], off[1:])
        shift = 14 - pb
        for p in range(1 << pb):
            for i in range(37):
                x = ids[int(bounds[p, i]):int(bounds[p + 1, i])]
                # brute force: the set's IDs whose top bits are p
                want = ids[int(off[i]):int(off[i + 1])]
                want = want[(want >> np.uint64(shift)) == p]
                assert np.array_equal(x, want)


def test_gather_packs_one_part_as_csr():
    spec = synth.bernoulli(0.05, rows_log2=12, n=20, seed=2)
    ids, off = synth.generate(spec)
    bounds = stream.plan_parts(ids, off, 12, 2)
    dst = np.zeros(ids.size, dtype=np.uint64)
    with ThreadPoolExecutor(4) as pool:
        o = stream._gather(ids, bounds[1], bounds[2], dst, pool, 4)
    for i in range(20):
        x = dst[o[i]:o[i + 1]]
        assert np.array_equal(x, ids[int(bounds[1, i]):int(bounds[2, i])])
        assert np.all((x >> np.uint64(10)) == 1)
    # relabelled to offsets in the part's ID range [1 << 10, 2 << 10)
    with ThreadPoolExecutor(4) as pool:
        o2 = stream._gather(ids, bounds[1], bounds[2], dst, pool, 4, base=1 << 10)
    assert np.array_equal(o2, o)
    for i in range(20):
        x = dst[o[i]:o[i + 1]]
        assert np.array_equal(x + np.uint64(1 << 10), ids[int(bounds[1, i]):int(bounds[2, i])])
        assert np.all(x < (1 << 10))


def test_unsorted_or_out_of_range_sets_are_refused():
    ids = np.array([5, 3, 9], dtype=np.uint64)
    off = np.array([0, 3], dtype=np.uint64)
    with pytest.raises(ValueError, match="ascending"):
        stream.plan_parts(ids, off, 8, 1)
    with pytest.raises(ValueError, match="2\\^universe_bits"):
        stream.plan_parts(np.array([1, 300], dtype=np.uint64), off[:2] * 0 + np.array([0, 2], np.uint64), 8, 1)
    with pytest.raises(ValueError):
        stream.plan_parts(ids, off, 8, 9)
