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


def _sets(ids, off):
    return [ids[int(off[i]):int(off[i + 1])].astype(np.int64) for i in range(off.size - 1)]


def test_bernoulli_sets_are_increasing_rows():
    s = synth.bernoulli(0.02, rows_log2=14, n=64)
    ids, off = synth.generate(s)
    for x in _sets(ids, off):
        assert x.size == 0 or (x.min() >= 0 and x.max() < (1 << 14))
        assert np.all(np.diff(x) > 0)
    c, co = synth.generate_samples(s, [5, 63, 0])
    for k, i in enumerate([5, 63, 0]):
        assert np.array_equal(c[int(co[k]):int(co[k + 1])], ids[int(off[i]):int(off[i + 1])])


def test_bernoulli_entry_statistics():
    # every entry present with probability p, independently (Sec. V-A3's synthetic matrices):
    # set sizes have mean m p; a row follows a present row with probability p
    # (a skip off by one makes that 0 or 1); the rows are spread evenly
    m_log2, n, p = 16, 400, 0.01
    m = 1 << m_log2
    ids, off = synth.generate(synth.bernoulli(p, rows_log2=m_log2, n=n))
    sizes = np.diff(off.astype(np.int64))
    mean_sd = np.sqrt(m * p * (1 - p) / n)
    assert abs(sizes.mean() - m * p) < 6 * mean_sd
    assert abs(sizes.var() / (m * p * (1 - p)) - 1) < 0.25  # binomial variance
    follow = sum(int(np.count_nonzero(np.diff(x) == 1)) for x in _sets(ids, off))
    trials = int(sizes.sum()) - n
    assert abs(follow / trials - p) < 6 * np.sqrt(p * (1 - p) / trials)
    per_block = np.bincount(ids.astype(np.int64) >> (m_log2 - 4), minlength=16)
    expect = n * (m / 16) * p
    assert np.all(np.abs(per_block - expect) < 6 * np.sqrt(expect))


def test_bernoulli_degenerate_densities():
    ids, off = synth.generate(synth.bernoulli(1.0, rows_log2=10, n=3))
    assert np.array_equal(off, np.arange(4, dtype=np.uint64) * 1024)
    assert np.array_equal(ids, np.tile(np.arange(1024, dtype=np.uint64), 3))
    ids, off = synth.generate(synth.bernoulli(0.0, rows_log2=10, n=3))
    assert ids.size == 0 and np.all(off == 0)


def test_bernoulli_sweep_sizes():
    for name, (p, rl) in synth.BERNOULLI.items():
        s = synth.workload(name)
        assert s.n == 10000 and s.rows == 1 << rl and s.universe_bits == rl and synth.BATCH_BITS[name] == rl
        assert s.density == p


def test_rmat_neighbourhoods_form_an_undirected_simple_graph():
    ids, off = synth.rmat_graph(10, 16, seed=1)
    n = 1 << 10
    assert off.size == n + 1 and ids.max() < n
    edges = set()
    for v in range(n):
        nb = ids[int(off[v]):int(off[v + 1])].astype(np.int64)
        assert np.all(np.diff(nb) > 0) and v not in nb  # ascending, no repeats, no self loop
        edges.update((v, int(u)) for u in nb)
    assert all((u, v) in edges for v, u in edges)  # u in N(v) <=> v in N(u)
    deg = np.diff(off.astype(np.int64))
    assert deg.max() > 10 * deg.mean() and (deg == 0).any()  # R-MAT's skew: hubs and isolated vertices
    a, ao = synth.rmat_graph(10, 16, seed=1)
    assert np.array_equal(a, ids) and np.array_equal(ao, off)


def test_graph_collections_behave_like_specs():
    g = synth.workload("graph_s13_ef64")
    assert g.n == 8192 and g.universe_bits == 13 and synth.BATCH_BITS["graph_s13_ef64"] == 13
    ids, off = synth.generate(g)
    c, co = synth.generate_samples(g, [9, 2])
    assert np.array_equal(c[:int(co[1])], ids[int(off[9]):int(off[10])])
    assert np.array_equal(synth.offsets(g), off)
