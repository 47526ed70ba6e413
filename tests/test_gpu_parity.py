"""HIP path vs the CPU oracle, element by element (needs a gfx950 GPU).

B and the unions are compared as integers, J bit for bit (binary64), |X_i|
exactly.  Sizes here finish in seconds on the oracle and still span several
128-column tiles, many row batches and ragged tails.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_04200_amd as jas  # noqa: E402
from paper_1911_04200_amd import jas as cabi  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def gpu_all_pairs(ids, off, U, batch_bits=0, dmin=0, upper=False, flags=0):
    db, st = jas.encode(dev(ids), dev(off), universe_bits=U, batch_bits=batch_bits, dense_min_degree=dmin)
    out = jas.gram(db, upper=upper, flags=flags)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    db.close()
    return res, st


def assert_matches(res, ref, upper=False):
    n = ref["card"].size
    assert np.array_equal(res["card"], ref["card"]), "|X_i|"
    if upper:
        iu = np.triu_indices(n)
        want = {"B": ref["inter"][iu], "den": ref["union"][iu], "J": ref["J"][iu]}
    else:
        want = {"B": ref["inter"], "den": ref["union"], "J": ref["J"]}
    bad = np.argwhere(res["B"] != want["B"])
    assert bad.size == 0, f"B differs at {bad[:5].tolist()}"
    assert np.array_equal(res["den"], want["den"]), "unions differ"
    assert np.array_equal(res["J"].view(np.uint64), want["J"].view(np.uint64)), "J differs"


@pytest.fixture(scope="module")
def tiny():
    spec = synth.workload("tiny")
    ids, off = synth.generate(spec)
    return spec, ids, off, oracle.all_pairs(ids, off)


# (batch_bits, dense_min_degree, upper): one batch .. 2^20 batches, every row packed .. no row packed
VARIANTS = [(24, 0, False), (24, 0, True), (16, 2, False), (10, 3, False), (4, 5, True), (24, 1000, False),
            (12, 8, False), (20, 4, True)]


@pytest.mark.parametrize("bb,dmin,upper", VARIANTS)
@pytest.mark.parametrize("path", ["popcount", "mfma"])
def test_tiny_workload(tiny, bb, dmin, upper, path):
    spec, ids, off, ref = tiny
    flags = cabi.JAS_FORCE_POPCOUNT if path == "popcount" else cabi.JAS_FORCE_MFMA
    res, st = gpu_all_pairs(ids, off, spec.universe_bits, bb, dmin, upper, flags)
    assert_matches(res, ref, upper)
    assert st["n_ids"] == ids.size
    assert st["n_pairs"] == int(ref["card"].sum())


SCALED = {
    # structure of each workload at sizes the oracle finishes in seconds
    "paperlike": dict(n=300, size_scale=0.004, pool_scale=0.004),
    "precision": dict(n=257, size_scale=0.01, pool_scale=0.01),
    "batching": dict(n=400, size_scale=0.004, pool_scale=0.004),
    "serving_db": dict(n=200, size_scale=0.01, pool_scale=0.005),
}


@pytest.mark.parametrize("name", sorted(SCALED))
@pytest.mark.parametrize("dmin", [0, 2, 6])
def test_scaled_workloads(name, dmin):
    spec = synth.scaled(synth.workload(name), **SCALED[name])
    ids, off = synth.generate(spec)
    ref = oracle.all_pairs(ids, off)
    res, st = gpu_all_pairs(ids, off, spec.universe_bits, synth.BATCH_BITS[name], dmin, upper=(dmin == 6))
    assert_matches(res, ref, upper=(dmin == 6))
    assert st["n_packed_rows"] + st["n_list_rows"] == st["n_shared_rows"] > 0
    if dmin == 2:
        assert st["n_packed_rows"] == st["n_shared_rows"]
    elif dmin == 6:
        assert st["n_list_rows"] > 0
    else:
        assert st["dense_min_degree"] >= 2


# The paper's synthetic indicator matrices (Sec. V-A3): each entry 1 with
# probability p.  From rows of degree ~0.3 (row lists) to p = 1, where every
# set holds every row (B = m, J = 1); one batch of all rows and 16 batches.
BERNOULLI_CASES = [(1e-3, 16, 300), (1e-2, 14, 200), (0.1, 12, 150), (0.5, 10, 130), (1.0, 9, 70)]


@pytest.mark.parametrize("p,rows_log2,n", BERNOULLI_CASES)
@pytest.mark.parametrize("batches", [1, 16])
@pytest.mark.parametrize("path", ["auto", "popcount"])
def test_bernoulli_matrices(p, rows_log2, n, batches, path):
    spec = synth.bernoulli(p, rows_log2, n, seed=batches)
    ids, off = synth.generate(spec)
    ref = oracle.all_pairs(ids, off)
    flags = cabi.JAS_FORCE_POPCOUNT if path == "popcount" else 0
    bb = rows_log2 - (batches.bit_length() - 1)
    res, st = gpu_all_pairs(ids, off, rows_log2, bb, 0, flags=flags)
    assert_matches(res, ref)
    if p == 1.0:
        assert np.all(res["B"] == 1 << rows_log2) and np.all(res["J"] == 1.0)
        assert st["n_packed_rows"] == 1 << rows_log2


# Vertex similarity (Sec. II-F): the sets are the neighbourhoods of an R-MAT
# graph (hubs of degree ~ n/5 next to isolated vertices), A its adjacency.
@pytest.mark.parametrize("dmin", [0, 2, 1 << 20])
def test_graph_neighbourhood_similarity(dmin):
    ids, off = synth.rmat_graph(10, 16, seed=2)
    ref = oracle.all_pairs(ids, off)
    res, st = gpu_all_pairs(ids, off, 10, 10, dmin)
    assert_matches(res, ref)


def test_graph_link_prediction_queries():
    ids, off = synth.rmat_graph(12, 8, seed=3)
    n = off.size - 1
    db, _ = jas.encode(dev(ids), dev(off), universe_bits=12, batch_bits=12, keep_ids=True)
    # queries: neighbourhoods of some vertices, one with an edge added, and an empty set
    qs = [ids[int(off[v]):int(off[v + 1])] for v in (0, 17, 4095)]
    qs.append(np.union1d(qs[1], np.array([5], np.uint64)))
    qs.append(np.zeros(0, np.uint64))
    qo = np.zeros(len(qs) + 1, np.uint64)
    qo[1:] = np.cumsum([q.size for q in qs])
    qi = np.concatenate(qs).astype(np.uint64)
    out = jas.query(db, dev(qi), dev(qo))
    torch.cuda.synchronize()
    ref = oracle.cross(qi, qo, ids, off)
    assert np.array_equal(out["B"].cpu().numpy(), ref["inter"])
    assert np.array_equal(out["den"].cpu().numpy(), ref["union"])
    assert np.array_equal(out["J"].cpu().numpy().view(np.uint64), ref["J"].view(np.uint64))
    db.close()


def test_duplicates_and_empty_sets():
    spec = synth.scaled(synth.workload("tiny"), n=40, dup_rate=0.3)
    ids, off = synth.generate(spec)
    # make sets 3, 17 and 39 empty and set 20 a copy of set 5
    sets = [ids[int(off[i]):int(off[i + 1])] for i in range(40)]
    sets[3] = sets[17] = sets[39] = np.zeros(0, np.uint64)
    sets[20] = sets[5].copy()
    off2 = np.zeros(41, np.uint64)
    off2[1:] = np.cumsum([s.size for s in sets])
    ids2 = np.concatenate(sets)
    ref = oracle.all_pairs(ids2, off2)
    for dmin in (0, 4):
        res, _ = gpu_all_pairs(ids2, off2, 24, 14, dmin)
        assert_matches(res, ref)
    assert res["J"][3, 17] == 1.0 and res["J"][3, 5] == 0.0 and res["J"][5, 20] == 1.0


def encode_timed(ids, off, U, **kw):
    """Encode and Gram with the library's timers on; returns (result, stats, timer names)."""
    cabi.jas_timing_report()
    cabi.jas_timing_enable(True)
    try:
        res, st = gpu_all_pairs(ids, off, U, **kw)
    finally:
        names = set(cabi.jas_timing_report())
        cabi.jas_timing_enable(False)
    return res, st, names


def csr(sets):
    off = np.zeros(len(sets) + 1, np.uint64)
    off[1:] = np.cumsum([s.size for s in sets])
    return np.concatenate(sets).astype(np.uint64), off


@pytest.mark.parametrize("case", ["uniform", "uniform_u24", "narrow_ids", "one_hot_id"])
def test_bucket_ranges_and_fallback(case):
    """Keys are sorted on their top ID bits only and each range of whole buckets is
    finished in LDS (keys held in 32 bits relative to the range's first bucket when
    they fit, as with U=24 here, else in 64); a bucket too large for LDS (IDs crowded
    into a narrow range, or one ID repeated many times) must take the full sort and
    give the same result."""
    rng = np.random.default_rng({"uniform": 1, "uniform_u24": 4, "narrow_ids": 2, "one_hot_id": 3}[case])
    if case.startswith("uniform"):
        U, n = (36, 90) if case == "uniform" else (24, 90)
        core = rng.integers(0, 1 << U, 4000, dtype=np.uint64)
        sets = [np.concatenate([rng.choice(core, int(rng.integers(0, 3000))),
                                rng.integers(0, 1 << U, int(rng.integers(0, 3000)), dtype=np.uint64)])
                for _ in range(n)]
    elif case == "narrow_ids":
        U, n = 40, 60
        sets = [rng.choice(1 << 12, int(rng.integers(500, 2500)), replace=False).astype(np.uint64)
                for _ in range(n)]
    else:
        U, n = 32, 40
        sets = [rng.integers(0, 1 << 32, 2000, dtype=np.uint64) for _ in range(n)]
        sets[7] = np.concatenate([sets[7], np.full(20000, 12345, np.uint64)])
        sets[9] = np.concatenate([sets[9], np.array([12345], np.uint64)])
    ids, off = csr(sets)
    ref = oracle.all_pairs(ids, off)
    res, st, names = encode_timed(ids, off, U, dmin=0)
    assert_matches(res, ref)
    assert st["n_pairs"] == int(ref["card"].sum())
    if case == "uniform":  # relative keys need 37 bits
        assert "local_cls_wide" in names and "host:classify_fallback" not in names
    elif case == "uniform_u24":  # relative keys fit 32 bits
        assert "local_cls" in names and "local_cls_wide" not in names and "host:classify_fallback" not in names
    else:
        assert "host:classify_fallback" in names and "cls_write" in names


def max_range_len(ids, off, U, stride):
    """Longest range [first bucket edge >= c*stride, first edge >= (c+1)*stride)
    of the keys sorted by their top ID bits, as the encoder forms them."""
    n = off.size - 1
    N = ids.size
    sbits = max(1, int(np.ceil(np.log2(n))))
    # the encoder's choice of sorted top bits: buckets of about 512 keys, or
    # about 1024 when a range's keys still fit 32 bits (4 bits for its span)
    tb = min(U, int(np.ceil(np.log2(-(-N // 512)))))
    fewer = min(U, int(np.ceil(np.log2(-(-N // 1024)))))
    if fewer > 0 and (U - fewer) + 4 + sbits <= 32:
        tb = fewer
    bucket = np.sort(ids >> np.uint64(U - tb), kind="stable")
    edges = np.flatnonzero(np.diff(bucket)) + 1
    edges = np.concatenate([[0], edges, [N]])
    starts = [edges[np.searchsorted(edges, min(c * stride, N))] for c in range(-(-N // stride) + 1)]
    return int(np.max(np.diff(starts)))


@pytest.mark.parametrize("declined", [False, True])
def test_first_sort_pass_forms_the_keys(monkeypatch, declined):
    """With a global sort the digits are counted from the IDs alone and the
    sort's first pass forms the keys (id << s | sample) itself, the sample of
    each tile found once; when the single-pass sort declines (a digit total
    above its look-back counts, forced here by a lowered test limit), the keys
    are formed by a kernel of their own and sorted by reduce-then-scan
    passes.  Both give the oracle's result."""
    spec = synth.scaled(synth.workload("paperlike"), n=300, size_scale=0.004, pool_scale=0.004)
    ids, off = synth.generate(spec)
    # a few empty sets and many short ones, so that tiles hold several samples
    sets = [ids[int(off[i]):int(off[i + 1])] for i in range(spec.n)]
    sets[1] = sets[7] = np.zeros(0, np.uint64)
    sets[20:120] = [s[:37] for s in sets[20:120]]
    ids, off = csr(sets)
    if declined:
        monkeypatch.setenv("JAS_TEST_SCATTER_LIMIT", "100")
    ref = oracle.all_pairs(ids, off)
    res, st, names = encode_timed(ids, off, spec.universe_bits)
    assert_matches(res, ref)
    assert "count_digits" in names
    if declined:
        assert "build_keys" in names and "radix_scatter" in names and "radix_onesweep" not in names
    else:
        assert "build_keys" not in names and "radix_onesweep" in names


def test_concurrent_encodes_on_two_streams():
    """Two host threads encode different collections on their own streams at
    once (each encode puts its row-list pairs on the library's side stream
    while it packs on its own stream); both results are the oracle's."""
    import threading

    cases = []
    for k, name in enumerate(("paperlike", "precision")):
        spec = synth.scaled(synth.workload(name), **SCALED[name])
        ids, off = synth.generate(spec)
        cases.append((spec, ids, off, oracle.all_pairs(ids, off)))
    results, errors = [None, None], []

    def work(k):
        try:
            spec, ids, off, _ = cases[k]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for _ in range(3):
                    db, _ = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, dense_min_degree=6)
                    out = jas.gram(db)
                    st.synchronize()
                    results[k] = {key: v.cpu().numpy() for key, v in out.items()}
                    db.close()
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        assert_matches(results[k], cases[k][3])


@pytest.mark.parametrize("N", [6145, 8192, 8193, 16384, 16385, 24577])
def test_scatter_tile_edges(N):
    """Entry counts around the single-pass scatter's 8192-entry tiles (the
    global sort runs from 6145 entries on), with set boundaries exactly on,
    just before and just after tile boundaries and empty sets there, so that
    the first pass's per-tile samples (first and last entry of each tile, the
    starts inside it) meet every case."""
    rng = np.random.default_rng(N)
    U = 30
    cuts = sorted({0, N} | {c for t in range(8192, N, 8192) for c in (t - 1, t, t + 1) if 0 < c < N}
                  | {int(x) for x in rng.integers(1, N, 6)})
    sizes = [b - a for a, b in zip(cuts, cuts[1:])]
    sets = []
    for k, sz in enumerate(sizes):
        sets.append(rng.integers(0, 1 << U, sz, dtype=np.uint64))
        if k % 3 == 1:
            sets.append(np.zeros(0, np.uint64))  # an empty set at this boundary
    # shared IDs, so that rows of several samples exist
    pool = rng.integers(0, 1 << U, 64, dtype=np.uint64)
    for st in sets:
        if st.size:
            st[: min(st.size, 5)] = rng.choice(pool, min(st.size, 5))
    ids, off = csr(sets)
    assert ids.size == N
    ref = oracle.all_pairs(ids, off)
    res, st, names = encode_timed(ids, off, U)
    assert_matches(res, ref)
    assert "radix_onesweep" in names and "count_digits" in names


def test_every_id_bit_sorted_globally():
    """A small universe and many entries (U = 8, 90,000 entries with repeats):
    the global sort covers every ID bit, so each bucket is one ID with its
    keys in sample order and the ranges (from 4096-key strides) are finished
    in LDS with no sort passes."""
    rng = np.random.default_rng(21)
    sets = [rng.integers(0, 256, 300, dtype=np.uint64) for _ in range(300)]
    sets[4] = np.zeros(0, np.uint64)
    ids, off = csr(sets)
    assert -(-ids.size // 512) > 128  # ceil(log2(N / 512)) >= U
    ref = oracle.all_pairs(ids, off)
    cabi.jas_timing_report()
    cabi.jas_timing_enable(True)
    try:
        res, st = gpu_all_pairs(ids, off, 8)
    finally:
        rep = cabi.jas_timing_report()
        cabi.jas_timing_enable(False)
    assert_matches(res, ref)
    assert rep["range_starts"][0] == 1 and "local_cls" in rep and "host:classify_fallback" not in rep


@pytest.mark.parametrize("U,per_cluster,tries", [(36, 26, 1), (36, 36, 2), (28, 36, 2)])
def test_longer_ranges_when_a_bucket_is_large(U, per_cluster, tries):
    """Clusters of IDs make buckets of 90 * per_cluster keys.  With 26 per
    cluster (~2300 keys) some 3072-key-stride range exceeds the 4096 keys the
    four-blocks-per-CU kernel holds, so the kernel for 6144-key ranges runs;
    with 36 (~3200 keys) some range exceeds even 6144 keys at that stride and
    the encoder tries 2048.  Either way the ranges are finished in LDS, with
    keys held in 64 bits there for U = 36 and in 32 for U = 28 (where the
    encoder sorts one top bit fewer, as the 32-bit keys still fit)."""
    rng = np.random.default_rng(11)
    n = 90
    sets = []
    for _ in range(n):
        parts = [rng.integers(0, 1 << U, 2000, dtype=np.uint64)]
        for k in range(8):
            parts.append((np.uint64(k << (U - 4)) + rng.choice(1 << 20, per_cluster, replace=False)).astype(np.uint64))
        sets.append(np.concatenate(parts))
    ids, off = csr(sets)
    if tries == 1:
        assert 6144 >= max_range_len(ids, off, U, 3072) > 4096
    else:
        assert max_range_len(ids, off, U, 3072) > 6144 >= max_range_len(ids, off, U, 2048) > 4096
    ref = oracle.all_pairs(ids, off)
    cabi.jas_timing_report()
    cabi.jas_timing_enable(True)
    try:
        res, st = gpu_all_pairs(ids, off, U)
    finally:
        rep = cabi.jas_timing_report()
        cabi.jas_timing_enable(False)
    assert_matches(res, ref)
    assert rep["range_starts"][0] == tries and "host:classify_fallback" not in rep
    assert ("local_cls_wide" if U == 36 else "local_cls") in rep


@pytest.mark.parametrize("case", ["uniform", "uniform_u24", "narrow_ids"])
def test_query_index_on_both_classification_paths(case):
    """With JAS_KEEP_IDS the distinct keys form the query index, whether the
    ranges were finished in LDS (keys held in 64 or in 32 bits there) or the
    full sort had to run."""
    rng = np.random.default_rng(7)
    if case.startswith("uniform"):
        U, n = (36, 70) if case == "uniform" else (24, 70)
        core = rng.integers(0, 1 << U, 3000, dtype=np.uint64)
        sets = [np.concatenate([rng.choice(core, int(rng.integers(0, 2500))),
                                rng.integers(0, 1 << U, int(rng.integers(0, 2500)), dtype=np.uint64)])
                for _ in range(n)]
    else:
        U, n = 40, 60
        sets = [rng.choice(1 << 12, int(rng.integers(500, 2500)), replace=False).astype(np.uint64)
                for _ in range(n)]
    ids, off = csr(sets)
    cabi.jas_timing_report()
    cabi.jas_timing_enable(True)
    try:
        db, st = jas.encode(dev(ids), dev(off), universe_bits=U, keep_ids=True)
        torch.cuda.synchronize()
    finally:
        names = set(cabi.jas_timing_report())
        cabi.jas_timing_enable(False)
    assert ("host:classify_fallback" in names) == (case == "narrow_ids")
    assert ("local_cls_wide" in names) == (case == "uniform")
    qsets = [sets[3], sets[11][::2], np.concatenate([sets[20][:50], np.array([(1 << U) - 1], np.uint64)])]
    qi, qo = csr(qsets)
    out = jas.query(db, dev(qi), dev(qo))
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    db.close()
    ref = oracle.cross(qi, qo, ids, off)
    assert np.array_equal(res["q_card"], ref["q_card"])
    assert np.array_equal(res["B"], ref["inter"])
    assert np.array_equal(res["J"].view(np.uint64), ref["J"].view(np.uint64))


def test_pack_long_and_short_rows():
    """Word rows whose 64 rows hold 64 samples or more on average are packed a
    row per wave, the others an entry per thread; both must give the oracle."""
    rng = np.random.default_rng(21)
    n = 200
    core = rng.choice(1 << 30, 700, replace=False).astype(np.uint64)  # rows of degree ~150-200
    sets = [np.concatenate([rng.choice(core, int(rng.integers(500, 700)), replace=False),
                            rng.integers(0, 1 << 30, int(rng.integers(0, 400)), dtype=np.uint64)])
            for _ in range(n)]
    ids, off = csr(sets)
    ref = oracle.all_pairs(ids, off)
    for dmin in (2, 100):
        res, st = gpu_all_pairs(ids, off, 30, 0, dmin)
        assert st["n_packed_rows"] > 0
        assert_matches(res, ref)


@pytest.mark.parametrize("n,dmin", [(300, 1000), (10300, 0)])
def test_row_lists_by_sample_and_by_row(n, dmin):
    """Rows kept as lists are summed sample by sample (their pairs sorted by the
    smaller sample, an LDS row of counters per sample, up to 10240 samples; long
    and short runs of one sample take different flushes) or, for more samples,
    pair by pair per row."""
    rng = np.random.default_rng(n)
    pool = rng.choice(1 << 20, 3000, replace=False).astype(np.uint64)
    sets = [np.unique(rng.choice(pool, int(rng.integers(0, 7)))) for _ in range(n)]
    sets[5] = pool[:40].copy()  # one sample in many rows
    sets[0] = pool[:2500].copy()  # a long run of pairs (0, b): counted without a touched list
    ids, off = csr(sets)
    ref = oracle.all_pairs(ids, off)
    res, st = gpu_all_pairs(ids, off, 20, 0, dmin)
    assert st["n_list_rows"] > 0
    assert_matches(res, ref)
    res, _ = gpu_all_pairs(ids, off, 20, 0, dmin, upper=True)
    assert_matches(res, ref, upper=True)


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 255, 257])
@pytest.mark.parametrize("path", ["popcount", "mfma"])
def test_tile_edges(n, path):
    flags = cabi.JAS_FORCE_POPCOUNT if path == "popcount" else cabi.JAS_FORCE_MFMA
    rng = np.random.default_rng(n)
    core = rng.choice(1 << 20, 3000, replace=False).astype(np.uint64)
    sets = [np.concatenate([rng.choice(core, int(rng.integers(0, 2000)), replace=False),
                            rng.integers(0, 1 << 20, int(rng.integers(0, 300))).astype(np.uint64)])
            for _ in range(n)]
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([s.size for s in sets])
    ids = np.concatenate(sets) if n else np.zeros(0, np.uint64)
    ref = oracle.all_pairs(ids, off)
    res, _ = gpu_all_pairs(ids, off, 20, 12, 0, flags=flags)
    assert_matches(res, ref)
    res, _ = gpu_all_pairs(ids, off, 20, 0, 0, upper=True, flags=flags)
    assert_matches(res, ref, upper=True)


def test_all_sets_empty():
    off = np.zeros(6, np.uint64)
    ids = np.zeros(0, np.uint64)
    db, st = jas.encode(dev(np.zeros(1, np.uint64))[:0], dev(off), universe_bits=16)
    out = jas.gram(db)
    torch.cuda.synchronize()
    assert st["n_pairs"] == 0
    assert np.all(out["B"].cpu().numpy() == 0)
    assert np.all(out["J"].cpu().numpy() == 1.0)
    assert np.all(out["den"].cpu().numpy() == 0)
    db.close()
    ref = oracle.all_pairs(ids, off)
    assert np.all(ref["J"] == 1.0)


def test_zero_sets():
    db, st = jas.encode(dev(np.zeros(1, np.uint64))[:0], dev(np.zeros(1, np.uint64)), universe_bits=16)
    assert db.n == 0
    out = jas.gram(db)
    assert out["B"].numel() == 0
    db.close()


@pytest.mark.parametrize("U,n", [(63, 2), (62, 3), (1, 3), (2, 5), (40, 1024)])
def test_universe_extremes(U, n):
    rng = np.random.default_rng(U * 1000 + n)
    top = (1 << U) - 1
    base = np.array([top, top - 1, 0, top // 2, top // 3], dtype=np.uint64)[: min(5, 1 << U)]
    sets = [np.unique(np.concatenate([rng.choice(base, int(rng.integers(0, base.size + 1))),
                                      rng.integers(0, top, 3, dtype=np.uint64, endpoint=True)]))
            for _ in range(n)]
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([s.size for s in sets])
    ids = np.concatenate(sets)
    ref = oracle.all_pairs(ids, off)
    res, _ = gpu_all_pairs(ids, off, U, 0, 0)
    assert_matches(res, ref)


def test_id_outside_universe_is_rejected():
    ids = np.array([1, 2, 1 << 20], dtype=np.uint64)
    with pytest.raises(jas.JasError) as e:
        jas.encode(dev(ids), dev(np.array([0, 3], np.uint64)), universe_bits=20)
    assert e.value.status == cabi.JAS_EINVAL


def test_budget_is_enforced():
    spec = synth.workload("tiny")
    ids, off = synth.generate(spec)
    with pytest.raises(jas.JasError) as e:
        jas.encode(dev(ids), dev(off), universe_bits=24, hbm_budget_bytes=1 << 20)
    assert e.value.status == cabi.JAS_ENOMEM


def test_host_pointers_match_device_path(tiny):
    spec, ids, off, ref = tiny
    opts = cabi.jas_encode_opts(24, 16, 0, cabi.JAS_HOST_PTRS, 0)
    db, st = cabi.jas_encode(ids, off, 32, opts)
    B = np.empty((32, 32), np.int32)
    card = np.empty(32, np.int64)
    den = np.empty((32, 32), np.int64)
    J = np.empty((32, 32), np.float64)
    cabi.jas_gram(db, cabi.JAS_HOST_PTRS, None, B, card, den, J)
    db.close()
    assert_matches({"B": B, "card": card, "den": den, "J": J}, ref)


@pytest.mark.parametrize("name", ["precision", "paperlike"])
def test_mfma_equals_popcount_on_dense_tiles(name):
    spec = synth.scaled(synth.workload(name), n=384, size_scale=0.01, pool_scale=0.01)
    ids, off = synth.generate(spec)
    db, st = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, batch_bits=synth.BATCH_BITS[name])
    a = jas.gram(db, flags=cabi.JAS_FORCE_POPCOUNT)
    b = jas.gram(db, flags=cabi.JAS_FORCE_MFMA)
    c = jas.gram(db)
    torch.cuda.synchronize()
    assert st["n_word_rows"] > 0
    assert torch.equal(a["B"], b["B"]) and torch.equal(a["B"], c["B"])
    assert torch.equal(a["J"], b["J"])
    db.close()
    ref = oracle.all_pairs(ids, off)
    assert_matches({k: v.cpu().numpy() for k, v in b.items()}, ref)


def test_gram_autotuner_keeps_results_exact():
    spec = synth.scaled(synth.workload("precision"), n=300, size_scale=0.01, pool_scale=0.01)
    ids, off = synth.generate(spec)
    db, st = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, dense_min_degree=2)
    assert st["n_word_rows"] > 0
    plain = jas.gram(db, upper=True)
    tuned = jas.gram(db, upper=True, flags=cabi.JAS_TUNE)    # times every tile variant, then runs the fastest
    again = jas.gram(db, upper=True)                          # the kept choice
    torch.cuda.synchronize()
    for k in ("B", "den", "J", "card"):
        assert torch.equal(plain[k], tuned[k]) and torch.equal(plain[k], again[k]), k
    db.close()
    ref = oracle.all_pairs(ids, off)
    assert_matches({k: v.cpu().numpy() for k, v in tuned.items()}, ref, upper=True)


@pytest.mark.parametrize("n", [130, 300, 513])
def test_every_mfma_tile_variant_is_exact(n):
    """Each MFMA tile variant (128 x 128 and 256 x 256 tiles, word rows per
    step, K split) gives the oracle's B, C and J, with ragged column tiles."""
    spec = synth.scaled(synth.workload("precision"), n=n, size_scale=0.01, pool_scale=0.01)
    ids, off = synth.generate(spec)
    db, st = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, dense_min_degree=2)
    assert st["n_word_rows"] > 0
    ref = oracle.all_pairs(ids, off)
    nv = cabi.jas_gram_variants()
    assert nv >= 2
    for v in range(nv):
        for upper in (False, True):
            out = jas.gram(db, upper=upper, flags=cabi.JAS_GRAM_VARIANT(v))
            torch.cuda.synchronize()
            assert_matches({k: x.cpu().numpy() for k, x in out.items()}, ref, upper=upper)
    with pytest.raises(cabi.JasError):
        jas.gram(db, flags=cabi.JAS_GRAM_VARIANT(nv))
    db.close()


def test_repeat_runs_are_identical():
    spec = synth.scaled(synth.workload("precision"), n=300, size_scale=0.01, pool_scale=0.01)
    ids, off = synth.generate(spec)
    db, _ = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, dense_min_degree=4)
    a = jas.gram(db)["B"].cpu().numpy()
    b = jas.gram(db)["B"].cpu().numpy()
    c = jas.gram(db, flags=cabi.JAS_FORCE_POPCOUNT)["B"].cpu().numpy()
    assert np.array_equal(a, c)
    db.close()
    assert np.array_equal(a, b)


# --- query path -------------------------------------------------------------
@pytest.mark.parametrize("query_only", [False, True])
def test_query_matches_oracle(query_only):
    """A query against every database set; with JAS_QUERY_ONLY the db holds only the
    query index (less device memory, the same answers) and jas_gram refuses it."""
    spec = synth.scaled(synth.workload("serving_db"), n=150, size_scale=0.01, pool_scale=0.005)
    ids, off = synth.generate(spec)
    db, st = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, batch_bits=26, keep_ids=True,
                        dense_min_degree=5, query_only=query_only)
    if query_only:
        full, st_full = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, batch_bits=26,
                                   keep_ids=True, dense_min_degree=5)
        assert st["device_bytes"] < st_full["device_bytes"]
        assert st["n_packed_rows"] == 0 and st["n_list_rows"] == 0 and st["n_pairs"] == st_full["n_pairs"]
        full.close()
        with pytest.raises(cabi.JasError) as e:
            jas.gram(db)
        assert e.value.status == cabi.JAS_EINVAL
    qspec = synth.scaled(synth.query_spec(spec, 0, 9), size_scale=0.01)
    qi, qo = synth.generate(qspec)
    # add DB sets 0 and 7, an empty set, and a set with repeats and IDs absent from the DB
    extra = [ids[int(off[0]):int(off[1])], ids[int(off[7]):int(off[8])], np.zeros(0, np.uint64),
             np.array([5, 5, 5, (1 << 36) - 1, 123456789], np.uint64)]
    sets = [qi[int(qo[i]):int(qo[i + 1])] for i in range(9)] + extra
    qoff = np.zeros(len(sets) + 1, np.uint64)
    qoff[1:] = np.cumsum([s.size for s in sets])
    qids = np.concatenate(sets)
    ref = oracle.cross(qids, qoff, ids, off)
    out = jas.query(db, dev(qids), dev(qoff))
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    db.close()
    assert np.array_equal(res["q_card"], ref["q_card"])
    assert np.array_equal(res["B"], ref["inter"])
    assert np.array_equal(res["den"], ref["union"])
    assert np.array_equal(res["J"].view(np.uint64), ref["J"].view(np.uint64))


def test_query_row_equals_gram_row():
    spec = synth.scaled(synth.workload("batching"), n=120, size_scale=0.004, pool_scale=0.004)
    ids, off = synth.generate(spec)
    db, _ = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, batch_bits=26, keep_ids=True)
    g = jas.gram(db)
    rows = [3, 50, 119]
    qs = [ids[int(off[i]):int(off[i + 1])] for i in rows]
    qoff = np.zeros(4, np.uint64)
    qoff[1:] = np.cumsum([s.size for s in qs])
    out = jas.query(db, dev(np.concatenate(qs)), dev(qoff))
    torch.cuda.synchronize()
    assert torch.equal(out["B"], g["B"][rows])
    assert torch.equal(out["J"], g["J"][rows])
    db.close()


def test_query_requires_index_and_rejects_bad_ids():
    spec = synth.workload("tiny")
    ids, off = synth.generate(spec)
    db, _ = jas.encode(dev(ids), dev(off), universe_bits=24)
    with pytest.raises(jas.JasError):
        jas.query(db, dev(ids[:10]), dev(np.array([0, 10], np.uint64)))
    db.close()
    db, _ = jas.encode(dev(ids), dev(off), universe_bits=24, keep_ids=True)
    with pytest.raises(jas.JasError) as e:
        jas.query(db, dev(np.array([1 << 24], np.uint64)), dev(np.array([0, 1], np.uint64)))
    assert e.value.status == cabi.JAS_EINVAL
    db.close()


def test_gram_captured_in_a_graph_replays_exactly():
    spec = synth.scaled(synth.workload("paperlike"), n=200, size_scale=0.004, pool_scale=0.004)
    ids, off = synth.generate(spec)
    db, st = jas.encode(dev(ids), dev(off), universe_bits=spec.universe_bits, batch_bits=26, dense_min_degree=4)
    assert st["n_list_rows"] > 0 and st["n_packed_rows"] > 0
    eager = jas.gram(db)
    torch.cuda.synchronize()
    n = spec.n
    B = torch.full((n, n), -7, dtype=torch.int32, device="cuda")
    card = torch.empty(n, dtype=torch.int64, device="cuda")
    den = torch.empty((n, n), dtype=torch.int64, device="cuda")
    J = torch.empty((n, n), dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        cabi.jas_gram(db, 0, side, B, card, den, J)  # warm the path outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        cabi.jas_gram(db, 0, torch.cuda.current_stream(), B, card, den, J)
    for rep in range(3):
        B.fill_(-1)
        J.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(B, eager["B"]), f"replay {rep}"
        assert torch.equal(J, eager["J"]) and torch.equal(den, eager["den"]) and torch.equal(card, eager["card"])
        _ = (eager["B"].float() * 2).sum().item()  # eager work between replays
    db.close()
