"""Full-size workloads on the GPU, in the configuration bench.py times.

The oracle cannot run all pairs at these sizes inside a test, so a committed
CPU-only script (tests/golden/make_fullsize_digests.py, which calls nothing
but the oracle and the generator) has run it once and stored, per workload,
the digest of the generated input and one digest of every output row of B,
C and J (tests/digests.py).  Each test here
  - regenerates the input and checks its digest first (a generator that drew
    something else is reported as such, not as a wrong result);
  - computes the whole result on the GPU and compares the digest of every
    row; at the first row that differs it recomputes that row with the
    oracle and names the first differing entry.
Where no digest file exists (the p = 1e-2 Bernoulli matrix, resident and
streamed), sampled pairs are recomputed by the oracle one by one, and two
identities that hold at any size are checked over the whole result: the
row sums of B equal sum over k in X_i of deg_k (B 1 = A^T (A 1)), with the
row degrees deg_k counted on the host, and 1^T B 1 = sum_k deg_k^2.
"""
import os

import numpy as np
import pytest

import digests
import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_1911_04200_amd import jas as cabi  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_fullsize_digests.py {name})")
    return digests.read_golden(path)


def resident(spec, with_digest=False):
    """Generate the whole collection into pinned memory and copy it to the GPU."""
    off = synth.offsets(spec)
    N = int(off[-1])
    host = torch.empty(N, dtype=torch.int64, pin_memory=True)
    ids = host.numpy().view(np.uint64)
    synth.generate(spec, out=ids)
    dig = digests.input_digest(ids, off) if with_digest else None
    ids_d = host.cuda()
    off_d = torch.from_numpy(off.view(np.int64)).cuda()
    torch.cuda.synchronize()
    del host, ids
    return ids_d, off_d, off, dig


def all_pairs_on_gpu(spec, name, upper, with_digest):
    n = spec.n
    ids_d, off_d, off, dig = resident(spec, with_digest)
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS[name], 0, 0, 0)
    db, st = cabi.jas_encode(ids_d, off_d, n, opts, None)
    del ids_d
    length = n * (n + 1) // 2 if upper else n * n
    out = {"B": torch.empty(length, dtype=torch.int32, device="cuda"),
           "card": torch.empty(n, dtype=torch.int64, device="cuda"),
           "den": torch.empty(length, dtype=torch.int64, device="cuda"),
           "J": torch.empty(length, dtype=torch.float64, device="cuda")}
    cabi.jas_gram(db, cabi.JAS_UPPER if upper else 0, None, out["B"], out["card"], out["den"], out["J"])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    del out
    assert st["n_ids"] == int(off[-1])
    return db, res, off, dig


def oracle_row(spec, i, cols=None):
    """Row i (against every set, or the listed ones) recomputed by the oracle."""
    n = spec.n
    cols = np.arange(n) if cols is None else np.asarray(cols)
    qi, qo = synth.generate_samples(spec, [i])
    xs, xo = synth.generate_samples(spec, cols)
    r = oracle.cross(qi, qo, xs, xo)
    return r["inter"][0], r["union"][0], r["J"][0]


def compare_rows(spec, res, gold, upper):
    """Every row's digest against the stored one; explain the first mismatch."""
    n = spec.n
    got = digests.row_digests(res["B"], res["den"], res["J"], n, upper)
    bad = [i for i in range(n) if got[i] != gold["rows"][i]]
    if not bad:
        return
    i = bad[0]
    sl = digests.upper_row(i, n) if upper else slice(i * n, (i + 1) * n)
    cols = np.arange(i, n) if upper else np.arange(n)
    wi, wu, wj = oracle_row(spec, i, cols)
    gb, gc, gj = res["B"][sl], res["den"][sl], res["J"][sl]
    diff = np.flatnonzero((gb != wi) | (gc != wu) | (gj.view(np.uint64) != wj.view(np.uint64)))
    detail = (f"first at column {cols[diff[0]]}: B {gb[diff[0]]} vs {wi[diff[0]]}, C {gc[diff[0]]} vs {wu[diff[0]]}, "
              f"J {gj[diff[0]]!r} vs {wj[diff[0]]!r}" if diff.size else "the oracle row matches (digest file stale?)")
    pytest.fail(f"{len(bad)} of {n} rows differ from the oracle's digests; row {i}: {diff.size} entries differ, {detail}")


def self_check(res, n, upper):
    """What the result must satisfy by construction (C is formed from B and
    |X_i|, the lower triangle mirrors the upper one); a self-check of the
    epilogue, not a parity check."""
    B, C, J, card = res["B"], res["den"], res["J"], res["card"]
    if upper:
        i, j = np.triu_indices(n)
    else:
        B2, C2, J2 = B.reshape(n, n), C.reshape(n, n), J.reshape(n, n)
        assert np.array_equal(B2, B2.T) and np.array_equal(C2, C2.T) and np.array_equal(J2, J2.T)
        i, j = np.indices((n, n))
        i, j = i.ravel(), j.ravel()
    ci, cj = card[i], card[j]
    assert np.all(B >= 0) and np.all(B <= np.minimum(ci, cj))
    assert np.array_equal(C, ci + cj - B)
    assert np.all((J >= 0) & (J <= 1))
    d = i == j
    assert np.array_equal(B[d], ci[d]) and np.all(J[d] == 1.0)


def full_matrix(B, n, upper):
    if not upper:
        return B.reshape(n, n).astype(np.int64)
    M = np.zeros((n, n), dtype=np.int64)
    M[np.triu_indices(n)] = B
    return M + M.T - np.diag(np.diag(M))


def check_row_sums(ids, off, B, n, upper, rows):
    """B 1 = A^T (A 1) and 1^T B 1 = sum_k deg_k^2, deg_k counted on the host
    (the IDs are row indices below `rows`, each set without repeats)."""
    deg = np.zeros(rows, dtype=np.int64)
    step = 1 << 27
    for a in range(0, ids.size, step):
        deg += np.bincount(ids[a:a + step].astype(np.int64), minlength=rows)
    want = np.array([int(deg[ids[int(off[i]):int(off[i + 1])]].sum()) for i in range(n)], dtype=np.int64)
    M = full_matrix(B, n, upper)
    got = M.sum(axis=1)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"row sums differ at rows {bad[:5].tolist()}: {got[bad[:5]]} vs {want[bad[:5]]}"
    assert int(M.sum()) == int((deg * deg).sum())


def sample_pairs(n, sizes, rng, k=40):
    big = list(np.argsort(sizes)[-3:])
    small = list(np.argsort(sizes)[:2])
    pts = set(int(x) for x in big + small)
    while len(pts) < 14:
        pts.add(int(rng.integers(0, n)))
    pts = sorted(pts)
    pairs = [(a, a) for a in pts[:4]]
    while len(pairs) < k:
        a, b = rng.choice(pts, 2, replace=False)
        pairs.append((int(min(a, b)), int(max(a, b))))
    return pts, pairs


def check_sampled(spec, res, pts, pairs, upper):
    n = spec.n
    ids, off = synth.generate_samples(spec, pts)
    s, so = oracle.normalize(ids, off)
    loc = {p: k for k, p in enumerate(pts)}
    qi = np.array([loc[a] for a, _ in pairs])
    xi = np.array([loc[b] for _, b in pairs])
    inter, uni, jac = oracle.pairs_normalized(s, so, s, so, qi, xi)
    for k, (a, b) in enumerate(pairs):
        pos = a * n - a * (a - 1) // 2 + (b - a) if upper else a * n + b
        assert res["B"][pos] == inter[k], f"B[{a},{b}]"
        assert res["den"][pos] == uni[k], f"C[{a},{b}]"
        assert res["J"][pos].view(np.uint64) == jac[k].view(np.uint64), f"J[{a},{b}]"
    assert np.array_equal(res["card"][pts], np.diff(so.astype(np.int64)))


def check_bernoulli_means(res, spec, upper):
    """Entries 1 with probability p, independently: off the diagonal B_ij has
    mean m p^2 and J_ij about p / (2 - p); the sample sizes have mean m p."""
    n, m, p = spec.n, spec.rows, spec.density
    if upper:
        i, j = np.triu_indices(n)
        off_diag = i != j
        B, J = res["B"][off_diag], res["J"][off_diag]
    else:
        mask = ~np.eye(n, dtype=bool)
        B, J = res["B"].reshape(n, n)[mask], res["J"].reshape(n, n)[mask]
    assert abs(res["card"].mean() / (m * p) - 1) < 1e-3
    assert abs(B.mean() / (m * p * p) - 1) < 5e-3
    assert abs(J.mean() / (p / (2 - p)) - 1) < 5e-3


@pytest.mark.parametrize("name,upper", [("paperlike", False), ("precision", False), ("batching", True),
                                        ("bernoulli_p1e-3", True), ("graph_s13_ef64", False)])
def test_full_size_every_row_matches_the_oracle(name, upper):
    gold = golden(name)
    spec = synth.workload(name)
    n = spec.n
    assert int(gold["n"]) == n and gold["layout"] == ("upper" if upper else "full")
    db, res, off, dig = all_pairs_on_gpu(spec, name, upper, with_digest=True)
    assert dig == gold["input"], "the generator drew a different input than the one the digests were made from"
    compare_rows(spec, res, gold, upper)
    self_check(res, n, upper)
    B = res["B"].astype(np.int64)
    upper_sum = B.sum() if upper else (B.sum() + B[np.arange(n) * (n + 1)].sum()) // 2
    assert int(upper_sum) == int(gold["sum_B_upper"])
    # the popcount path gives the same bytes as the MFMA path on this db
    if not upper:
        B2 = torch.empty(n * n, dtype=torch.int32, device="cuda")
        cabi.jas_gram(db, cabi.JAS_FORCE_POPCOUNT, None, B2, None, None, None)
        torch.cuda.synchronize()
        assert np.array_equal(B2.cpu().numpy(), res["B"])
    db.close()
    cabi.jas_trim()


def test_full_size_bernoulli_p1e2_identities_and_samples():
    """The p = 1e-2 matrix (3.36e9 IDs, every row in one batch): the row-sum
    identities over the whole result, sampled pairs against the oracle, the
    self-check and the means the model fixes."""
    name = "bernoulli_p1e-2"
    spec = synth.workload(name)
    n = spec.n
    db, res, off, _ = all_pairs_on_gpu(spec, name, True, with_digest=False)
    db.close()
    cabi.jas_trim()
    ids, off = synth.generate(spec)
    check_row_sums(ids, off, res["B"], n, True, spec.rows)
    del ids
    pts, pairs = sample_pairs(n, np.diff(off.astype(np.int64)), np.random.default_rng(11))
    check_sampled(spec, res, pts, pairs, True)
    self_check(res, n, True)
    check_bernoulli_means(res, spec, True)


def test_full_size_serving_requests_match_the_oracle():
    """32 seeded requests (1-64 query sets each) against the whole 8192-set
    database: every query row's digest against the oracle's."""
    gold = golden("serving")
    spec = synth.workload("serving_db")
    n = spec.n
    ids_d, off_d, off, dig = resident(spec, with_digest=True)
    assert dig == gold["input"], "the generator drew a different database than the one the digests were made from"
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS["serving_db"], 0, cabi.JAS_KEEP_IDS, 0)
    db, st = cabi.jas_encode(ids_d, off_d, n, opts, None)
    del ids_d
    torch.cuda.synchronize()
    assert len(gold["requests"]) >= 32
    for req in gold["requests"]:
        r, nq = req["request"], req["nq"]
        qi, qo = synth.generate(synth.query_spec(spec, r, nq))
        assert digests.input_digest(qi, qo) == req["input"], f"request {r}: a different query input"
        B = torch.empty((nq, n), dtype=torch.int32, device="cuda")
        qc = torch.empty(nq, dtype=torch.int64, device="cuda")
        den = torch.empty((nq, n), dtype=torch.int64, device="cuda")
        J = torch.empty((nq, n), dtype=torch.float64, device="cuda")
        cabi.jas_query(db, torch.from_numpy(qi.view(np.int64)).cuda(), torch.from_numpy(qo.view(np.int64)).cuda(),
                       nq, 0, None, B, qc, den, J)
        torch.cuda.synchronize()
        Bh, qch, dh, Jh = B.cpu().numpy(), qc.cpu().numpy(), den.cpu().numpy(), J.cpu().numpy()
        assert int(qch.sum()) == req["q_card_sum"], f"request {r}: |Q| differs"
        got = [digests.row_digest(Bh[q], dh[q], Jh[q]) for q in range(nq)]
        bad = [q for q in range(nq) if got[q] != req["rows"][q]]
        if bad:
            q = bad[0]
            xs, xo = synth.generate_samples(spec, np.arange(n))
            ref = oracle.cross(qi[int(qo[q]):int(qo[q + 1])], np.array([0, qo[q + 1] - qo[q]], np.uint64), xs, xo)
            d = np.flatnonzero(Bh[q] != ref["inter"][0])
            pytest.fail(f"request {r}: {len(bad)} of {nq} query rows differ; row {q}: B differs at columns "
                        f"{d[:5].tolist()}")
    db.close()
    cabi.jas_trim()


def test_full_size_streamed_bernoulli():
    """The p = 1e-2 matrix (3.36e9 IDs) streamed from host memory in 8 parts of
    2^22 rows: the row-sum identities, sampled pairs against the oracle, the
    self-check and the model means."""
    from paper_1911_04200_amd import stream
    spec = synth.workload("bernoulli_p1e-2")
    n = spec.n
    ids, off = synth.generate(spec)
    res = stream.all_pairs_streamed(ids, off, spec.universe_bits, 3, upper=True, check_sorted=False)
    torch.cuda.synchronize()
    out = {k: res[k].cpu().numpy() for k in ("B", "card", "den", "J")}
    assert res["n_parts"] == 8 and sum(s["n_ids"] for s in res["parts"]) == ids.size
    # each part's device footprint is about an eighth of the resident encoding's
    assert max(s["device_bytes"] for s in res["parts"]) < 40 << 30
    del res
    check_row_sums(ids, off, out["B"], n, True, spec.rows)
    del ids
    sizes = np.diff(off.astype(np.int64))
    pts, pairs = sample_pairs(n, sizes, np.random.default_rng(3))
    check_sampled(spec, out, pts, pairs, True)
    self_check(out, n, True)
    check_bernoulli_means(out, spec, True)


def test_full_size_graph_link_prediction():
    """Neighbourhoods of the 2^20 vertices of a scale-20 R-MAT graph as the
    database; queries are some vertices' neighbourhoods, with and without an
    added edge: every column's bounds, sampled columns against the oracle."""
    g = synth.workload("graph_s20_ef16")
    n = g.n
    ids_d, off_d, off, _ = resident(g)
    opts = cabi.jas_encode_opts(g.universe_bits, synth.BATCH_BITS["graph_s20_ef16"], 0, cabi.JAS_KEEP_IDS, 0)
    db, st = cabi.jas_encode(ids_d, off_d, n, opts, None)
    del ids_d
    rng = np.random.default_rng(9)
    deg = np.diff(off.astype(np.int64))
    verts = [int(np.argmax(deg))] + [int(v) for v in rng.choice(np.flatnonzero(deg > 0), 14, replace=False)]
    qs = [g.ids[int(off[v]):int(off[v + 1])] for v in verts]
    qs.append(np.union1d(qs[1], rng.choice(n, 3, replace=False).astype(np.uint64)))
    qo = np.zeros(len(qs) + 1, np.uint64)
    qo[1:] = np.cumsum([q.size for q in qs])
    qi = np.concatenate(qs).astype(np.uint64)
    nq = len(qs)
    B = torch.empty((nq, n), dtype=torch.int32, device="cuda")
    qc = torch.empty(nq, dtype=torch.int64, device="cuda")
    den = torch.empty((nq, n), dtype=torch.int64, device="cuda")
    J = torch.empty((nq, n), dtype=torch.float64, device="cuda")
    cabi.jas_query(db, torch.from_numpy(qi.view(np.int64)).cuda(), torch.from_numpy(qo.view(np.int64)).cuda(), nq,
                   0, None, B, qc, den, J)
    torch.cuda.synchronize()
    B, qc, den, J = B.cpu().numpy(), qc.cpu().numpy(), den.cpu().numpy(), J.cpu().numpy()
    db.close()
    cabi.jas_trim()
    cols = np.unique(np.concatenate([np.array(verts), rng.choice(n, 40, replace=False)]))
    xs, xo = synth.generate_samples(g, cols)
    ref = oracle.cross(qi, qo, xs, xo)
    assert np.array_equal(qc, ref["q_card"])
    assert np.array_equal(B[:, cols], ref["inter"])
    assert np.array_equal(den[:, cols], ref["union"])
    assert np.array_equal(J[:, cols].view(np.uint64), ref["J"].view(np.uint64))
    # a vertex's own neighbourhood: J = 1 with its own column
    for k, v in enumerate(verts):
        assert J[k, v] == 1.0
    assert np.all(B >= 0) and np.all(B <= qc[:, None]) and np.all(B <= deg[None, :])
    assert np.all((J >= 0) & (J <= 1))
    # B 1 = A^T (A 1) over every column, degrees from the host's copy of the graph
    vdeg = np.bincount(g.ids.astype(np.int64), minlength=n)
    want = np.array([int(vdeg[qi[int(qo[k]):int(qo[k + 1])]].sum()) for k in range(nq)])
    assert np.array_equal(B.astype(np.int64).sum(axis=1), want)
