"""Full-size workloads on the GPU, in the configuration bench.py times.

The oracle cannot do all pairs at these sizes, so each test checks
  - sampled pairs (i, j), recomputed one by one by the oracle from the same
    seeded sets (regenerated on the host), bit for bit: B, the union and J;
  - properties of the whole result that hold at any size: symmetry,
    B_ii = |X_i|, 0 <= B_ij <= min(|X_i|, |X_j|), C_ij = |X_i| + |X_j| - B_ij,
    J in [0, 1], J_ii = 1.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_1911_04200_amd import jas as cabi  # noqa: E402


def resident(spec):
    """Generate the whole collection into pinned memory and copy it to the GPU."""
    off = synth.offsets(spec)
    N = int(off[-1])
    host = torch.empty(N, dtype=torch.int64, pin_memory=True)
    synth.generate(spec, out=host.numpy().view(np.uint64))
    ids_d = host.cuda()
    off_d = torch.from_numpy(off.view(np.int64)).cuda()
    torch.cuda.synchronize()
    del host
    return ids_d, off_d, off


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
    card = res["card"]
    for k, (a, b) in enumerate(pairs):
        pos = a * n - a * (a - 1) // 2 + (b - a) if upper else a * n + b
        assert res["B"][pos] == inter[k], f"B[{a},{b}]"
        assert res["den"][pos] == uni[k], f"C[{a},{b}]"
        assert res["J"][pos].view(np.uint64) == jac[k].view(np.uint64), f"J[{a},{b}]"
    assert np.array_equal(card[pts], np.diff(so.astype(np.int64)))


def check_properties(res, n, upper):
    B, C, J, card = res["B"], res["den"], res["J"], res["card"]
    if upper:
        i, j = np.triu_indices(n)
    else:
        B, C, J = B.reshape(n, n), C.reshape(n, n), J.reshape(n, n)
        assert np.array_equal(B, B.T) and np.array_equal(C, C.T) and np.array_equal(J, J.T)
        i, j = np.indices((n, n))
        i, j = i.ravel(), j.ravel()
        B, C, J = B.ravel(), C.ravel(), J.ravel()
    ci, cj = card[i], card[j]
    assert np.all(B >= 0) and np.all(B <= np.minimum(ci, cj))
    assert np.array_equal(C, ci + cj - B)
    assert np.all((J >= 0) & (J <= 1))
    d = i == j
    assert np.array_equal(B[d], ci[d]) and np.all(J[d] == 1.0)


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
                                        ("bernoulli_p1e-3", True), ("bernoulli_p1e-2", True),
                                        ("graph_s13_ef64", False)])
def test_full_size_all_pairs(name, upper):
    spec = synth.workload(name)
    n = spec.n
    ids_d, off_d, off = resident(spec)
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS[name], 0, 0, 0)
    db, st = cabi.jas_encode(ids_d, off_d, n, opts, None)
    del ids_d
    length = n * (n + 1) // 2 if upper else n * n
    out = {"B": torch.empty(length, dtype=torch.int32, device="cuda"),
           "card": torch.empty(n, dtype=torch.int64, device="cuda"),
           "den": torch.empty(length, dtype=torch.int64, device="cuda"),
           "J": torch.empty(length, dtype=torch.float64, device="cuda")}
    flags = cabi.JAS_UPPER if upper else 0
    cabi.jas_gram(db, flags, None, out["B"], out["card"], out["den"], out["J"])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    del out
    assert st["n_ids"] == int(off[-1])
    sizes = np.diff(off.astype(np.int64))
    rng = np.random.default_rng(11)
    pts, pairs = sample_pairs(n, sizes, rng)
    check_sampled(spec, res, pts, pairs, upper)
    check_properties(res, n, upper)
    if spec.size_kind == 2:
        check_bernoulli_means(res, spec, upper)
    # the popcount path gives the same bytes as the MFMA path on this db
    if not upper:
        B2 = torch.empty(length, dtype=torch.int32, device="cuda")
        cabi.jas_gram(db, cabi.JAS_FORCE_POPCOUNT, None, B2, None, None, None)
        torch.cuda.synchronize()
        assert np.array_equal(B2.cpu().numpy(), res["B"])
    db.close()
    cabi.jas_trim()


def test_full_size_serving_queries():
    spec = synth.workload("serving_db")
    n = spec.n
    ids_d, off_d, off = resident(spec)
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS["serving_db"], 0, cabi.JAS_KEEP_IDS, 0)
    db, st = cabi.jas_encode(ids_d, off_d, n, opts, None)
    del ids_d
    torch.cuda.synchronize()
    q = synth.query_spec(spec, 3, 12)
    qi, qo = synth.generate(q)
    nq = q.n
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
    rng = np.random.default_rng(5)
    cols = np.sort(rng.choice(n, 24, replace=False))
    xs, xo = synth.generate_samples(spec, cols)
    ref = oracle.cross(qi, qo, xs, xo)
    assert np.array_equal(qc, ref["q_card"])
    assert np.array_equal(B[:, cols], ref["inter"])
    assert np.array_equal(den[:, cols], ref["union"])
    assert np.array_equal(J[:, cols].view(np.uint64), ref["J"].view(np.uint64))
    # any size: bounds and the union identity over every column
    assert np.all(B >= 0) and np.all(B <= qc[:, None])
    assert np.all((J >= 0) & (J <= 1))


def test_full_size_streamed_bernoulli():
    """The p = 1e-2 matrix (3.36e9 IDs) streamed from host memory in 8 parts of
    2^22 rows: sampled pairs against the oracle, properties and model means."""
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
    del res, ids
    sizes = np.diff(off.astype(np.int64))
    pts, pairs = sample_pairs(n, sizes, np.random.default_rng(3))
    check_sampled(spec, out, pts, pairs, True)
    check_properties(out, n, True)
    check_bernoulli_means(out, spec, True)


def test_full_size_graph_link_prediction():
    """Neighbourhoods of the 2^20 vertices of a scale-20 R-MAT graph as the
    database; queries are some vertices' neighbourhoods, with and without an
    added edge: every column's bounds, sampled columns against the oracle."""
    g = synth.workload("graph_s20_ef16")
    n = g.n
    ids_d, off_d, off = resident(g)
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
