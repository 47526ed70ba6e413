"""Row batches streamed from host memory (JAS_ACCUMULATE + jas_finalize) vs the oracle."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1911_04200_amd import jas as cabi  # noqa: E402
from paper_1911_04200_amd import stream  # noqa: E402


def host(res):
    return {k: res[k].cpu().numpy() for k in ("B", "card", "den", "J")}


def check(res, ref, upper):
    n = ref["card"].size
    assert np.array_equal(res["card"], ref["card"])
    if upper:
        iu = np.triu_indices(n)
        want = {"B": ref["inter"][iu], "den": ref["union"][iu], "J": ref["J"][iu]}
    else:
        want = {"B": ref["inter"].ravel(), "den": ref["union"].ravel(), "J": ref["J"].ravel()}
    bad = np.argwhere(res["B"] != want["B"])
    assert bad.size == 0, f"B differs at {bad[:5].tolist()}"
    assert np.array_equal(res["den"], want["den"])
    assert np.array_equal(res["J"].view(np.uint64), want["J"].view(np.uint64))


@pytest.mark.parametrize("part_bits", [0, 2, 5])
@pytest.mark.parametrize("upper", [False, True])
def test_streamed_bernoulli_matches_the_oracle(part_bits, upper):
    spec = synth.bernoulli(0.02, rows_log2=14, n=150, seed=7)
    ids, off = synth.generate(spec)
    ref = oracle.all_pairs(ids, off)
    res = stream.all_pairs_streamed(ids, off, 14, part_bits, batch_bits=12, upper=upper)
    torch.cuda.synchronize()
    assert res["n_parts"] == 1 << part_bits
    check(host(res), ref, upper)


def test_streamed_sorted_paperlike_sets_with_lists_and_packed_rows():
    spec = synth.scaled(synth.workload("paperlike"), n=200, size_scale=0.004, pool_scale=0.004)
    ids, off = synth.generate(spec)
    for i in range(spec.n):  # ascending within each set, as sorted k-mer files are
        ids[int(off[i]):int(off[i + 1])].sort()
    ref = oracle.all_pairs(ids, off)
    for dmin in (0, 2):
        res = stream.all_pairs_streamed(ids, off, spec.universe_bits, 3, batch_bits=synth.BATCH_BITS["paperlike"],
                                        dense_min_degree=dmin)
        torch.cuda.synchronize()
        check(host(res), ref, False)
        st = res["parts"]
        assert sum(s["n_ids"] for s in st) == ids.size and len(st) == 8


def test_accumulate_flag_rules():
    spec = synth.bernoulli(0.05, rows_log2=10, n=20, seed=1)
    ids, off = synth.generate(spec)
    d_ids = torch.from_numpy(ids.view(np.int64)).cuda()
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    db, _ = cabi.jas_encode(d_ids, d_off, 20, cabi.jas_encode_opts(10, 0, 0, 0, 0), None)
    B = torch.zeros(400, dtype=torch.int32, device="cuda")
    card = torch.zeros(20, dtype=torch.int64, device="cuda")
    den = torch.empty(400, dtype=torch.int64, device="cuda")
    for flags, kw in [(cabi.JAS_ACCUMULATE, {}), (cabi.JAS_ACCUMULATE, {"den": den}),
                      (cabi.JAS_ACCUMULATE | cabi.JAS_TUNE, {"card": card})]:
        with pytest.raises(cabi.JasError) as e:
            cabi.jas_gram(db, flags, None, B, kw.get("card"), kw.get("den"))
        assert e.value.status == cabi.JAS_EINVAL
    # the same db added twice counts every intersection twice
    cabi.jas_gram(db, cabi.JAS_ACCUMULATE, None, B, card)
    cabi.jas_gram(db, cabi.JAS_ACCUMULATE, None, B, card)
    J = torch.empty(400, dtype=torch.float64, device="cuda")
    cabi.jas_finalize(20, 0, None, B, card, den, J)
    torch.cuda.synchronize()
    ref = oracle.all_pairs(ids, off)
    assert np.array_equal(card.cpu().numpy(), 2 * ref["card"])
    assert np.array_equal(B.cpu().numpy().reshape(20, 20), 2 * ref["inter"])
    db.close()


def test_streamed_graph_neighbourhoods():
    # skewed rows (hubs next to isolated vertices) split over 4 ID ranges
    ids, off = synth.rmat_graph(10, 16, seed=4)
    ref = oracle.all_pairs(ids, off)
    res = stream.all_pairs_streamed(ids, off, 10, 2, batch_bits=8, upper=True)
    torch.cuda.synchronize()
    check(host(res), ref, True)


def test_overflow_is_reported_by_encode_and_by_finalize(monkeypatch):
    """With the set-size bound lowered to 100 (test hook): a set of 150
    distinct IDs is refused by jas_encode, and the same set cut into two ID
    ranges of 75 each encodes part by part but is refused by jas_finalize,
    whose summed |X_i| reaches the bound."""
    monkeypatch.setenv("JAS_TEST_CARD_LIMIT", "100")
    assert cabi.jas_card_limit() == 100
    big = np.arange(0, 300, 2, dtype=np.uint64)  # 150 distinct IDs
    sets = [big, np.arange(0, 40, dtype=np.uint64), np.array([1, 2, 3, 299], dtype=np.uint64)]
    off = np.zeros(4, np.uint64)
    off[1:] = np.cumsum([x.size for x in sets])
    ids = np.concatenate(sets)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()  # noqa: E731
    with pytest.raises(cabi.JasError) as e:
        cabi.jas_encode(d(ids), d(off), 3, cabi.jas_encode_opts(9, 0, 0, 0, 0), None)
    assert e.value.status == cabi.JAS_EOVERFLOW
    B = torch.zeros(9, dtype=torch.int32, device="cuda")
    card = torch.zeros(3, dtype=torch.int64, device="cuda")
    for lo, hi in [(0, 150), (150, 300)]:  # two ID ranges: 75 IDs of the big set in each
        part = [x[(x >= lo) & (x < hi)] for x in sets]
        po = np.zeros(4, np.uint64)
        po[1:] = np.cumsum([x.size for x in part])
        db, st = cabi.jas_encode(d(np.concatenate(part)), d(po), 3, cabi.jas_encode_opts(9, 0, 0, 0, 0), None)
        cabi.jas_gram(db, cabi.JAS_ACCUMULATE, None, B, card)
        db.close()
    torch.cuda.synchronize()
    assert card.cpu().tolist() == [150, 40, 4]
    with pytest.raises(cabi.JasError) as e:
        cabi.jas_finalize(3, 0, None, B, card)
    assert e.value.status == cabi.JAS_EOVERFLOW
    # below the bound the same sums finalize
    monkeypatch.setenv("JAS_TEST_CARD_LIMIT", "151")
    den = torch.empty(9, dtype=torch.int64, device="cuda")
    cabi.jas_finalize(3, 0, None, B, card, den)
    torch.cuda.synchronize()
    ref = oracle.all_pairs(ids, off)
    assert np.array_equal(B.cpu().numpy().reshape(3, 3), ref["inter"])
    assert np.array_equal(den.cpu().numpy().reshape(3, 3), ref["union"])
