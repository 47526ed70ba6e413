"""Encode plans: the batching form as one captured launch sequence.

A plan is made from one collection; jas_plan_encode then encodes other
collections of the same shape with no host synchronisation and no
allocation.  Checked against the oracle bit for bit: the planning collection
and a second seeded collection encoded through the plan, eagerly and as one
HIP graph (plan encode + Gram + finalize) replayed several times with other
work between the replays; a collection beyond the plan's capacities is
reported, not computed wrongly.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1911_04200_amd import jas as cabi  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def batching_like(seed_offset, n=600, scale=0.01):
    spec = synth.scaled(synth.workload("batching"), n=n, size_scale=scale, pool_scale=0.01,
                        seed_offset=seed_offset)
    return spec, synth.generate(spec)


def upper(ref, key):
    n = ref["card"].size
    return ref[key][np.triu_indices(n)]


def gram_upper(db, n):
    L = n * (n + 1) // 2
    out = {"B": torch.empty(L, dtype=torch.int32, device="cuda"),
           "card": torch.empty(n, dtype=torch.int64, device="cuda"),
           "den": torch.empty(L, dtype=torch.int64, device="cuda"),
           "J": torch.empty(L, dtype=torch.float64, device="cuda")}
    cabi.jas_gram(db, cabi.JAS_UPPER, None, out["B"], out["card"], out["den"], out["J"])
    return out


def check(out, ref, tag):
    got = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.array_equal(got["card"], ref["card"]), tag
    bad = np.flatnonzero(got["B"] != upper(ref, "inter"))
    assert bad.size == 0, f"{tag}: B differs at {bad[:5].tolist()}"
    assert np.array_equal(got["den"], upper(ref, "union")), tag
    assert np.array_equal(got["J"].view(np.uint64), upper(ref, "J").view(np.uint64)), tag


@pytest.mark.parametrize("case,dmin,word_bits", [("batching", 0, 64), ("batching", 3, 64),
                                                 ("paperlike", 0, 64), ("paperlike", 5, 32)])
def test_planned_encode_matches_the_oracle(case, dmin, word_bits):
    if case == "batching":
        make = lambda k: batching_like(k)  # noqa: E731
    else:
        def make(k):
            spec = synth.scaled(synth.workload("paperlike"), n=300, size_scale=0.004, pool_scale=0.004,
                                seed_offset=k, dup_rate=0.01)
            return spec, synth.generate(spec)
    spec, (ids, off) = make(0)
    n = spec.n
    opts = cabi.jas_encode_opts(spec.universe_bits, synth.BATCH_BITS[case], dmin, 0, 0, word_bits)
    plan = cabi.jas_plan_create(dev(ids), dev(off), n, opts, headroom=2.0)
    for k in (0, 1, 2):  # the planning collection, then two others of the same shape
        _, (ids_k, off_k) = make(k)
        cabi.jas_plan_encode(plan, dev(ids_k), dev(off_k))
        st = cabi.jas_plan_check(plan)
        assert st["n_ids"] == int(off_k[-1])
        out = gram_upper(plan.db, n)
        torch.cuda.synchronize()
        check(out, oracle.all_pairs(ids_k, off_k), f"{case} collection {k}")
    plan.close()


def test_captured_encode_gram_finalize_replays_exactly():
    spec, (ids0, off0) = batching_like(0, n=800)
    n = spec.n
    others = [batching_like(k, n=800)[1] for k in (1, 2)]
    cap = max(int(o[1][-1]) for o in [(ids0, off0)] + others)
    ids_buf = torch.zeros(cap, dtype=torch.int64, device="cuda")
    off_buf = torch.zeros(n + 1, dtype=torch.int64, device="cuda")

    def load(ids, off):
        ids_buf[:ids.size].copy_(torch.from_numpy(ids.view(np.int64)))
        off_buf.copy_(torch.from_numpy(off.view(np.int64)))

    load(ids0, off0)
    opts = cabi.jas_encode_opts(spec.universe_bits, 26, 0, 0, 0)
    plan = cabi.jas_plan_create(ids_buf, off_buf, n, opts, headroom=2.0)
    L = n * (n + 1) // 2
    B = torch.empty(L, dtype=torch.int32, device="cuda")
    card = torch.empty(n, dtype=torch.int64, device="cuda")
    den = torch.empty(L, dtype=torch.int64, device="cuda")
    J = torch.empty(L, dtype=torch.float64, device="cuda")
    db = plan.db
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # one eager run on the capture stream first
        cabi.jas_plan_encode(plan, ids_buf, off_buf, s)
        cabi.jas_gram(db, cabi.JAS_UPPER, s, B, card, den, J)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cabi.jas_plan_encode(plan, ids_buf, off_buf, s)
        cabi.jas_gram(db, cabi.JAS_UPPER, s, B, card, den, J)
    sets = [(ids0, off0)] + others + [(ids0, off0)]
    for rep, (ids, off) in enumerate(sets):
        load(ids, off)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        cabi.jas_plan_check(plan)
        got = {"B": B.clone(), "card": card.clone(), "den": den.clone(), "J": J.clone()}
        # other eager work between the replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
        check(got, oracle.all_pairs(ids, off), f"replay {rep}")
    del g
    plan.close()


def test_plan_reports_a_collection_beyond_its_capacity():
    spec, (ids, off) = batching_like(0, n=300, scale=0.004)
    opts = cabi.jas_encode_opts(spec.universe_bits, 26, 0, 0, 0)
    plan = cabi.jas_plan_create(dev(ids), dev(off), spec.n, opts, headroom=0.0)
    big = synth.scaled(spec, size_scale=3.0)
    ids2, off2 = synth.generate(big)
    cabi.jas_plan_encode(plan, dev(ids2), dev(off2))
    with pytest.raises(cabi.JasError) as e:
        cabi.jas_plan_check(plan)
    assert e.value.status == cabi.JAS_ENOMEM
    # the plan still works for what it holds
    cabi.jas_plan_encode(plan, dev(ids), dev(off))
    cabi.jas_plan_check(plan)
    out = gram_upper(plan.db, spec.n)
    torch.cuda.synchronize()
    check(out, oracle.all_pairs(ids, off), "after an overrun")
    plan.close()


def test_tuned_threshold_is_timed_and_exact():
    spec, (ids, off) = batching_like(0, n=400)
    opts = cabi.jas_encode_opts(spec.universe_bits, 26, 0, cabi.JAS_TUNE, 0)
    plan = cabi.jas_plan_create(dev(ids), dev(off), spec.n, opts, headroom=0.2)
    tun = plan.tuning()
    assert len(tun) >= 3 and all(ms > 0 for _, ms in tun)
    assert plan.threshold == min(tun, key=lambda x: x[1])[0]
    cabi.jas_plan_encode(plan, dev(ids), dev(off))
    cabi.jas_plan_check(plan)
    out = gram_upper(plan.db, spec.n)
    torch.cuda.synchronize()
    check(out, oracle.all_pairs(ids, off), "tuned")
    plan.close()


def test_plan_refuses_a_collection_that_needs_the_fallback_sort():
    """One ID repeated 20,000 times makes a bucket too large to finish in LDS:
    the eager encode takes the full sort (checked against the oracle), and a
    plan, which prepares only the single-pass path, is refused up front."""
    rng = np.random.default_rng(3)
    sets = [rng.integers(0, 1 << 32, 2000, dtype=np.uint64) for _ in range(40)]
    sets[7] = np.concatenate([sets[7], np.full(20000, 12345, np.uint64)])
    sets[9] = np.concatenate([sets[9], np.array([12345], np.uint64)])
    off = np.zeros(len(sets) + 1, np.uint64)
    off[1:] = np.cumsum([s.size for s in sets])
    ids = np.concatenate(sets)
    opts = cabi.jas_encode_opts(32, 0, 0, 0, 0)
    db, _ = cabi.jas_encode(dev(ids), dev(off), 40, opts, None)
    out = gram_upper(db, 40)
    torch.cuda.synchronize()
    check(out, oracle.all_pairs(ids, off), "eager with the fallback sort")
    db.close()
    with pytest.raises(cabi.JasError) as e:
        cabi.jas_plan_create(dev(ids), dev(off), 40, opts, headroom=0.5)
    assert e.value.status == cabi.JAS_EUNSUPPORTED
    assert "fallback" in e.value.message
