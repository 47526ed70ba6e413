"""Serving loop: admission and batching logic (CPU) and alone-vs-mix equality (GPU)."""
import numpy as np
import pytest

from paper_1911_04200_amd import serve


class _StubDb:
    n = 100
    handle = None


def _req(rid, nq, ids_per_set=10):
    off = np.arange(nq + 1, dtype=np.uint64) * np.uint64(ids_per_set)
    return serve.Request(rid, np.zeros(nq * ids_per_set, np.uint64), off)


def test_batches_take_fifo_requests_up_to_the_set_limit():
    s = serve.Server(_StubDb(), slots=2, budget_bytes=1 << 40, max_batch_sets=10)
    for rid, nq in enumerate([4, 5, 3, 1]):
        s.submit(_req(rid, nq))
    batch, cost = s._take()
    assert [r.rid for r in batch] == [0, 1]       # 4 + 5 <= 10, + 3 would exceed
    batch, cost = s._take()
    assert [r.rid for r in batch] == [2, 3]
    assert s._take() is None


def test_admission_respects_the_budget():
    s = serve.Server(_StubDb(), slots=2, budget_bytes=0, max_batch_sets=64)
    one = s.cost([_req(0, 2)])
    s.budget = one + one // 2
    for rid in range(3):
        s.submit(_req(rid, 2))
    batch, c = s._take()            # only one request fits
    assert [r.rid for r in batch] == [0]
    assert s._take() is None         # the next waits for memory
    s.in_use -= c
    batch, c = s._take()
    assert [r.rid for r in batch] == [1]


def test_an_oversized_request_runs_alone_when_nothing_else_is_in_flight():
    s = serve.Server(_StubDb(), slots=1, budget_bytes=1, max_batch_sets=64)
    s.submit(_req(0, 3))
    batch, c = s._take()
    assert [r.rid for r in batch] == [0]


def test_poisson_arrivals_are_seeded_and_increasing():
    a = serve.poisson_arrivals(100, 50.0, 3)
    assert a == serve.poisson_arrivals(100, 50.0, 3)
    assert all(x < y for x, y in zip(a, a[1:]))
    assert 1.0 < a[-1] < 3.5


@pytest.mark.gpu
def test_each_result_is_the_same_alone_and_in_the_mix():
    import torch
    import oracle
    import synth
    from paper_1911_04200_amd import jas as cabi
    spec = synth.scaled(synth.workload("serving_db"), n=256, size_scale=0.01, pool_scale=0.005)
    ids, off = synth.generate(spec)
    opts = cabi.jas_encode_opts(spec.universe_bits, 26, 0, cabi.JAS_KEEP_IDS, 0)
    db, _ = cabi.jas_encode(torch.from_numpy(ids.view(np.int64)).cuda(),
                            torch.from_numpy(off.view(np.int64)).cuda(), spec.n, opts, None)
    reqs = serve.make_requests(spec, 40, seed=9, max_sets=12, size_scale=0.01)
    alone = serve.Server(db, slots=1, max_batch_sets=1)
    alone.run(reqs)
    solo = {r.rid: (r.B.copy(), r.q_card.copy(), r.den.copy(), r.J.copy()) for r in reqs}
    for r in reqs:
        r.B = r.q_card = r.den = r.J = None
    mixed = serve.Server(db, slots=4, max_batch_sets=32)
    # Poisson arrivals (batching depends on timing), then a closed batch (all
    # queued before the slots start, so calls take several requests)
    for arrivals in (serve.poisson_arrivals(len(reqs), 400.0, 1), None):
        done = mixed.run(reqs, arrivals)
        assert len(done) == len(reqs)
        if arrivals is None:
            assert max(r.batch_size for r in reqs) > 1, "no request was batched with another"
        for r in reqs:
            B, qc, den, J = solo[r.rid]
            assert np.array_equal(r.B, B) and np.array_equal(r.q_card, qc) and np.array_equal(r.den, den)
            assert np.array_equal(r.J.view(np.uint64), J.view(np.uint64))
            r.B = r.q_card = r.den = r.J = None
    # and against the oracle for a few requests
    mixed.run(reqs[:3])
    for r in reqs[:3]:
        ref = oracle.cross(r.ids, r.offsets, ids, off)
        assert np.array_equal(r.B, ref["inter"]) and np.array_equal(r.J, ref["J"])
    db.close()
