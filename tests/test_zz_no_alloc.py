"""jas_query_noalloc (the query with a fixed device workspace) against jas_query.

Called through the C ABI (raw ctypes), on two requests in a row, the second
smaller, over one database: every output must equal jas_query's bit for bit,
the calls must allocate no device memory, and requests beyond the fixed
workspace must be refused before any work is enqueued.  With JAS_NO_WAIT a
call either runs as usual or, while another thread's call holds the
workspace, returns JAS_EBUSY without enqueueing anything.
"""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1911_04200_amd import jas as cabi  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def outputs(nq, n):
    return (torch.full((nq, n), -7, dtype=torch.int32, device="cuda"),
            torch.full((nq,), -7, dtype=torch.int64, device="cuda"),
            torch.full((nq, n), -7, dtype=torch.int64, device="cuda"),
            torch.full((nq, n), -7.0, dtype=torch.float64, device="cuda"))


def call(fn, db, qids, qoff, nq, outs, flags=0):
    lib = cabi.load()
    s = torch.cuda.current_stream().cuda_stream
    B, qc, den, J = outs
    return getattr(lib, fn)(db.handle, ctypes.c_void_p(qids.data_ptr() if qids.numel() else None),
                            ctypes.c_void_p(qoff.data_ptr()), nq, flags, ctypes.c_void_p(s),
                            ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(qc.data_ptr()),
                            ctypes.c_void_p(den.data_ptr()), ctypes.c_void_p(J.data_ptr()))


def request(spec, ids, off, r, nq, size_scale):
    q = synth.scaled(synth.query_spec(spec, r, nq), size_scale=size_scale)
    qi, qo = synth.generate(q)
    # a database set, an empty set and a set with repeats and absent IDs as well
    extra = [ids[int(off[3]):int(off[4])], np.zeros(0, np.uint64),
             np.array([9, 9, 9, (1 << 36) - 1, 123456789], np.uint64)]
    sets = [qi[int(qo[i]):int(qo[i + 1])] for i in range(nq)] + extra
    qoff = np.zeros(len(sets) + 1, np.uint64)
    qoff[1:] = np.cumsum([s.size for s in sets])
    return np.concatenate(sets), qoff


def test_noalloc_query_equals_query_on_two_calls():
    spec = synth.scaled(synth.workload("serving_db"), n=300, size_scale=0.01, pool_scale=0.005)
    ids, off = synth.generate(spec)
    n = spec.n
    db, _ = cabi.jas_encode(dev(ids), dev(off), n, cabi.jas_encode_opts(spec.universe_bits, 26, 0,
                                                                        cabi.JAS_KEEP_IDS, 0), None)
    reqs = [request(spec, ids, off, 1, 40, 0.05), request(spec, ids, off, 2, 6, 0.01)]  # the second smaller
    assert reqs[1][0].size < reqs[0][0].size and reqs[0][0].size > 100000
    want = []
    for qids, qoff in reqs:
        nq = qoff.size - 1
        o = outputs(nq, n)
        assert call("jas_query", db, dev(qids), dev(qoff), nq, o) == cabi.JAS_OK
        torch.cuda.synchronize()
        want.append([x.cpu() for x in o])
    dq = [(dev(qids), dev(qoff)) for qids, qoff in reqs]
    outs = [outputs(qoff.size - 1, n) for _, qoff in reqs]
    # the first call on the device looks up its copy of the fixed workspace,
    # which the runtime maps then (once per process); later calls allocate nothing
    o = outputs(1, n)
    assert call("jas_query_noalloc", db, dq[1][0], dev(np.array([0, 5], np.uint64)), 1, o) == cabi.JAS_OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k, ((qids, qoff), o) in enumerate(zip(dq, outs)):
        nq = reqs[k][1].size - 1
        assert call("jas_query_noalloc", db, qids, qoff, nq, o) == cabi.JAS_OK, cabi.jas_last_error()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0, "jas_query_noalloc changed the free device memory"
    for k in range(2):
        got = [x.cpu() for x in outs[k]]
        for name, g, w in zip(("B", "q_card", "den", "J"), got, want[k]):
            assert torch.equal(g, w), f"call {k}: {name} differs from jas_query"
    # repeated on the first request after the smaller one: the workspace's
    # leftovers from the previous call do not leak into the result
    o = outputs(reqs[0][1].size - 1, n)
    assert call("jas_query_noalloc", db, dq[0][0], dq[0][1], reqs[0][1].size - 1, o) == cabi.JAS_OK
    torch.cuda.synchronize()
    assert all(torch.equal(g.cpu(), w) for g, w in zip(o, want[0]))
    db.close()


def test_noalloc_query_refuses_what_the_workspace_cannot_hold():
    spec = synth.scaled(synth.workload("serving_db"), n=20, size_scale=0.001, pool_scale=0.001)
    ids, off = synth.generate(spec)
    db, _ = cabi.jas_encode(dev(ids), dev(off), 20, cabi.jas_encode_opts(spec.universe_bits, 26, 0,
                                                                         cabi.JAS_KEEP_IDS, 0), None)
    # too many query sets (all empty)
    nq = (1 << 16) + 1
    qoff = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    o = outputs(nq, 20)
    assert call("jas_query_noalloc", db, qoff[:0], qoff, nq, o) == cabi.JAS_ENOMEM
    assert "fixed workspace" in cabi.jas_last_error()
    # too many query IDs
    big = (1 << 23) + 1
    qids = torch.zeros(big, dtype=torch.int64, device="cuda")
    qoff = torch.tensor([0, big], dtype=torch.int64, device="cuda")
    o = outputs(1, 20)
    assert call("jas_query_noalloc", db, qids, qoff, 1, o) == cabi.JAS_ENOMEM
    assert "fixed workspace" in cabi.jas_last_error()
    # host pointers are not accepted (staging would allocate)
    assert call("jas_query_noalloc", db, qids[:4], torch.tensor([0, 4], device="cuda"), 1, o,
                cabi.JAS_HOST_PTRS) == cabi.JAS_EINVAL
    # the largest request it takes still runs
    qoff = torch.tensor([0, 1 << 23], dtype=torch.int64, device="cuda")
    o2 = outputs(1, 20)
    assert call("jas_query_noalloc", db, qids[:1 << 23], qoff, 1, o2) == cabi.JAS_OK, cabi.jas_last_error()
    o3 = outputs(1, 20)
    assert call("jas_query", db, qids[:1 << 23], qoff, 1, o3) == cabi.JAS_OK
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(o2, o3))
    db.close()


def test_noalloc_no_wait_is_busy_or_the_same_result():
    """With JAS_NO_WAIT a call runs as usual, or, while another thread's call
    holds the fixed workspace, returns JAS_EBUSY at once and enqueues nothing
    (its outputs keep their fill)."""
    import threading

    spec = synth.scaled(synth.workload("serving_db"), n=300, size_scale=0.01, pool_scale=0.005)
    ids, off = synth.generate(spec)
    n = spec.n
    db, _ = cabi.jas_encode(dev(ids), dev(off), n, cabi.jas_encode_opts(spec.universe_bits, 26, 0,
                                                                        cabi.JAS_KEEP_IDS, 0), None)
    qids, qoff = request(spec, ids, off, 1, 40, 0.05)
    nq = qoff.size - 1
    dq, dqo = dev(qids), dev(qoff)
    want = outputs(nq, n)
    assert call("jas_query", db, dq, dqo, nq, want) == cabi.JAS_OK
    torch.cuda.synchronize()
    want = [x.cpu() for x in want]
    o = outputs(nq, n)
    assert call("jas_query_noalloc", db, dq, dqo, nq, o, cabi.JAS_NO_WAIT) == cabi.JAS_OK, cabi.jas_last_error()
    torch.cuda.synchronize()
    assert all(torch.equal(g.cpu(), w) for g, w in zip(o, want))

    stop, errors = threading.Event(), []

    def worker():  # keeps the workspace busy with waiting calls on its own stream
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(200):
                    if stop.is_set():
                        break
                    st = call("jas_query_noalloc", db, dq, dqo, nq, outputs(nq, n))
                    if st != cabi.JAS_OK:
                        errors.append(st)
                        break
        except Exception as e:  # reported by the main thread
            errors.append(repr(e))

    t = threading.Thread(target=worker)
    t.start()
    busy = 0
    try:
        for _ in range(400):
            o = outputs(nq, n)
            torch.cuda.synchronize()
            st = call("jas_query_noalloc", db, dq, dqo, nq, o, cabi.JAS_NO_WAIT)
            torch.cuda.synchronize()
            if st == cabi.JAS_EBUSY:
                busy += 1
                assert "in use" in cabi.jas_last_error()
                assert bool((o[0] == -7).all()) and bool((o[1] == -7).all()), "a refused call wrote its outputs"
            else:
                assert st == cabi.JAS_OK, cabi.jas_last_error()
                assert all(torch.equal(g.cpu(), w) for g, w in zip(o, want))
            if busy >= 3 or not t.is_alive():
                break
    finally:
        stop.set()
        t.join()
    assert not errors, errors
    db.close()
    if busy == 0:
        pytest.skip("no call overlapped the other thread's calls")
