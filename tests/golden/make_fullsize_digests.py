"""Write the full-size parity digests, from the CPU oracle alone.

For each named workload, at the full size the benchmark runs, this script
generates the seeded input (synth/), computes every pair's |X_i cap X_j|,
|X_i cup X_j| and J with the oracle (oracle/: sorted sets, one counting walk
per pair), and writes tests/golden/fullsize_<workload>.txt holding the input's
digest and one digest per output row (tests/digests.py).  Nothing from the GPU
library is imported.  The all-pairs workloads take the pairs i <= j (the
definition is symmetric) and mirror them; the serving workload takes a fixed,
seeded set of query requests against every database set.

Run on the CPU (hours for the largest workloads; every available core):
    python tests/golden/make_fullsize_digests.py [--cache DIR] [workload ...]
--cache keeps finished blocks of rows so an interrupted run resumes.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
sys.path[:0] = [ROOT, TESTS]

import digests  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402

# all-pairs workloads and the layout the GPU test reads back
ALL_PAIRS = {"graph_s13_ef64": False, "paperlike": False, "bernoulli_p1e-3": True, "precision": False,
             "batching": True}
SERVING_REQUESTS = 32
SERVING_SEED = 20261203


def serving_requests():
    """(request index, number of query sets) of the checked serving requests."""
    rng = np.random.default_rng(SERVING_SEED)
    return [(int(r), int(q)) for r, q in zip(range(SERVING_REQUESTS), rng.integers(1, 65, SERVING_REQUESTS))]


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def all_pairs_rows(name: str, cache: str | None):
    spec = synth.workload(name)
    n = spec.n
    ids, off = synth.generate(spec)
    ind = digests.input_digest(ids, off)
    log(name, "generated", ids.size, "IDs, input", ind[:16])
    s, so = oracle.normalize(ids, off)
    del ids
    card = np.diff(so.astype(np.int64))
    B = np.empty((n, n), dtype=np.int64)
    C = np.empty((n, n), dtype=np.int64)
    J = np.empty((n, n), dtype=np.float64)
    # blocks of rows with about 2^21 pairs (i, j >= i) each
    i0 = 0
    t0 = time.time()
    while i0 < n:
        i1, cnt = i0, 0
        while i1 < n and cnt < (1 << 21):
            cnt += n - i1
            i1 += 1
        path = os.path.join(cache, f"{name}_{i0}_{i1}.npz") if cache else None
        if path and os.path.exists(path):
            z = np.load(path)
            inter, uni, jac = z["inter"], z["uni"], z["jac"]
        else:
            qi = np.concatenate([np.full(n - i, i, np.int32) for i in range(i0, i1)])
            xi = np.concatenate([np.arange(i, n, dtype=np.int32) for i in range(i0, i1)])
            inter, uni, jac = oracle.pairs_normalized(s, so, s, so, qi, xi)
            if path:
                np.savez(path + ".tmp.npz", inter=inter, uni=uni, jac=jac)
                os.replace(path + ".tmp.npz", path)
        k = 0
        for i in range(i0, i1):
            m = n - i
            B[i, i:], C[i, i:], J[i, i:] = inter[k:k + m], uni[k:k + m], jac[k:k + m]
            B[i:, i], C[i:, i], J[i:, i] = inter[k:k + m], uni[k:k + m], jac[k:k + m]
            k += m
        log(name, f"rows {i1}/{n}", f"{time.time() - t0:.0f} s")
        i0 = i1
    assert np.array_equal(np.diag(B), card)
    if B.max() >= 2 ** 31:
        raise SystemExit(f"{name}: an intersection exceeds int32")
    return spec, ind, B, C, J


def write_all_pairs(name: str, cache: str | None):
    upper = ALL_PAIRS[name]
    spec, ind, B, C, J = all_pairs_rows(name, cache)
    n = spec.n
    if upper:
        iu = np.triu_indices(n)
        rows = digests.row_digests(B[iu].astype(np.int32), C[iu], J[iu], n, True)
    else:
        rows = digests.row_digests(B.astype(np.int32), C, J, n, False)
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    with open(path, "w") as f:
        f.write(f"# Full-size parity digests of the {name} workload, written by\n"
                f"# tests/golden/make_fullsize_digests.py from the CPU oracle alone.\n"
                f"# row i: first {digests.ROW_HEX} hex digits of SHA-256 over row i of B (int32),\n"
                f"# C (int64) and J (binary64), little-endian, in the {'packed upper (j >= i)' if upper else 'full'}"
                f" layout.\n")
        f.write(f"workload {name}\nn {n}\nlayout {'upper' if upper else 'full'}\ninput {ind}\n")
        f.write(f"sum_B_upper {int(np.triu(B).sum())}\n")
        for i, d in enumerate(rows):
            f.write(f"row {i} {d}\n")
    log("wrote", path)


def write_serving(cache: str | None):
    spec = synth.workload("serving_db")
    n = spec.n
    reqs = serving_requests()
    qsets = {}
    for r, nq in reqs:
        qi, qo = synth.generate(synth.query_spec(spec, r, nq))
        qsets[r] = (digests.input_digest(qi, qo),) + oracle.normalize(qi, qo)
    res = {r: [np.empty((nq, n), np.int64), np.empty((nq, n), np.int64), np.empty((nq, n), np.float64)]
           for r, nq in reqs}
    # the database in two halves of columns (each half normalised once)
    half = n // 2
    per_sample = []
    import hashlib
    for h in range(2):
        cols = np.arange(h * half, (h + 1) * half)
        xi, xo = synth.generate_samples(spec, cols)
        # per-set hashes, combined into the whole input's digest below
        for i in range(half):
            per_sample.append(hashlib.sha256(
                memoryview(np.ascontiguousarray(xi[int(xo[i]):int(xo[i + 1])], dtype="<u8")).cast("B")).digest())
        xs, xso = oracle.normalize(xi, xo)
        del xi
        for r, nq in reqs:
            path = os.path.join(cache, f"serving_{r}_{h}.npz") if cache else None
            if path and os.path.exists(path):
                z = np.load(path)
                inter, uni, jac = z["inter"], z["uni"], z["jac"]
            else:
                _, qs, qso = qsets[r]
                inter, uni, jac = oracle.cross_normalized(qs, qso, xs, xso)
                if path:
                    np.savez(path + ".tmp.npz", inter=inter, uni=uni, jac=jac)
                    os.replace(path + ".tmp.npz", path)
            res[r][0][:, cols], res[r][1][:, cols], res[r][2][:, cols] = inter, uni, jac
            log("serving half", h, "request", r, "nq", nq)
        del xs
    hh = hashlib.sha256(np.ascontiguousarray(synth.offsets(spec), dtype="<u8").tobytes())
    for d in per_sample:
        hh.update(d)
    ind = hh.hexdigest()
    path = os.path.join(HERE, "fullsize_serving.txt")
    with open(path, "w") as f:
        f.write("# Full-size parity digests of serving requests against the whole serving_db\n"
                "# database, written by tests/golden/make_fullsize_digests.py from the CPU oracle alone.\n"
                f"# request r: query sets synth.query_spec(db, r, nq); row q: first {digests.ROW_HEX} hex digits\n"
                "# of SHA-256 over B[q, :] (int32), C[q, :] (int64), J[q, :] (binary64), little-endian.\n")
        f.write(f"workload serving_db\nn {n}\nlayout query\ninput {ind}\n")
        for r, nq in reqs:
            qd, qs, qso = qsets[r]
            B, C, J = res[r]
            qc = int(np.diff(qso.astype(np.int64)).sum())
            f.write(f"request {r} nq {nq} input {qd} q_card_sum {qc}\n")
            for q in range(nq):
                f.write(f"row {q} {digests.row_digest(B[q].astype(np.int32), C[q], J[q])}\n")
    log("wrote", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default=None)
    ap.add_argument("workloads", nargs="*")
    a = ap.parse_args()
    names = a.workloads or list(ALL_PAIRS) + ["serving"]
    if a.cache:
        os.makedirs(a.cache, exist_ok=True)
    log("oracle threads", oracle.threads())
    for name in names:
        if name == "serving":
            write_serving(a.cache)
        else:
            write_all_pairs(name, a.cache)


if __name__ == "__main__":
    main()
