"""Pins of the CPU oracle: checks against things other than the oracle itself.

Each check returns a list of failure strings (empty when it holds), so the
same checks serve the oracle tests and the planted-mistake test.

  brute_force   - tiny collections; B = A^T A by an integer matrix product of
                  the dense 0/1 indicator matrix (Sec. III-A), unions as
                  column-OR counts, J as the correctly rounded value of the
                  exact fraction (Python's Fraction -> float rounds correctly).
  python_sets   - the same quantities from Python's own set type.
  closed_forms  - families whose answer is known in closed form.
  golden_hand   - hand-worked examples (tests/golden/hand_examples.txt).
  invariants    - symmetry, B_ii = |X_i|, bounds, inclusion-exclusion
                  (Sec. III-A: |X_i cup X_j| = |X_i| + |X_j| - B_ij),
                  1^T B 1 = sum_k deg_k^2 and row sums of B = sum over the
                  set of row degrees, with degrees from numpy's unique counts.
  triangle      - d_J = 1 - J is a metric (Sec. II-A): triangle inequality in
                  exact rational arithmetic.
  two_collections - query sets against a different collection (Q != X, of
                  other sizes and offsets), every pair and selected pairs,
                  against Python's set type: catches the two collections'
                  offsets or sizes mixed up, which Q = X cannot show.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_examples.txt")


def _collection(sets):
    off = np.zeros(len(sets) + 1, dtype=np.uint64)
    for i, s in enumerate(sets):
        off[i + 1] = off[i] + len(s)
    ids = np.array([x for s in sets for x in s], dtype=np.uint64)
    return ids, off


def _random_tiny(rng, n, m, empty_p=0.1, dup_p=0.2):
    sets = []
    for i in range(n):
        r = rng.random()
        if r < empty_p:
            sets.append([])
            continue
        if i > 0 and r < empty_p + 0.1:
            sets.append(list(sets[rng.integers(0, i)]))  # an identical set
            continue
        size = int(rng.integers(1, max(2, m // 2)))
        s = list(rng.integers(0, m, size=size))
        if rng.random() < dup_p and s:
            s += list(rng.choice(s, size=max(1, len(s) // 3)))
        rng.shuffle(s)
        sets.append([int(x) for x in s])
    return sets


def _check_equal(tag, got, want, fails):
    got = np.asarray(got)
    want = np.asarray(want)
    if got.shape != want.shape or not np.array_equal(got, want):
        bad = np.argwhere(got != want) if got.shape == want.shape else "shape"
        fails.append(f"{tag}: mismatch at {bad if isinstance(bad, str) else bad[:5].tolist()}")


def brute_force(lib=None, seeds=range(6)):
    fails = []
    for seed in seeds:
        rng = np.random.default_rng(1000 + seed)
        n = int(rng.integers(1, 17))
        m = int(2 ** rng.integers(2, 13))
        sets = _random_tiny(rng, n, m)
        ids, off = _collection(sets)
        r = oracle.all_pairs(ids, off, lib=lib)
        A = np.zeros((m, n), dtype=np.int64)
        for i, s in enumerate(sets):
            for x in s:
                A[x, i] = 1
        B = A.T @ A
        Cu = np.zeros((n, n), dtype=np.int64)
        for i in range(n):
            for j in range(n):
                Cu[i, j] = int(np.count_nonzero(A[:, i] | A[:, j]))
        Jw = np.array([[1.0 if Cu[i, j] == 0 else float(Fraction(int(B[i, j]), int(Cu[i, j])))
                        for j in range(n)] for i in range(n)], dtype=np.float64).reshape(n, n)
        _check_equal(f"bf seed {seed} B", r["inter"], B, fails)
        _check_equal(f"bf seed {seed} union", r["union"], Cu, fails)
        _check_equal(f"bf seed {seed} card", r["card"], A.sum(axis=0), fails)
        if not np.array_equal(r["J"].view(np.uint64), Jw.view(np.uint64)):
            fails.append(f"bf seed {seed} J bits differ")
    return fails


def python_sets(lib=None, seeds=range(4)):
    fails = []
    for seed in seeds:
        rng = np.random.default_rng(2000 + seed)
        n = int(rng.integers(2, 12))
        sets = _random_tiny(rng, n, int(2 ** rng.integers(3, 10)))
        # large IDs exercise the full 64-bit range
        sets = [[(x * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF for x in s] for s in sets]
        ids, off = _collection(sets)
        r = oracle.all_pairs(ids, off, lib=lib)
        S = [set(s) for s in sets]
        for i in range(n):
            for j in range(n):
                inter, uni = len(S[i] & S[j]), len(S[i] | S[j])
                if r["inter"][i, j] != inter or r["union"][i, j] != uni:
                    fails.append(f"sets seed {seed} ({i},{j}) counts")
                jw = 1.0 if uni == 0 else float(Fraction(inter, uni))
                if r["J"][i, j] != jw:
                    fails.append(f"sets seed {seed} ({i},{j}) J")
    return fails


def closed_forms(lib=None):
    fails = []
    # disjoint sets: B = 0 off the diagonal, J = 0
    sets = [list(range(100 * i, 100 * i + 10 + i)) for i in range(6)]
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    off = ~np.eye(6, dtype=bool)
    if np.any(r["inter"][off] != 0) or np.any(r["J"][off] != 0.0):
        fails.append("disjoint")
    # identical sets: B = |X|, J = 1
    sets = [list(range(50))] * 4
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    if np.any(r["inter"] != 50) or np.any(r["J"] != 1.0):
        fails.append("identical")
    # nested chain X_1 c X_2 c ... : B_ij = |X_min(i,j)|, J_ij = |X_min| / |X_max|
    sizes = [3, 7, 20, 21, 64]
    sets = [list(range(s)) for s in sizes]
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    for i in range(5):
        for j in range(5):
            a, b = sizes[min(i, j)], sizes[max(i, j)]
            if r["inter"][i, j] != a or r["union"][i, j] != b or r["J"][i, j] != float(Fraction(a, b)):
                fails.append(f"nested ({i},{j})")
    # shared core plus private parts: B_ij = |core| for i != j
    core = list(range(1000, 1040))
    sets = [core + list(range(10000 * (i + 1), 10000 * (i + 1) + 5 * i)) for i in range(5)]
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    for i in range(5):
        for j in range(5):
            if i != j and r["inter"][i, j] != 40:
                fails.append(f"core ({i},{j})")
            if i != j and r["union"][i, j] != 40 + 5 * i + 5 * j:
                fails.append(f"core union ({i},{j})")
    # empty sets: J(empty, empty) = 1 (Sec. II-A), J(empty, X) = 0
    sets = [[], [1, 2], []]
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    if r["J"][0, 2] != 1.0 or r["J"][0, 0] != 1.0 or r["J"][0, 1] != 0.0 or r["J"][1, 1] != 1.0:
        fails.append("empty")
    return fails


def golden_hand(lib=None, path=GOLDEN):
    fails = []
    for ln, line in enumerate(open(path)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        xs, ys, ci, cu, jf = [p.strip() for p in line.split(";")]
        X = [int(t) for t in xs.split()]
        Y = [int(t) for t in ys.split()]
        num, den = (int(t) for t in jf.split("/"))
        r = oracle.all_pairs(*_collection([X, Y]), lib=lib)
        if r["inter"][0, 1] != int(ci) or r["union"][0, 1] != int(cu):
            fails.append(f"golden line {ln + 1}: counts")
        if r["J"][0, 1] != float(Fraction(num, den)) or r["J"][1, 0] != r["J"][0, 1]:
            fails.append(f"golden line {ln + 1}: J")
    return fails


def invariants_of(r, ids, off):
    """Invariants of one all-pairs result r (dict from oracle.all_pairs) on (ids, off)."""
    fails = []
    B, C, J, card = r["inter"], r["union"], r["J"], r["card"]
    n = card.size
    if not np.array_equal(B, B.T) or not np.array_equal(C, C.T) or not np.array_equal(J, J.T):
        fails.append("symmetry")
    if not np.array_equal(np.diag(B), card):
        fails.append("B_ii = |X_i|")
    mn = np.minimum(card[:, None], card[None, :])
    mx = np.maximum(card[:, None], card[None, :])
    if np.any(B < 0) or np.any(B > mn) or np.any(C < mx):
        fails.append("bounds")
    if not np.array_equal(C, card[:, None] + card[None, :] - B):
        fails.append("inclusion-exclusion")
    if np.any(J < 0) or np.any(J > 1) or np.any(np.diag(J) != 1.0):
        fails.append("J range / diagonal")
    # degrees from numpy, independent of the oracle
    uniq = [np.unique(ids[int(off[i]):int(off[i + 1])]) for i in range(n)]
    if not np.array_equal(np.array([u.size for u in uniq], dtype=np.int64), card):
        fails.append("card vs numpy unique")
    allu = np.concatenate(uniq) if n else np.zeros(0, np.uint64)
    vals, deg = np.unique(allu, return_counts=True)
    if int(B.sum()) != int((deg.astype(np.int64) ** 2).sum()):
        fails.append("1^T B 1 = sum deg^2")
    degmap = dict(zip(vals.tolist(), deg.tolist()))
    for i in range(min(n, 8)):
        if int(B[i].sum()) != sum(degmap[x] for x in uniq[i].tolist()):
            fails.append(f"row sum {i}")
    return fails


def invariants(lib=None):
    import synth
    s = synth.scaled(synth.workload("tiny"), n=24, size_scale=0.2)
    ids, off = synth.generate(s)
    return invariants_of(oracle.all_pairs(ids, off, lib=lib), ids, off)


def triangle(lib=None, trials=400):
    fails = []
    rng = np.random.default_rng(7)
    sets = _random_tiny(rng, 14, 40, empty_p=0.15)
    r = oracle.all_pairs(*_collection(sets), lib=lib)
    B, C = r["inter"], r["union"]

    def d(i, j):
        return Fraction(1) - (Fraction(1) if C[i, j] == 0 else Fraction(int(B[i, j]), int(C[i, j])))

    n = len(sets)
    for _ in range(trials):
        i, j, k = (int(x) for x in rng.integers(0, n, 3))
        if d(i, k) > d(i, j) + d(j, k):
            fails.append(f"triangle ({i},{j},{k})")
    for i in range(n):
        if d(i, i) != 0:
            fails.append(f"d(i,i) {i}")
    return fails


def two_collections(lib=None, seeds=range(3)):
    fails = []
    for seed in seeds:
        rng = np.random.default_rng(4000 + seed)
        m = int(2 ** rng.integers(4, 10))
        # different counts and sizes on the two sides, so that no offset of
        # one collection is also a valid offset of the other by chance
        if seed % 2 == 1:  # fewer query sets than database sets
            qsets = _random_tiny(rng, int(rng.integers(2, 7)), m, empty_p=0.15)
            xsets = [s + [int(v) for v in rng.integers(0, m, 3)] for s in _random_tiny(rng, int(rng.integers(7, 13)), m)]
        else:  # more, smaller query sets: a mixed-up offset stays inside the other collection
            qsets = [[int(v) for v in rng.integers(0, m, int(rng.integers(0, 4)))] for _ in range(int(rng.integers(9, 14)))]
            xsets = [[int(v) for v in rng.integers(0, m, m // 2)] for _ in range(int(rng.integers(3, 7)))]
        qn, qo = oracle.normalize(*_collection(qsets), lib=lib)
        xn, xo = oracle.normalize(*_collection(xsets), lib=lib)
        Q, X = [set(s) for s in qsets], [set(s) for s in xsets]
        nq, nx = len(Q), len(X)
        want_i = np.array([[len(Q[a] & X[b]) for b in range(nx)] for a in range(nq)], dtype=np.int64)
        want_u = np.array([[len(Q[a] | X[b]) for b in range(nx)] for a in range(nq)], dtype=np.int64)
        want_j = np.array([[1.0 if want_u[a, b] == 0 else float(Fraction(int(want_i[a, b]), int(want_u[a, b])))
                            for b in range(nx)] for a in range(nq)], dtype=np.float64)
        ci, cu, cj = oracle.cross_normalized(qn, qo, xn, xo, lib=lib)
        _check_equal(f"two seed {seed} cross inter", ci, want_i, fails)
        _check_equal(f"two seed {seed} cross union", cu, want_u, fails)
        _check_equal(f"two seed {seed} cross J", cj.view(np.uint64), want_j.view(np.uint64), fails)
        qi = rng.integers(0, nq, 50)
        xi = rng.integers(0, nx, 50)
        pi, pu, pj = oracle.pairs_normalized(qn, qo, xn, xo, qi, xi, lib=lib)
        _check_equal(f"two seed {seed} pairs inter", pi, want_i[qi, xi], fails)
        _check_equal(f"two seed {seed} pairs union", pu, want_u[qi, xi], fails)
        _check_equal(f"two seed {seed} pairs J", pj.view(np.uint64), want_j[qi, xi].view(np.uint64), fails)
        if fails:
            break  # one failing case is enough (a later one may read out of bounds)
    return fails


ALL = [brute_force, python_sets, closed_forms, golden_hand, invariants, triangle, two_collections]


def run_all(lib=None):
    out = []
    for f in ALL:
        out += f(lib=lib)
    return out
