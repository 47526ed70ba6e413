"""The k-mer oracle against the paper's worked example and brute force (no GPU)."""
import itertools
import os

import numpy as np

import oracle
import synth

CODE = {"A": 0, "C": 1, "G": 2, "T": 3}
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kmers_paper_example.txt")


def codes(s):
    return np.array([CODE[c] for c in s], dtype=np.uint8)


def decode(v, k):
    """Base-4 digits of v, first base most significant, as a string."""
    return "".join("ACGT"[(int(v) >> (2 * (k - 1 - j))) & 3] for j in range(k))


def revcomp(s):
    return s[::-1].translate(str.maketrans("ACGT", "TGCA"))


def test_paper_example():
    lines = [ln for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(lines) == 2
    for ln in lines:
        seq, k, want = (x.strip() for x in ln.split(";"))
        k = int(k)
        got = oracle.kmers(codes(seq), k)
        assert [decode(v, k) for v in got] == want.split()


def test_ids_order_like_the_strings_and_canonical_form_by_brute_force():
    for k in (1, 2, 3, 4):
        words = ["".join(p) for p in itertools.product("ACGT", repeat=k)]
        ids = [int(oracle.kmers(codes(w), k)[0]) for w in words]
        assert ids == list(range(4 ** k))  # lexicographic order = numeric order
        for w in words:
            c = int(oracle.kmers(codes(w), k, canonical=True)[0])
            assert decode(c, k) == min(w, revcomp(w))
    # odd k: no k-mer is its own reverse complement, so both strands give the same ID
    for w in ["".join(p) for p in itertools.product("ACGT", repeat=3)]:
        assert w != revcomp(w)
        assert oracle.kmers(codes(w), 3, True)[0] == oracle.kmers(codes(revcomp(w)), 3, True)[0]


def test_long_kmers_and_short_sequences():
    rng = np.random.default_rng(1)
    s = rng.integers(0, 4, size=100, dtype=np.uint8)
    text = "".join("ACGT"[c] for c in s)
    for k in (19, 31):
        got = oracle.kmers(s, k)
        assert got.size == 100 - k + 1
        assert all(decode(v, k) == text[i:i + k] for i, v in enumerate(got))
        got_c = oracle.kmers(s, k, canonical=True)
        assert all(decode(v, k) == min(text[i:i + k], revcomp(text[i:i + k])) for i, v in enumerate(got_c))
    assert oracle.kmers(s[:5], 6).size == 0 and oracle.kmers(s[:6], 6).size == 1


def test_packing_of_sequences():
    seqs = [codes("AATGTC"), codes(""), codes("G" * 40)]
    words, off = synth.pack_2bit(seqs)
    assert list(off) == [0, 6, 6, 46]
    flat = np.concatenate(seqs)
    for b in range(46):
        assert (int(words[b // 32]) >> (2 * (b % 32))) & 3 == flat[b]
    g = synth.random_genomes(5, 300, n_refs=2, mutation=0.05, seqs_per_sample=3, seed=1)
    assert len(g) == 5 and all(len(x) == 3 and sum(p.size for p in x) == 300 for x in g)
