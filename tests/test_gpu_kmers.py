"""The GPU k-mer front end against the oracle, and sequences -> Jaccard end to end."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1911_04200_amd as jas  # noqa: E402
from paper_1911_04200_amd import jas as cabi  # noqa: E402


def gpu_kmers(samples, k, canonical):
    seqs = [s for smp in samples for s in smp]
    words, seq_off = synth.pack_2bit(seqs)
    smp_off = np.zeros(len(samples) + 1, dtype=np.uint64)
    np.cumsum([len(x) for x in samples], out=smp_off[1:])
    ids_off = cabi.jas_kmer_offsets(seq_off, smp_off, k)
    ids = torch.empty(max(1, int(ids_off[-1])), dtype=torch.int64, device="cuda")
    cabi.jas_kmers(torch.from_numpy(words.view(np.int64)).cuda(), seq_off, k,
                   cabi.JAS_CANONICAL if canonical else 0, None, ids)
    torch.cuda.synchronize()
    return ids, ids_off


@pytest.mark.parametrize("k", [1, 3, 19, 31])
@pytest.mark.parametrize("canonical", [False, True])
def test_kmers_match_the_oracle(k, canonical):
    rng = np.random.default_rng(k)
    lens = [0, 1, 5, 31, 32, 33, 63, 64, 65, 1000, 4097, 30]
    samples = [[rng.integers(0, 4, size=L, dtype=np.uint8) for L in lens[i::3]] for i in range(3)]
    samples.append([])  # a sample without sequences
    ids, off = gpu_kmers(samples, k, canonical)
    want, want_off = oracle.kmer_sets(samples, k, canonical)
    assert np.array_equal(off, want_off)
    assert np.array_equal(ids.cpu().numpy().view(np.uint64)[:want.size], want)


def test_argument_checks():
    with pytest.raises(cabi.JasError):
        cabi.jas_kmer_offsets(np.array([0, 5], np.uint64), np.array([0, 1], np.uint64), 32)
    with pytest.raises(cabi.JasError):
        cabi.jas_kmer_offsets(np.array([0, 5], np.uint64), np.array([0, 2], np.uint64), 3)
    with pytest.raises(cabi.JasError):
        cabi.jas_kmers(None, np.array([0, 5], np.uint64), 3, 0x1, None, None)


def test_sequences_to_jaccard_end_to_end():
    # mutated copies of 4 reference genomes, 3 sequences each; k = 19 canonical
    samples = synth.random_genomes(40, 20000, n_refs=4, mutation=0.01, seqs_per_sample=3, seed=5)
    k = 19
    ids, off = gpu_kmers(samples, k, True)
    res_db, st = jas.encode(ids[:int(off[-1])], torch.from_numpy(off.view(np.int64)).cuda(), universe_bits=2 * k,
                            batch_bits=30)
    out = jas.gram(res_db, upper=False)
    torch.cuda.synchronize()
    want_ids, want_off = oracle.kmer_sets(samples, k, True)
    ref = oracle.all_pairs(want_ids, want_off)
    assert np.array_equal(out["card"].cpu().numpy(), ref["card"])
    assert np.array_equal(out["B"].cpu().numpy().reshape(40, 40), ref["inter"])
    J = out["J"].cpu().numpy().reshape(40, 40)
    assert np.array_equal(J.view(np.uint64), ref["J"].view(np.uint64))
    # copies of one reference are far more alike than copies of two
    assert J.max(initial=0, where=~np.eye(40, dtype=bool)) > 0.5
    res_db.close()


@pytest.mark.parametrize("U", [20, 62, 64])
def test_relabel_is_the_rank_among_distinct_ids(U):
    rng = np.random.default_rng(U)
    base = rng.integers(0, 1 << 62, size=5000, dtype=np.uint64) >> np.uint64(max(0, 62 - U))
    if U == 64:
        base = base | np.uint64(1 << 63)
    ids = rng.choice(base, size=200000)  # repeats
    ids[:3] = [0, (1 << U) - 1 if U < 64 else (1 << 64) - 1, ids[5]]
    uniq, inv = np.unique(ids, return_inverse=True)
    d = torch.from_numpy(ids.view(np.int64)).cuda()
    out = torch.empty_like(d)
    D, newU = cabi.jas_relabel(d, ids.size, U, None, out)
    assert D == uniq.size and newU == max(1, int(uniq.size - 1).bit_length())
    assert np.array_equal(out.cpu().numpy().view(np.uint64), inv.astype(np.uint64))
    # in place
    D2, _ = cabi.jas_relabel(d, ids.size, U, None, d)
    assert D2 == D and torch.equal(d, out)
    if U < 64:
        bad = torch.from_numpy(np.array([1 << U], np.uint64).view(np.int64)).cuda()
        with pytest.raises(cabi.JasError) as e:
            cabi.jas_relabel(bad, 1, U, None, bad)
        assert e.value.status == cabi.JAS_EINVAL


def test_k31_sequences_to_jaccard_through_the_relabel():
    """k = 31 canonical k-mers (IDs below 2^62) of 64 genomes: 62 + 6 key bits
    do not fit, so the encoder refuses them as they are; relabelled by rank
    they fit 23 bits, and B, C and J equal the oracle's on the k-mer sets."""
    samples = synth.random_genomes(64, 20000, n_refs=4, mutation=0.01, seqs_per_sample=2, seed=9)
    k = 31
    ids, off = gpu_kmers(samples, k, True)
    N = int(off[-1])
    d_off = torch.from_numpy(off.view(np.int64)).cuda()
    with pytest.raises(cabi.JasError) as e:
        cabi.jas_encode(ids[:N], d_off, 64, cabi.jas_encode_opts(2 * k, 0, 0, 0, 0), None)
    assert e.value.status == cabi.JAS_EINVAL
    D, U = cabi.jas_relabel(ids, N, 2 * k, None, ids)
    assert U <= 64 - 6
    db, st = jas.encode(ids[:N], d_off, universe_bits=U)
    out = jas.gram(db)
    torch.cuda.synchronize()
    want_ids, want_off = oracle.kmer_sets(samples, k, True)
    assert D == np.unique(want_ids).size
    ref = oracle.all_pairs(want_ids, want_off)
    assert np.array_equal(out["card"].cpu().numpy(), ref["card"])
    assert np.array_equal(out["B"].cpu().numpy().reshape(64, 64), ref["inter"])
    assert np.array_equal(out["den"].cpu().numpy().reshape(64, 64), ref["union"])
    assert np.array_equal(out["J"].cpu().numpy().reshape(64, 64).view(np.uint64), ref["J"].view(np.uint64))
    db.close()
