"""The CPU oracle against its pins (no GPU)."""
import os
import shutil

import numpy as np
import pytest

import oracle
import pins


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(check):
    fails = check()
    assert not fails, fails


def test_cross_is_a_block_of_all_pairs():
    import synth
    s = synth.scaled(synth.workload("tiny"), n=12, size_scale=0.1)
    ids, off = synth.generate(s)
    whole = oracle.all_pairs(ids, off)
    q = [2, 5, 11]
    qi, qo = synth.generate_samples(s, q)
    r = oracle.cross(qi, qo, ids, off)
    assert np.array_equal(r["inter"], whole["inter"][q])
    assert np.array_equal(r["union"], whole["union"][q])
    assert np.array_equal(r["J"].view(np.uint64), whole["J"][q].view(np.uint64))
    assert np.array_equal(r["q_card"], whole["card"][q])


def test_selected_pairs_match_all_pairs():
    import synth
    s = synth.scaled(synth.workload("tiny"), n=10, size_scale=0.1)
    ids, off = synth.generate(s)
    whole = oracle.all_pairs(ids, off)
    ns, no = oracle.normalize(ids, off)
    rng = np.random.default_rng(3)
    I = rng.integers(0, 10, 40)
    J = rng.integers(0, 10, 40)
    inter, uni, jac = oracle.pairs_normalized(ns, no, ns, no, I, J)
    assert np.array_equal(inter, whole["inter"][I, J])
    assert np.array_equal(uni, whole["union"][I, J])
    assert np.array_equal(jac, whole["J"][I, J])


def test_rejects_bad_offsets():
    with pytest.raises(ValueError):
        oracle.normalize(np.arange(4, dtype=np.uint64), np.array([0, 3, 2, 4], dtype=np.uint64))


# Planted mistakes: each edit below is a plausible slip in the oracle (a
# dropped term, a wrong branch or operand, a wrong convention).  Built from a
# copy of oracle.c, every mutant must fail at least one pin.
MUTANTS = {
    "count_on_wrong_branch": ("c += p == q;", "c += p <= q;"),
    "union_drops_tails": ("*uni = u + (nx - a) + (ny - b);", "*uni = u + (nx - a);"),
    "union_counts_match_twice": ("++u;\n    }", "u += 1 + (p == q);\n    }"),
    "empty_pair_is_zero": ("if (uni == 0) return 1.0;", "if (uni == 0) return 0.0;"),
    "keeps_repeats": ("if (dst[t] != dst[k - 1]) dst[k++] = dst[t];", "dst[k++] = dst[t];"),
    "transposed_ratio": ("return (double)inter / (double)uni;", "return (double)uni / (double)(inter ? inter : 1);"),
    "float_quotient": ("return (double)inter / (double)uni;", "return (double)((float)inter / (float)uni);"),
    "off_by_one_start": ("uint64_t a = 0, b = 0, c = 0, u = 0;", "uint64_t a = 1, b = 0, c = 0, u = 0;"),
    "signed_compare": ("return (x > y) - (x < y);", "return ((int64_t)x > (int64_t)y) - ((int64_t)x < (int64_t)y);"),
    # the two collections' offsets confused: invisible while Q = X
    "pairs_mix_offsets": ("*b = x + xoff[xi[k]];", "*b = x + qoff[xi[k]];"),
    "pairs_mix_sizes": ("nb = xoff[xi[k] + 1] - xoff[xi[k]];", "nb = qoff[xi[k] + 1] - qoff[xi[k]];"),
    "cross_mix_offsets": ("*b = x + xoff[j];", "*b = x + qoff[j];"),
}


_CHILD = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, pins
lib = oracle.load({lib!r})
failed = 0
for check in pins.ALL:
    if check(lib=lib):
        failed += 1
        print("PINS_FAILED", check.__name__, flush=True)
print("PINS_PASSED" if not failed else "DONE", flush=True)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    """The mutant's pins run in a child process: a mistake that makes the
    oracle read out of bounds may crash it, and a crash is a detection too."""
    import subprocess
    import sys
    src = open(oracle._SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    msrc = tmp_path / "oracle_mut.c"
    msrc.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(msrc), out=str(tmp_path / "liboracle_mut.so"))
    tests = os.path.dirname(os.path.abspath(__file__))
    code = _CHILD.format(root=os.path.dirname(tests), tests=tests, lib=lib)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if "PINS_FAILED" in r.stdout:
        return  # a pin failed (a later one may have crashed on the mutant's reads)
    assert r.returncode < 0, f"planted mistake {name} passed every pin:\n{r.stdout}\n{r.stderr[-2000:]}"
