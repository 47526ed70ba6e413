"""The host C code of the tests under AddressSanitizer and
UndefinedBehaviorSanitizer (gcc; no GPU).

oracle/oracle.c and synth/synth.c are built with -fsanitize=address,undefined
(no recovery from undefined behaviour) and driven through their Python
bindings in a child process that preloads the sanitizer runtime: every oracle
pin, the generator's workloads at small scale (clustered pools with repeats,
Bernoulli matrices, R-MAT graphs, serving queries, single samples regenerated
alone) and the oracle's all-pairs and cross products on them.  Any invalid
access, leak of bounds or undefined operation aborts the child.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1",
         "-fPIC", "-shared", "-std=c11"]


def asan_runtime():
    if not shutil.which("gcc"):
        return None
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    rt = asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    d = tmp_path_factory.mktemp("sanitized")
    lo, ls = str(d / "liboracle_san.so"), str(d / "libsynth_san.so")
    subprocess.check_call(["gcc", *FLAGS, "-fno-fast-math", "-ffp-contract=off", "-o", lo,
                           os.path.join(ROOT, "oracle", "oracle.c")])
    subprocess.check_call(["gcc", *FLAGS, "-o", ls, os.path.join(ROOT, "synth", "synth.c"), "-lm"])
    return rt, lo, ls


CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import numpy as np
import synth
synth.use_library({synth_lib!r})
import oracle
import pins
lib = oracle.load({oracle_lib!r})
failed = [c.__name__ for c in pins.ALL if c(lib=lib)]
assert not failed, failed
cases = [
    synth.workload("tiny"),
    synth.scaled(synth.workload("paperlike"), n=48, size_scale=0.002, pool_scale=0.002, dup_rate=0.05),
    synth.scaled(synth.workload("batching"), n=96, size_scale=0.001, pool_scale=0.001),
    synth.bernoulli(0.02, rows_log2=12, n=40),
    synth.Graph(9, 8),
]
for spec in cases:
    ids, off = synth.generate(spec)
    ref = oracle.all_pairs(ids, off, lib=lib)
    n = off.size - 1
    assert ref["inter"].shape == (n, n) and np.array_equal(ref["inter"], ref["inter"].T)
    assert np.array_equal(np.diag(ref["inter"]), ref["card"])
    if hasattr(spec, "size_kind"):
        pick = [0, n // 2, n - 1]
        sub_ids, sub_off = synth.generate_samples(spec, pick)
        for k, i in enumerate(pick):
            assert np.array_equal(sub_ids[sub_off[k]:sub_off[k + 1]], ids[off[i]:off[i + 1]])
db = synth.scaled(synth.workload("serving_db"), n=64, size_scale=0.001, pool_scale=0.001)
ids, off = synth.generate(db)
q = synth.scaled(synth.query_spec(db, 3, 8), size_scale=0.01)
qi, qo = synth.generate(q)
c = oracle.cross(qi, qo, ids, off, lib=lib)
assert c["inter"].shape == (qo.size - 1, off.size - 1)
print("SANITIZED_OK", flush=True)
"""


def test_oracle_and_generator_under_sanitizers(sanitized):
    rt, lo, ls = sanitized
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")
    code = CHILD.format(root=ROOT, tests=TESTS, synth_lib=ls, oracle_lib=lo)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0 and "SANITIZED_OK" in r.stdout, (r.stdout[-2000:] + "\n" + r.stderr[-4000:])
