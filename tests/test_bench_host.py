"""bench.py's host-side contract (no GPU): refusals and the roofline's algorithmic amounts."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_streaming_needs_ascending_sets():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "paperlike",
                        "--stream-part-bits", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "ascending" in r.stdout


def test_algorithmic_amounts():
    b = load_bench()
    st = {"n_pairs": 1000, "n_rows": 600, "n_shared_rows": 100, "list_pairs": 500, "n_word_rows": 10,
          "n_list_rows": 50}
    # a scatter pass reads and writes every 8-byte key once
    assert b.algorithmic("radix_onesweep", st, 1024, 10 ** 9, 3)[1] == 16.0
    # pair words are 4 bytes: sort passes read + write, emission writes, counting reads
    assert b.algorithmic("pair_sort", st, 1024, 0, 0)[1] == 8.0 * 500 / 1e9
    assert b.algorithmic("pair_emit", st, 1024, 0, 0)[1] == 4.0 * 500 / 1e9
    # packed words: H word rows of n rounded up to 128 columns
    assert b.algorithmic("pack", st, 130, 0, 0)[1] == 8.0 * 10 * 256 / 1e9
    # Gram: 2 ops per bit pair of every 128 x 128 tile pair of the upper triangle
    bound, amount, unit, _ = b.algorithmic("gram_fp4", st, 256, 0, 0)
    assert bound == "mfma_fp4" and unit == "TFLOP/s"
    assert amount == 2.0 * 10 * 64 * 3 * 128 * 128 / 1e12
    assert b.algorithmic("no_such_kernel", st, 1, 1, 1) is None
