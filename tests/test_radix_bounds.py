"""Bounds of the single-pass radix scatter's indexing, emulated on the host.

tests/radix_bounds_emul.cpp walks the kernel's tiles, look-back status words,
digit starts and output positions with the kernel's own index expressions
(csrc/onesweep_index.hpp) and checks every address against its buffer: at the
paper-like workload's full size (N = 1,676,543,805 keys, 8192-key tiles, the
three passes of 8, 8 and 6 bits its 22 sorted ID bits take), with and without
look-back waits that give up, and key by key on smaller inputs.  No GPU.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "radix_bounds_emul.cpp")
INC = os.path.join(ROOT, "paper_1911_04200_amd", "csrc")
PAPERLIKE_N = 1676543805


@pytest.fixture(scope="module")
def emul(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("emul") / "radix_bounds_emul")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", INC, "-o", exe, SRC])
    return exe


def run(exe, *args):
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.parametrize("n,widths,dist,giveup,seed", [
    (1_000_000, "8,8,6", "uniform", 0, 1),
    (1_000_000, "8,8,6", "uniform", 200, 2),
    (999_999, "8,8", "skew", 0, 3),
    (8193, "8", "uniform", 0, 4),
    (8191, "7,7", "skew", 5000, 5),
])
def test_every_key_lands_in_bounds(emul, n, widths, dist, giveup, seed):
    out = run(emul, n, 8192, widths, dist, giveup, seed, "exact")
    assert "fails 0" in out


@pytest.mark.parametrize("giveup", [0, 50])
def test_paperlike_size_in_bounds(emul, giveup):
    out = run(emul, PAPERLIKE_N, 8192, "8,8,6", "uniform", giveup, 11 + giveup)
    assert "tiles 204657" in out and "fails 0" in out
    if giveup:
        assert "giveups 0 " not in out
