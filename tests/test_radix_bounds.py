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


@pytest.mark.parametrize("sizes", ["large", "small", "empty_runs"])
def test_sample_of_an_entry_from_its_tile(sizes):
    """The first scatter pass forms key id << s | sample: the sample of entry t
    in a tile [t0, t1) is the sample s0 of the tile's first entry plus the
    number of sample starts off[k], s0 < k <= s1 (s1 = the sample of the
    tile's last entry), at or before t, each compared as a position in the
    tile (off[k] - t0 < 8192).  Checked for every entry against the plain
    definition (the last sample whose start is <= t) on offsets with large
    sets, small sets and runs of empty sets."""
    import numpy as np

    rng = np.random.default_rng({"large": 1, "small": 2, "empty_runs": 3}[sizes])
    if sizes == "large":
        lens = rng.integers(5000, 40000, 60)
    elif sizes == "small":
        lens = rng.integers(1, 40, 3000)
    else:
        lens = rng.integers(0, 200, 2000) * (rng.random(2000) < 0.3)
        lens[:5] = 0
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N, tk = int(off[-1]), 8192
    want = np.searchsorted(off, np.arange(N), side="right") - 1  # last s with off[s] <= t
    for t0 in range(0, N, tk):
        t1 = min(N, t0 + tk)
        s0, s1 = int(want[t0]), int(want[t1 - 1])
        starts = off[s0 + 1:s1 + 1] - t0
        assert np.all((starts > 0) & (starts < tk))
        li = np.arange(t1 - t0)
        got = s0 + (li[:, None] >= starts[None, :]).sum(axis=1)
        assert np.array_equal(got, want[t0:t1]), t0
