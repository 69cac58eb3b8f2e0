"""Pins of the oracle's Philox4x32-10 against an independent implementation.

The oracle writes Philox4x32-10 from its published definition (Salmon,
Moraes, Dror, Shaw, SC'11).  The pin is PyTorch's ATen PhiloxRNGEngine.h, an
installed source implementation written by others, compiled here into a small
harness.  ATen's engine with key = seed, counter words 2..3 = subsequence and
counter words 0..1 = offset reproduces the oracle's layout
counter = (i_lo, i_hi, t, block) with subsequence = t + 2^32 * block, offset = i.
"""
import os
import subprocess
import sysconfig

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def aten_harness(tmp_path_factory):
    torch_inc = None
    for base in (sysconfig.get_paths()["purelib"], sysconfig.get_paths()["platlib"]):
        cand = os.path.join(base, "torch", "include")
        if os.path.exists(os.path.join(cand, "ATen", "core", "PhiloxRNGEngine.h")):
            torch_inc = cand
    if torch_inc is None:
        pytest.skip("ATen PhiloxRNGEngine.h not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_aten")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I" + torch_inc, "-o", exe,
                           os.path.join(HERE, "harness", "philox_aten.cpp")])
    return exe


def _aten_words(exe, seeds, subseq, offsets):
    rec = np.stack([seeds, subseq, offsets], axis=1).astype(np.uint64)
    out = subprocess.run([exe], input=rec.tobytes(), stdout=subprocess.PIPE, check=True).stdout
    return np.frombuffer(out, np.uint32).reshape(-1, 4)


def test_philox_block_matches_aten(oracle_lib, aten_harness):
    O = oracle_lib
    rng = np.random.default_rng(11)
    n = 20000
    seeds = rng.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n).astype(np.uint64)
    i = rng.integers(0, 2**63, size=n, dtype=np.uint64)
    t = rng.integers(0, 2**32, size=n, dtype=np.uint64)
    b = rng.integers(0, 2**32, size=n, dtype=np.uint64)
    # include small / structured counters too
    i[:100] = np.arange(100)
    t[:100] = 0
    b[:100] = 0
    seeds[:100] = 1
    ref = _aten_words(aten_harness, seeds, t + (b << np.uint64(32)), i)
    for q in range(n):
        ctr = [int(i[q]) & 0xFFFFFFFF, int(i[q]) >> 32, int(t[q]), int(b[q])]
        key = [int(seeds[q]) & 0xFFFFFFFF, int(seeds[q]) >> 32]
        got = O.philox(ctr, key)
        assert np.array_equal(got, ref[q]), (q, ctr, key, got, ref[q])


def test_word_layout(oracle_lib):
    """word(seed, i, t, m) is output m mod 4 of block m // 4."""
    O = oracle_lib
    for seed, i, t in ((1, 0, 0), (3, 123456789012, 7), (2**64 - 1, 2**40 + 5, 0x80000000)):
        for m in range(12):
            blk = O.philox([i & 0xFFFFFFFF, i >> 32, t, m // 4], [seed & 0xFFFFFFFF, seed >> 32])
            assert O.word(seed, i, t, m) == int(blk[m % 4])


def test_words_look_uniform(oracle_lib):
    """Sanity: mean of 2e4 words / 2^32 ~ 1/2, no repeated words."""
    O = oracle_lib
    w = np.array([O.word(5, i, 0, 0) for i in range(20000)], np.float64) / 2**32
    assert abs(w.mean() - 0.5) < 5 * (1 / np.sqrt(12 * 20000))
    assert len(np.unique(w)) == 20000
