"""Pins of the oracle's MRG32k3a generator and streams (Sec. 4.4, eq.
mrg32k3a and eq. rngstream; reading R28) against an independent
implementation and against plain stepping:

* rocRAND's mrg32k3a engine header (installed, written by others, with its
  own precomputed jump tables), compiled into a harness: outputs after
  skipping g streams (2^127 outputs), i substreams (2^76) and an offset agree
  word for word with the oracle's jumps by repeated squaring;
* jumps by small offsets equal stepping the recursion one output at a time;
* integration with the MRG32k3a streams is unbiased: pulls against the
  closed form over many seeds have mean 0 and standard deviation 1.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import closed_forms as cf
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
M1 = 4294967087


@pytest.fixture(scope="module")
def rocrand_harness(tmp_path_factory):
    inc = "/opt/rocm/include"
    if not os.path.exists(os.path.join(inc, "rocrand", "rocrand_mrg32k3a.h")):
        pytest.skip("rocRAND headers not installed")
    exe = str(tmp_path_factory.mktemp("mrg") / "mrg32k3a_rocrand")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + inc,
                           "-o", exe, os.path.join(HERE, "harness", "mrg32k3a_rocrand.cpp")])
    return exe


def test_streams_and_substreams_match_rocrand(oracle_lib, rocrand_harness):
    rng = np.random.default_rng(5)
    n = 3000
    g = rng.integers(0, 2**63, n, dtype=np.uint64)
    i = rng.integers(0, 2**40, n, dtype=np.uint64)
    off = rng.integers(0, 2**38, n, dtype=np.uint64)
    # small and structured positions: the start, single jumps, stream 1024 s + c
    g[:64] = np.arange(64, dtype=np.uint64)
    i[:64] = 0
    off[:64] = 0
    g[64:128] = 1024 * 3 + np.arange(64, dtype=np.uint64)
    i[64:128] = np.arange(64, dtype=np.uint64)
    off[64:128] = 64 * np.arange(64, dtype=np.uint64)
    rec = np.stack([g, i, off], axis=1).astype(np.uint64)
    out = subprocess.run([rocrand_harness], input=rec.tobytes(), stdout=subprocess.PIPE,
                         check=True).stdout
    ref = np.frombuffer(out, np.uint32).reshape(-1, 8)
    for q in range(n):
        got = oracle_lib.mrg_outputs(int(g[q]), int(i[q]), int(off[q]), 8)
        assert np.array_equal(got, ref[q]), (q, int(g[q]), int(i[q]), int(off[q]))
    assert ref.min() >= 1 and ref.max() <= M1


def test_jumps_equal_stepping(oracle_lib):
    seq = oracle_lib.mrg_outputs(7, 11, 0, 20000)
    rng = np.random.default_rng(6)
    for k in rng.integers(0, 19990, 200):
        assert np.array_equal(oracle_lib.mrg_outputs(7, 11, int(k), 8), seq[k:k + 8])


def test_outputs_are_uniform(oracle_lib):
    from scipy.stats import chisquare
    z = oracle_lib.mrg_outputs(1, 2, 3, 200_000).astype(np.float64) / (M1 + 1)
    h, _ = np.histogram(z, bins=64, range=(0, 1))
    assert chisquare(h).pvalue > 1e-4


def _c1_wide():
    p = W.config1()
    cl = p.chan_loc + np.array([[0.03, -0.02], [-0.02, 0.04]])
    return p.with_(chan_loc=cl, chan_width=p.chan_width * 1.6, name="c1_wide", rng=1)


def test_integration_with_mrg_streams_is_unbiased(oracle_lib):
    p = _c1_wide()
    I = cf.integral(p)
    z = []
    for s in range(3000, 3150):
        o = oracle_lib.Oracle(p.with_(seed=s))
        o.sample_iteration(2000)
        z.append((o.history[0, 0] - I) / o.history[0, 1])
    z = np.array(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(len(z)), z.mean()
    assert 0.8 < z.std(ddof=1) < 1.25, z.std(ddof=1)


def test_mrg_words_differ_by_call_channel_iteration(oracle_lib):
    p = W.gauss_mixture(3, 3, 10, seed=5).with_(rng=1)
    o = oracle_lib.Oracle(p)
    a = o.trace(3000, 0, 0, 3000)
    b = o.trace(3000, 1, 0, 3000)
    assert not np.array_equal(a["words"], b["words"])
    # no two calls of a pass share their words
    assert len({tuple(r) for r in a["words"]}) == 3000
    # seeds must leave room for 1024 streams per seed
    with pytest.raises(ValueError):
        oracle_lib.Oracle(p.with_(seed=2**54))
