"""Pins of the oracle parts that have no closed form of their own, checked
against statistics and exact integer arithmetic rather than against the
oracle's own formulas:

* the error of a pass (Sec. 3.1: the error shrinks as sqrt(V/N); Sec. 3.4:
  per-channel variances of the multi-channel estimator; reading R10) --
  pulls (E - I) / sigma over many independent seeds have mean 0 and standard
  deviation 1 against the closed-form integral;
* the combination of iterations (Sec. 3.5, last paragraph of the iteration
  organisation; reading R17) -- over the same seeds, iterations of very
  different sizes combine into pulls of standard deviation 1 (a plain mean
  would give about 2.7 here) with chi^2/ndf averaging 1;
* the word -> (bin, fraction) rule (reading R3) -- for identity channels on
  flat grids the point is x = (j + fraction) / n with j and the fraction
  computed from the Philox word with Python big integers.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import closed_forms as cf
import workloads as W

SEEDS = range(1000, 1200)


def _bw_pair():
    """d = 2: two Breit-Wigner peaks (one on both axes, one on axis 0 only),
    channels with the peaks' own shapes."""
    pk = np.array([[2, 2], [2, 0]], np.int32)
    pl = np.array([[0.35, 0.6], [0.7, 0.5]])
    pw = np.array([[0.08, 0.12], [0.05, 1.0]])
    wt = np.array([0.7, 0.3])
    return W.Problem(2, 16, pk, pl, pw, wt, pk.copy(), pl.copy(), pw.copy(), seed=1,
                     name="bw_pair")


def _c1_wide():
    """C1's integrand with channel maps that do not match its peaks (wider and
    off-centre Gaussians), so the weights vary inside every channel (C1's own
    channels make them constant per channel and the variance 0)."""
    p = W.config1()
    cl = p.chan_loc + np.array([[0.03, -0.02], [-0.02, 0.04]])
    return p.with_(chan_loc=cl, chan_width=p.chan_width * 1.6, name="c1_wide")


def _pulls(oracle_lib, problem, n_points):
    I = cf.integral(problem)
    pulls = []
    for s in SEEDS:
        o = oracle_lib.Oracle(problem.with_(seed=s))
        o.sample_iteration(n_points)
        E, sig = o.history[0, 0], o.history[0, 1]
        assert sig > 0
        pulls.append((E - I) / sig)
    return np.array(pulls)


@pytest.mark.parametrize("maker,n_points", [(_c1_wide, 2000), (_bw_pair, 4000)])
def test_pass_error_pulls(oracle_lib, maker, n_points):
    p = maker()
    z = _pulls(oracle_lib, p, n_points)
    n = len(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(n), z.mean()
    assert 0.8 < z.std(ddof=1) < 1.25, z.std(ddof=1)


@pytest.mark.parametrize("maker", [_c1_wide, _bw_pair])
def test_iteration_combination_pulls_and_chi2(oracle_lib, maker):
    p = maker()
    I = cf.integral(p)
    sizes = [500, 2000, 8000, 32000]
    z, chi2 = [], []
    for s in SEEDS:
        o = oracle_lib.Oracle(p.with_(seed=s))
        for n in sizes:  # fixed grids and weights: independent iterations
            o.sample_iteration(n)
        r = o.result(0)
        assert r["n_iter"] == len(sizes)
        z.append((r["integral"] - I) / r["error"])
        chi2.append(r["chi2_ndf"])
        # the combined error is below the best single iteration's
        assert r["error"] < o.history[-1, 1]
    z, chi2 = np.array(z), np.array(chi2)
    n = len(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(n), z.mean()
    assert 0.8 < z.std(ddof=1) < 1.25, z.std(ddof=1)
    # chi^2 with 3 degrees of freedom, divided by 3: mean 1, s.d. sqrt(2/3)
    assert abs(chi2.mean() - 1.0) < 4.0 * math.sqrt(2.0 / 3.0 / n), chi2.mean()


def _exact_point(u, n, fp32, edges):
    """x from word u by reading R3, in exact rationals: j = floor(u n / 2^32),
    lo = u n mod 2^32, fraction (lo + 1/2) 2^-32 (FP64 rules) or
    (floor(lo / 2^9) + 1/2) 2^-23 (FP32 rules); x = e_j + fraction (e_{j+1} - e_j)."""
    prod = int(u) * int(n)
    j = prod >> 32
    lo = prod & 0xFFFFFFFF
    frac = Fraction(2 * (lo >> 9) + 1, 1 << 24) if fp32 else Fraction(2 * lo + 1, 1 << 33)
    e0, e1 = Fraction(float(edges[j])), Fraction(float(edges[j + 1]))
    return j, e0 + frac * (e1 - e0)


@pytest.mark.parametrize("n", [1, 3, 20, 100, 256])
@pytest.mark.parametrize("fp32", [False, True])
def test_word_to_bin_and_fraction_big_int(oracle_lib, n, fp32):
    d = 3
    p = W.constant_problem(d, 1, n).with_(precision=1 if fp32 else 0)
    o = oracle_lib.Oracle(p)
    edges = o.edges[0]  # flat (FP32-snapped under FP32 rules)
    # flat edges are j/n correctly rounded (then rounded to FP32 under FP32 rules)
    for k in range(d):
        for j in range(n + 1):
            want = float(Fraction(j, n))
            if fp32:
                want = float(np.float32(want))
            assert edges[k, j] == want
    N = 4000
    tr = o.trace(N, 5, 0, N, n_words=d)
    for q in range(0, N, 7):
        for k in range(d):
            j, x = _exact_point(tr["words"][q, k], n, fp32, edges[k])
            assert tr["bins"][q, 0, k] == j
            assert 0 <= j < n
            got = Fraction(float(tr["p"][q, k]))
            if n & (n - 1) == 0:
                # e_j, the width and the fraction are exact and so is x
                assert got == x, (n, q, k)
            else:
                # one rounding of the product and one of the sum
                assert abs(got - x) <= Fraction(2 ** -52) * max(abs(x), Fraction(2 ** -60))


def test_pass_is_independent_of_the_worker_split(oracle_lib):
    """Sec. 4.4: with counter-based random numbers every call's words depend
    only on (seed, call, iteration), so a pass split over any number of
    workers (contiguous call ranges, combined in order) gives the same
    per-channel sums and per-bin sums up to the rounding of the combination;
    this is what lets the pass shard over GPUs with one reduction.  1 worker
    against 7 (ragged ranges), importance and stratified passes."""
    import workloads as W
    for p in (W.config2(), W.mixed_problem(6, 4, 3, 40, seed=61),
              W.config2().with_(strat=2)):
        a, b = oracle_lib.Oracle(p), oracle_lib.Oracle(p)
        for _ in range(2):
            a.sample_iteration(30_011, 1)
            b.sample_iteration(30_011, 7)
            np.testing.assert_array_equal(a.alloc, b.alloc)
            sa, sb = a.channel_stats, b.channel_stats
            assert np.max(np.abs(sa[:, :3] - sb[:, :3]) / np.abs(sa[:, :3]).clip(1e-300)) < 1e-13
            assert np.max(np.abs(a.hist - b.hist) / np.abs(a.hist).clip(1e-300)) < 1e-12
            assert abs(a.history[-1, 0] - b.history[-1, 0]) <= 1e-13 * abs(a.history[-1, 0])
            a.refine()
            b.refine()
            # the grids stay the same to rounding, so the next pass is comparable
            assert np.max(np.abs(a.edges - b.edges)) < 1e-12
