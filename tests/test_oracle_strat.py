"""Pins of the oracle's pseudo-stratified sampling (Sec. 3.3: r space of a
channel cut into n_r^d boxes, the same number s >= 2 of uniform calls in
every box, then the VEGAS map; reading R30 for the layout, the bin rule and
the box variance), against counting, exact integers and statistics:

* the layout: s n_r^d <= N_c < s (n_r + 1)^d by brute force;
* coverage: with identity channels on flat grids a call's point is its r, and
  every box of every channel holds exactly its number of calls;
* the bin and fraction of each axis from the box digit and the word, with
  Python big integers (exact for n and n_r powers of two);
* the error: pulls against the closed form over many seeds have mean 0 and
  standard deviation 1 with the box-variance estimate (a plain per-call
  variance would overstate it several times);
* the point of stratifying: at equal calls the error is smaller than with
  uniform sampling.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import closed_forms as cf
import workloads as W


def _layout(oracle_lib, n, d, s):
    import ctypes as C
    nr, pb = C.c_int64(0), C.c_int64(0)
    oracle_lib.lib().orc_strat_layout(n, d, s, C.byref(nr), C.byref(pb))
    return nr.value, pb.value


def test_layout_brute_force(oracle_lib):
    rng = np.random.default_rng(8)
    for _ in range(300):
        d = int(rng.integers(1, 11))
        s = int(rng.integers(2, 6))
        n = int(rng.integers(s, 10**7))
        nr, pb = _layout(oracle_lib, n, d, s)
        assert 1 <= nr <= 2**20
        assert s * nr**d <= n or nr == 1
        assert nr == 2**20 or s * (nr + 1)**d > n
        assert pb == n // nr**d and pb >= min(s, n)


def _flat_strat(d, n_bins, K, s, fp32=False):
    return W.constant_problem(d, K, n_bins).with_(strat=s, precision=1 if fp32 else 0)


@pytest.mark.parametrize("d,K,s", [(2, 1, 2), (3, 2, 3), (1, 3, 2)])
def test_every_box_gets_its_calls(oracle_lib, d, K, s):
    p = _flat_strat(d, 16, K, s)
    o = oracle_lib.Oracle(p)
    N = 5000
    nc_pre, _ = oracle_lib.allocation(np.full(K, 1.0 / K), N, 10)
    tr_alloc = None
    o.sample_iteration(N)
    nc = o.alloc
    starts = np.concatenate([[0], np.cumsum(nc[:-1])])
    tr = o.trace(N, 0, 0, int(nc[-1]))
    for c in range(K):
        nr, pb = _layout(oracle_lib, int(nc_pre[c]), d, s)
        assert nc[c] == pb * nr**d
        pts = tr["p"][starts[c]:starts[c] + nc[c]]
        digits = np.floor(pts * nr).astype(np.int64)
        box = np.zeros(len(pts), np.int64)
        for k in reversed(range(d)):
            box = box * nr + digits[:, k]
        counts = np.bincount(box, minlength=nr**d)
        assert np.all(counts == pb), (c, nr, pb)
        # and a call's box is its index in the channel over the calls per box
        np.testing.assert_array_equal(box, np.arange(nc[c]) // pb)


@pytest.mark.parametrize("fp32", [False, True])
def test_stratified_bin_and_fraction_big_int(oracle_lib, fp32):
    d, n, s = 3, 16, 2
    p = _flat_strat(d, n, 1, s, fp32)
    o = oracle_lib.Oracle(p)
    N = 4096
    nr, pb = _layout(oracle_lib, N, d, s)  # one channel: N_c = N
    tr = o.trace(N, 2, 0, pb * nr**d)
    for q in range(0, pb * nr**d, 5):
        box = q // pb
        for k in range(d):
            b = (box // nr**k) % nr
            u = int(tr["words"][q, k])
            Rn = ((b << 32) | u) * n
            j, rem = divmod(Rn, nr << 32)
            assert tr["bins"][q, 0, k] == j
            frac = Fraction(2 * rem + 1, 2 * (nr << 32))
            x = (j + frac) / n  # flat grid, identity channel
            got = Fraction(float(tr["p"][q, k]))
            if fp32:
                assert abs(got - x) <= Fraction(1, n * 2**24)
            elif nr & (nr - 1) == 0:
                assert got == x
            else:
                assert abs(got - x) <= Fraction(2 ** -52) * x


def _c1_wide():
    p = W.config1()
    cl = p.chan_loc + np.array([[0.03, -0.02], [-0.02, 0.04]])
    return p.with_(chan_loc=cl, chan_width=p.chan_width * 1.6, name="c1_wide")


def test_stratified_pulls(oracle_lib):
    p = _c1_wide().with_(strat=2)
    I = cf.integral(p)
    z = []
    for s in range(4000, 4200):
        o = oracle_lib.Oracle(p.with_(seed=s))
        o.sample_iteration(4000)
        z.append((o.history[0, 0] - I) / o.history[0, 1])
    z = np.array(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(len(z)), z.mean()
    assert 0.8 < z.std(ddof=1) < 1.25, z.std(ddof=1)


def test_stratified_error_below_uniform(oracle_lib):
    p = _c1_wide()
    sig = {}
    for strat in (0, 2):
        o = oracle_lib.Oracle(p.with_(strat=strat))
        o.sample_iteration(20_000)
        sig[strat] = o.history[0, 1]
        N = o.history[0, 2]
    assert sig[2] < 0.5 * sig[0], sig
    # both estimate the same integral
    I = cf.integral(p)
    o = oracle_lib.Oracle(p.with_(strat=2))
    o.sample_iteration(20_000)
    assert abs(o.history[0, 0] - I) < 5 * o.history[0, 1]


@pytest.mark.parametrize("maker,s", [(_c1_wide, 2), (_c1_wide, 5), (W.config2, 3)])
def test_box_variance_exact(oracle_lib, maker, s):
    """V_c of a stratified pass against exact rational arithmetic over the
    pass's own weights (re-derived call by call with the trace): per box of m
    calls (call i_c in box floor(i_c / m)), sum w^2 - (sum w)^2 / k over its k
    weights, summed over boxes, times m/(m-1), over N_c.  A wrong box split, a
    dropped factor or a mean over the wrong count fails it; so would the
    cancellation of S2 - Q/m in floating point, at the spreads of C1."""
    p = maker().with_(strat=s)
    o = oracle_lib.Oracle(p)
    N = 4000
    o.sample_iteration(N)
    nc = o.alloc[:-1]  # calls per channel (the last entry is their total)
    starts = np.concatenate([[0], np.cumsum(nc[:-1])])
    tr = o.trace(N, 0, 0, int(nc.sum()))
    st = o.channel_stats
    for c in range(p.n_channels):
        nr, m = _layout(oracle_lib, int(nc[c]), p.dim, s)
        w = tr["w"][starts[c]:starts[c] + nc[c]]
        assert np.all(np.isfinite(w)) and len(w) == m * nr**p.dim
        ssw = Fraction(0)
        for b in range(nr**p.dim):
            box = [Fraction(float(x)) for x in w[b * m:(b + 1) * m]]
            ssw += sum(x * x for x in box) - sum(box) ** 2 / len(box)
        v = float(Fraction(m, m - 1) * ssw / int(nc[c]))
        assert v > 0
        assert abs(st[c, 6] - v) <= 1e-13 * v, (c, st[c, 6], v)
