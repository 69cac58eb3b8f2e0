"""Parity of the kernel the sample pass actually runs (k_sample: grouped
hint-cell lookups, the term-bound skip of channel terms that cannot change g,
the FP64 partial-exponent skip, per-lane sums folded every 16 rounds) with the
FP64 CPU oracle:

* call by call, through the kernel's trace instantiation (the same template
  and grid, writing f, g, w for a window of calls) -- Sec. 3.5 eq. g(p) and
  eq. vamp-master;
* at the full loop shape: passes of 1.6e7 calls, where every lane of every
  workgroup folds its per-lane sums at least twice, compared on the estimate, the per-channel
  sums of w and w^2, the largest weights and the per-bin sums of w^2
  (Sec. 3.1, Sec. 3.2 eq. 31);
* in precision mode: Philox words, channels and own bins bit-exact; other
  channels' bins equal to the bin that holds the GPU's own point among the
  FP32-rounded p-space edges (computed here from the oracle's maps), except
  within one FP32 ulp of such an edge.
"""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import inject, pair, random_alpha, random_edges, rel

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
FULL_N = 16_000_000


def _problems():
    return {
        "C3_fp64": W.config3(precision=0),
        "mixed_d10_K12": W.mixed_problem(10, 8, 4, 100, seed=31),
        "C2": W.config2(),
        "C1": W.config1(),
    }


def _windows(N, count):
    return [0, N // 2 - count // 2, N - count]


@pytest.mark.parametrize("name", list(_problems()))
def test_timed_kernel_calls_match_oracle_fp64(name):
    p = _problems()[name]
    gpu, orc = pair(p)
    rng = np.random.default_rng(300)
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins),
           random_alpha(rng, p.n_channels))
    N, count = 8_000_000, 2000
    for first in _windows(N, count):
        t = gpu.sample_trace(N, 4, first, count)
        o = orc.trace(N, 4, first, count)
        g = gpu.trace(N, 4, first, count)  # every channel term, no skips
        ok = ~np.any(o["near"], axis=(1, 2))
        assert ok.mean() > 0.9
        for key in ("f", "g", "w"):
            assert rel(t[key][ok], o[key][ok]) < 1e-10, key
            # the skipped terms are below half an ulp of the running sums:
            # the timed kernel and the full evaluation agree to rounding order
            assert rel(t[key], g[key]) < 1e-13, key


def _full_pass(p, seed):
    gpu, orc = pair(p)
    rng = np.random.default_rng(seed)
    fp32 = p.precision != 0
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=fp32),
           random_alpha(rng, p.n_channels))
    gpu.sample_iteration(FULL_N)
    orc.sample_iteration(FULL_N, THREADS)
    _, G = gpu.pass_timing(0)
    # calls per lane of a workgroup: the per-lane sums fold every 16 of them
    assert FULL_N / G / 256 >= 2 * 16
    return gpu, orc


def test_full_size_pass_matches_oracle_fp64():
    gpu, orc = _full_pass(W.config3(precision=0), 301)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    hg, ho = gpu.history[0], orc.history[0]
    assert rel(hg[0], ho[0]) < 1e-12
    assert rel(hg[1], ho[1]) < 1e-9
    assert rel(hg[3], ho[3]) < 1e-12
    assert hg[2] == ho[2] and hg[4] == ho[4]
    sg, so = gpu.channel_stats, orc.channel_stats
    for q in (0, 1, 2, 4, 5):  # S1, S2, w_max, E_c, W_c
        assert rel(sg[:, q], so[:, q]) < 1e-12, q
    hgs, hos = gpu.hist, orc.hist
    m = hos > 0
    assert np.all((hgs > 0) == m)
    # eq. 31's per-bin sums of w^2 are sums of positive terms, so each bin is
    # within twice the per-call bound on w (1e-10: the maps' conditioning
    # near an arctan pole, checked call by call above) plus summation order;
    # at 1.6e7 calls a few sparsely filled bins are dominated by such calls,
    # the rest agree at the estimate's 1e-12
    r = np.abs(hgs[m] - hos[m]) / hos[m]
    assert r.max() < 2.5e-10
    assert np.quantile(r, 0.999) < 1e-12


def test_full_size_pass_matches_oracle_fp32_mode():
    gpu, orc = _full_pass(W.config3(precision=1), 302)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    hg, ho = gpu.history[0], orc.history[0]
    assert rel(hg[0], ho[0]) < 1e-5
    assert hg[2] == ho[2] and hg[4] == ho[4]
    sg, so = gpu.channel_stats, orc.channel_stats
    assert rel(sg[:, 0].sum(), so[:, 0].sum()) < 1e-5
    assert rel(sg[:, 1].sum(), so[:, 1].sum()) < 1e-4


def _fp32_edge_counts(orc, p, edges, pts):
    """For every call, channel and axis: the number of interior p-space edges
    (the oracle's map of each x-space edge, rounded to FP32) at or below the
    point, and whether the point lies within one FP32 ulp of such an edge."""
    import oracle as O
    K, d, n = p.n_channels, p.dim, p.n_bins
    count = pts.shape[0]
    J = np.zeros((count, K, d), np.int64)
    near = np.zeros((count, K, d), bool)
    for c in range(K):
        for k in range(d):
            kind, loc, width = int(p.chan_kind[c, k]), float(p.chan_loc[c, k]), float(p.chan_width[c, k])
            P = np.array([O.map_forward(kind, loc, width, float(edges[c, k, j]))
                          for j in range(1, n)])
            P32 = P.astype(np.float32).astype(np.float64)
            x = pts[:, k]
            J[:, c, k] = np.searchsorted(P32, x, side="right")
            ulp = np.spacing(np.abs(P32).astype(np.float32)).astype(np.float64)
            dist = np.abs(x[:, None] - P32[None, :]) <= ulp[None, :]
            near[:, c, k] = dist.any(axis=1)
    return J, near


@pytest.mark.parametrize("name,maker", [
    ("C3", lambda: W.config3(precision=1)),
    ("mixed_d10_K12", lambda: W.mixed_problem(10, 8, 4, 100, seed=31, precision=1)),
    ("C2_fp32", lambda: W.config2().with_(precision=1)),
])
def test_trace_fp32_mode(name, maker):
    p = maker()
    gpu, orc = pair(p)
    rng = np.random.default_rng(303)
    edges = random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=True)
    inject(gpu, orc, edges, random_alpha(rng, p.n_channels))
    N, count = 1_000_003, 1500
    nw = 4 * ((p.dim + 3 + 3) // 4)
    for first in _windows(N, count):
        g = gpu.trace(N, 6, first, count, n_words=nw)
        o = orc.trace(N, 6, first, count, n_words=nw)
        np.testing.assert_array_equal(g["words"], o["words"])
        np.testing.assert_array_equal(g["chan"], o["chan"])
        idx = g["chan"][:, None, None].repeat(p.dim, 2)
        np.testing.assert_array_equal(np.take_along_axis(g["bins"], idx, 1),
                                      np.take_along_axis(o["bins"], idx, 1))
        # other channels: the bin of the GPU's own FP32 point among the
        # FP32-rounded p-space edges, exact away from a one-ulp window
        J, near = _fp32_edge_counts(orc, p, edges, g["p"])
        other = np.ones_like(near)
        other[np.arange(count), g["chan"], :] = False
        chk = other & ~near
        assert chk[other].mean() > 0.95
        np.testing.assert_array_equal(g["bins"][chk], J[chk])
        # the GPU's FP32 point is the oracle's to FP32 accuracy of the maps
        assert np.median(np.abs(g["p"] - o["p"])) < 1e-6
        # weights of the timed kernel in FP32 against the oracle's FP64 ones
        # where every bin agrees: FP32 evaluation of f and g at the same
        # point (relative rounding of exp2 of an exponent of at most ~30)
        t = gpu.sample_trace(N, 6, first, count)
        same = np.all(g["bins"] == o["bins"], axis=(1, 2))
        assert same.mean() > 0.9
        r = np.abs(t["w"][same] - o["w"][same]) / np.abs(o["w"][same])
        assert np.median(r) < 2e-6, np.median(r)
        assert np.quantile(r, 0.999) < 5e-5, np.quantile(r, 0.999)


@pytest.mark.parametrize("name,maker", [
    ("C3", lambda: W.config3(precision=1)),
    ("mixed_d10_K12", lambda: W.mixed_problem(10, 8, 4, 100, seed=31, precision=1)),
])
def test_timed_fp32_equals_direct_evaluation(name, maker):
    """The timed FP32 kernel -- hint-cell reads in groups, term-bound skips
    (reading R25), crowded hint cells first bounded by their largest density
    and walked only where that bound lets the term change g -- against the
    direct FP32 evaluation of eq. g(p) (Sec. 3.5) in the trace kernel, which
    adds every channel term with its exact bins: the same calls, on grids
    with bin widths over four decades, so that many hint cells hold several
    edges.  A density taken from the wrong bin, or a term dropped that could
    change g, moves w by far more than the rounding allowed here."""
    p = maker()
    gpu, _ = pair(p)
    rng = np.random.default_rng(304)
    edges = random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=True, spread=4.0)
    gpu.set_state_for_test(edges, random_alpha(rng, p.n_channels))
    N, count = 1_000_003, 4000
    for first in _windows(N, count):
        direct = gpu.trace(N, 7, first, count)
        timed = gpu.sample_trace(N, 7, first, count)
        # both FP32 at the same point: f and g differ by the rounding of
        # their association only (calls whose every term underflows, f = g
        # = 0, are zero or not finite on both sides alike)
        for key in ("f", "g", "w"):
            a, b = timed[key], direct[key]
            ok = np.isfinite(b) & (b != 0)
            np.testing.assert_array_equal(ok, np.isfinite(a) & (a != 0))
            assert ok.mean() > 0.9
            r = np.abs(a[ok] - b[ok]) / np.abs(b[ok])
            assert np.median(r) < 1e-6, (key, np.median(r))
            assert r.max() < 1e-5, (key, r.max())
