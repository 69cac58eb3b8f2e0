"""Pseudo-stratified passes on the GPU (Sec. 3.3; reading R30) against the
oracle: the layout (calls per channel), every call's words, box, bins, point
and weight, and the pass (estimate, box-variance error, per-channel sums,
per-bin sums) over adapting iterations; with Philox words and MRG32k3a
streams; in FP64 and precision mode."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import inject, pair, random_alpha, random_edges, rel

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def _problems():
    return {
        "C1_s2": W.config1().with_(strat=2),
        "C2_s3": W.config2().with_(strat=3),
        "mixed_d10_K12_s2": W.mixed_problem(10, 8, 4, 100, seed=31).with_(strat=2),
        "C2_s2_mrg": W.config2().with_(strat=2, rng=1),
    }


@pytest.mark.parametrize("name", list(_problems()))
def test_stratified_calls_match_oracle(name):
    p = _problems()[name]
    gpu, orc = pair(p)
    rng = np.random.default_rng(600)
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins),
           random_alpha(rng, p.n_channels))
    N = 1_000_000
    gpu.sample_iteration(N)
    orc.sample_iteration(N, THREADS)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    ntot = int(orc.alloc[-1])
    count = 1500
    nw = p.dim
    for first in (0, ntot // 2, ntot - count):
        g = gpu.trace(N, 1, first, count, n_words=nw)
        o = orc.trace(N, 1, first, count, n_words=nw)
        np.testing.assert_array_equal(g["words"], o["words"])
        np.testing.assert_array_equal(g["chan"], o["chan"])
        idx = g["chan"][:, None, None].repeat(p.dim, 2)
        np.testing.assert_array_equal(np.take_along_axis(g["bins"], idx, 1),
                                      np.take_along_axis(o["bins"], idx, 1))
        ok = ~np.any(o["near"], axis=(1, 2))
        assert rel(g["p"][ok], o["p"][ok]) < 1e-12 or np.max(np.abs(g["p"][ok] - o["p"][ok])) < 1e-12
        assert rel(g["w"][ok], o["w"][ok]) < 1e-10


@pytest.mark.parametrize("name", ["C1_s2", "C2_s3", "mixed_d10_K12_s2", "C2_s2_mrg"])
def test_stratified_passes_match_oracle(name):
    p = _problems()[name]
    gpu, orc = pair(p)
    N = 400_000
    for it in range(3):
        gpu.sample_iteration(N)
        orc.sample_iteration(N, THREADS)
        np.testing.assert_array_equal(gpu.alloc, orc.alloc)
        hg, ho = gpu.history[it], orc.history[it]
        assert rel(hg[0], ho[0]) < 1e-12 * 10 ** it
        assert rel(hg[1], ho[1]) < 1e-9 * 10 ** it  # the box-variance error
        assert hg[2] == ho[2]
        if it == 0:
            sg, so = gpu.channel_stats, orc.channel_stats
            assert rel(sg[:, [0, 1, 2]], so[:, [0, 1, 2]]) < 1e-11
            # V_c = m/(m-1) SSW / N_c, SSW = sum over boxes of the squared
            # deviations from the box mean.  Weights within a relative delta
            # of each other move SSW by at most 2 delta sqrt(SSW S2) +
            # delta^2 S2 (Cauchy-Schwarz over the calls, then the boxes);
            # delta = 1e-10 is the per-call bar, m/(m-1) <= 2.  Channels
            # whose weights barely spread inside the boxes (V_c near 1e-28
            # with S2/SSW near 1e22) only keep that bound.
            nc = orc.alloc[:-1].astype(np.float64)
            ssw, s2, delta = so[:, 6] * nc, so[:, 1], 1e-10
            bound = 2.0 / nc * (2 * delta * np.sqrt(ssw * s2) + delta**2 * s2)
            assert np.all(np.abs(sg[:, 6] - so[:, 6]) <= bound), (sg[:, 6], so[:, 6], bound)
            m = orc.hist > 0
            r = np.abs(gpu.hist[m] - orc.hist[m]) / orc.hist[m]
            assert r.max() < 2.5e-10 and np.quantile(r, 0.999) < 1e-12
        gpu.refine()
        orc.refine()


def test_stratified_precision_mode():
    p = W.mixed_problem(6, 4, 3, 40, seed=37, precision=1).with_(strat=2)
    gpu, orc = pair(p)
    for _ in range(2):
        gpu.sample_iteration(500_000)
        orc.sample_iteration(500_000, THREADS)
        np.testing.assert_array_equal(gpu.alloc, orc.alloc)
        gpu.refine()
        orc.refine()
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < 1e-5
    assert rel(gpu.history[:, 1], orc.history[:, 1]) < 1e-3


def test_stratified_unweighting_samples_importance_wise():
    p = W.config1().with_(strat=2)
    gpu, orc = pair(p)
    for _ in range(2):
        gpu.sample_iteration(10_000)
        orc.sample_iteration(10_000)
        gpu.refine()
        orc.refine()
    gpu.sample_iteration(10_000)
    orc.sample_iteration(10_000)
    orc.edges = gpu.edges
    orc.wmax = gpu.history[-1, 3]
    ev_g, st_g = gpu.unweight(2000, batch=4096)
    ev_o, st_o = orc.unweight(2000, batch=4096)
    assert st_o["accept_ties"] == 0
    assert st_g["trials"] == st_o["trials"]
    assert np.max(np.abs(ev_g.cpu().numpy() - ev_o)) < 1e-12
