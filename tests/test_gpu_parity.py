"""Parity of the HIP sample pass with the FP64 CPU oracle.

Bit-exact: Philox words, channel of every call, the call's own bins.  FP64
mode: other-channel bins identical except where the oracle flags the point as
within 1e-12 of a bin edge; weights, integral estimates, histograms, grids
and channel weights within 1e-12 relative.  FP32-mixed mode: integral within
1e-5 relative of the oracle run with the same FP32 rules.
"""
import math

import numpy as np
import pytest

import closed_forms as cf
import workloads as W
from gpu_util import inject, pair, random_alpha, random_edges, rel

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _problems():
    return {
        "C1": W.config1(),
        "C2": W.config2(),
        "mixed_d10_K12": W.mixed_problem(10, 8, 4, 100, seed=31),
        "C3_fp64": W.config3(precision=0),
        "gauss_d3_K5_n17": W.gauss_mixture(3, 5, 17, seed=32),
        "const_d4_K3": W.constant_problem(4, 3, 16),
    }


@pytest.mark.parametrize("name", list(_problems()))
def test_trace_bit_exact_fp64(name):
    p = _problems()[name]
    gpu, orc = pair(p)
    rng = np.random.default_rng(100)
    fp32 = p.precision != 0
    e = random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=fp32)
    a = random_alpha(rng, p.n_channels)
    inject(gpu, orc, e, a)
    N = 20_000 + 37
    count = 3000
    firsts = [0, N // 2 - count // 2, N + p.n_channels * 10 - count - 5]
    nw = 4 * ((p.dim + 3 + 3) // 4)
    for first in firsts:
        first = max(0, min(first, N - count))
        g = gpu.trace(N, 3, first, count, n_words=nw)
        o = orc.trace(N, 3, first, count, n_words=nw)
        np.testing.assert_array_equal(g["words"], o["words"])
        np.testing.assert_array_equal(g["chan"], o["chan"])
        own = np.take_along_axis(g["bins"], g["chan"][:, None, None].repeat(p.dim, 2), 1)[:, 0]
        own_o = np.take_along_axis(o["bins"], o["chan"][:, None, None].repeat(p.dim, 2), 1)[:, 0]
        np.testing.assert_array_equal(own, own_o)
        diff = g["bins"] != o["bins"]
        assert not np.any(diff & (o["near"] == 0)), "other-channel bin differs away from an edge"
        ok = ~np.any(diff, axis=(1, 2))
        # per call: p and w carry the conditioning of the maps (tan near its
        # pole); the 1e-12 bar applies to the integral estimates below
        assert np.max(np.abs(g["p"][ok] - o["p"][ok])) < 1e-12
        assert rel(g["w"][ok], o["w"][ok]) < 1e-10


@pytest.mark.parametrize("name", ["C1", "C2", "mixed_d10_K12", "C3_fp64", "gauss_d3_K5_n17"])
@pytest.mark.parametrize("N", [None, 12_345])
def test_single_pass_parity_fp64(name, N):
    p = _problems()[name]
    gpu, orc = pair(p)
    rng = np.random.default_rng(7)
    e = random_edges(rng, p.n_channels, p.dim, p.n_bins)
    a = random_alpha(rng, p.n_channels)
    inject(gpu, orc, e, a)
    N = N or min(p.n_points or 100_000, 200_000)
    gpu.sample_iteration(N)
    orc.sample_iteration(N, 8)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    hg, ho = gpu.history[0], orc.history[0]
    assert rel(hg[0], ho[0]) < FP64_TOL
    assert rel(hg[1], ho[1]) < 1e-9
    assert hg[2] == ho[2] and hg[4] == ho[4]
    assert rel(hg[3], ho[3]) < FP64_TOL
    sg, so = gpu.channel_stats, orc.channel_stats
    assert rel(sg[:, [0, 1, 2, 4, 5]], so[:, [0, 1, 2, 4, 5]]) < FP64_TOL
    hgs, hos = gpu.hist, orc.hist
    m = hos > 0
    assert np.all((hgs > 0) == m)
    assert rel(hgs[m], hos[m]) < 1e-11


@pytest.mark.parametrize("name", ["C1", "C2", "mixed_d10_K12"])
def test_refine_parity_fp64(name):
    p = _problems()[name]
    gpu, orc = pair(p)
    for it in range(3):
        gpu.sample_iteration(50_000)
        orc.sample_iteration(50_000, 8)
        gpu.refine()
        orc.refine()
        assert rel(gpu.edges, orc.edges) < FP64_TOL
        assert rel(gpu.alpha, orc.alpha) < FP64_TOL
        assert np.all(np.diff(gpu.edges, axis=-1) > 0)
        assert gpu.alpha.sum() == pytest.approx(1.0, rel=1e-14)
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < FP64_TOL


def test_config1_full_end_to_end():
    p = W.config1()
    gpu, orc = pair(p)
    for _ in range(p.n_iterations):
        gpu.sample_iteration(p.n_points)
        orc.sample_iteration(p.n_points)
        gpu.refine()
        orc.refine()
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < FP64_TOL
    rg, ro = gpu.result(), orc.result()
    assert rel(rg["integral"], ro["integral"]) < FP64_TOL
    I = cf.integral(p)
    # C1's channels match its peaks, so an iteration's weights can be constant
    # per channel up to rounding: its variance W - E^2 then rounds to <= 0 and
    # is clamped to 0, and the combined result is that iteration's estimate
    # with error 0.  What remains is the rounding of the weights (the oracle
    # itself is 4e-15 off the closed form), hence the absolute 1e-14.
    assert abs(rg["integral"] - I) < 5 * rg["error"] + 1e-14


def test_config2_full_end_to_end():
    p = W.config2()
    gpu, orc = pair(p)
    for _ in range(p.n_iterations):
        gpu.sample_iteration(p.n_points)
        orc.sample_iteration(p.n_points, 16)
        gpu.refine()
        orc.refine()
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < FP64_TOL
    assert rel(gpu.edges, orc.edges) < 1e-11
    I = cf.integral(p)
    r = gpu.result(5)
    assert abs(r["integral"] - I) < 5 * r["error"]


def test_precision_mode_vs_oracle():
    p = W.mixed_problem(10, 12, 4, 100, seed=33, precision=1)
    gpu, orc = pair(p)
    for _ in range(3):
        gpu.sample_iteration(200_000)
        orc.sample_iteration(200_000, 16)
        gpu.refine()
        orc.refine()
    hg, ho = gpu.history, orc.history
    assert rel(hg[:, 0], ho[:, 0]) < 1e-5
    e = gpu.edges
    assert np.all(e.astype(np.float32).astype(np.float64) == e)


def test_zero_variance_alpha_star_full_c3_size():
    """At the full C3 size: flat grids and alpha* make every weight I up to
    the allocation rounding (|N_c/N - alpha*_c| <= 1/N), for both modes."""
    for prec in (0, 1):
        p = W.config3(precision=prec)
        from gpu_util import mcv
        gpu = mcv().Integrator(p)
        astar = np.array(cf.zero_variance_alpha(p))
        gpu.set_state_for_test(alpha=astar)
        N = p.n_points
        gpu.sample_iteration(N)
        nc = gpu.alloc
        alpha = nc[:-1] / nc[-1]
        spread = max(np.max(astar / alpha) - 1, 1 - np.min(astar / alpha))
        I = cf.integral(p)
        E = gpu.history[0, 0]
        tol = spread + (1e-12 if prec == 0 else 2e-6)
        assert abs(E - I) / I < tol
        st = gpu.channel_stats
        wmax = st[:, 2].max()
        assert wmax / I < 1 + tol + (0 if prec == 0 else 1e-4)
