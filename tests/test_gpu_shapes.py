"""Parity at the edges of the problem shapes the library accepts: one
dimension, one channel and one bin; the largest bin count (start bins up to
255 in the hint-cell records); dimensions that do not fill their kernel
bucket (guarded axes) and the largest bucket; Breit-Wigner channels of the
smallest width next to flat axes; Gaussian channels with a width per axis.  Per call: Philox words, channels and own
bins bit-exact, other-channel bins bit-exact away from the oracle's near-edge
flags; per pass: FP64 integral estimates within 1e-12 of the oracle, FP32
mode within 1e-5 of the oracle run with the same FP32 rules."""
import numpy as np
import pytest

import workloads as W
from gpu_util import inject, pair, random_alpha, random_edges, rel

pytestmark = pytest.mark.gpu


def _shapes():
    return {
        "d1_K1_n1": W.gauss_mixture(1, 1, 1, seed=51),
        "d1_K3_n256": W.gauss_mixture(1, 3, 256, seed=52),
        "d3_K4_n256": W.mixed_problem(3, 2, 2, 256, seed=53),
        "d13_K5_n40": W.mixed_problem(13, 3, 2, 40, seed=54),
        "d32_K3_n8": W.mixed_problem(32, 2, 1, 8, seed=55),
        "bw_flat_d11_K64_n37": W.batch_job(4_000_100).with_(n_bins=37),
        # Gaussian on every axis with a width per axis: the general density
        # kernel with the linear hint map (one width per channel takes the
        # isotropic form)
        "aniso_d7_K6_n60": W.gauss_mixture(7, 6, 60, seed=56, anisotropic=True),
    }


@pytest.mark.parametrize("name", list(_shapes()))
def test_trace_bit_exact(name):
    p = _shapes()[name]
    if p.n_channels > 64 or p.dim * p.n_channels > 2000:
        pytest.skip("trace output size")
    gpu, orc = pair(p)
    rng = np.random.default_rng(60)
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins),
           random_alpha(rng, p.n_channels))
    N = 5_000 + 13
    count = 1500
    nw = 4 * ((p.dim + 3 + 3) // 4)
    for first in (0, N - count):
        g = gpu.trace(N, 2, first, count, n_words=nw)
        o = orc.trace(N, 2, first, count, n_words=nw)
        np.testing.assert_array_equal(g["words"], o["words"])
        np.testing.assert_array_equal(g["chan"], o["chan"])
        diff = g["bins"] != o["bins"]
        assert not np.any(diff & (o["near"] == 0)), "a bin differs away from an edge"
        ok = ~np.any(diff, axis=(1, 2))
        assert np.max(np.abs(g["p"][ok] - o["p"][ok])) < 1e-12
        assert rel(g["w"][ok], o["w"][ok]) < 1e-10


@pytest.mark.parametrize("name", list(_shapes()))
def test_single_pass_parity(name):
    p = _shapes()[name]
    gpu, orc = pair(p)
    rng = np.random.default_rng(61)
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins),
           random_alpha(rng, p.n_channels))
    N = 40_000
    gpu.sample_iteration(N)
    orc.sample_iteration(N, 8)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    assert rel(gpu.history[0, 0], orc.history[0, 0]) < 1e-12
    gpu.refine()
    orc.refine()
    assert rel(gpu.edges, orc.edges) < 1e-11
    gpu.sample_iteration(N)
    orc.sample_iteration(N, 8)
    assert rel(gpu.history[1, 0], orc.history[1, 0]) < 1e-12


@pytest.mark.parametrize("name", ["d1_K3_n256", "d13_K5_n40", "bw_flat_d11_K64_n37", "aniso_d7_K6_n60"])
def test_precision_mode(name):
    p = _shapes()[name].with_(precision=1)
    gpu, orc = pair(p)
    for _ in range(2):
        gpu.sample_iteration(40_000)
        orc.sample_iteration(40_000, 8)
        gpu.refine()
        orc.refine()
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < 1e-5
