"""Channel equivalences on the GPU (Sec. 3.5: equivalent channels pool the
bin weights their grids adapt to) against the oracle: after the same pass,
the rebinned grids agree to 1e-12 for random lists of equivalences (trivial
entries, permuted axes, every mode), and stay in step over iterations."""
import numpy as np
import pytest

import workloads as W
from gpu_util import inject, pair, random_alpha, random_edges, rel

pytestmark = pytest.mark.gpu


def _random_list(rng, K, d, n_rows, with_invariant=True):
    rows = []
    for c in range(K):  # the trivial entry for most channels
        if rng.random() < 0.8:
            rows.append([c, c] + list(range(d)) + [0] * d)
    for _ in range(n_rows):
        c, c2 = rng.integers(0, K, 2)
        perm = rng.permutation(d)
        modes = rng.choice([0, 1, 2, 3] if with_invariant else [0, 1, 2], d,
                           p=[0.4, 0.3, 0.25, 0.05] if with_invariant else [0.4, 0.3, 0.3])
        rows.append([int(c), int(c2)] + [int(a) for a in perm] + [int(m) for m in modes])
    order = rng.permutation(len(rows))
    return [rows[i] for i in order]


@pytest.mark.parametrize("name,maker", [
    ("mixed_d10_K12", lambda: W.mixed_problem(10, 8, 4, 100, seed=31)),
    ("C2", W.config2),
    ("mixed_fp32", lambda: W.mixed_problem(6, 4, 3, 40, seed=34, precision=1)),
])
def test_equivalences_match_oracle(name, maker):
    p = maker()
    gpu, orc = pair(p)
    rng = np.random.default_rng(400)
    fp32 = p.precision != 0
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=fp32),
           random_alpha(rng, p.n_channels))
    eq = _random_list(rng, p.n_channels, p.dim, 3 * p.n_channels)
    gpu.set_equivalences(eq)
    orc.set_equivalences(eq)
    tol = 1e-12 if not fp32 else 0.0
    for it in range(3):
        gpu.sample_iteration(200_000)
        orc.sample_iteration(200_000, 8)
        gpu.refine()
        orc.refine()
        eg, eo = gpu.edges, orc.edges
        if fp32:
            # FP32-snapped grids from sums that agree to ~1e-6: the same to a
            # few FP32 ulps where a rounding boundary falls between them
            assert np.max(np.abs(eg - eo)) < 1e-5
        else:
            assert rel(eg, eo) < 1e-12 * (10 ** it)
        assert np.all(np.diff(eg, axis=-1) > 0)


def test_equivalences_removed_and_refused():
    p = W.gauss_mixture(3, 3, 16, seed=41)
    gpu, orc = pair(p)
    M = __import__("gpu_util").mcv()
    with pytest.raises(M.MCVError) as e:
        gpu.set_equivalences([[0, 3, 0, 1, 2, 0, 0, 0]])
    assert e.value.status == M.MCV_E_INVALID
    with pytest.raises(M.MCVError):
        gpu.set_equivalences([[0, 1, 0, 0, 2, 0, 0, 0]])
    gpu.set_equivalences([[0, 1, 0, 1, 2, 1, 1, 1]])
    gpu.set_equivalences([])  # removed: plain rebinning again
    gpu.sample_iteration(50_000)
    orc.sample_iteration(50_000)
    gpu.refine()
    orc.refine()
    assert rel(gpu.edges, orc.edges) < 1e-12


def test_mirrored_channels_get_mirrored_grids_on_gpu():
    pk = np.array([[1, 2], [1, 2]], np.int32)
    pl = np.array([[0.3, 0.2], [0.7, 0.8]])
    pw = np.array([[0.07, 0.05], [0.07, 0.05]])
    p = W.Problem(2, 24, pk, pl, pw, np.array([0.5, 0.5]), pk.copy(), pl.copy(), pw.copy(),
                  seed=11, name="mirror")
    gpu, _ = pair(p)
    gpu.set_equivalences([[0, 0, 0, 1, 0, 0], [0, 1, 0, 1, 1, 1],
                          [1, 1, 0, 1, 0, 0], [1, 0, 0, 1, 1, 1]])
    for _ in range(3):
        gpu.sample_iteration(100_000)
        gpu.refine()
        e = gpu.edges
        np.testing.assert_allclose(e[1], 1.0 - e[0][:, ::-1], rtol=0, atol=1e-13)
