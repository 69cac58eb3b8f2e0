"""GPU tests of the rest of the boundary: unweighting (Sec. 2 eq. efficiency,
Sec. 3.5 event generation), iteration combination, checkpoint / resume,
determinism of the pass, and precision-mode unweighting statistics."""
import numpy as np
import pytest

import closed_forms as cf
import workloads as W
from gpu_util import mcv, pair, rel

pytestmark = pytest.mark.gpu


def _adapt(gpu, orc, p, n_iter, N):
    for _ in range(n_iter):
        gpu.sample_iteration(N)
        orc.sample_iteration(N, 8)
        gpu.refine()
        orc.refine()
    # last pass without refinement: alpha = N_c / N_tot on both sides
    gpu.sample_iteration(N)
    orc.sample_iteration(N, 8)


@pytest.mark.parametrize("maker,N,n_ev,batch", [
    (W.config1, 10_000, 5_000, 4096),
    (W.config2, 200_000, 3_000, 65_536),
    (lambda: W.mixed_problem(6, 4, 3, 40, seed=51), 100_000, 2_000, 8_192),
    # batches that end in a partial 1024-trial compaction tile, or are one
    (W.config1, 10_000, 3_000, 5_000),
    (lambda: W.mixed_problem(6, 4, 3, 40, seed=52), 100_000, 500, 700),
])
def test_unweight_parity_fp64(maker, N, n_ev, batch):
    p = maker()
    gpu, orc = pair(p)
    _adapt(gpu, orc, p, 3, N)
    # identical state: grids from the GPU, w_max of the GPU's last pass
    orc.edges = gpu.edges
    orc.wmax = gpu.history[-1, 3]
    import torch
    ev_g, st_g = gpu.unweight(n_ev, batch=batch)
    ev_o, st_o = orc.unweight(n_ev, batch=batch)
    # no accept decision of the oracle is within 1e-12 of its threshold, so
    # both sides must keep the same trials
    assert st_o["accept_ties"] == 0
    assert st_g["trials"] == st_o["trials"]
    # "w > w_max" is decided at the last ulp for weights that sit at the
    # maximum (C1's adapted weights cluster there); the two sides round exp
    # differently, so an overweight flag may differ only where the oracle's
    # weight ties the batch's w_max within 1e-12 (flagged per event)
    assert abs(st_g["n_overweight"] - st_o["n_overweight"]) <= st_o["overweight_ties"]
    assert st_g["w_max"] == pytest.approx(st_o["w_max"], rel=1e-12)
    ev_g = ev_g.cpu().numpy()
    assert np.max(np.abs(ev_g - ev_o)) < 1e-12
    # a second call continues the trial sequence on both sides
    ev_g2, st_g2 = gpu.unweight(n_ev // 2, batch=batch)
    ev_o2, st_o2 = orc.unweight(n_ev // 2, batch=batch)
    assert st_g2["trials"] == st_o2["trials"]
    assert np.max(np.abs(ev_g2.cpu().numpy() - ev_o2)) < 1e-12
    assert not np.allclose(ev_g2.cpu().numpy()[:, :10], ev_g[:, :10])


@pytest.mark.parametrize("maker,N,n_ev,batch", [
    (lambda: W.mixed_problem(6, 4, 3, 40, seed=53, precision=1), 200_000, 2_000, 8_192),
    (lambda: W.config2().with_(precision=1), 200_000, 3_000, 65_536),
])
def test_unweight_parity_fp32_mode(maker, N, n_ev, batch):
    """Precision mode against the oracle under the FP32 rules, from the same
    state (FP32-snapped grids and weights injected on both sides, one pass):
    the channel and point of every trial are the same, and the weights, FP32
    arithmetic on the GPU, agree with the oracle's to about 1e-5 relative.
    So an accept decision within 1e-4 of its threshold counts as a tie; up to
    the first tie both sides keep the same trials in the same order, with the
    events equal to FP32 precision."""
    from gpu_util import inject, random_alpha, random_edges
    p = maker()
    gpu, orc = pair(p)
    rng = np.random.default_rng(700)
    inject(gpu, orc, random_edges(rng, p.n_channels, p.dim, p.n_bins, fp32=True, spread=1.0),
           random_alpha(rng, p.n_channels))
    gpu.sample_iteration(N)
    orc.sample_iteration(N, 8)
    np.testing.assert_array_equal(gpu.alloc, orc.alloc)
    orc.wmax = gpu.history[-1, 3]
    ev_g, st_g = gpu.unweight(n_ev, batch=batch)
    ev_o, st_o = orc.unweight(n_ev, batch=batch, tie_rel=1e-4)
    k = st_o["first_tie"]
    assert k >= n_ev // 4, st_o  # ties are rare: most of the sequence is compared
    ev_g = ev_g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(ev_g[:, :k] - ev_o[:, :k])) < 2e-6
    if st_o["accept_ties"] == 0:
        assert st_g["trials"] == st_o["trials"]


def test_unweight_fp32_follows_integrand_d2():
    """Precision mode: accepted events follow f/I (chi^2 in 10x10 cells) and
    the acceptance matches <w>/w_max."""
    from scipy.stats import chi2
    p = W.config1().with_(precision=1)
    gpu = mcv().Integrator(p)
    for _ in range(4):
        gpu.sample_iteration(20_000)
        gpu.refine(mcv().MCV_REFINE_GRID)
    gpu.sample_iteration(20_000)
    n_ev = 40_000
    ev, st = gpu.unweight(n_ev, batch=16_384)
    ev = ev.cpu().numpy().astype(np.float64)
    assert ev.shape == (2, n_ev)
    I = cf.integral(p)
    edges = np.linspace(0, 1, 11)
    H, _, _ = np.histogram2d(ev[0], ev[1], bins=[edges, edges])
    exp = np.array([[cf.cell_mass(p, (edges[a], edges[b]), (edges[a + 1], edges[b + 1])) / I
                     for b in range(10)] for a in range(10)]) * n_ev
    m = exp > 5
    stat = float(((H[m] - exp[m]) ** 2 / exp[m]).sum())
    assert chi2.sf(stat, int(m.sum()) - 1) > 1e-4
    assert st["efficiency"] == pytest.approx(I / st["w_max"], rel=0.05)


def test_result_combination_matches_oracle():
    p = W.config2()
    gpu, orc = pair(p)
    for _ in range(4):
        gpu.sample_iteration(100_000)
        orc.sample_iteration(100_000, 8)
        gpu.refine()
        orc.refine()
    for first in (0, 2, 3):
        rg, ro = gpu.result(first), orc.result(first)
        assert rel(rg["integral"], ro["integral"]) < 1e-12
        assert rel(rg["error"], ro["error"]) < 1e-9
        assert rg["chi2_ndf"] == pytest.approx(ro["chi2_ndf"], rel=1e-6, abs=1e-12)
        assert rg["n_iter"] == ro["n_iter"]


def test_pass_is_deterministic():
    """Same state, same iteration index: bit-identical sums (ordered
    workgroup partials)."""
    p = W.mixed_problem(10, 12, 4, 100, seed=52, precision=1)
    a = mcv().Integrator(p)
    b = mcv().Integrator(p)
    for g in (a, b):
        g.sample_iteration(500_000)
    assert np.array_equal(a.history, b.history)
    assert np.array_equal(a.channel_stats[:, [0, 1, 2]], b.channel_stats[:, [0, 1, 2]])


def test_checkpoint_resume():
    p = W.config2()
    a = mcv().Integrator(p)
    for _ in range(3):
        a.sample_iteration(200_000)
        a.refine()
    blob = a.save_state()
    b = mcv().Integrator(p)
    b.load_state(blob)
    for g in (a, b):
        for _ in range(2):
            g.sample_iteration(200_000)
            g.refine()
    ha, hb = a.history, b.history
    assert ha.shape == hb.shape == (5, 5)
    assert rel(ha[:, 0], hb[:, 0]) < 1e-13
    assert rel(a.edges, b.edges) < 1e-13
    # a state from another problem shape is refused
    c = mcv().Integrator(W.config1())
    with pytest.raises(mcv().MCVError):
        c.load_state(blob)


def test_state_errors_on_gpu():
    p = W.config1()
    g = mcv().Integrator(p)
    M = mcv()
    with pytest.raises(M.MCVError) as e:
        g.result(0)
    assert e.value.status == M.MCV_E_STATE
    with pytest.raises(M.MCVError) as e:
        g.refine()
    assert e.value.status == M.MCV_E_STATE
    with pytest.raises(M.MCVError) as e:
        g.sample_iteration(5)  # below K * min_calls
    assert e.value.status == M.MCV_E_INVALID
    with pytest.raises(M.MCVError) as e:
        g.set_state_for_test(edges=np.zeros((2, 2, 21)))
    assert e.value.status == M.MCV_E_INVALID


def test_min_calls_floor_and_tiny_pass():
    """N = K * min_calls exactly; a channel with vanishing weight keeps the
    floor (Sec. 3.4 safeguard) and the pass still estimates I."""
    p = W.gauss_mixture(2, 3, 8, seed=53)
    gpu, orc = pair(p)
    alpha = np.array([0.999, 0.0005, 0.0005])
    gpu.set_state_for_test(alpha=alpha)
    orc.alpha = alpha
    gpu.sample_iteration(30)
    orc.sample_iteration(30)
    assert list(gpu.alloc) == list(orc.alloc)
    assert np.all(gpu.alloc[:-1] >= 10)
    assert rel(gpu.history[0, 0], orc.history[0, 0]) < 1e-12
