"""Pins of the oracle's sample pass, adaptation and result against what the
paper and the mathematics fix: closed-form integrals, the zero-variance
channel weights, the constant integrand, the normalisation of the
multi-channel density, the rebinning walk and the allocation rules.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import closed_forms as cf
import workloads as W

FLAT, GAUSS, BW = 0, 1, 2


# --------------------------------------------------------------------------
# Sec. 3.1 / 3.4: estimator and error
# --------------------------------------------------------------------------
def test_config1_full_matches_closed_form(oracle_lib):
    """C1 at full size: every iteration within 5 sigma of the closed form."""
    p = W.config1()
    o = oracle_lib.Oracle(p)
    I = cf.integral(p)
    for _ in range(p.n_iterations):
        o.sample_iteration(p.n_points)
        o.refine()
    h = o.history
    assert np.all(np.abs(h[:, 0] - I) <= 5 * h[:, 1] + 1e-15)
    r = o.result(0)
    assert abs(r["integral"] - I) <= 5 * r["error"] + 1e-15


def test_config2_reduced_matches_closed_form(oracle_lib):
    p = W.config2()
    o = oracle_lib.Oracle(p)
    I = cf.integral(p)
    for _ in range(3):
        o.sample_iteration(200_000, n_threads=8)
        o.refine()
    h = o.history
    assert np.all(np.abs(h[:, 0] - I) <= 5 * h[:, 1])
    # Each channel maps its peak exactly, so the flat grid is already optimal
    # and the channel weights carry the adaptation: eq. 15 alone drives the
    # error down by orders of magnitude (grid updates only add noise here).
    o2 = oracle_lib.Oracle(p)
    for _ in range(4):
        o2.sample_iteration(200_000, n_threads=8)
        o2.refine(oracle_lib.REFINE_ALPHA)
    h2 = o2.history
    assert np.all(np.abs(h2[:, 0] - I) <= 5 * h2[:, 1] + 1e-14)
    assert h2[-1, 1] < 0.01 * h2[0, 1]


def test_threaded_mode_matches_single_thread(oracle_lib):
    p = W.mixed_problem(5, 3, 2, 30, seed=21)
    a = oracle_lib.Oracle(p)
    b = oracle_lib.Oracle(p)
    a.sample_iteration(20_000, 1)
    b.sample_iteration(20_000, 7)
    assert b.history[0, 0] == pytest.approx(a.history[0, 0], rel=1e-14)
    assert b.history[0, 1] == pytest.approx(a.history[0, 1], rel=1e-12)
    np.testing.assert_allclose(b.hist, a.hist, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(b.channel_stats[:, 2], a.channel_stats[:, 2])


# --------------------------------------------------------------------------
# Zero-variance channel weights: with flat grids and alpha*_c = w_c M_c / I
# the multi-channel density equals f / I, so every weight equals I.  A dropped
# term, a wrong sign, index or a transposed operand in the weight breaks this.
# --------------------------------------------------------------------------
def test_config1_zero_variance_alpha(oracle_lib):
    p = W.config1()
    o = oracle_lib.Oracle(p)
    I = cf.integral(p)
    o.alpha = cf.zero_variance_alpha(p)  # (0.4, 0.6)
    o.sample_iteration(10_000)
    assert list(o.alloc) == [4000, 6000, 10000]
    E, sig = o.history[0, :2]
    assert E == pytest.approx(I, rel=2e-15)
    # V = N/(N-1) (<w^2> - <w>^2) in FP64 (Sec. 3.1) cannot resolve a variance
    # below the rounding of <w^2>: sigma sits at the floor sqrt(eps / N) * I.
    assert sig <= math.sqrt(4 * 2.2e-16 / 10_000) * I
    tr = o.trace(10_000, 0, 0, 10_000)
    np.testing.assert_allclose(tr["w"], I, rtol=5e-15)


@pytest.mark.parametrize("maker", [W.config2, lambda: W.mixed_problem(6, 5, 3, 40, seed=8),
                                   lambda: W.gauss_mixture(3, 4, 25, seed=9)])
def test_zero_variance_alpha_general(oracle_lib, maker):
    """alpha after allocation differs from alpha* by <= 0.5/N per channel, so
    w/I stays within [min alpha*/alpha, max alpha*/alpha]."""
    p = maker()
    o = oracle_lib.Oracle(p)
    I = cf.integral(p)
    astar = np.array(cf.zero_variance_alpha(p))
    N = 400_000
    o.alpha = astar
    o.sample_iteration(N)
    nc = o.alloc
    alpha = nc[:-1] / nc[-1]
    lo, hi = np.min(astar / alpha), np.max(astar / alpha)
    tr = o.trace(N, 0, 0, 3000)
    tr2 = o.trace(N, 0, N - 3000, 3000)
    w = np.concatenate([tr["w"], tr2["w"]]) / I
    assert np.all(w >= lo * (1 - 1e-13)) and np.all(w <= hi * (1 + 1e-13))
    assert o.history[0, 0] == pytest.approx(I, rel=max(hi - 1, 1 - lo) + 1e-14)


# --------------------------------------------------------------------------
# Constant integrand, identity channels, flat grids (n a power of two, so
# every bin density is exactly 1): every weight is the same double.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("d,K,n", [(1, 1, 16), (3, 4, 32), (5, 7, 64), (2, 3, 20)])
def test_constant_integrand(oracle_lib, d, K, n):
    p = W.constant_problem(d, K, n)
    o = oracle_lib.Oracle(p)
    o.sample_iteration(5000)
    E, sig = o.history[0, :2]
    assert E == pytest.approx(1.0, abs=4e-16)
    assert sig <= math.sqrt(4 * 2.2e-16 / 5000)  # rounding floor of <w^2> - <w>^2
    st = o.channel_stats
    assert np.all(st[:, 6] <= 4 * 2.2e-16)  # per-channel variance
    if n in (16, 32, 64):
        w = o.trace(5000, 0, 0, 500)["w"]
        assert np.all(w == w[0])


# --------------------------------------------------------------------------
# Sec. 3.2 eq. g(x) and Sec. 3.5 eq. g(p): every channel density and the
# multi-channel density integrate to one, for any grids and weights.
# Tensor Gauss-Legendre on cells split at every channel's p-space bin edge.
# --------------------------------------------------------------------------
def _cells_1d(o, k, extra):
    bps = set(np.linspace(0, 1, extra + 1))
    e = o.edges
    for c in range(o.K):
        kind = int(o.problem.chan_kind[c, k])
        loc, wid = float(o.problem.chan_loc[c, k]), float(o.problem.chan_width[c, k])
        for x in e[c, k, 1:-1]:
            bps.add(oracle_map_forward(kind, loc, wid, x))
    return np.array(sorted(bps))


oracle_map_forward = None


def _quad2(o, fn_index, extra=200, order=8):
    global oracle_map_forward
    import oracle
    oracle_map_forward = oracle.map_forward
    bx = _cells_1d(o, 0, extra)
    by = _cells_1d(o, 1, extra)
    t, wt = leggauss(order)
    def nodes(b):
        a0, a1 = b[:-1, None], b[1:, None]
        x = (0.5 * (a1 - a0) * t[None, :] + 0.5 * (a1 + a0)).ravel()
        w = (0.5 * (a1 - a0) * wt[None, :]).ravel()
        return x, w
    x, wx = nodes(bx)
    y, wy = nodes(by)
    total = 0.0
    for j0 in range(0, len(y), 512):
        yy = y[j0:j0 + 512]
        P = np.stack(np.meshgrid(x, yy, indexing="ij"), axis=-1).reshape(-1, 2)
        vals = o.eval_fg(P)[fn_index].reshape(len(x), len(yy))
        total += float(wx @ vals @ wy[j0:j0 + 512])
    return total


def test_multichannel_density_normalised_d2(oracle_lib):
    p = W.config1()
    o = oracle_lib.Oracle(p)
    rng = np.random.default_rng(4)
    e = np.zeros((2, 2, p.n_bins + 1))
    for c in range(2):
        for k in range(2):
            inner = np.sort(rng.uniform(0, 1, p.n_bins - 1))
            e[c, k] = np.concatenate([[0.0], inner, [1.0]])
    o.edges = e
    o.alpha = [0.27, 0.73]
    assert _quad2(o, 1) == pytest.approx(1.0, abs=2e-12)
    assert _quad2(o, 0) == pytest.approx(cf.integral(p), abs=2e-12)


def test_bw_multichannel_density_normalised_d2(oracle_lib):
    """Two BW channels on different axes plus a flat one."""
    pk = np.array([[BW, FLAT], [FLAT, BW], [FLAT, FLAT]], np.int32)
    pl = np.array([[0.4, 0.5], [0.5, 0.6], [0.5, 0.5]])
    pw = np.array([[0.01, 1.0], [1.0, 0.03], [1.0, 1.0]])
    p = W.Problem(2, 16, pk, pl, pw, np.array([0.5, 0.3, 0.2]), pk.copy(), pl.copy(), pw.copy())
    o = oracle_lib.Oracle(p)
    rng = np.random.default_rng(5)
    e = np.zeros((3, 2, 17))
    for c in range(3):
        for k in range(2):
            e[c, k] = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, 15)), [1.0]])
    o.edges = e
    o.alpha = [0.2, 0.5, 0.3]
    assert _quad2(o, 1, extra=400) == pytest.approx(1.0, abs=1e-10)


# --------------------------------------------------------------------------
# Sec. 3.4 eq. 15: channel-weight update.  From alpha = (1/2, 1/2) on C1 the
# per-channel second moments are W_1 = (0.8 I)^2, W_2 = (1.2 I)^2 (away from
# the far tails), so one update with beta = 1/2 gives alpha = (0.4, 0.6), the
# zero-variance weights, and the next pass has (almost) no variance.
# --------------------------------------------------------------------------
def test_config1_alpha_converges_to_zero_variance(oracle_lib):
    p = W.config1()
    o = oracle_lib.Oracle(p)
    I = cf.integral(p)
    o.sample_iteration(10_000)
    o.refine(oracle_lib.REFINE_ALPHA)
    np.testing.assert_allclose(o.alpha, [0.4, 0.6], rtol=1e-9)
    o.sample_iteration(10_000)
    assert list(o.alloc) == [4000, 6000, 10000]
    assert o.history[1, 1] <= math.sqrt(4 * 2.2e-16 / 10_000) * I
    assert o.history[1, 0] == pytest.approx(I, rel=1e-13)


def test_alpha_update_fixed_point_and_degenerate(oracle_lib):
    a = np.array([0.1, 0.2, 0.7])
    np.testing.assert_allclose(oracle_lib.update_alpha(a, [2.0, 2.0, 2.0]), a, rtol=1e-15)
    np.testing.assert_array_equal(oracle_lib.update_alpha(a, [0.0, 0.0, 0.0]), a)
    b = oracle_lib.update_alpha(a, [4.0, 1.0, 1.0])
    assert b.sum() == pytest.approx(1.0, rel=1e-15)
    assert np.all(b >= 0) and b[0] > a[0]


# --------------------------------------------------------------------------
# Sec. 3.4: integer allocation N_c, floor N_min.
# --------------------------------------------------------------------------
def test_allocation_invariants(oracle_lib):
    rng = np.random.default_rng(6)
    for trial in range(200):
        K = int(rng.integers(1, 70))
        a = rng.dirichlet(np.full(K, 0.3))
        N = int(rng.integers(K * 10, 10**7))
        nc, alpha = oracle_lib.allocation(a, N, 10)
        assert np.all(nc >= 10)
        raw = np.floor(a * N)
        free = raw >= 10
        if nc.sum() == N:
            assert np.all(np.abs(nc[free] - a[free] * N) < 1.0 + 1e-9)
        else:
            assert nc.sum() > N and np.all(nc[free] == raw[free])
        assert alpha.sum() == pytest.approx(1.0, rel=1e-14)
        np.testing.assert_array_equal(alpha, nc / nc.sum())


def test_allocation_floor_raises_total(oracle_lib):
    nc, alpha = oracle_lib.allocation([1 / 3, 1 / 3, 1 / 3], 10, 10)
    assert list(nc) == [10, 10, 10]
    nc, alpha = oracle_lib.allocation([0.5, 0.5], 10_000, 10)
    assert list(nc) == [5000, 5000]


# --------------------------------------------------------------------------
# Sec. 3.2 eq. 30/31: rebinning walk.
# --------------------------------------------------------------------------
def test_rebin_equal_weights_keeps_grid(oracle_lib):
    rng = np.random.default_rng(7)
    for n in (4, 20, 100):
        e = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, n - 1)), [1.0]])
        out = oracle_lib.rebin_axis(e, np.full(n, 3.7))
        np.testing.assert_allclose(out, e, rtol=0, atol=1e-14)  # rounding of the running sums


def test_rebin_worked_example(oracle_lib):
    """n = 4, uniform grid, all weight in the last bin: omega = (0,0,0,1),
    r = (0,0,0,1), m = (0,0,0,1) by the limits r->0 and r=1, M = 1, and the
    three interior edges split the last bin into quarters:
    0.75 + 0.25 * i/4 = 0.8125, 0.875, 0.9375 (exact binary fractions)."""
    out = oracle_lib.rebin_axis([0, 0.25, 0.5, 0.75, 1.0], [0, 0, 0, 1.0])
    assert list(out) == [0.0, 0.8125, 0.875, 0.9375, 1.0]


def test_rebin_zero_bins_are_avoided(oracle_lib):
    out = oracle_lib.rebin_axis(np.linspace(0, 1, 5), [0, 2.0, 0, 2.0])
    inner = out[1:-1]
    assert np.all(((inner >= 0.25) & (inner <= 0.5)) | ((inner >= 0.75) & (inner <= 1.0)))


def test_rebin_power_zero_keeps_grid(oracle_lib):
    """a = 0 makes m_j = 1 for every non-empty bin: grid unchanged."""
    rng = np.random.default_rng(8)
    e = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, 29)), [1.0]])
    out = oracle_lib.rebin_axis(e, rng.uniform(0.1, 5, 30), power=0.0)
    np.testing.assert_allclose(out, e, atol=4e-16)


def test_rebin_quantiles_of_piecewise_linear_measure(oracle_lib):
    """New edges are the i/n quantiles of the measure that puts m_j uniformly
    on old bin j (computed here with numpy interpolation)."""
    rng = np.random.default_rng(9)
    for n in (5, 50, 128):
        e = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, n - 1)), [1.0]])
        h = rng.uniform(0.01, 10, n) ** 3
        a = 1.5
        om = np.sqrt(h)
        r = om / om.sum()
        m = ((r - 1) / np.log(r)) ** a
        cum = np.concatenate([[0.0], np.cumsum(m)])
        want = np.interp(np.arange(n + 1) / n * cum[-1], cum, e)
        out = oracle_lib.rebin_axis(e, h, power=a)
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-13)
        assert np.all(np.diff(out) > 0)


def test_rebin_monotone_and_bounded_random(oracle_lib):
    rng = np.random.default_rng(10)
    for n in (2, 7, 64, 256):
        for _ in range(20):
            e = np.concatenate([[0.0], np.sort(rng.uniform(0, 1, n - 1)), [1.0]])
            h = rng.uniform(0, 1, n) ** 8 * (rng.uniform(0, 1, n) < 0.3)
            for snap in (False, True):
                out = oracle_lib.rebin_axis(e, h, snap32=snap)
                assert out[0] == 0.0 and out[-1] == 1.0
                assert np.all(np.diff(out) > 0)
                if snap:
                    assert np.all(out.astype(np.float32).astype(np.float64) == out)


# --------------------------------------------------------------------------
# Iteration combination.
# --------------------------------------------------------------------------
def test_result_single_iteration_is_that_iteration(oracle_lib):
    p = W.config1()
    o = oracle_lib.Oracle(p)
    for _ in range(3):
        o.sample_iteration(10_000)
        o.refine()
    h = o.history
    r = o.result(2)
    assert r["integral"] == h[2, 0] and r["error"] == pytest.approx(h[2, 1], rel=1e-15)
    r = o.result(1)
    assert min(h[1, 0], h[2, 0]) <= r["integral"] <= max(h[1, 0], h[2, 0])
    assert r["error"] < min(h[1, 1], h[2, 1])


# --------------------------------------------------------------------------
# Unweighting (eq. efficiency; Sec. 3.5 last paragraph).
# --------------------------------------------------------------------------
def test_unweighted_events_follow_integrand_d2(oracle_lib):
    from scipy.stats import chi2
    p = W.config1()
    o = oracle_lib.Oracle(p)
    for _ in range(4):
        o.sample_iteration(10_000)
        o.refine(oracle_lib.REFINE_GRID)
    o.sample_iteration(10_000)
    n_ev = 20_000
    ev, st = o.unweight(n_ev, batch=4096)
    I = cf.integral(p)
    edges = np.linspace(0, 1, 11)
    H, _, _ = np.histogram2d(ev[0], ev[1], bins=[edges, edges])
    exp = np.array([[cf.cell_mass(p, (edges[a], edges[b]), (edges[a + 1], edges[b + 1])) / I
                     for b in range(10)] for a in range(10)]) * n_ev
    mask = exp > 5
    stat = float(((H[mask] - exp[mask]) ** 2 / exp[mask]).sum())
    dof = int(mask.sum()) - 1
    assert chi2.sf(stat, dof) > 1e-4
    assert H[~mask].sum() <= 5 * max(exp[~mask].sum(), 1)
    # acceptance ~ <w>/w_max (eq. efficiency)
    assert st["efficiency"] == pytest.approx(I / st["w_max"], rel=0.05)


def test_allocation_exact_rational_rule_on_knife_edges(oracle_lib):
    """Reading R16 (Sec. 3.4: N_c = alpha_c N made integer, floor N_min):
    base_c = max(N_min, floor(alpha_c N)), the remainder one call each to the
    largest fractional parts (ties to the lower channel; floored channels
    last).  With N a power of two alpha_c N is exact in FP64, so the oracle's
    IEEE sequence must reproduce the rule evaluated in exact rationals, bit for
    bit, on tied remainders, remainders one ulp apart and products one ulp
    from an integer."""
    from fractions import Fraction

    import alpha_cases
    checked = 0
    for alpha, N, kind in alpha_cases.cases():
        if kind not in ("tied", "ulp_apart", "near_integer"):
            continue
        K = len(alpha)
        v = [Fraction(float(a)) * N for a in alpha]
        base, frac = [], []
        for c in range(K):
            b = v[c].numerator // v[c].denominator
            if b < 10:
                base.append(10)
                frac.append(Fraction(-1))
            else:
                base.append(b)
                frac.append(v[c] - b)
        nc = list(base)
        rem = N - sum(base)
        order = sorted(range(K), key=lambda c: (-frac[c], c))
        i = 0
        while rem > 0:
            nc[order[i % K]] += 1
            i += 1
            rem -= 1
        got, _ = oracle_lib.allocation(alpha, N, 10)
        assert list(got) == nc, (kind, N, list(alpha))
        checked += 1
    assert checked >= 100
