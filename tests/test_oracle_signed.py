"""Integrands of either sign (Sec. 3.1: an NLO integrand need not be positive
semidefinite; reading R27): the estimate stays unbiased with a correct error
(pulls against the closed form over many seeds), the largest weight is the
largest |w|, and unweighted events carry signs whose histogram follows f/I
(closed-form cell integrals; the events are distributed as |f|, their signed
counts as f)."""
import math

import numpy as np
import pytest

import closed_forms as cf
import workloads as W


def test_signed_integrand_changes_sign():
    p = W.signed_problem()
    # at the second centre: 1 * pdf_0 - 0.3 * pdf_1 < 0 in d = 2
    g0 = math.exp(-0.5 * (0.1 / 0.15) ** 2 * 2) / (2 * math.pi * 0.15 ** 2)
    g1 = 1.0 / (2 * math.pi * 0.04 ** 2)
    assert g0 - 0.3 * g1 < 0
    assert cf.integral(p) > 0


def test_signed_pulls(oracle_lib):
    p = W.signed_problem()
    I = cf.integral(p)
    z = []
    for s in range(2000, 2200):
        o = oracle_lib.Oracle(p.with_(seed=s))
        o.sample_iteration(4000)
        E, sig = o.history[0, 0], o.history[0, 1]
        z.append((E - I) / sig)
    z = np.array(z)
    assert abs(z.mean()) < 3.0 / math.sqrt(len(z)), z.mean()
    assert 0.8 < z.std(ddof=1) < 1.25, z.std(ddof=1)


def test_signed_largest_weight_is_largest_magnitude(oracle_lib):
    p = W.signed_problem()
    o = oracle_lib.Oracle(p)
    o.sample_iteration(20_000)
    tr = o.trace(20_000, 0, 0, 20_000)
    w = tr["w"]
    assert np.any(w < 0) and np.any(w > 0)
    assert o.history[0, 3] == np.max(np.abs(w))


def test_signed_events_follow_the_integrand(oracle_lib):
    from scipy.stats import chi2
    p = W.signed_problem()
    o = oracle_lib.Oracle(p)
    for _ in range(3):
        o.sample_iteration(20_000)
        o.refine()
    o.sample_iteration(20_000)
    n_ev = 60_000
    ev, sg, st = o.unweight(n_ev, batch=16_384, signs=True)
    assert set(np.unique(sg)) == {-1, 1}
    I = cf.integral(p)
    # every kept event is the sign of |f|-distributed points: the signed
    # counts per cell estimate n_signed * (integral of f over the cell) / I
    edges = np.linspace(0, 1, 9)
    n_signed = float(sg.sum())
    stat, dof = 0.0, 0
    for a in range(8):
        for b in range(8):
            inside = ((ev[0] >= edges[a]) & (ev[0] < edges[a + 1]) &
                      (ev[1] >= edges[b]) & (ev[1] < edges[b + 1]))
            n_cell = int(inside.sum())
            if n_cell < 30:
                continue
            s_cell = float(sg[inside].sum())
            expect = n_signed * cf.cell_mass(p, (edges[a], edges[b]), (edges[a + 1], edges[b + 1])) / I
            stat += (s_cell - expect) ** 2 / n_cell
            dof += 1
    assert dof > 20
    assert chi2.sf(stat, dof - 1) > 1e-4, (stat, dof)
    # (n_plus - n_minus) / trials * w_max estimates I
    est = n_signed / st["trials"] * st["w_max"]
    assert est == pytest.approx(I, rel=0.05)
