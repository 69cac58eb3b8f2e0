"""Pins of the oracle's 1-d channel maps, densities and erfcinv.

The oracle's maps play the role of the paper's channel mappings phi_c
(Sec. 3.1: p = phi(x), dmu = phi'(x) d^d x; Sec. 3.4: q_c = 1/phi_c').
They are checked against scipy's own truncated-normal and Cauchy
distributions (independent implementations), against mpmath numerical
differentiation, and by round trips.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special, stats

FLAT, GAUSS, BW = 0, 1, 2


def test_erfcinv_vs_scipy(oracle_lib):
    O = oracle_lib
    ys = np.concatenate([np.logspace(-300, 0, 400), np.linspace(0.01, 1.99, 199)])
    for y in ys:
        got = O.erfcinv(y)
        ref = special.erfcinv(y)
        assert got == pytest.approx(ref, rel=4e-15, abs=1e-300), y


def test_erfcinv_round_trip_mpmath(oracle_lib):
    O = oracle_lib
    mp.mp.dps = 40
    for y in (1e-250, 3e-100, 1e-20, 1e-5, 0.03, 0.5, 0.999, 1.0 - 1e-12):
        x = O.erfcinv(y)
        back = float(mp.erfc(mp.mpf(x)))
        assert back == pytest.approx(y, rel=1e-14)


@pytest.mark.parametrize("mu,sigma", [(0.3, 0.05), (0.7, 0.05), (0.15, 0.01), (0.85, 0.1), (0.5, 0.3)])
def test_gauss_map_vs_scipy_truncnorm(oracle_lib, mu, sigma):
    O = oracle_lib
    a, b = (0 - mu) / sigma, (1 - mu) / sigma
    dist = stats.truncnorm(a, b, loc=mu, scale=sigma)
    for x in np.concatenate([np.linspace(1e-6, 1 - 1e-6, 57), [1e-12, 0.5, 1 - 1e-9]]):
        p = O.map_forward(GAUSS, mu, sigma, x)
        assert p == pytest.approx(dist.ppf(x), rel=1e-12, abs=1e-13), x
        assert O.map_cdf(GAUSS, mu, sigma, p) == pytest.approx(x, rel=1e-10, abs=1e-14)
        assert O.map_density(GAUSS, mu, sigma, p) == pytest.approx(dist.pdf(p), rel=1e-12)


@pytest.mark.parametrize("m,gamma", [(0.5, 1e-3), (0.2, 1e-1), (0.83, 1e-2), (0.1, 5e-3)])
def test_bw_map_vs_scipy_cauchy(oracle_lib, m, gamma):
    O = oracle_lib
    h = gamma / 2
    F = stats.cauchy(loc=m, scale=h)
    F0, F1 = F.cdf(0.0), F.cdf(1.0)
    for p in np.concatenate([np.linspace(0, 1, 41), m + h * np.linspace(-5, 5, 21)]):
        if not 0 <= p <= 1:
            continue
        x_ref = (F.cdf(p) - F0) / (F1 - F0)
        assert O.map_cdf(BW, m, gamma, p) == pytest.approx(x_ref, rel=1e-11, abs=1e-14)
        assert O.map_density(BW, m, gamma, p) == pytest.approx(F.pdf(p) / (F1 - F0), rel=1e-12)
    for x in np.linspace(1e-4, 1 - 1e-4, 31):
        p = O.map_forward(BW, m, gamma, x)
        assert O.map_cdf(BW, m, gamma, p) == pytest.approx(x, rel=1e-10)


def test_flat_map_identity(oracle_lib):
    O = oracle_lib
    for x in (1e-9, 0.25, 0.5, 0.999):
        assert O.map_forward(FLAT, 0.5, 1.0, x) == x
        assert O.map_cdf(FLAT, 0.5, 1.0, x) == x
        assert O.map_density(FLAT, 0.5, 1.0, x) == 1.0


@pytest.mark.parametrize("kind,loc,width", [(GAUSS, 0.3, 0.05), (GAUSS, 0.62, 0.013), (BW, 0.4, 0.02)])
def test_density_is_cdf_derivative(oracle_lib, kind, loc, width):
    """q(p) = d x(p) / dp by mpmath numerical differentiation; CDF(0)=0, CDF(1)=1."""
    O = oracle_lib
    mp.mp.dps = 30
    assert O.map_cdf(kind, loc, width, 0.0) == pytest.approx(0.0, abs=1e-15)
    assert O.map_cdf(kind, loc, width, 1.0) == pytest.approx(1.0, abs=1e-15)
    for p in np.linspace(loc - 3 * width, loc + 3 * width, 13):
        if not 0 < p < 1:
            continue
        num = mp.diff(lambda t: O.map_cdf(kind, loc, width, float(t)), mp.mpf(p), h=mp.mpf(width) * 1e-5)
        assert O.map_density(kind, loc, width, p) == pytest.approx(float(num), rel=1e-6)


@pytest.mark.parametrize("kind,loc,width", [(GAUSS, 0.3, 0.05), (GAUSS, 0.85, 0.01), (BW, 0.4, 1e-3)])
def test_density_integrates_to_one(oracle_lib, kind, loc, width):
    O = oracle_lib
    mp.mp.dps = 20
    pts = [0, max(0, loc - 20 * width), loc, min(1, loc + 20 * width), 1]
    tot = mp.quad(lambda t: O.map_density(kind, loc, width, float(t)), pts)
    assert float(tot) == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("kind,loc,width", [(GAUSS, 0.3, 0.05), (BW, 0.4, 2e-2)])
def test_peak_pdf_normalised(oracle_lib, kind, loc, width):
    """The integrand's peak factors are untruncated normalised pdfs: their
    mass on [0,1] is the closed-form truncation mass."""
    O = oracle_lib
    mp.mp.dps = 20
    pts = [0, loc - 10 * width, loc, loc + 10 * width, 1]
    pts = sorted(min(1, max(0, t)) for t in pts)
    tot = float(mp.quad(lambda t: O.peak_pdf(kind, loc, width, float(t)), pts))
    if kind == GAUSS:
        s2 = width * math.sqrt(2)
        ref = 0.5 * (math.erf((1 - loc) / s2) + math.erf(loc / s2))
    else:
        h = width / 2
        ref = (math.atan((1 - loc) / h) - math.atan(-loc / h)) / math.pi
    assert tot == pytest.approx(ref, rel=1e-9)
