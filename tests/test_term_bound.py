"""The sample pass skips a channel's grid lookups when its term of g(p)
(Sec. 3.5, eq. g(p)) provably cannot change the running sum: the term is
non-negative, g only grows, and the test (alpha gbound) r < g, evaluated in
the pass precision with gbound = RU(2^s (1 + m) cnorm prod_k max_j dens_kj),
must imply that the term -- however the pass rounds it -- is below half an
ulp of g, so that g + term rounds back to g.  These tests check that
implication with exact rational arithmetic on adversarial draws (the bin
densities at their maxima, g just above the test value, powers of two,
tiny and huge magnitudes), in both precisions, following the kernel's
evaluation order: term = ((alpha cnorm) G) r with G the product of the d
densities in axis order, either rounded or fused into g + term."""
from fractions import Fraction
import math

import numpy as np
import pytest

# (pass precision, s, m) as in the bound kernel
CASES = [(np.float32, 25, 2.0 ** -16), (np.float64, 54, 2.0 ** -40)]


def _ulp(x, dt):
    """ulp of a positive finite x of type dt (spacing to the next value up)."""
    return Fraction(float(np.nextafter(dt(x), dt(np.inf)))) - Fraction(float(x))


def _round_up(g, dt):
    f = dt(g)
    if not np.isfinite(f):
        return f  # the bound kernel stores +inf: such a channel is never skipped
    if Fraction(float(f)) < Fraction(g):
        f = np.nextafter(f, dt(np.inf))
    return f


def _bound(cnorm, dmax, s, m, dt):
    g = float(cnorm)
    for v in dmax:
        g *= float(v)
    return _round_up(g * 2.0 ** s * (1.0 + m), dt)


def _draw(rng, dt):
    d = int(rng.integers(1, 33))
    dmax = (10.0 ** rng.uniform(-2, 3, size=d)).astype(dt)
    # the densities of the bins the point falls into: at the maxima (the
    # worst case for the bound) or below them
    dens = dmax if rng.random() < 0.5 else (dmax * rng.uniform(0, 1, size=d)).astype(dt)
    cnorm = dt(10.0 ** rng.uniform(-8, 8))
    alpha = dt(rng.uniform(1e-6, 1.0))
    r = dt(10.0 ** rng.uniform(-30, 10) if dt == np.float32 else 10.0 ** rng.uniform(-200, 100))
    return d, dmax, dens, cnorm, alpha, r


@pytest.mark.parametrize("dt,s,m", CASES)
def test_skipped_terms_cannot_change_g(dt, s, m):
    rng = np.random.default_rng(2024)
    checked = 0
    with np.errstate(over="ignore", under="ignore"):
        for _ in range(3000):
            d, dmax, dens, cnorm, alpha, r = _draw(rng, dt)
            gb = _bound(cnorm, dmax, s, m, dt)
            v = dt(dt(alpha * gb) * r)  # the kernel's test value
            # the term as the pass evaluates it: ((alpha cnorm) G) r
            G = dt(1)
            for x in dens:
                G = dt(G * x)
            X = dt(dt(alpha * cnorm) * G)
            if not np.isfinite(dt(X * r)):
                assert not np.isfinite(v)  # an overflowing term is never skipped
                continue
            if not np.isfinite(v) or v == 0:
                continue
            exact = Fraction(float(X)) * Fraction(float(r))  # fused: g + X r exactly
            rounded = Fraction(float(dt(X * r)))           # unfused: g + fl(X r)
            term = max(exact, rounded)
            # g values that pass the test: just above v, and powers of two
            gs = [np.nextafter(v, dt(np.inf)), dt(v * dt(1.5))]
            e = math.frexp(float(v))[1]
            gs.append(dt(2.0 ** e))
            for g in gs:
                if not (np.isfinite(g) and np.isfinite(np.nextafter(g, dt(np.inf))) and v < g):
                    continue
                assert term < _ulp(g, dt) / 2, (d, float(g), float(term))
                checked += 1
    assert checked > 3000


@pytest.mark.parametrize("dt,s,m", CASES)
def test_half_ulp_leaves_g_unchanged(dt, s, m):
    """The rounding fact the skip rests on: g + t == g for 0 <= t < ulp(g)/2
    (round to nearest), including at powers of two."""
    rng = np.random.default_rng(7)
    for _ in range(2000):
        g = dt(10.0 ** rng.uniform(-30, 30))
        if rng.random() < 0.3:
            g = dt(2.0 ** int(rng.integers(-60, 60)))
        half = _ulp(g, dt) / 2
        t = dt(float(half * Fraction(rng.uniform(0, 0.999))))
        assert Fraction(float(t)) < half
        assert dt(g + t) == g


def test_bound_rounds_up():
    for g in (1.0 / 3.0, 1e38 * 3.1, 1e-40, 2.0 ** 100 + 1.0):
        f = _round_up(g, np.float32)
        assert Fraction(float(f)) >= Fraction(g)


def _floor_log2(x):
    return math.frexp(float(x))[1] - 1


def _skip_offsets(tw, a, gb, dt):
    """The exponent offsets (EA, EB) the allocation writes for a channel."""
    P, s = (24, 25) if dt == np.float32 else (53, 54)
    ea = -100000 if tw == 0 else _floor_log2(tw) + P + 4
    eb = _floor_log2(a) + _floor_log2(gb) + 4 - s + P
    return ea, eb


@pytest.mark.parametrize("dt,s,m", CASES)
def test_partial_exponent_skip_cannot_change_f_or_g(dt, s, m):
    """An all-Gaussian channel is skipped when its partial exponent sum S (of
    the first axes) is at least max(EA - ex(f), EB - ex(g)) (ex = floor log2,
    of max(x, smallest normal)).  The full sum is at least S and r is
    2^-(full sum) up to the exponential's rounding (taken as 2^-20 here), so
    both of the channel's terms must then lie below half an ulp of f and of
    g -- checked exactly."""
    rng = np.random.default_rng(99)
    tiny = np.finfo(dt).tiny
    skipped = 0
    with np.errstate(over="ignore", under="ignore"):
        for _ in range(4000):
            d, dmax, dens, cnorm, alpha, _ = _draw(rng, dt)
            gb = _bound(cnorm, dmax, s, m, dt)
            if not np.isfinite(gb):
                continue
            tw = dt(10.0 ** rng.uniform(-5, 20)) if rng.random() < 0.9 else dt(0)
            f = dt(10.0 ** rng.uniform(-30, 30)) if rng.random() < 0.9 else dt(0)
            g = dt(10.0 ** rng.uniform(-30, 30)) if rng.random() < 0.9 else dt(0)
            ea, eb = _skip_offsets(tw, alpha, gb, dt)
            thr = max(ea - _floor_log2(max(f, tiny)), eb - _floor_log2(max(g, tiny)))
            S = dt(max(thr, 0) + rng.uniform(0, 3))  # a partial sum that passes
            if not S >= thr:
                continue
            full = S + Fraction(rng.uniform(0, 5))
            r_hi = Fraction(2) ** -math.floor(full) * Fraction(1 + 2.0 ** -20)  # >= r
            G = dt(1)
            for x in dens:
                G = dt(G * x)
            X = dt(dt(alpha * cnorm) * G)
            tg = Fraction(float(X)) * r_hi * (1 + Fraction(2) ** -20)  # >= the term of g
            tf = Fraction(float(tw)) * r_hi * (1 + Fraction(2) ** -20)  # >= the term of f
            half_f = _ulp(max(f, tiny), dt) / 2
            half_g = _ulp(max(g, tiny), dt) / 2
            assert tf < half_f and tg < half_g, (float(f), float(g), float(tw), thr)
            skipped += 1
    assert skipped > 2000
