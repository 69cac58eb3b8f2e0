"""The FP32 erfcinv of the sample pass's Gaussian maps (fast_erfcinv in
mcv_device.h): its literal coefficients are the ones erfcinv_fit.py fits, and
the same evaluation in float32 (log2, the two Horner branches, the (1 - y)
factor) stays within 4e-7 of scipy's erfcinv over the argument range the
branches serve (the library function takes y < 7.5e-9)."""
import os
import re
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_09711_amd", "csrc")


def _fit():
    sys.path.insert(0, CSRC)
    try:
        import erfcinv_fit
    finally:
        sys.path.pop(0)
    pc, ec = erfcinv_fit.central()
    (pt, et), (c, h) = erfcinv_fit.tail()
    return pc, ec, pt, et, c, h


def _source_coefficients():
    src = open(os.path.join(CSRC, "mcv_device.h")).read()
    body = src[src.index("__device__ inline float fast_erfcinv"):]
    body = body[:body.index("\n}\n")]
    central, tail = body.split("if (L >= -26.0f)")
    num = r"(-?\d\.\d+e[+-]\d+)f"
    def coefs(part):
        first = re.search(r"float P = " + num, part).group(1)
        rest = re.findall(r"P = fmaf\(P, t, " + num + r"\)", part)
        return np.array([float(first)] + [float(v) for v in rest])
    tline = re.search(r"\(sqrtf\(-L\) - " + num + r"\) \* " + num, tail)
    return coefs(central), coefs(tail), float(tline.group(1)), float(tline.group(2))


def test_source_holds_the_fitted_coefficients():
    pc, ec, pt, et, c, h = _fit()
    sc, st, s_c, s_ih = _source_coefficients()
    assert ec < 5e-8 and et < 5e-8
    np.testing.assert_allclose(sc, pc, rtol=1e-9, atol=0)
    np.testing.assert_allclose(st, pt, rtol=1e-9, atol=0)
    assert abs(s_c - c) < 1e-8 * c and abs(s_ih - 1.0 / h) < 1e-8 / h


def test_float32_evaluation_against_scipy():
    from scipy.special import erfcinv
    sc, st, s_c, s_ih = _source_coefficients()
    f32 = np.float32
    rng = np.random.default_rng(3)
    y = np.concatenate([np.exp(rng.uniform(np.log(7.6e-9), 0, 400_000)),
                        rng.uniform(0, 1, 400_000),
                        1 - np.exp(rng.uniform(np.log(1e-7), np.log(0.5), 100_000))]).astype(f32)
    y = y[(y > 0) & (y <= 1)]
    L = np.log2(y * (f32(2) - y)).astype(f32)
    keep = L >= f32(-26)
    y, L = y[keep], L[keep]
    x = f32(1) - y
    t = (L * f32(-0.2) - f32(1)).astype(f32)
    P = np.full_like(t, f32(sc[0]))
    for k in sc[1:]:
        P = (P * t + f32(k)).astype(f32)
    tt = ((np.sqrt(np.maximum(-L, f32(0))) - f32(s_c)) * f32(s_ih)).astype(f32)
    Pt = np.full_like(tt, f32(st[0]))
    for k in st[1:]:
        Pt = (Pt * tt + f32(k)).astype(f32)
    v = (x * np.where(L >= f32(-10), P, Pt)).astype(np.float64)
    ref = erfcinv(y.astype(np.float64))
    big = np.abs(ref) > 1e-3
    assert np.max(np.abs(v[big] - ref[big]) / np.abs(ref[big])) < 4e-7
    # small results (y near 1): within 2e-7 of |1 - y|
    dist = np.maximum(np.abs(1.0 - y[~big].astype(np.float64)), 1e-30)
    assert np.max(np.abs(v[~big] - ref[~big]) / dist) < 2e-7
