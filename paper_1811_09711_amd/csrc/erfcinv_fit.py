"""Coefficients of the FP32 erfcinv in mcv_device.h (fast_erfcinv).

Structure of M. Giles, "Approximating the erfinv function" (GPU Computing
Gems, Jade Edition, 2011): with w = -log2(y (2 - y)) for the argument y of
erfcinv, erfcinv(y) = erfinv(1 - y) = (1 - y) P(w); P is fitted here as a
polynomial in t = (w - 5) / 5 for 0 <= w <= 10 and in t = (sqrt(w) - c) / h
over 10 < w <= 26 (sqrt(10) .. sqrt(26) onto [-1, 1]), weighted Chebyshev
least squares in relative error against scipy.special.erfcinv, then written
in the power basis of t for Horner's rule.  Prints the coefficient arrays
(highest power first) and the largest relative error of each fit.

    python erfcinv_fit.py
"""
import numpy as np
from numpy.polynomial import chebyshev as Ch
from scipy.special import erfcinv

W_MID, W_TAIL, W_END = 10.0, 10.0, 26.0
DEG_CENTRAL, DEG_TAIL = 11, 8


def _p_of_w(w):
    q = np.exp2(-w)                  # y (2 - y) = 1 - x^2, x = 1 - y
    x = np.sqrt(1.0 - q)
    y = q / (1.0 + x)                # 1 - x without cancellation
    with np.errstate(invalid="ignore", divide="ignore"):
        small = x < 1e-6             # P(0) = sqrt(pi)/2 (1 + pi x^2 / 12 + ...)
        return np.where(small, np.sqrt(np.pi) / 2 * (1 + np.pi / 12 * x * x), erfcinv(y) / x)


def fit(t, P, deg):
    c = Ch.chebfit(t, P, deg, w=1.0 / P)
    pw = Ch.cheb2poly(c)[::-1]       # highest power first
    return pw, float(np.max(np.abs(np.polyval(pw, t) / P - 1)))


def central():
    w = np.linspace(0.0, W_MID, 200001)
    return fit((w - W_MID / 2) / (W_MID / 2), _p_of_w(w), DEG_CENTRAL)


def tail():
    s = np.linspace(np.sqrt(W_TAIL), np.sqrt(W_END), 200001)
    c, h = (s[0] + s[-1]) / 2, (s[-1] - s[0]) / 2
    return fit((s - c) / h, _p_of_w(s * s), DEG_TAIL), (c, h)


if __name__ == "__main__":
    pc, ec = central()
    (pt, et), (c, h) = tail()
    print("// central, t = (w - 5) / 5: max rel err %.2e" % ec)
    print("{" + ", ".join("%.9ef" % v for v in pc) + "}")
    print("// tail, t = (sqrt(w) - %.17g) / %.17g: max rel err %.2e" % (c, h, et))
    print("{" + ", ".join("%.9ef" % v for v in pt) + "}")
