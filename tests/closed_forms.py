"""Closed-form integrals of the synthetic peak mixtures over the unit cube.

I = sum_i w_i prod_k M_ik with the mass of each 1-d factor on [0, 1]:
Gaussian (mu, sigma): (erf((1-mu)/(sigma sqrt 2)) + erf(mu/(sigma sqrt 2))) / 2;
Breit-Wigner (m, FWHM Gamma, h = Gamma/2): (atan((1-m)/h) + atan(m/h)) / pi;
flat: 1.  Evaluated with mpmath at 40 digits, independently of the oracle.
"""
import mpmath as mp

FLAT, GAUSS, BW = 0, 1, 2


def factor_mass(kind, loc, width, lo=0.0, hi=1.0):
    mp.mp.dps = 40
    loc, width, lo, hi = mp.mpf(loc), mp.mpf(width), mp.mpf(lo), mp.mpf(hi)
    if kind == GAUSS:
        s2 = width * mp.sqrt(2)
        return (mp.erf((hi - loc) / s2) - mp.erf((lo - loc) / s2)) / 2
    if kind == BW:
        h = width / 2
        return (mp.atan((hi - loc) / h) - mp.atan((lo - loc) / h)) / mp.pi
    return hi - lo


def peak_masses(problem):
    """M_i = prod_k M_ik for every peak (mpf)."""
    out = []
    for i in range(problem.n_peaks):
        m = mp.mpf(1)
        for k in range(problem.dim):
            m *= factor_mass(int(problem.peak_kind[i, k]), float(problem.peak_loc[i, k]),
                             float(problem.peak_width[i, k]))
        out.append(m)
    return out


def integral(problem):
    return float(sum(mp.mpf(float(problem.peak_weight[i])) * m
                     for i, m in enumerate(peak_masses(problem))))


def zero_variance_alpha(problem):
    """alpha*_c = w_c M_c / I when channel c maps peak c with the peak's own
    shape: then sum_c alpha*_c q_c = f / I and every weight equals I."""
    ms = peak_masses(problem)
    tot = sum(mp.mpf(float(problem.peak_weight[i])) * m for i, m in enumerate(ms))
    return [float(mp.mpf(float(problem.peak_weight[i])) * m / tot) for i, m in enumerate(ms)]


def cell_mass(problem, lo, hi):
    """Integral of f over the box [lo, hi] (per-dim bounds)."""
    tot = mp.mpf(0)
    for i in range(problem.n_peaks):
        m = mp.mpf(float(problem.peak_weight[i]))
        for k in range(problem.dim):
            m *= factor_mass(int(problem.peak_kind[i, k]), float(problem.peak_loc[i, k]),
                             float(problem.peak_width[i, k]), lo[k], hi[k])
        tot += m
    return float(tot)
