"""Seeded synthetic problem generators for the multi-channel VEGAS sample pass.

This module is the ONLY code shared by the FP64 CPU oracle (``oracle/``) and the
HIP library (``paper_1811_09711_amd``).  It draws problem *descriptions* (peak
positions, widths, mixture weights, job sizes, arrival times) from a seeded
numpy generator and holds none of the integration method's arithmetic: no
mappings, no densities, no grids, no random numbers the method itself draws
(those come from the counter-based Philox stream that each side implements on
its own).

A problem is a product-form peak mixture (the integrand) plus one channel
mapping per peak.  Every shape is a product over dimensions of 1-d factors:

* ``FLAT``  -- constant 1 on [0, 1];
* ``GAUSS`` -- normal density with centre ``loc`` and standard deviation ``width``;
* ``BW``    -- Breit-Wigner (Cauchy) density with centre ``loc`` and full width
  at half maximum ``width``.

The paper's physics processes (matrix elements built from Feynman graphs, the
phase-space channels built from them) are not available, so these synthetic
mixtures stand in for them, in the roles the paper gives to the integrand f and
to the channel mappings phi_c (Sec. 3.1 and Sec. 3.4).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FLAT, GAUSS, BW = 0, 1, 2
FP64, FP32_MIXED = 0, 1


@dataclasses.dataclass
class Problem:
    """One integration job.  Arrays are row-major [shape][dim]."""

    dim: int
    n_bins: int
    peak_kind: np.ndarray      # int32 [P, d]
    peak_loc: np.ndarray       # float64 [P, d]
    peak_width: np.ndarray     # float64 [P, d]
    peak_weight: np.ndarray    # float64 [P]
    chan_kind: np.ndarray      # int32 [K, d]
    chan_loc: np.ndarray       # float64 [K, d]
    chan_width: np.ndarray     # float64 [K, d]
    seed: int = 1
    precision: int = FP64
    grid_power: float = 1.5
    channel_power: float = 0.5
    min_calls: int = 10
    name: str = ""
    n_points: int = 0          # points per iteration of the workload
    n_iterations: int = 0      # adaptation iterations of the workload
    rng: int = 0               # 0: Philox4x32-10 words; 1: MRG32k3a streams
    strat: int = 0             # 0: importance sampling; s >= 2: pseudo-stratified, s calls per box

    @property
    def n_peaks(self) -> int:
        return int(self.peak_kind.shape[0])

    @property
    def n_channels(self) -> int:
        return int(self.chan_kind.shape[0])

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _shape_arrays(n: int, d: int):
    return (np.zeros((n, d), np.int32), np.full((n, d), 0.5), np.ones((n, d)))


def _same_channels(peak_kind, peak_loc, peak_width):
    """Channel c maps peak c with the peak's own shape (one channel per peak)."""
    return peak_kind.copy(), peak_loc.copy(), peak_width.copy()


def config1() -> Problem:
    """d=2, K=2, n=20: two isotropic Gaussians sigma=0.05 at (0.3,0.3) w=0.4 and
    (0.7,0.7) w=0.6; channel i is the erf inverse-CDF map of peak i; FP64;
    5 iterations x 1e4 points; Philox seed 1."""
    d = 2
    pk, pl, pw = _shape_arrays(2, d)
    pk[:] = GAUSS
    pl[0] = 0.3
    pl[1] = 0.7
    pw[:] = 0.05
    weight = np.array([0.4, 0.6])
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, 20, pk, pl, pw, weight, ck, cl, cw, seed=1, name="C1",
                   n_points=10_000, n_iterations=5)


def _bw_peaks(rng: np.random.Generator, d: int, n: int):
    """Product Breit-Wigner peaks on 2 distinct random dims, flat elsewhere;
    centres U[0.1, 0.9]; FWHM log-uniform [1e-3, 1e-1] per listed dim."""
    pk, pl, pw = _shape_arrays(n, d)
    for i in range(n):
        centre = rng.uniform(0.1, 0.9, size=d)
        dims = rng.choice(d, size=min(2, d), replace=False)
        for k in dims:
            pk[i, k] = BW
            pl[i, k] = centre[k]
            pw[i, k] = math.exp(rng.uniform(math.log(1e-3), math.log(1e-1)))
    return pk, pl, pw


def config2() -> Problem:
    """d=6, K=P=8, n=50: product Breit-Wigner peaks on 2 random dims each, flat
    elsewhere, w=1/8; channel i is the arctan map of peak i; FP64;
    10 iterations x 1e6 points; problem and sampling seed 2."""
    d, n_peaks = 6, 8
    rng = np.random.default_rng(2)
    pk, pl, pw = _bw_peaks(rng, d, n_peaks)
    weight = np.full(n_peaks, 1.0 / n_peaks)
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, 50, pk, pl, pw, weight, ck, cl, cw, seed=2, name="C2",
                   n_points=1_000_000, n_iterations=10)


def config3(precision: int = FP32_MIXED) -> Problem:
    """d=10, K=P=32, n=100: 24 isotropic Gaussians (sigma log-uniform
    [0.01, 0.1], centres U[0.1, 0.9]^10) and 8 Breit-Wigner ridges (FWHM 1e-3
    on a random pair of dims, centres U[0.1, 0.9], flat on the other 8);
    w = 1/32; channel per peak; 10 iterations x 1e8 points; seed 3."""
    d, n_gauss, n_bw = 10, 24, 8
    rng = np.random.default_rng(3)
    pk, pl, pw = _shape_arrays(n_gauss + n_bw, d)
    for i in range(n_gauss):
        pk[i] = GAUSS
        pl[i] = rng.uniform(0.1, 0.9, size=d)
        pw[i] = math.exp(rng.uniform(math.log(0.01), math.log(0.1)))
    for i in range(n_gauss, n_gauss + n_bw):
        centre = rng.uniform(0.1, 0.9, size=d)
        dims = rng.choice(d, size=2, replace=False)
        for k in dims:
            pk[i, k] = BW
            pl[i, k] = centre[k]
            pw[i, k] = 1e-3
    weight = np.full(n_gauss + n_bw, 1.0 / (n_gauss + n_bw))
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, 100, pk, pl, pw, weight, ck, cl, cw, seed=3, precision=precision,
                   name="C3", n_points=100_000_000, n_iterations=10)


def batch_job(seed: int, n_bins: int = 50) -> Problem:
    """One job of the batched / serving workloads: d ~ U{2..12},
    K = P ~ U{1..64}, N ~ round(exp(U[ln 1e4, ln 1e7])), BW peaks as config2."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(2, 13))
    n_peaks = int(rng.integers(1, 65))
    n_points = int(round(math.exp(rng.uniform(math.log(1e4), math.log(1e7)))))
    pk, pl, pw = _bw_peaks(rng, d, n_peaks)
    weight = np.full(n_peaks, 1.0 / n_peaks)
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, n_bins, pk, pl, pw, weight, ck, cl, cw, seed=seed,
                   name=f"job{seed}", n_points=n_points, n_iterations=10)


def config4(n_jobs: int = 256) -> List[Problem]:
    """256 independent jobs, seeds 4,000,000 + j, 10 iterations each."""
    return [batch_job(4_000_000 + j) for j in range(n_jobs)]


def config5_arrivals(duration_s: float = 30.0, rate: float = 200.0,
                     seed: int = 5) -> np.ndarray:
    """Poisson arrival times (seconds) of serving requests at `rate` per second."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration_s]


def config5_job(q: int) -> Problem:
    """Serving job q: sizes as the batched jobs, 8 iterations + 1e5 events."""
    return batch_job(5_000_000 + q).with_(n_iterations=8)


def constant_problem(d: int, n_channels: int, n_bins: int) -> Problem:
    """f = 1 (one all-flat peak of weight 1), identity channels."""
    pk, pl, pw = _shape_arrays(1, d)
    ck, cl, cw = _shape_arrays(n_channels, d)
    return Problem(d, n_bins, pk, pl, pw, np.ones(1), ck, cl, cw, seed=7,
                   name=f"const_d{d}_K{n_channels}_n{n_bins}")


def gauss_mixture(d: int, n_peaks: int, n_bins: int, seed: int,
                  sigma_range=(0.02, 0.1), anisotropic: bool = False) -> Problem:
    """Gaussian peaks with random centres U[0.1, 0.9]^d and sigma log-uniform
    in sigma_range, one sigma per peak (isotropic) or, with anisotropic, one
    per peak and axis; unequal weights; channel per peak."""
    rng = np.random.default_rng(seed)
    pk, pl, pw = _shape_arrays(n_peaks, d)
    for i in range(n_peaks):
        pk[i] = GAUSS
        pl[i] = rng.uniform(0.1, 0.9, size=d)
        lo, hi = math.log(sigma_range[0]), math.log(sigma_range[1])
        pw[i] = np.exp(rng.uniform(lo, hi, size=d)) if anisotropic else math.exp(rng.uniform(lo, hi))
    weight = rng.uniform(0.5, 1.5, size=n_peaks)
    weight /= weight.sum()
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, n_bins, pk, pl, pw, weight, ck, cl, cw, seed=seed,
                   name=f"gauss_d{d}_K{n_peaks}" + ("_aniso" if anisotropic else ""))


def mixed_problem(d: int, n_gauss: int, n_bw: int, n_bins: int, seed: int,
                  precision: int = FP64) -> Problem:
    """A scaled-down config3: isotropic Gaussians plus BW ridges on a random
    pair of dims; used for parity at sizes the oracle finishes in seconds."""
    rng = np.random.default_rng(seed)
    n = n_gauss + n_bw
    pk, pl, pw = _shape_arrays(n, d)
    for i in range(n_gauss):
        pk[i] = GAUSS
        pl[i] = rng.uniform(0.1, 0.9, size=d)
        pw[i] = math.exp(rng.uniform(math.log(0.01), math.log(0.1)))
    for i in range(n_gauss, n):
        centre = rng.uniform(0.1, 0.9, size=d)
        dims = rng.choice(d, size=min(2, d), replace=False)
        for k in dims:
            pk[i, k] = BW
            pl[i, k] = centre[k]
            pw[i, k] = 1e-3
    weight = np.full(n, 1.0 / n)
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, n_bins, pk, pl, pw, weight, ck, cl, cw, seed=seed,
                   precision=precision, name=f"mixed_d{d}_G{n_gauss}_B{n_bw}")


def signed_problem(d: int = 2, n_bins: int = 20, seed: int = 9) -> Problem:
    """An integrand that changes sign (the role of an NLO integrand): a wide
    positive Gaussian minus a narrower one inside it, weights +1 and -0.3 (the
    difference is negative near the second centre); one channel per peak."""
    pk, pl, pw = _shape_arrays(2, d)
    pk[:] = GAUSS
    pl[0] = 0.45
    pl[1] = 0.55
    pw[0] = 0.15
    pw[1] = 0.04
    weight = np.array([1.0, -0.3])
    ck, cl, cw = _same_channels(pk, pl, pw)
    return Problem(d, n_bins, pk, pl, pw, weight, ck, cl, cw, seed=seed,
                   name=f"signed_d{d}", n_points=20_000, n_iterations=5)
