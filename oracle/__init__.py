"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never does, and this package never
imports the product library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)
_u8p = C.POINTER(C.c_uint8)
_dp = C.POINTER(C.c_double)

REFINE_GRID, REFINE_ALPHA = 1, 2
TAG_UNWEIGHT = 0x80000000


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_channels", C.c_int32), ("n_bins", C.c_int32),
                ("n_peaks", C.c_int32), ("fp32_rules", C.c_int32),
                ("peak_kind", _i32p), ("peak_loc", _dp), ("peak_width", _dp),
                ("peak_weight", _dp), ("chan_kind", _i32p), ("chan_loc", _dp),
                ("chan_width", _dp), ("seed", C.c_uint64), ("grid_power", C.c_double),
                ("channel_power", C.c_double), ("min_calls", C.c_int64), ("rng", C.c_int32),
                ("strat", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp = C.c_void_p
        sig = {
            "orc_philox": (None, [_u32p, _u32p, _u32p]),
            "orc_word": (C.c_uint32, [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]),
            "orc_erfcinv": (C.c_double, [C.c_double]),
            "orc_strat_layout": (None, [C.c_int64, C.c_int32, C.c_int64, _i64p, _i64p]),
            "orc_mrg_outputs": (None, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int32, _u32p]),
            "orc_map_forward": (C.c_double, [C.c_int32, C.c_double, C.c_double, C.c_double]),
            "orc_map_cdf": (C.c_double, [C.c_int32, C.c_double, C.c_double, C.c_double]),
            "orc_map_density": (C.c_double, [C.c_int32, C.c_double, C.c_double, C.c_double]),
            "orc_peak_pdf": (C.c_double, [C.c_int32, C.c_double, C.c_double, C.c_double]),
            "orc_create": (vp, [C.POINTER(_Problem), C.c_int32]),
            "orc_destroy": (None, [vp]),
            "orc_allocate": (C.c_int, [vp, C.c_int64]),
            "orc_sample_iteration": (C.c_int, [vp, C.c_int64, C.c_int32]),
            "orc_refine": (C.c_int, [vp, C.c_uint32]),
            "orc_result": (C.c_int, [vp, C.c_int32, _dp]),
            "orc_trace": (C.c_int, [vp, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                    _u32p, _i32p, _i32p, _u8p, _dp, _dp]),
            "orc_eval_fg": (C.c_int, [vp, C.c_int64, _dp, _dp, _dp]),
            "orc_unweight": (C.c_int, [vp, C.c_int64, C.c_int64, _dp, _dp]),
            "orc_unweight_ex": (C.c_int, [vp, C.c_int64, C.c_int64, _dp, C.POINTER(C.c_int8),
                                          _dp]),
            "orc_get_edges": (C.c_int, [vp, _dp]),
            "orc_set_edges": (C.c_int, [vp, _dp]),
            "orc_get_alpha": (C.c_int, [vp, _dp]),
            "orc_set_alpha": (C.c_int, [vp, _dp]),
            "orc_get_alloc": (C.c_int, [vp, _i64p]),
            "orc_get_hist": (C.c_int, [vp, _dp]),
            "orc_get_channel_stats": (C.c_int, [vp, _dp]),
            "orc_unweight_tol": (C.c_int, [vp, C.c_int64, C.c_int64, C.c_double, _dp,
                                           C.POINTER(C.c_int8), _dp, _i64p]),
            "orc_n_iterations": (C.c_int32, [vp]),
            "orc_get_history": (C.c_int, [vp, _dp]),
            "orc_rebin_axis": (C.c_int, [C.c_int32, _dp, _dp, C.c_double, C.c_int32, _dp]),
            "orc_update_alpha": (C.c_int, [C.c_int32, _dp, _dp, C.c_double]),
            "orc_allocation": (C.c_int, [C.c_int32, _dp, C.c_int64, C.c_int64, _i64p, _dp]),
            "orc_set_equivalences": (C.c_int, [vp, C.c_int32, _i32p]),
            "orc_get_equivalent_hist": (C.c_int, [vp, _dp]),
            "orc_wmax": (C.c_double, [vp]),
            "orc_set_wmax": (None, [vp, C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def word(seed, i, t, m):
    return int(lib().orc_word(seed, i, t, m))


def mrg_outputs(g, i, offset, count):
    """MRG32k3a outputs z of substream i of stream g, `offset` steps in."""
    z = np.zeros(count, np.uint32)
    lib().orc_mrg_outputs(int(g), int(i), int(offset), int(count), _ptr(z, _u32p))
    return z


def erfcinv(y):
    return float(lib().orc_erfcinv(float(y)))


def map_forward(kind, loc, width, x):
    return float(lib().orc_map_forward(kind, loc, width, x))


def map_cdf(kind, loc, width, p):
    return float(lib().orc_map_cdf(kind, loc, width, p))


def map_density(kind, loc, width, p):
    return float(lib().orc_map_density(kind, loc, width, p))


def peak_pdf(kind, loc, width, p):
    return float(lib().orc_peak_pdf(kind, loc, width, p))


def rebin_axis(edges, hist, power=1.5, snap32=False):
    e = np.ascontiguousarray(edges, np.float64)
    h = np.ascontiguousarray(hist, np.float64)
    n = h.shape[0]
    out = np.zeros(n + 1)
    lib().orc_rebin_axis(n, _ptr(e, _dp), _ptr(h, _dp), power, int(snap32), _ptr(out, _dp))
    return out


def update_alpha(alpha, w2, beta=0.5):
    a = np.array(alpha, np.float64)
    w = np.ascontiguousarray(w2, np.float64)
    lib().orc_update_alpha(a.shape[0], _ptr(a, _dp), _ptr(w, _dp), beta)
    return a


def allocation(alpha, n_points, min_calls=10):
    a = np.ascontiguousarray(alpha, np.float64)
    nc = np.zeros(a.shape[0], np.int64)
    out = np.zeros(a.shape[0])
    lib().orc_allocation(a.shape[0], _ptr(a, _dp), n_points, min_calls, _ptr(nc, _i64p),
                         _ptr(out, _dp))
    return nc, out


class Oracle:
    """One integration job on the CPU oracle."""

    def __init__(self, problem, max_iter: int = 1000):
        p = problem
        self.problem = p
        self.d, self.K, self.n, self.P = p.dim, p.n_channels, p.n_bins, p.n_peaks
        self._keep = [np.ascontiguousarray(a, dt) for a, dt in (
            (p.peak_kind, np.int32), (p.peak_loc, np.float64), (p.peak_width, np.float64),
            (p.peak_weight, np.float64), (p.chan_kind, np.int32), (p.chan_loc, np.float64),
            (p.chan_width, np.float64))]
        k = self._keep
        st = _Problem(p.dim, p.n_channels, p.n_bins, p.n_peaks, int(p.precision != 0),
                      _ptr(k[0], _i32p), _ptr(k[1], _dp), _ptr(k[2], _dp), _ptr(k[3], _dp),
                      _ptr(k[4], _i32p), _ptr(k[5], _dp), _ptr(k[6], _dp), p.seed,
                      p.grid_power, p.channel_power, p.min_calls, int(getattr(p, "rng", 0)),
                      int(getattr(p, "strat", 0)))
        self._h = lib().orc_create(C.byref(st), max_iter)
        if not self._h:
            raise ValueError("oracle rejected the problem")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def sample_iteration(self, n_points: int, n_threads: int = 1):
        rc = lib().orc_sample_iteration(self._h, n_points, n_threads)
        if rc != 0:
            raise RuntimeError(f"orc_sample_iteration failed ({rc})")

    def refine(self, what: int = REFINE_GRID | REFINE_ALPHA):
        rc = lib().orc_refine(self._h, what)
        if rc != 0:
            raise RuntimeError(f"orc_refine failed ({rc})")

    def allocate(self, n_points):
        lib().orc_allocate(self._h, n_points)

    def result(self, first_iter: int = 0):
        out = np.zeros(4)
        rc = lib().orc_result(self._h, first_iter, _ptr(out, _dp))
        if rc != 0:
            raise RuntimeError(f"orc_result failed ({rc})")
        return {"integral": out[0], "error": out[1], "chi2_ndf": out[2], "n_iter": int(out[3])}

    @property
    def edges(self):
        e = np.zeros((self.K, self.d, self.n + 1))
        lib().orc_get_edges(self._h, _ptr(e, _dp))
        return e

    @edges.setter
    def edges(self, e):
        e = np.ascontiguousarray(e, np.float64).reshape(self.K, self.d, self.n + 1)
        lib().orc_set_edges(self._h, _ptr(e, _dp))

    @property
    def alpha(self):
        a = np.zeros(self.K)
        lib().orc_get_alpha(self._h, _ptr(a, _dp))
        return a

    @alpha.setter
    def alpha(self, a):
        a = np.ascontiguousarray(a, np.float64)
        lib().orc_set_alpha(self._h, _ptr(a, _dp))

    @property
    def alloc(self):
        nc = np.zeros(self.K + 1, np.int64)
        lib().orc_get_alloc(self._h, _ptr(nc, _i64p))
        return nc

    @property
    def hist(self):
        h = np.zeros((self.K, self.d, self.n))
        lib().orc_get_hist(self._h, _ptr(h, _dp))
        return h

    @property
    def channel_stats(self):
        st = np.zeros((self.K, 7))
        lib().orc_get_channel_stats(self._h, _ptr(st, _dp))
        return st

    @property
    def history(self):
        n = lib().orc_n_iterations(self._h)
        h = np.zeros((n, 5))
        if n:
            lib().orc_get_history(self._h, _ptr(h, _dp))
        return h

    def set_equivalences(self, eq):
        """eq: [n_eq][2 + 2d] int rows (c, c', perm[d], mode[d]); [] clears."""
        e = np.ascontiguousarray(np.asarray(eq, np.int32).reshape(-1, 2 + 2 * self.d))
        rc = lib().orc_set_equivalences(self._h, e.shape[0], _ptr(e, _i32p))
        if rc != 0:
            raise ValueError("malformed equivalence list")

    @property
    def equivalent_hist(self):
        h = np.zeros((self.K, self.d, self.n))
        lib().orc_get_equivalent_hist(self._h, _ptr(h, _dp))
        return h

    @property
    def wmax(self):
        return lib().orc_wmax(self._h)

    @wmax.setter
    def wmax(self, w):
        lib().orc_set_wmax(self._h, float(w))

    def trace(self, n_points, iteration, first, count, n_words=None):
        d, K = self.d, self.K
        n_words = d if n_words is None else n_words
        words = np.zeros((count, n_words), np.uint32)
        chan = np.zeros(count, np.int32)
        bins = np.zeros((count, K, d), np.int32)
        near = np.zeros((count, K, d), np.uint8)
        p = np.zeros((count, d))
        fgw = np.zeros((count, 3))
        rc = lib().orc_trace(self._h, n_points, iteration, first, count, n_words,
                             _ptr(words, _u32p), _ptr(chan, _i32p), _ptr(bins, _i32p),
                             _ptr(near, _u8p), _ptr(p, _dp), _ptr(fgw, _dp))
        if rc != 0:
            raise RuntimeError("orc_trace failed")
        return {"words": words, "chan": chan, "bins": bins, "near": near, "p": p,
                "f": fgw[:, 0], "g": fgw[:, 1], "w": fgw[:, 2]}

    def eval_fg(self, p):
        p = np.ascontiguousarray(p, np.float64).reshape(-1, self.d)
        f = np.zeros(p.shape[0])
        g = np.zeros(p.shape[0])
        lib().orc_eval_fg(self._h, p.shape[0], _ptr(p, _dp), _ptr(f, _dp), _ptr(g, _dp))
        return f, g

    def unweight(self, n_events, batch=65536, signs=False, tie_rel=1e-12):
        """Events [d][n_events] and stats; overweight_ties / accept_ties count
        the decisions within tie_rel of their threshold (see orc_unweight_ex
        and orc_unweight_tol), first_tie the events kept before the first
        tied accept decision.  signs: also return the sign (+1 / -1) of each
        event's weight."""
        ev = np.zeros((self.d, n_events))
        sg = np.zeros(n_events, np.int8)
        st = np.zeros(6)
        ft = np.zeros(1, np.int64)
        rc = lib().orc_unweight_tol(self._h, n_events, batch, tie_rel, _ptr(ev, _dp),
                                    _ptr(sg, C.POINTER(C.c_int8)), _ptr(st, _dp),
                                    _ptr(ft, _i64p))
        if rc != 0:
            raise RuntimeError(f"orc_unweight failed ({rc})")
        stats = {"trials": int(st[0]), "n_overweight": int(st[1]), "w_max": st[2],
                 "efficiency": st[3], "overweight_ties": int(st[4]), "accept_ties": int(st[5]),
                 "first_tie": int(ft[0])}
        if signs:
            return ev, sg, stats
        return ev, stats
