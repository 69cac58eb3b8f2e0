"""Python binding of libmcv (include/mcv.h): argument marshalling only.

Every step of the sample pass, the adaptation and the unweighting runs in the
HIP library; this module converts numpy/torch arguments into C-ABI calls.
PyTorch provides device memory and the HIP stream: when the library is
loaded, torch's caching allocator is installed as the library's allocator
(mcv_set_allocator), so integrators, batches and servers take their device
memory from torch.  The library must be built (``__graft_entry__.build()`` or
``python -m paper_1811_09711_amd.build``); importing without it raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
from typing import Optional

import numpy as np

import torch  # noqa: F401  (loads the process's HIP runtime before libmcv)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcv.so")

MCV_OK, MCV_E_INVALID, MCV_E_NOMEM, MCV_E_DEVICE, MCV_E_STATE, MCV_E_NUMERIC = 0, -1, -2, -3, -4, -5
MCV_FP64, MCV_FP32_MIXED = 0, 1
MCV_RNG_PHILOX, MCV_RNG_MRG32K3A = 0, 1
MCV_FLAT, MCV_GAUSS, MCV_BW = 0, 1, 2
MCV_REFINE_GRID, MCV_REFINE_ALPHA = 1, 2
MCV_EQ_IDENTITY, MCV_EQ_INVERT, MCV_EQ_SYMMETRIC, MCV_EQ_INVARIANT = 0, 1, 2, 3

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_u32p = C.POINTER(C.c_uint32)
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p


class mcv_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_channels", C.c_int32), ("n_bins", C.c_int32),
                ("n_peaks", C.c_int32), ("precision", C.c_int32),
                ("peak_kind", _i32p), ("peak_loc", _dp), ("peak_width", _dp),
                ("peak_weight", _dp), ("chan_kind", _i32p), ("chan_loc", _dp),
                ("chan_width", _dp), ("seed", C.c_uint64), ("grid_power", C.c_double),
                ("channel_power", C.c_double), ("min_calls", C.c_int64),
                ("max_iterations", C.c_int32), ("rng", C.c_int32), ("strat", C.c_int32)]


class mcv_summary(C.Structure):
    _fields_ = [("integral", C.c_double), ("error", C.c_double), ("chi2_ndf", C.c_double),
                ("w_max", C.c_double), ("n_iter_used", C.c_int32), ("n_points", C.c_int64),
                ("n_bad", C.c_int64)]


class mcv_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("unit_calls", C.c_int32), ("launch_bound", C.c_int32),
                ("term_bound", C.c_int32)]


class mcv_server_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_active", C.c_int32), ("hbm_budget", C.c_int64),
                ("unweight_batch", C.c_int64), ("tuning", mcv_tuning), ("keep_events", C.c_int32)]


class mcv_job_report(C.Structure):
    _fields_ = [("state", C.c_int32), ("iterations_done", C.c_int32), ("result", mcv_summary),
                ("n_events", C.c_int64), ("trials", C.c_int64), ("n_overweight", C.c_int64),
                ("w_max", C.c_double), ("efficiency", C.c_double), ("submit_time", C.c_double),
                ("admit_time", C.c_double), ("finish_time", C.c_double),
                ("device_bytes", C.c_int64)]


class mcv_step_info(C.Structure):
    _fields_ = [("n_integrating", C.c_int32), ("n_generating", C.c_int32),
                ("n_admitted", C.c_int32), ("n_finished", C.c_int32), ("n_queued", C.c_int32),
                ("n_active", C.c_int32), ("bytes_in_use", C.c_int64)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_SIGNATURES = {
    "mcv_set_allocator": (C.c_int, [_ALLOC_FN, _FREE_FN, _vp]),
    "mcv_create_integrator": (C.c_int, [C.POINTER(mcv_problem), _vp, C.POINTER(_vp)]),
    "mcv_set_stream": (C.c_int, [_vp, _vp]),
    "mcv_sample_iteration": (C.c_int, [_vp, C.c_int64]),
    "mcv_refine": (C.c_int, [_vp, C.c_uint32]),
    "mcv_set_equivalences": (C.c_int, [_vp, C.c_int32, _i32p]),
    "mcv_result": (C.c_int, [_vp, C.c_int32, C.POINTER(mcv_summary)]),
    "mcv_get_history": (C.c_int, [_vp, _dp, C.c_int32, _i32p]),
    "mcv_unweight": (C.c_int, [_vp, C.c_int64, C.c_int64, _vp, _dp]),
    "mcv_unweight_signed": (C.c_int, [_vp, C.c_int64, C.c_int64, _vp, _vp, _dp]),
    "mcv_unweight_noalloc": (C.c_int, [_vp, C.c_int64, C.c_int64, _vp, _dp]),
    "mcv_get_state": (C.c_int, [_vp, _dp, _dp, _i64p]),
    "mcv_set_state_for_test": (C.c_int, [_vp, _dp, _dp]),
    "mcv_get_pass_stats": (C.c_int, [_vp, _dp, _dp]),
    "mcv_debug_trace": (C.c_int, [_vp, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_int32,
                                  _u32p, _i32p, _i32p, _dp, _dp]),
    "mcv_debug_sample_trace": (C.c_int, [_vp, C.c_int64, C.c_int64, C.c_int64, C.c_int64, _dp]),
    "mcv_save_state": (C.c_int, [_vp, _vp, C.POINTER(C.c_size_t)]),
    "mcv_load_state": (C.c_int, [_vp, _vp, C.c_size_t]),
    "mcv_pass_timing": (C.c_int, [_vp, C.c_int32, _dp, _i32p]),
    "mcv_destroy": (None, [_vp]),
    "mcv_batch_create": (C.c_int, [C.POINTER(mcv_problem), _i64p, C.c_int32,
                                   C.POINTER(mcv_tuning), _vp, C.POINTER(_vp)]),
    "mcv_batch_iterate": (C.c_int, [_vp, C.c_uint32, C.c_int32]),
    "mcv_batch_get_history": (C.c_int, [_vp, C.c_int32, _dp, C.c_int32, _i32p]),
    "mcv_batch_result": (C.c_int, [_vp, C.c_int32, C.c_int32, C.POINTER(mcv_summary)]),
    "mcv_batch_get_state": (C.c_int, [_vp, C.c_int32, _dp, _dp, _i64p]),
    "mcv_batch_info": (C.c_int, [_vp, _i32p, _i32p, _i32p, C.POINTER(mcv_tuning)]),
    "mcv_batch_timing": (C.c_int, [_vp, C.c_int32, _dp, _dp]),
    "mcv_batch_destroy": (None, [_vp]),
    "mcv_autotune": (C.c_int, [C.POINTER(mcv_problem), _i64p, C.c_int32, _vp, C.c_char_p,
                               C.POINTER(mcv_tuning), _dp]),
    "mcv_tuning_key": (C.c_int, [C.POINTER(mcv_problem), _i64p, C.c_int32, C.c_char_p,
                                 C.c_size_t]),
    "mcv_server_create": (C.c_int, [C.POINTER(mcv_server_config), _vp, C.POINTER(_vp)]),
    "mcv_server_clock": (C.c_int, [_vp, _dp]),
    "mcv_server_submit": (C.c_int, [_vp, C.POINTER(mcv_problem), C.c_int64, C.c_int32,
                                    C.c_int64, _i64p]),
    "mcv_server_step": (C.c_int, [_vp, C.POINTER(mcv_step_info)]),
    "mcv_server_finished": (C.c_int, [_vp, _i64p, C.c_int32, _i32p]),
    "mcv_server_report": (C.c_int, [_vp, C.c_int64, C.POINTER(mcv_job_report)]),
    "mcv_server_events": (C.c_int, [_vp, C.c_int64, _vp]),
    "mcv_server_destroy": (None, [_vp]),
    "mcv_last_error": (C.c_char_p, []),
    "mcv_version": (C.c_char_p, []),
}

_lib = None
_exiting = False


def _torch_alloc(nbytes, ctx):
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes)))
    except Exception:  # reported to the library as an allocation failure
        return None


def _torch_free(ptr, ctx):
    if not _exiting and ptr:
        torch.cuda.caching_allocator_delete(ptr)


# kept alive for the life of the process (the library holds the pointers)
_torch_alloc_c = _ALLOC_FN(_torch_alloc)
_torch_free_c = _FREE_FN(_torch_free)


@atexit.register
def _at_exit():
    # objects collected during interpreter teardown must not call into torch
    global _exiting
    _exiting = True


def lib():
    """Load libmcv.so (raises if it was not built) and install torch's
    caching allocator as its device allocator."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        use_torch_allocator(True)
    return _lib


def use_torch_allocator(enable: bool = True):
    """mcv_set_allocator: torch's caching allocator (enable) or the library's
    own hipMalloc / hipFree.  Blocks already made are returned to the
    allocator that made them."""
    L = lib()
    if enable:
        _check(L.mcv_set_allocator(_torch_alloc_c, _torch_free_c, None))
    else:
        _check(L.mcv_set_allocator(_ALLOC_FN(), _FREE_FN(), None))


class MCVError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mcv status {status}: {msg}")
        self.status = status


def _check(status):
    if status != MCV_OK:
        raise MCVError(status, lib().mcv_last_error().decode())


def _p(a, t):
    return a.ctypes.data_as(t)


def current_stream_handle() -> int:
    """The HIP stream torch is using on the current device."""
    return int(torch.cuda.current_stream().cuda_stream)


# Thin wrappers with the C-ABI names -------------------------------------------------
def mcv_create_integrator(problem: mcv_problem, stream: Optional[int] = None):
    h = _vp()
    _check(lib().mcv_create_integrator(C.byref(problem), stream, C.byref(h)))
    return h


def mcv_sample_iteration(h, n_points: int):
    _check(lib().mcv_sample_iteration(h, int(n_points)))


def mcv_refine(h, what: int):
    _check(lib().mcv_refine(h, int(what)))


def mcv_result(h, first_iter: int = 0) -> mcv_summary:
    s = mcv_summary()
    _check(lib().mcv_result(h, int(first_iter), C.byref(s)))
    return s


def mcv_destroy(h):
    lib().mcv_destroy(h)


def problem_struct(p, max_iterations: int, keep: list) -> mcv_problem:
    """An mcv_problem over contiguous copies of the problem's arrays (appended
    to `keep`, which must outlive the call that reads the struct)."""
    arrs = [np.ascontiguousarray(a, dt) for a, dt in (
        (p.peak_kind, np.int32), (p.peak_loc, np.float64), (p.peak_width, np.float64),
        (p.peak_weight, np.float64), (p.chan_kind, np.int32), (p.chan_loc, np.float64),
        (p.chan_width, np.float64))]
    keep.extend(arrs)
    k = arrs
    return mcv_problem(p.dim, p.n_channels, p.n_bins, p.n_peaks, int(p.precision),
                       _p(k[0], _i32p), _p(k[1], _dp), _p(k[2], _dp), _p(k[3], _dp),
                       _p(k[4], _i32p), _p(k[5], _dp), _p(k[6], _dp), p.seed,
                       p.grid_power, p.channel_power, p.min_calls, max_iterations,
                       int(getattr(p, "rng", 0)), int(getattr(p, "strat", 0)))


def _tuning(t) -> Optional[mcv_tuning]:
    if t is None:
        return None
    if isinstance(t, mcv_tuning):
        return t
    return mcv_tuning(int(t["block"]), int(t["unit_calls"]), int(t.get("launch_bound", 0)),
                      int(t.get("term_bound", 1)))


def tuning_dict(t: mcv_tuning) -> dict:
    return {"block": t.block, "unit_calls": t.unit_calls, "launch_bound": t.launch_bound,
            "term_bound": t.term_bound}


def _problem_array(problems, max_iterations):
    keep: list = []
    arr = (mcv_problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = problem_struct(p, max_iterations, keep)
    return arr, keep


class Integrator:
    """One integration job on the GPU (owns an mcv_integrator handle)."""

    def __init__(self, problem, stream: Optional[int] = None, max_iterations: int = 1000):
        p = problem
        self.problem = p
        self.d, self.K, self.n, self.P = p.dim, p.n_channels, p.n_bins, p.n_peaks
        self.precision = int(p.precision)
        self._keep: list = []
        st = problem_struct(p, max_iterations, self._keep)
        if stream is None:
            stream = current_stream_handle()
        self._h = mcv_create_integrator(st, stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().mcv_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_stream(self, stream: Optional[int]):
        _check(lib().mcv_set_stream(self._h, stream))

    def sample_iteration(self, n_points: int):
        mcv_sample_iteration(self._h, n_points)

    def refine(self, what: int = MCV_REFINE_GRID | MCV_REFINE_ALPHA):
        mcv_refine(self._h, what)

    def set_equivalences(self, eq):
        """mcv_set_equivalences: rows (c, c', perm[d], mode[d]); [] removes."""
        e = np.ascontiguousarray(np.asarray(eq, np.int32).reshape(-1, 2 + 2 * self.d))
        _check(lib().mcv_set_equivalences(self._h, e.shape[0], _p(e, _i32p)))

    def result(self, first_iter: int = 0) -> dict:
        s = mcv_result(self._h, first_iter)
        return {"integral": s.integral, "error": s.error, "chi2_ndf": s.chi2_ndf,
                "w_max": s.w_max, "n_iter": s.n_iter_used, "n_points": s.n_points,
                "n_bad": s.n_bad}

    @property
    def history(self) -> np.ndarray:
        n = C.c_int32(0)
        _check(lib().mcv_get_history(self._h, None, 0, C.byref(n)))
        out = np.zeros((n.value, 5))
        if n.value:
            _check(lib().mcv_get_history(self._h, _p(out, _dp), n.value, C.byref(n)))
        return out

    def get_state(self):
        e = np.zeros((self.K, self.d, self.n + 1))
        a = np.zeros(self.K)
        nc = np.zeros(self.K + 1, np.int64)
        _check(lib().mcv_get_state(self._h, _p(e, _dp), _p(a, _dp), _p(nc, _i64p)))
        return e, a, nc

    @property
    def edges(self):
        return self.get_state()[0]

    @property
    def alpha(self):
        return self.get_state()[1]

    @property
    def alloc(self):
        return self.get_state()[2]

    def set_state_for_test(self, edges=None, alpha=None):
        e = None if edges is None else np.ascontiguousarray(edges, np.float64)
        a = None if alpha is None else np.ascontiguousarray(alpha, np.float64)
        _check(lib().mcv_set_state_for_test(self._h, None if e is None else _p(e, _dp),
                                            None if a is None else _p(a, _dp)))

    def pass_stats(self):
        h = np.zeros((self.K, self.d, self.n))
        st = np.zeros((self.K, 7))
        _check(lib().mcv_get_pass_stats(self._h, _p(h, _dp), _p(st, _dp)))
        return h, st

    @property
    def hist(self):
        return self.pass_stats()[0]

    @property
    def channel_stats(self):
        return self.pass_stats()[1]

    def trace(self, n_points, iteration, first, count, n_words=None):
        d, K = self.d, self.K
        n_words = d if n_words is None else n_words
        words = np.zeros((count, max(n_words, 1)), np.uint32)
        chan = np.zeros(count, np.int32)
        bins = np.zeros((count, K, d), np.int32)
        p = np.zeros((count, d))
        fgw = np.zeros((count, 3))
        _check(lib().mcv_debug_trace(self._h, n_points, iteration, first, count, n_words,
                                     _p(words, _u32p), _p(chan, _i32p), _p(bins, _i32p),
                                     _p(p, _dp), _p(fgw, _dp)))
        return {"words": words[:, :n_words], "chan": chan, "bins": bins, "p": p,
                "f": fgw[:, 0], "g": fgw[:, 1], "w": fgw[:, 2]}

    def sample_trace(self, n_points, iteration, first, count):
        """f, g, w of calls [first, first+count) as the sample-pass kernel
        computes them (mcv_debug_sample_trace)."""
        fgw = np.zeros((count, 3))
        _check(lib().mcv_debug_sample_trace(self._h, n_points, iteration, first, count,
                                            _p(fgw, _dp)))
        return {"f": fgw[:, 0], "g": fgw[:, 1], "w": fgw[:, 2]}

    def unweight(self, n_events: int, batch: int = 65536, out: Optional[torch.Tensor] = None):
        dt = torch.float32 if self.precision == MCV_FP32_MIXED else torch.float64
        if out is None:
            out = torch.empty((self.d, n_events), dtype=dt, device="cuda")
        assert out.dtype == dt and out.is_contiguous() and tuple(out.shape) == (self.d, n_events)
        st = np.zeros(4)
        _check(lib().mcv_unweight(self._h, n_events, batch, C.c_void_p(out.data_ptr()),
                                  _p(st, _dp)))
        return out, {"trials": int(st[0]), "n_overweight": int(st[1]), "w_max": st[2],
                     "efficiency": st[3]}

    def unweight_signed(self, n_events: int, batch: int = 65536):
        """mcv_unweight_signed: events [d][n_events], their weights' signs
        (int8 tensor, +1 / -1) and the stats."""
        dt = torch.float32 if self.precision == MCV_FP32_MIXED else torch.float64
        out = torch.empty((self.d, n_events), dtype=dt, device="cuda")
        sg = torch.empty(n_events, dtype=torch.int8, device="cuda")
        st = np.zeros(4)
        _check(lib().mcv_unweight_signed(self._h, n_events, batch, C.c_void_p(out.data_ptr()),
                                         C.c_void_p(sg.data_ptr()), _p(st, _dp)))
        return out, sg, {"trials": int(st[0]), "n_overweight": int(st[1]), "w_max": st[2],
                         "efficiency": st[3]}

    def pass_timing(self, iteration: int):
        """(sample-kernel ms, workgroups) of pass `iteration`."""
        ms = C.c_double(0.0)
        g = C.c_int32(0)
        _check(lib().mcv_pass_timing(self._h, int(iteration), C.byref(ms), C.byref(g)))
        return ms.value, g.value

    def save_state(self) -> bytes:
        n = C.c_size_t(0)
        _check(lib().mcv_save_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().mcv_save_state(self._h, buf, C.byref(n)))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(lib().mcv_load_state(self._h, buf, len(blob)))


def autotune(problems, n_points, cache_path: Optional[str] = None,
             stream: Optional[int] = None, max_iterations: int = 16):
    """mcv_autotune: the fastest launch shape of the batched sample kernel
    for these jobs (a dict) and its sample-pass time in ms."""
    arr, keep = _problem_array(problems, max_iterations)
    npts = np.ascontiguousarray(n_points, np.int64)
    out = mcv_tuning()
    ms = C.c_double(0.0)
    if stream is None:
        stream = current_stream_handle()
    _check(lib().mcv_autotune(arr, _p(npts, _i64p), len(problems), stream,
                              None if cache_path is None else cache_path.encode(),
                              C.byref(out), C.byref(ms)))
    return tuning_dict(out), ms.value


def tuning_key(problems, n_points) -> str:
    arr, keep = _problem_array(problems, 1)
    npts = np.ascontiguousarray(n_points, np.int64)
    buf = C.create_string_buffer(256)
    _check(lib().mcv_tuning_key(arr, _p(npts, _i64p), len(problems), buf, 256))
    return buf.value.decode()


class Batch:
    """Many integration jobs advancing one iteration together (mcv_batch)."""

    def __init__(self, problems, n_points, tuning=None, stream: Optional[int] = None,
                 max_iterations: int = 64):
        self.problems = list(problems)
        self.n_jobs = len(self.problems)
        self.precision = int(self.problems[0].precision)
        arr, keep = _problem_array(self.problems, max_iterations)
        npts = np.ascontiguousarray(n_points, np.int64)
        t = _tuning(tuning)
        if stream is None:
            stream = current_stream_handle()
        self._h = _vp()
        _check(lib().mcv_batch_create(arr, _p(npts, _i64p), self.n_jobs,
                                      None if t is None else C.byref(t), stream,
                                      C.byref(self._h)))
        self.n_iter = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().mcv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def iterate(self, what: int = MCV_REFINE_GRID | MCV_REFINE_ALPHA, graph: bool = True):
        _check(lib().mcv_batch_iterate(self._h, int(what), 1 if graph else 0))
        self.n_iter += 1

    def history(self, job: int) -> np.ndarray:
        n = C.c_int32(0)
        _check(lib().mcv_batch_get_history(self._h, job, None, 0, C.byref(n)))
        out = np.zeros((n.value, 5))
        if n.value:
            _check(lib().mcv_batch_get_history(self._h, job, _p(out, _dp), n.value, C.byref(n)))
        return out

    def result(self, job: int, first_iter: int = 0) -> dict:
        s = mcv_summary()
        _check(lib().mcv_batch_result(self._h, job, first_iter, C.byref(s)))
        return {"integral": s.integral, "error": s.error, "chi2_ndf": s.chi2_ndf,
                "w_max": s.w_max, "n_iter": s.n_iter_used, "n_points": s.n_points,
                "n_bad": s.n_bad}

    def get_state(self, job: int):
        p = self.problems[job]
        e = np.zeros((p.n_channels, p.dim, p.n_bins + 1))
        a = np.zeros(p.n_channels)
        nc = np.zeros(p.n_channels + 1, np.int64)
        _check(lib().mcv_batch_get_state(self._h, job, _p(e, _dp), _p(a, _dp), _p(nc, _i64p)))
        return e, a, nc

    def info(self) -> dict:
        u, g, l = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        t = mcv_tuning()
        _check(lib().mcv_batch_info(self._h, C.byref(u), C.byref(g), C.byref(l), C.byref(t)))
        return {"units": u.value, "workgroups": g.value, "lds_bytes": l.value,
                "tuning": tuning_dict(t)}

    def timing(self, iteration: int):
        """(iteration ms, sample-kernel ms or -1 for graph replays)."""
        a, b = C.c_double(0.0), C.c_double(0.0)
        _check(lib().mcv_batch_timing(self._h, int(iteration), C.byref(a), C.byref(b)))
        return a.value, b.value


JOB_STATES = {0: "queued", 1: "integrating", 2: "generating", 3: "done"}


def _summary_dict(s: mcv_summary) -> dict:
    return {"integral": s.integral, "error": s.error, "chi2_ndf": s.chi2_ndf, "w_max": s.w_max,
            "n_iter": s.n_iter_used, "n_points": s.n_points, "n_bad": s.n_bad}


class Server:
    """Continuous-batching server of integration requests (mcv_server)."""

    def __init__(self, precision: int = MCV_FP64, max_active: int = 4096, hbm_budget: int = 0,
                 unweight_batch: int = 65536, tuning=None, keep_events: bool = False,
                 stream: Optional[int] = None):
        self.precision = int(precision)
        t = _tuning(tuning) or mcv_tuning(0, 0, 0, 0)
        cfg = mcv_server_config(self.precision, max_active, hbm_budget, unweight_batch, t,
                                1 if keep_events else 0)
        if stream is None:
            stream = current_stream_handle()
        self._h = _vp()
        _check(lib().mcv_server_create(C.byref(cfg), stream, C.byref(self._h)))
        self.dims = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().mcv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def clock(self) -> float:
        t = C.c_double(0.0)
        _check(lib().mcv_server_clock(self._h, C.byref(t)))
        return t.value

    def submit(self, problem, n_points: int, n_iterations: int, n_events: int) -> int:
        keep: list = []
        st = problem_struct(problem, n_iterations, keep)
        t = C.c_int64(0)
        _check(lib().mcv_server_submit(self._h, C.byref(st), int(n_points), int(n_iterations),
                                       int(n_events), C.byref(t)))
        self.dims[t.value] = (problem.dim, int(n_events))
        return t.value

    def step(self) -> dict:
        info = mcv_step_info()
        _check(lib().mcv_server_step(self._h, C.byref(info)))
        return {f: getattr(info, f) for f, _ in mcv_step_info._fields_}

    def finished(self, cap: int = 4096):
        buf = (C.c_int64 * cap)()
        n = C.c_int32(0)
        _check(lib().mcv_server_finished(self._h, buf, cap, C.byref(n)))
        return [buf[i] for i in range(n.value)]

    def report(self, ticket: int) -> dict:
        r = mcv_job_report()
        _check(lib().mcv_server_report(self._h, int(ticket), C.byref(r)))
        return {"state": JOB_STATES[r.state], "iterations_done": r.iterations_done,
                "result": _summary_dict(r.result), "n_events": r.n_events, "trials": r.trials,
                "n_overweight": r.n_overweight, "w_max": r.w_max, "efficiency": r.efficiency,
                "submit_time": r.submit_time, "admit_time": r.admit_time,
                "finish_time": r.finish_time, "device_bytes": r.device_bytes}

    def events(self, ticket: int) -> torch.Tensor:
        d, n = self.dims[ticket]
        dt = torch.float32 if self.precision == MCV_FP32_MIXED else torch.float64
        out = torch.empty((d, n), dtype=dt, device="cuda")
        _check(lib().mcv_server_events(self._h, int(ticket), C.c_void_p(out.data_ptr())))
        return out

    def run_until_idle(self, max_steps: int = 100000):
        for _ in range(max_steps):
            info = self.step()
            if info["n_active"] == 0 and info["n_queued"] == 0:
                return
        raise RuntimeError("server did not drain")
