"""The C ABI validates problem descriptors before touching the device, so
these checks run without a GPU: each invalid descriptor is refused with
MCV_E_INVALID and a message."""
import ctypes as C

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def M():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(root, "paper_1811_09711_amd", "libmcv.so")):
        from paper_1811_09711_amd import build
        build.build()
    from paper_1811_09711_amd import mcv
    return mcv


def _create(M, p, **over):
    arrs = [np.ascontiguousarray(a, dt) for a, dt in (
        (p.peak_kind, np.int32), (p.peak_loc, np.float64), (p.peak_width, np.float64),
        (p.peak_weight, np.float64), (p.chan_kind, np.int32), (p.chan_loc, np.float64),
        (p.chan_width, np.float64))]
    P = lambda a, t: a.ctypes.data_as(t)
    fields = dict(dim=p.dim, n_channels=p.n_channels, n_bins=p.n_bins, n_peaks=p.n_peaks,
                  precision=p.precision, seed=p.seed, grid_power=p.grid_power,
                  channel_power=p.channel_power, min_calls=p.min_calls, max_iterations=10)
    fields.update(over)
    st = M.mcv_problem(fields["dim"], fields["n_channels"], fields["n_bins"], fields["n_peaks"],
                       fields["precision"], P(arrs[0], M._i32p), P(arrs[1], M._dp),
                       P(arrs[2], M._dp), P(arrs[3], M._dp), P(arrs[4], M._i32p),
                       P(arrs[5], M._dp), P(arrs[6], M._dp), fields["seed"],
                       fields["grid_power"], fields["channel_power"], fields["min_calls"],
                       fields["max_iterations"])
    h = C.c_void_p()
    rc = M.lib().mcv_create_integrator(C.byref(st), None, C.byref(h))
    return rc, M.lib().mcv_last_error().decode()


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 0, "dim"), ("dim", 33, "dim"), ("n_bins", 0, "n_bins"), ("n_bins", 257, "n_bins"),
    ("n_channels", 0, "n_channels"), ("precision", 7, "precision"),
    ("grid_power", -1.0, "grid_power"), ("channel_power", float("nan"), "channel_power"),
    ("min_calls", 0, "min_calls"), ("max_iterations", 0, "max_iterations"),
])
def test_invalid_descriptor_fields(M, field, value, msg):
    p = W.config1()
    rc, err = _create(M, p, **{field: value})
    assert rc == M.MCV_E_INVALID
    assert msg in err


@pytest.mark.parametrize("mutate,msg", [
    (lambda p: p.peak_width.__setitem__((0, 0), 0.0), "width"),
    (lambda p: p.chan_width.__setitem__((1, 1), -1e-3), "width"),
    (lambda p: p.peak_loc.__setitem__((0, 1), 1.5), "centre"),
    (lambda p: p.chan_loc.__setitem__((0, 0), float("nan")), "centre"),
    (lambda p: p.chan_kind.__setitem__((0, 0), 9), "kind"),
    (lambda p: p.peak_weight.__setitem__(0, float("inf")), "weight"),
])
def test_invalid_shapes(M, mutate, msg):
    p = W.config1()
    p = p.with_(peak_kind=p.peak_kind.copy(), peak_loc=p.peak_loc.copy(),
                peak_width=p.peak_width.copy(), peak_weight=p.peak_weight.copy(),
                chan_kind=p.chan_kind.copy(), chan_loc=p.chan_loc.copy(),
                chan_width=p.chan_width.copy())
    mutate(p)
    rc, err = _create(M, p)
    assert rc == M.MCV_E_INVALID
    assert msg in err


def test_null_arguments(M):
    h = C.c_void_p()
    assert M.lib().mcv_create_integrator(None, None, C.byref(h)) == M.MCV_E_INVALID
    assert M.lib().mcv_sample_iteration(None, 100) == M.MCV_E_INVALID
    assert M.lib().mcv_refine(None, 1) == M.MCV_E_INVALID
    assert M.lib().mcv_result(None, 0, None) == M.MCV_E_INVALID
    M.lib().mcv_destroy(None)
