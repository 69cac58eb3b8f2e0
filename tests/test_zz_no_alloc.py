"""mcv_unweight_noalloc: the unweighting entry point for callers that cannot
allocate device memory gives exactly mcv_unweight's events and statistics
(the same kernels, with the work buffers in a static per-device area), on two
calls in a row (the second smaller), allocates nothing, and refuses a batch
whose buffers do not fit the area."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_util import mcv

pytestmark = pytest.mark.gpu


def _pair(p, n_points):
    """Two integrators in the same adapted state (the second loads the
    first's saved state: rebinning sums per-bin weights with atomics, so two
    separately adapted integrators differ at the last bit)."""
    M = mcv()
    a, b = M.Integrator(p), M.Integrator(p)
    a.sample_iteration(n_points)
    a.refine()
    a.sample_iteration(n_points)
    b.load_state(a.save_state())
    return a, b


def _noalloc(integ, n_events, batch):
    import torch
    M = mcv()
    dt = torch.float32 if integ.precision == M.MCV_FP32_MIXED else torch.float64
    out = torch.empty((integ.d, n_events), dtype=dt, device="cuda")
    st = np.zeros(4)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    rc = M.lib().mcv_unweight_noalloc(integ._h, n_events, batch, C.c_void_p(out.data_ptr()),
                                      st.ctypes.data_as(C.POINTER(C.c_double)))
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before  # nothing allocated through torch
    return rc, out, st


@pytest.mark.parametrize("maker,prec", [(W.config2, 0), (lambda: W.mixed_problem(10, 8, 4, 100, seed=36), 1)])
def test_noalloc_matches_unweight_on_two_calls(maker, prec):
    M = mcv()
    p = maker().with_(precision=prec)
    a, b = _pair(p, 200_000)
    for n_ev, batch in ((4000, 32768), (700, 5000)):  # the second call smaller
        ev_a, st_a = a.unweight(n_ev, batch=batch)
        rc, ev_b, st_b = _noalloc(b, n_ev, batch)
        assert rc == M.MCV_OK, M.lib().mcv_last_error()
        assert st_b[0] == st_a["trials"] and st_b[1] == st_a["n_overweight"]
        assert st_b[2] == st_a["w_max"] and st_b[3] == st_a["efficiency"]
        assert ev_b.dtype == ev_a.dtype
        np.testing.assert_array_equal(ev_b.cpu().numpy(), ev_a.cpu().numpy())


def test_noalloc_refuses_a_batch_beyond_the_area():
    M = mcv()
    a, _ = _pair(W.config2(), 50_000)
    # d = 6, FP64: 9 + 48 bytes per trial; 2^18 trials need about 15 MB
    rc, _, _ = _noalloc(a, 100, 1 << 18)
    assert rc == M.MCV_E_INVALID
    assert b"work area" in M.lib().mcv_last_error()
    rc, ev, st = _noalloc(a, 100, 1 << 16)  # fits: works after the refusal
    assert rc == M.MCV_OK and st[0] > 0
