"""The library's device memory comes from the allocator installed with
mcv_set_allocator: the binding installs torch's caching allocator, so
integrators, batches and servers show up in torch's accounting and give their
memory back when released; results do not depend on the allocator."""
import numpy as np
import pytest

import workloads as W
from gpu_util import mcv

pytestmark = pytest.mark.gpu


def _allocated():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.memory_allocated()


def test_integrator_memory_is_torchs():
    M = mcv()
    M.lib()
    p = W.config2()
    base = _allocated()
    g = M.Integrator(p)
    held = _allocated() - base
    # the job block alone holds K d M cell records of 32 bytes (FP64)
    assert held >= p.n_channels * p.dim * 512 * 32
    g.sample_iteration(100_000)
    g.refine()
    ev, _ = g.unweight(500, batch=4096)  # grows the unweighting buffers
    del ev  # the event tensor is the caller's
    assert _allocated() - base > held
    h_torch = g.history
    g.close()
    assert _allocated() == base
    # the library's own hipMalloc gives the same results and leaves torch alone
    M.use_torch_allocator(False)
    try:
        before = _allocated()
        g2 = M.Integrator(p)
        assert _allocated() == before
        g2.sample_iteration(100_000)
        g2.refine()
        np.testing.assert_array_equal(g2.history, h_torch)
        g2.close()
    finally:
        M.use_torch_allocator(True)


def test_batch_and_server_memory_is_torchs():
    M = mcv()
    ps = W.config4(6)
    npts = [min(p.n_points, 50_000) for p in ps]
    base = _allocated()
    b = M.Batch(ps, npts, max_iterations=4)
    b.iterate()
    assert _allocated() > base
    b.close()
    assert _allocated() == base
    srv = M.Server(precision=0, unweight_batch=8192)
    t = srv.submit(ps[0], npts[0], 2, 100)
    srv.run_until_idle()
    assert srv.report(t)["state"] == "done"
    assert _allocated() > base  # the server's own work buffers
    srv.close()
    assert _allocated() == base


def test_set_allocator_rejects_half_a_pair():
    M = mcv()
    L = M.lib()
    st = L.mcv_set_allocator(M._torch_alloc_c, M._FREE_FN(), None)
    assert st == M.MCV_E_INVALID
    # the allocator in use is unchanged
    base = _allocated()
    g = M.Integrator(W.config1())
    assert _allocated() > base
    g.close()
    assert _allocated() == base
