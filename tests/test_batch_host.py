"""Host-side checks of the batch API that need no GPU: argument validation
before any device call, the autotuner's workload key, and its JSON cache
(a hit returns without touching the device; a malformed file is refused)."""
import json

import pytest

import workloads as W


def _mcv():
    from paper_1811_09711_amd import mcv
    return mcv


def _arr(ps, n_iter=16):
    import ctypes as C

    import numpy as np
    mcv = _mcv()
    arr, keep = mcv._problem_array(ps, n_iter)
    return arr, keep


def _create(ps, npts, tuning=None):
    import ctypes as C

    import numpy as np
    mcv = _mcv()
    arr, keep = _arr(ps)
    n = np.ascontiguousarray(npts, np.int64)
    h = C.c_void_p()
    t = None if tuning is None else C.byref(mcv._tuning(tuning))
    return mcv.lib().mcv_batch_create(arr, mcv._p(n, mcv._i64p), len(ps), t, None, C.byref(h))


def test_batch_create_rejects_mixed_precision():
    mcv = _mcv()
    ps = [W.batch_job(1), W.batch_job(2).with_(precision=1)]
    assert _create(ps, [50_000, 50_000]) == mcv.MCV_E_INVALID
    assert b"precision" in mcv.lib().mcv_last_error()


@pytest.mark.parametrize("tuning,msg", [
    ({"block": 100, "unit_calls": 4096}, b"block"),
    ({"block": 256, "unit_calls": 128}, b"unit_calls"),
    ({"block": 256, "unit_calls": 4096, "launch_bound": 768}, b"launch_bound"),
    ({"block": 1024, "unit_calls": 4096, "launch_bound": 512}, b"launch_bound"),
    ({"block": 512, "unit_calls": 4096, "launch_bound": 256}, b"launch_bound"),
    ({"block": 256, "unit_calls": 4096, "launch_bound": 256, "term_bound": 2}, b"term_bound"),
])
def test_batch_create_rejects_bad_tuning(tuning, msg):
    mcv = _mcv()
    assert _create([W.batch_job(1)], [50_000], tuning) == mcv.MCV_E_INVALID
    assert msg in mcv.lib().mcv_last_error()


def test_batch_create_names_the_bad_job():
    mcv = _mcv()
    bad = W.batch_job(3)
    bad.peak_width[0, 0] = -1.0
    bad.peak_kind[0, 0] = 1
    assert _create([W.batch_job(1), bad], [50_000, 50_000]) == mcv.MCV_E_INVALID
    assert mcv.lib().mcv_last_error().startswith(b"job 1:")


def test_tuning_key_buckets():
    mcv = _mcv()
    ps = [W.batch_job(4_000_000 + j) for j in range(16)]
    npts = [p.n_points for p in ps]
    key = mcv.tuning_key(ps, npts)
    assert key.startswith("fp64 d<=12 K<=2^6 n<=50 calls~2^")
    assert mcv.tuning_key([p.with_(precision=1) for p in ps], npts).startswith("fp32 ")


def test_cache_hit_needs_no_device(tmp_path):
    mcv = _mcv()
    ps = [W.batch_job(4_000_000 + j) for j in range(4)]
    npts = [p.n_points for p in ps]
    key = mcv.tuning_key(ps, npts)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"other": {"block": 64, "unit_calls": 64, "ms": 1},
                                key: {"block": 512, "unit_calls": 8192, "launch_bound": 512,
                                      "ms": 12.5}}))
    t, ms = mcv.autotune(ps, npts, cache_path=str(path), stream=0)
    # an entry without term_bound reads as term_bound 1
    assert t == {"block": 512, "unit_calls": 8192, "launch_bound": 512, "term_bound": 1}
    assert ms == 12.5
    path.write_text(json.dumps({key: {"block": 256, "unit_calls": 4096, "launch_bound": 256,
                                      "term_bound": 0, "ms": 3.0}}))
    t, ms = mcv.autotune(ps, npts, cache_path=str(path), stream=0)
    assert t == {"block": 256, "unit_calls": 4096, "launch_bound": 256, "term_bound": 0}
    assert ms == 3.0


def test_malformed_cache_is_refused(tmp_path):
    mcv = _mcv()
    ps = [W.batch_job(5)]
    path = tmp_path / "tune.json"
    path.write_text('{"x": {"block": }')
    with pytest.raises(mcv.MCVError) as ei:
        mcv.autotune(ps, [50_000], cache_path=str(path), stream=0)
    assert ei.value.status == mcv.MCV_E_INVALID
