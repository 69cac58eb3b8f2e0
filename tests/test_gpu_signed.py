"""Integrands of either sign on the GPU (Sec. 3.1: NLO integrands need not
be positive semidefinite; reading R27) against the oracle: the pass (estimate,
largest |w|, sums), and unweighting by |w| with the events' signs."""
import numpy as np
import pytest

import workloads as W
from gpu_util import pair, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d", [2, 5])
def test_signed_pass_and_events_match_oracle(d):
    p = W.signed_problem(d=d)
    gpu, orc = pair(p)
    for _ in range(3):
        gpu.sample_iteration(50_000)
        orc.sample_iteration(50_000, 8)
        gpu.refine()
        orc.refine()
    gpu.sample_iteration(50_000)
    orc.sample_iteration(50_000, 8)
    hg, ho = gpu.history, orc.history
    assert rel(hg[:, 0], ho[:, 0]) < 1e-12
    assert rel(hg[:, 3], ho[:, 3]) < 1e-12  # largest |w|
    st = gpu.channel_stats
    assert np.any(st[:, 0] < 0) or np.any(st[:, 4] < 0) or ho[-1, 0] > 0
    orc.edges = gpu.edges
    orc.wmax = hg[-1, 3]
    n_ev = 4000
    ev_g, sg_g, st_g = gpu.unweight_signed(n_ev, batch=8192)
    ev_o, sg_o, st_o = orc.unweight(n_ev, batch=8192, signs=True)
    assert st_o["accept_ties"] == 0
    assert st_g["trials"] == st_o["trials"]
    assert abs(st_g["n_overweight"] - st_o["n_overweight"]) <= st_o["overweight_ties"]
    assert np.max(np.abs(ev_g.cpu().numpy() - ev_o)) < 1e-12
    np.testing.assert_array_equal(sg_g.cpu().numpy(), sg_o)
    assert (sg_o < 0).sum() > 0


def test_signed_precision_mode_vs_oracle():
    p = W.signed_problem(d=4).with_(precision=1)
    gpu, orc = pair(p)
    for _ in range(2):
        gpu.sample_iteration(200_000)
        orc.sample_iteration(200_000, 8)
        gpu.refine()
        orc.refine()
    assert rel(gpu.history[:, 0], orc.history[:, 0]) < 1e-5
