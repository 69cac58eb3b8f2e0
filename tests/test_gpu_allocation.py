"""The integer channel allocation on the GPU repeats the oracle's IEEE
sequence (Sec. 3.4: N_c = alpha_c N made integer; reading R16), so N_c must
be equal, not merely close, on knife-edge weight vectors: tied remainders,
remainders one ulp apart, alpha_c N one ulp from an integer, inexact products
(where a fused multiply-add would see another remainder) and binding floors."""
import numpy as np
import pytest

import alpha_cases
import workloads as W
from gpu_util import mcv

pytestmark = pytest.mark.gpu


def test_allocation_equals_oracle_on_adversarial_alpha():
    import oracle
    p8 = W.gauss_mixture(2, 8, 8, seed=61)
    gpus = {}
    n = 0
    for alpha, N, kind in alpha_cases.cases():
        K = len(alpha)
        if K not in gpus:
            p = p8.with_(peak_kind=p8.peak_kind[:K], peak_loc=p8.peak_loc[:K],
                         peak_width=p8.peak_width[:K], peak_weight=p8.peak_weight[:K] * 0 + 1.0 / K,
                         chan_kind=p8.chan_kind[:K], chan_loc=p8.chan_loc[:K],
                         chan_width=p8.chan_width[:K])
            gpus[K] = mcv().Integrator(p, max_iterations=400)
        g = gpus[K]
        g.set_state_for_test(alpha=np.ascontiguousarray(alpha))
        g.sample_iteration(N)
        nc_o, alpha_o = oracle.allocation(alpha, N, 10)
        nc_g = g.alloc
        assert list(nc_g[:-1]) == list(nc_o), (kind, N, list(alpha))
        assert nc_g[-1] == nc_o.sum()
        np.testing.assert_array_equal(g.alpha, alpha_o)
        n += 1
    assert n == 300
