"""Pins of the channel equivalences (Sec. 3.5: bin weights of equivalent
channels are combined, with a permutation of the axes and an identity /
invert / symmetric / invariant mapping, before the grids are rebinned;
reading R26: a listed channel is rebinned with the sum of its listed
equivalences, its own weights entering through the trivial entry
(c, c, identity)), checked against the geometry they must produce rather
than against the oracle's own formula:

* the worked rebinning example (n = 4, weights (0,0,0,1) give the edges
  (0, 0.8125, 0.875, 0.9375, 1)) reached through an inverted partner;
* identity-equivalent twins (two channels with the same map) end up with the
  same grid, bit for bit;
* a channel and its mirror image (p -> 1 - p), equivalent under invert, end
  up with mirrored grids;
* a channel symmetric with itself gets a grid symmetric about 1/2;
* an invariant axis keeps its grid while the other axes adapt;
* a permutation pulls the partner's other axis.
"""
import numpy as np
import pytest

import workloads as W

I, V, S, N = 0, 1, 2, 3  # identity, invert, symmetric, invariant


def _row(c, c2, perm, modes):
    return [c, c2] + list(perm) + list(modes)


def _mirror_problem():
    """d = 2: peak A and its mirror image A' (p -> 1 - p on both axes), one
    channel per peak with the peak's own shape."""
    pk = np.array([[1, 2], [1, 2]], np.int32)
    pl = np.array([[0.3, 0.2], [0.7, 0.8]])
    pw = np.array([[0.07, 0.05], [0.07, 0.05]])
    wt = np.array([0.5, 0.5])
    return W.Problem(2, 24, pk, pl, pw, wt, pk.copy(), pl.copy(), pw.copy(), seed=11,
                     name="mirror")


def test_worked_example_through_an_inverted_partner(oracle_lib):
    # channel 0 has weights (0,0,0,1) after the equivalence when channel 1's
    # (1,0,0,0) are inverted onto it and its own are zero
    p = W.constant_problem(1, 2, 4)
    o = oracle_lib.Oracle(p)
    o.sample_iteration(100)
    o.set_equivalences([_row(0, 0, [0], [I]), _row(0, 1, [0], [V])])
    h = o.hist
    # equivalent weights: own (trivial entry) + inverted partner; channel 1
    # is not listed and keeps its own
    w = o.equivalent_hist
    np.testing.assert_array_equal(w[0, 0], h[0, 0] + h[1, 0][::-1])
    np.testing.assert_array_equal(w[1, 0], h[1, 0])
    e = oracle_lib.rebin_axis(np.linspace(0, 1, 5), [0, 0, 0, 2.0])
    np.testing.assert_array_equal(e, [0, 0.8125, 0.875, 0.9375, 1])
    e = oracle_lib.rebin_axis(np.linspace(0, 1, 5), np.array([0, 0, 0, 1.0]) + np.array([1.0, 0, 0, 0])[::-1])
    np.testing.assert_array_equal(e, [0, 0.8125, 0.875, 0.9375, 1])


def test_identity_twins_get_the_same_grid(oracle_lib):
    p = W.gauss_mixture(3, 2, 20, seed=21)
    # channel 1 = a copy of channel 0's map
    p = p.with_(chan_kind=np.repeat(p.chan_kind[:1], 2, 0), chan_loc=np.repeat(p.chan_loc[:1], 2, 0),
                chan_width=np.repeat(p.chan_width[:1], 2, 0))
    o = oracle_lib.Oracle(p)
    o.set_equivalences([_row(0, 0, [0, 1, 2], [I] * 3), _row(0, 1, [0, 1, 2], [I] * 3),
                        _row(1, 1, [0, 1, 2], [I] * 3), _row(1, 0, [0, 1, 2], [I] * 3)])
    for _ in range(3):
        o.sample_iteration(20_000)
        h = o.hist
        assert not np.array_equal(h[0], h[1])  # the channels' own sums differ
        o.refine(oracle_lib.REFINE_GRID)
        e = o.edges
        np.testing.assert_array_equal(e[0], e[1])
    # without the equivalence they differ
    q = oracle_lib.Oracle(p)
    q.sample_iteration(20_000)
    q.refine(oracle_lib.REFINE_GRID)
    assert not np.array_equal(q.edges[0], q.edges[1])


def test_inverted_mirror_channels_get_mirrored_grids(oracle_lib):
    p = _mirror_problem()
    o = oracle_lib.Oracle(p)
    o.set_equivalences([_row(0, 0, [0, 1], [I, I]), _row(0, 1, [0, 1], [V, V]),
                        _row(1, 1, [0, 1], [I, I]), _row(1, 0, [0, 1], [V, V])])
    for _ in range(3):
        o.sample_iteration(40_000)
        o.refine(oracle_lib.REFINE_GRID)
        e = o.edges
        # e1_j = 1 - e0_{n-j}, to the rounding of the rebinning walk
        np.testing.assert_allclose(e[1], 1.0 - e[0][:, ::-1], rtol=0, atol=1e-14)
        assert not np.allclose(e[0], np.linspace(0, 1, p.n_bins + 1)[None, :])


def test_self_symmetric_channel_gets_a_symmetric_grid(oracle_lib):
    p = W.constant_problem(2, 1, 30).with_(
        peak_kind=np.array([[1, 2]], np.int32), peak_loc=np.array([[0.3, 0.6]]),
        peak_width=np.array([[0.1, 0.05]]))
    o = oracle_lib.Oracle(p)
    o.set_equivalences([_row(0, 0, [0, 1], [S, S])])
    o.sample_iteration(50_000)
    o.refine(oracle_lib.REFINE_GRID)
    e = o.edges[0]
    np.testing.assert_allclose(e, 1.0 - e[:, ::-1], rtol=0, atol=1e-14)
    assert np.max(np.abs(e - np.linspace(0, 1, 31))) > 0.01  # it did adapt


def test_invariant_axis_keeps_its_grid(oracle_lib):
    p = W.gauss_mixture(2, 2, 20, seed=22)
    # identity channel maps: the grids must adapt to the peaks
    p = p.with_(chan_kind=np.zeros_like(p.chan_kind))
    o = oracle_lib.Oracle(p)
    o.set_equivalences([_row(0, 0, [0, 1], [I, I]), _row(0, 1, [0, 1], [I, N])])
    before = o.edges
    o.sample_iteration(20_000)
    w = o.equivalent_hist
    assert np.all(w[0, 1] == 1.0)
    o.refine(oracle_lib.REFINE_GRID)
    after = o.edges
    np.testing.assert_allclose(after[0, 1], before[0, 1], rtol=0, atol=1e-15)
    assert np.max(np.abs(after[0, 0] - before[0, 0])) > 0.01
    assert np.max(np.abs(after[1, 1] - before[1, 1])) > 0.01


def test_permutation_pulls_the_partners_other_axis(oracle_lib):
    p = W.gauss_mixture(2, 2, 16, seed=23)
    o = oracle_lib.Oracle(p)
    o.sample_iteration(20_000)
    h = o.hist
    o.set_equivalences([_row(0, 1, [1, 0], [I, V])])
    w = o.equivalent_hist
    # channel 0 is listed without its trivial entry: only the partner counts
    np.testing.assert_array_equal(w[0, 0], h[1, 1])
    np.testing.assert_array_equal(w[0, 1], h[1, 0][::-1])
    np.testing.assert_array_equal(w[1], h[1])


def test_malformed_equivalences_are_refused(oracle_lib):
    o = oracle_lib.Oracle(W.gauss_mixture(2, 2, 8, seed=24))
    for bad in ([_row(0, 2, [0, 1], [I, I])], [_row(0, 1, [0, 0], [I, I])],
                [_row(0, 1, [0, 1], [I, 4])], [_row(-1, 1, [0, 1], [I, I])]):
        with pytest.raises(ValueError):
            o.set_equivalences(bad)
