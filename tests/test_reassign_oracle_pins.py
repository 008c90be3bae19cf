"""Pins of the reassignment oracle (Alg. 1, `reassign`) against plain definitions."""
import numpy as np
import pytest

from oracle import reassign_ref as RA
from synth import scenes


def test_ord64_preserves_order():
    g = np.random.default_rng(0)
    v = np.concatenate([g.normal(0, 1e3, 500), g.normal(0, 1e-3, 500), [0.0, -0.0, 1e-300, -1e-300, 5.0, -5.0]])
    o = RA.ord64(v)
    i, j = g.integers(0, v.size, (2, 5000))
    lt = v[i] < v[j]
    assert np.all(o[i][lt] < o[j][lt])
    gt = v[i] > v[j]
    assert np.all(o[i][gt] > o[j][gt])


def test_selection_is_sorting_when_values_are_well_separated():
    g = np.random.default_rng(1)
    v = g.permutation(1000).astype(np.float64) * 1.7 - 300.0   # distinct, far apart
    assert np.array_equal(RA.select(v, 37, descending=False), np.argsort(v)[:37])
    assert np.array_equal(RA.select(v, 37, descending=True), np.argsort(-v)[:37])


def test_ties_go_to_the_lower_index():
    v = np.array([3.0, 1.0, 1.0, 2.0, 1.0 + 1e-12, 1.0])
    # values equal to ~2^-27 relative tie: indices 1, 2, 4, 5 all carry 1.0
    assert list(RA.select(v, 4, descending=False)) == [1, 2, 4, 5]
    assert list(RA.select(v, 2, descending=True)) == [0, 3]


def test_gumbel_top_n_samples_proportionally():
    # one draw: with N = 3 and n = 1, P(point i) = exp(-lse_i) / sum exp(-lse)
    lse = np.array([0.0, np.log(2.0), np.log(4.0)])
    p = np.exp(-lse) / np.exp(-lse).sum()
    hits = np.zeros(3)
    T = 20000
    for t in range(T):
        gm = scenes.gumbel_noise(3, t, cfg=99)
        pts, _ = RA.reassign(np.zeros((3, 2), np.float32), lse, gm, np.ones(3), 1)
        hits[pts[0]] += 1
    assert np.abs(hits / T - p).max() < 0.015


def test_reassign_moves_only_the_selected_means():
    X, pr = scenes.random_problem(300, 40, 3, seed=5)
    g = np.random.default_rng(2)
    lse = g.normal(-5, 3, 300)
    alpha = 1.0 + g.integers(0, 50, 40).astype(np.float64)
    gm = scenes.gumbel_noise(300, 0, cfg=98)
    pts, comps = RA.reassign(X, lse, gm, alpha, 10)
    assert len(set(pts)) == 10 and len(set(comps)) == 10
    # least used first
    assert np.all(np.diff(alpha[comps]) >= 0) and alpha[comps].max() <= np.sort(alpha)[9]
    mp, mq = RA.apply(pr.m0, pr.m0, X, pts, comps)
    assert np.array_equal(mp[comps], X[pts].astype(np.float64))
    others = np.setdiff1d(np.arange(40), comps)
    assert np.array_equal(mp[others], pr.m0[others]) and np.array_equal(mq, mp)


def test_reassign_zero_and_bounds():
    X = np.zeros((5, 2), np.float32)
    pts, comps = RA.reassign(X, np.zeros(5), np.zeros(5), np.ones(3), 0)
    assert pts.size == 0 and comps.size == 0
    with pytest.raises(ValueError):
        RA.reassign(X, np.zeros(5), np.zeros(5), np.ones(3), 4)
