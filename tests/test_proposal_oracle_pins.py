"""Pins of the proposal oracle (CPU only): gradients by central differences, top-C against
hand-built ties, C = K reducing to the dense E-step, captured mass by its definition, Adam's
closed form with beta1 = beta2 = 0."""
import numpy as np
import pytest

from oracle import proposal_ref as PR
from oracle import vbgs_ref as R
from synth import scenes


def _mlp(D, H, K, seed, X0=None):
    w = scenes.mlp_init(D, H, K, seed, X0)
    return PR.MLP(**{k: v.astype(np.float64) for k, v in w.items()})


def test_gradients_match_central_differences():
    g = np.random.default_rng(0)
    D, H, K, B, M = 6, 8, 64, 16, 5
    X = g.uniform(0, 1, (B, D))
    m = _mlp(D, H, K, 1, X)
    m.b1 += 0.1
    m.b2 += 0.1
    m.beta[:] = g.normal(0, 0.3, K)
    tk = np.stack([g.choice(K, M, replace=False) for _ in range(B)])
    tk[3, 2:] = -1
    tr = g.uniform(0.1, 1.0, (B, M))
    L, grads = PR.loss_and_grads(m, X, tk, tr)
    assert abs(L - PR.loss_only(m, X, tk, tr)) < 1e-14
    h = 1e-6
    for P, G in zip(m.params(), grads):
        idx = [tuple(g.integers(0, s) for s in P.shape) for _ in range(6)]
        for i in idx:
            old = P[i]
            P[i] = old + h
            lp = PR.loss_only(m, X, tk, tr)
            P[i] = old - h
            lm = PR.loss_only(m, X, tk, tr)
            P[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(fd)), (P.shape, i, fd, G[i])


def test_topc_ties_break_on_smaller_index():
    z = np.array([[1.0, 3.0, 3.0, 2.0, 3.0, -1.0]])
    assert PR.topc(z, 2).tolist() == [[1, 2]]
    assert PR.topc(z, 4).tolist() == [[1, 2, 3, 4]]
    assert PR.topc(z, 10).tolist() == [[0, 1, 2, 3, 4, 5]]
    g = np.random.default_rng(2)
    z = g.normal(size=(20, 50))
    c = PR.topc(z, 7)
    for n in range(20):
        thr = np.sort(z[n])[-7]
        assert set(c[n]) == set(np.nonzero(z[n] >= thr)[0])


def test_pruned_with_all_components_is_the_dense_estep():
    X, pr = scenes.random_problem(300, 12, 5, seed=4)
    q = R.NW.from_prior(pr)
    cand = np.tile(np.arange(12), (300, 1))
    lse_c, st = PR.pruned_estep(X, q, cand)
    ls = R.lse(X, q)
    ref = R.stats(X, q, ls, scatter=False)
    assert np.allclose(lse_c, ls, rtol=1e-13, atol=1e-12)
    assert np.allclose(st.Nk, ref.Nk, rtol=1e-11, atol=1e-12)
    assert np.allclose(st.S2, ref.S2, rtol=1e-11, atol=1e-12)


def test_captured_mass_is_the_candidates_share_of_r():
    X, pr = scenes.random_problem(200, 30, 6, seed=5)
    q = R.NW.from_prior(pr)
    g = np.random.default_rng(6)
    cand = np.stack([np.sort(g.choice(30, 8, replace=False)) for _ in range(200)])
    lse_c, _ = PR.pruned_estep(X, q, cand)
    cap = PR.captured_log_mass(lse_c, R.lse(X, q))
    Rr = R.responsibilities(X, q)
    share = np.take_along_axis(Rr, cand, axis=1).sum(axis=1)
    assert np.allclose(np.exp(cap), share, rtol=1e-10)
    assert (cap <= 1e-12).all()


def test_fallback_decision_cases():
    b = np.log1p(-1e-4)
    assert PR.fallback_decision(np.zeros(100))[0] is False
    assert PR.fallback_decision(np.full(100, -1.0))[0] is True
    cap = np.zeros(1000)
    cap[:5] = -1e-3           # 0.5% below the bound, aggregate still fine
    assert PR.fallback_decision(cap)[0] is False
    cap[:20] = -1e-3          # 2% below the bound
    assert PR.fallback_decision(cap)[0] is True


def test_adam_with_zero_betas_moves_by_lr_times_sign():
    w = [np.array([2.0, -3.0, 0.5])]
    g = [w[0].copy()]          # gradient of 0.5 w^2
    m1, m2 = [np.zeros(3)], [np.zeros(3)]
    PR.adam_step(w, g, m1, m2, 1, PR.Adam(lr=0.1, b1=0.0, b2=0.0, eps=0.0))
    assert np.allclose(w[0], [1.9, -2.9, 0.4], atol=1e-15)
