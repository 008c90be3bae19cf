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


def _hand_network():
    """D = 3, H = 2, K = 3 network whose outputs on two points are worked out by hand below:
    non-zero input centre and scales (normalisation order), a non-square W1 and a non-symmetric
    W2 (operand orientation), and pre-activations of both signs (the ReLUs)."""
    return PR.MLP(W1=np.array([[1.0, -1.0, 0.5], [0.0, 2.0, 1.0]]), b1=np.array([3.0, -1.0]),
                  W2=np.array([[1.0, 2.0], [-3.0, 0.5]]), b2=np.array([0.0, 6.0]),
                  E=np.array([[1.0, 0.0], [0.5, -1.0], [-2.0, 3.0]]), beta=np.array([0.0, 1.0, -1.0]),
                  mu_in=np.array([1.0, 0.0, -1.0]), inv_s_in=np.array([2.0, 0.5, 1.0]))


def test_forward_and_logits_on_a_hand_built_network():
    # point 0: x' = ((2-1)2, (4-0)0.5, (-3+1)1) = (2, 2, -2)
    #   W1 x' + b1 = (2 - 2 - 1 + 3, 4 - 2 - 1) = (2, 1) -> h1 = (2, 1)
    #   W2 h1 + b2 = (2 + 2 + 0, -6 + 0.5 + 6) = (4, 0.5) -> h2 = (4, 0.5)
    #   z = (4, 2 - 0.5 + 1, -8 + 1.5 - 1) = (4, 2.5, -7.5)
    # point 1: x' = (0, -1, 1); W1 x' + b1 = (1 + 0.5 + 3, -2 + 1 - 1) = (4.5, -2) -> h1 = (4.5, 0)
    #   W2 h1 + b2 = (4.5, -13.5 + 6) = (4.5, -7.5) -> h2 = (4.5, 0); z = (4.5, 3.25, -10)
    m = _hand_network()
    X = np.array([[2.0, 4.0, -3.0], [1.0, -2.0, 0.0]])
    x, h1, h2 = PR.forward(m, X)
    assert np.array_equal(x, [[2.0, 2.0, -2.0], [0.0, -1.0, 1.0]])
    assert np.array_equal(h1, [[2.0, 1.0], [4.5, 0.0]])
    assert np.array_equal(h2, [[4.0, 0.5], [4.5, 0.0]])
    assert np.array_equal(PR.logits(m, X), [[4.0, 2.5, -7.5], [4.5, 3.25, -10.0]])


def test_loss_and_beta_gradient_closed_form_with_zero_embeddings():
    """E = 0 makes every logit z_nk = beta_k. With beta = (0, ln 3, ln 4), LSE = ln 8 and
    softmax = (1/8, 3/8, 1/2). Rows: targets {2: 1, 0: 3} (renormalised to 1/4, 3/4; the padded
    slot's weight is ignored), one-hot {1}, none. Loss per row: ln 8 - ln 4 / 4 = 2.5 ln 2,
    ln 8 - ln 3, ln 8; the mean is (8.5 ln 2 - ln 3) / 3. dL/dbeta = mean(softmax - rbar) =
    ((-5/8 + 1/8 + 1/8), (3/8 - 5/8 + 3/8), (1/4 + 1/2 + 1/2)) / 3 = (-1/8, 1/24, 5/12), and no
    gradient reaches the layers below (dh2 = dz E = 0)."""
    m = _hand_network()
    m.E[:] = 0.0
    m.beta[:] = [0.0, np.log(3.0), np.log(4.0)]
    X = np.array([[2.0, 4.0, -3.0], [1.0, -2.0, 0.0], [0.0, 0.0, 0.0]])
    tk = np.array([[2, 0, -1], [1, -1, -1], [-1, -1, -1]])
    tr = np.array([[1.0, 3.0, 5.0], [0.2, 0.0, 0.0], [0.0, 0.0, 0.0]])
    want = (8.5 * np.log(2.0) - np.log(3.0)) / 3.0
    assert abs(PR.loss_only(m, X, tk, tr) - want) < 1e-15
    L, (gW1, gb1, gW2, gb2, gE, gbeta) = PR.loss_and_grads(m, X, tk, tr)
    assert abs(L - want) < 1e-15
    assert np.allclose(gbeta, [-1.0 / 8.0, 1.0 / 24.0, 5.0 / 12.0], rtol=0, atol=1e-15)
    for gz in (gW1, gb1, gW2, gb2):
        assert not gz.any()


def test_adam_two_steps_with_default_betas():
    """beta1 = 0.9, beta2 = 0.999, gradients 1 then -2 (exact fractions):
    step 1: m = 1/10, v = 1/1000, bias-corrected m^ = v^ = 1 -> move -lr.
    step 2: m = 9/100 - 2/10 = -11/100, v = 999/10^6 + 4/1000 = 4999/10^6,
    m^ = (-11/100) / (19/100) = -11/19, v^ = (4999/10^6) / (1999/10^6) = 4999/1999,
    move -lr m^ / sqrt(v^) = +0.36610352703584553 lr."""
    lr = 0.01
    w = [np.array([0.0])]
    m1, m2 = [np.zeros(1)], [np.zeros(1)]
    PR.adam_step(w, [np.array([1.0])], m1, m2, 1, PR.Adam(lr=lr, eps=0.0))
    assert abs(w[0][0] + lr) < 1e-15 * lr
    assert abs(m1[0][0] - 0.1) < 1e-15 and abs(m2[0][0] - 1e-3) < 1e-17
    PR.adam_step(w, [np.array([-2.0])], m1, m2, 2, PR.Adam(lr=lr, eps=0.0))
    assert abs(m1[0][0] + 0.11) < 1e-15 and abs(m2[0][0] - 4.999e-3) < 1e-16
    assert abs(w[0][0] - (-lr + 0.36610352703584553 * lr)) < 1e-15


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every step,
    so each step moves by lr sign(g) whatever the betas (eps = 0)."""
    w = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.3, -7.0, 1e-3])]
    m1, m2 = [np.zeros(3)], [np.zeros(3)]
    for t in range(1, 6):
        PR.adam_step(w, g, m1, m2, t, PR.Adam(lr=0.05, b1=0.9, b2=0.999, eps=0.0))
        assert np.allclose(w[0], np.array([1.0, -2.0, 3.0]) - 0.05 * t * np.sign(g[0]), rtol=0, atol=1e-12)
