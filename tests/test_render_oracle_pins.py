"""Pins of the rendering oracle against routes that do not share its formulas.

* Monte Carlo over the posterior (mu, Lambda) ~ NW of one component: the mean of the position
  block's precision ((Lambda^-1)_ss)^-1, the mean of its log-determinant and the mean score
  E[ln N(x_s | mu_s, Sigma_ss)] match the marginal Normal-Wishart; the mean colour given the
  position, E[mu_c + Sigma_cs Sigma_ss^-1 (x_s - mu_s)], matches m_c + B (x_s - m_s);
* special cases: one component (the regression line), well separated components (each mean's own
  colour), a two-factor model (a convex combination of the component colours, with weights from
  explicit-inverse scores);
* the PSNR closed form for a constant offset.
"""
import numpy as np
import pytest
from scipy import stats as sst
from scipy.special import logsumexp

from oracle import brute
from oracle import factorised_ref as FR
from oracle import render_ref as RR
from oracle import vbgs_ref as R


def _one_component(D, seed):
    g = np.random.default_rng(seed)
    A = g.normal(0, 1, (D, D))
    Psi = A @ A.T / D + 0.3 * np.eye(D)
    return R.NW(alpha=np.array([2.0]), kappa=np.array([3.5]), m=g.uniform(0, 1, (1, D)), Winv=Psi[None],
                nu=np.array([D + 4.0]))


def _samples(q, n, seed):
    g = np.random.default_rng(seed)
    W = np.linalg.inv(q.Winv[0])
    Lam = sst.wishart(df=q.nu[0], scale=W).rvs(size=n, random_state=g)
    Sig = np.linalg.inv(Lam)
    C = np.linalg.cholesky(Sig / q.kappa[0])
    mu = q.m[0] + np.einsum("nij,nj->ni", C, g.standard_normal((n, q.D)))
    return mu, Sig


def _close(mc_values, ref, z=5.0):
    mc_values = np.asarray(mc_values)
    se = mc_values.std(axis=0) / np.sqrt(mc_values.shape[0])
    return np.all(np.abs(mc_values.mean(axis=0) - ref) <= z * se + 1e-12), (mc_values.mean(axis=0), ref, se)


@pytest.mark.parametrize("D,s", [(5, 2), (6, 3)])
def test_marginal_by_monte_carlo(D, s):
    q = _one_component(D, 10 + D)
    qs, mc, B = RR.marginal(q, s)
    mu, Sig = _samples(q, 200000, 3)
    Lss = np.linalg.inv(Sig[:, :s, :s])
    ok, info = _close(Lss.reshape(len(Lss), -1), (qs.nu[0] * np.linalg.inv(qs.Winv[0])).ravel())
    assert ok, info
    ok, info = _close(np.linalg.slogdet(Lss)[1], R.expectations(qs).ElnLam[0])
    assert ok, info
    # the score of a position: E[ln N(x_s | mu_s, Sigma_ss)] + E[ln pi] (E[ln pi] = 0 for K = 1)
    x = q.m[0, :s] + 0.2
    d = x - mu[:, :s]
    quad = np.einsum("ni,nij,nj->n", d, Lss, d)
    lnN = -0.5 * s * np.log(2 * np.pi) + 0.5 * np.linalg.slogdet(Lss)[1] - 0.5 * quad
    score = R.pair_scores(x[None], qs, np.array([0]), np.array([0]))[0]
    ok, info = _close(lnN, score)
    assert ok, info
    # the colour given the position
    reg = Sig[:, s:, :s] @ np.linalg.inv(Sig[:, :s, :s])
    col = mu[:, s:] + np.einsum("ncj,nj->nc", reg, x - mu[:, :s])
    ok, info = _close(col, mc[0] + B[0] @ (x - q.m[0, :s]))
    assert ok, info


def test_one_component_renders_its_regression_line():
    q = _one_component(5, 4)
    qs, mc, B = RR.marginal(q, 2)
    X = q.m[0, :2] + np.array([[0.0, 0.0], [0.1, -0.05], [0.2, -0.1], [0.3, -0.15]])
    col, _ = RR.render(X, qs, mc, B)
    assert np.allclose(col[0], q.m[0, 2:], atol=1e-14)
    assert np.allclose(np.diff(col, n=2, axis=0), 0.0, atol=1e-12)         # affine along the line
    assert np.allclose(col[1] - col[0], np.linalg.solve(q.Winv[0, :2, :2], q.Winv[0, :2, 2:]).T @ X[1] -
                       np.linalg.solve(q.Winv[0, :2, :2], q.Winv[0, :2, 2:]).T @ X[0], atol=1e-12)


def test_separated_components_render_their_own_colour():
    g = np.random.default_rng(5)
    K, D = 6, 5
    m = np.concatenate([np.stack([np.arange(K) * 1.0, np.zeros(K)], 1), g.uniform(0, 1, (K, 3))], 1)
    q = R.NW(alpha=np.full(K, 3.0), kappa=np.full(K, 5.0), m=m, Winv=np.broadcast_to(np.eye(D) * 1e-4, (K, D, D)).copy(),
             nu=np.full(K, 12.0))
    qs, mc, B = RR.marginal(q, 2)
    col, _ = RR.render(m[:, :2], qs, mc, B)
    assert np.allclose(col, m[:, 2:], atol=1e-9)


def test_two_factor_render_is_a_convex_combination():
    g = np.random.default_rng(6)
    K, D, s = 9, 6, 3
    q = FR.NW2(alpha=g.uniform(1, 5, K), kappa=g.uniform(1, 4, (K, 2)), m=g.uniform(0, 1, (K, D)),
               Winv=np.zeros((K, D, D)), nu=D + g.uniform(1, 5, (K, 2)), split=s)
    for b, i in enumerate((np.arange(0, s), np.arange(s, D))):
        A = g.normal(0, 0.1, (K, len(i), len(i)))
        q.Winv[:, i[:, None], i[None, :]] = np.einsum("kij,klj->kil", A, A) + 0.01 * np.eye(len(i))
    qs, mc, B = RR.marginal_factorised(q)
    X = g.uniform(0, 1, (40, s))
    col, lse = RR.render(X, qs, mc, B)
    r = brute.rho(X, q.alpha, q.kappa[:, 0], q.m[:, :s], q.Winv[:, :s, :s], q.nu[:, 0])
    w = np.exp(r - logsumexp(r, axis=1, keepdims=True))
    assert np.allclose(col, w @ q.m[:, s:], atol=1e-12)
    assert np.allclose(lse, logsumexp(r, axis=1), atol=1e-10)
    assert np.all(col >= q.m[:, s:].min(0) - 1e-12) and np.all(col <= q.m[:, s:].max(0) + 1e-12)


def test_psnr_closed_forms():
    g = np.random.default_rng(7)
    ref = g.uniform(0.2, 0.8, (32, 32, 3))
    assert RR.psnr(ref, ref)[1] == np.inf
    for delta, db in ((0.1, 20.0), (0.01, 40.0)):
        mse, p = RR.psnr(ref + delta, ref)
        assert abs(mse - (255 * delta) ** 2) < 1e-9 and abs(p - db) < 1e-10
    # values outside [0, 1] are clamped before the difference
    assert RR.psnr(np.full(3, 1.5), np.ones(3))[1] == np.inf
