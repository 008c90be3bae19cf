"""Pins of the two-factor (spatial / colour) oracle of Sec. 2.1.2 against independent routes.

* block scores by explicit inverses summed with E[ln pi] counted once (brute.rho per factor);
* the seven-term bound of PRML 10.70 summed over the two factors (brute.elbo_bishop_blocks);
* K = 1 at the exact posterior: the bound equals ln p(X), which factorises into the two
  closed-form Normal-Wishart marginals (brute.log_marginal_k1 on each coordinate group);
* the update through natural parameters per factor (brute.update_natural);
* an uninformative colour factor (identical across components) leaves the spatial model's
  responsibilities, a textbook one-factor mixture.
"""
import numpy as np
import pytest
from scipy.special import digamma, logsumexp

from oracle import brute
from oracle import factorised_ref as F
from oracle import vbgs_ref as R
from synth import scenes


def _perturbed(p: F.NW2, seed: int) -> F.NW2:
    g = np.random.default_rng(seed)
    K, D = p.m.shape
    Winv = np.zeros_like(p.Winv)
    for b in (0, 1):
        i = p.idx(b)
        A = g.normal(0, 0.3, (K, len(i), len(i)))
        base = p.Winv[:, i][:, :, i]
        Winv[:, i[:, None], i[None, :]] = (base * g.uniform(0.5, 2.0, (K, 1, 1))
                                           + np.einsum("kij,klj->kil", A, A) * base[:, :1, :1])
    return F.NW2(alpha=p.alpha * g.uniform(0.5, 5.0, K), kappa=p.kappa * g.uniform(0.5, 4.0, (K, 2)),
                 m=p.m + g.normal(0, 0.02, p.m.shape), Winv=Winv, nu=p.nu + g.uniform(0.0, 6.0, (K, 2)),
                 split=p.split)


def _problem(N, K, D, split, seed):
    X, pr = scenes.random_problem(N, K, D, seed=seed)
    p = F.NW2.from_prior(pr, split)
    return X.astype(np.float64), p, _perturbed(p, seed + 1)


def _brute_rho(X, q: F.NW2):
    Elnpi = digamma(q.alpha) - digamma(q.alpha.sum())
    r = -Elnpi[None, :]
    for b in (0, 1):
        i = q.idx(b)
        r = r + brute.rho(X[:, i], q.alpha, q.kappa[:, b], q.m[:, i], q.Winv[:, i][:, :, i], q.nu[:, b])
    return r


@pytest.mark.parametrize("D,split", [(6, 3), (5, 2), (2, 1), (4, 1)])
def test_scores_are_factor_sums(D, split):
    X, p, q = _problem(60, 7, D, split, seed=D * 10 + split)
    r = _brute_rho(X, q)
    assert np.allclose(F.lse(X, q), logsumexp(r, axis=1), rtol=0, atol=1e-10)
    assert np.allclose(F.responsibilities(X, q), np.exp(r - logsumexp(r, axis=1, keepdims=True)),
                       rtol=0, atol=1e-12)


@pytest.mark.parametrize("D,split,K", [(6, 3, 5), (5, 2, 4), (2, 1, 3)])
def test_elbo_equals_seven_terms_per_factor(D, split, K):
    X, p, q = _problem(50, K, D, split, seed=7 + D)
    got = F.elbo(F.lse(X, q).sum(), q, p)
    ref = brute.elbo_bishop_blocks(X, q, p, split)
    assert abs(got - ref) < 1e-8 * max(1.0, abs(ref)), (got, ref)


@pytest.mark.parametrize("D,split", [(6, 3), (5, 2), (3, 1)])
def test_k1_bound_at_exact_posterior_is_product_of_marginals(D, split):
    X, p, _ = _problem(40, 1, D, split, seed=31 + D)
    e = F.expectations(p)
    q = F.update(p, F.stats(X, p, F.lse(X, p, e), e))
    got = F.elbo(F.lse(X, q).sum(), q, p)
    ref = 0.0
    for b in (0, 1):
        i = p.idx(b)
        ref += brute.log_marginal_k1(X[:, i], p.m[0, i], p.kappa[0, b], p.Winv[0][np.ix_(i, i)], p.nu[0, b])
    assert abs(got - ref) < 1e-9 * max(1.0, abs(ref)), (got, ref)


def test_update_matches_natural_parameters_per_factor():
    X, p, q = _problem(80, 6, 6, 3, seed=77)
    Rr = F.responsibilities(X, q)
    got = F.update(p, F.stats(X, q, F.lse(X, q)))
    assert np.allclose(got.alpha, p.alpha + Rr.sum(0), rtol=1e-12)
    for b in (0, 1):
        i = p.idx(b)
        pb = R.NW(alpha=p.alpha, kappa=p.kappa[:, b], m=p.m[:, i], Winv=p.Winv[:, i][:, :, i], nu=p.nu[:, b])
        nat = brute.update_natural(pb, Rr, X[:, i])
        assert np.allclose(got.kappa[:, b], nat["kappa"], rtol=1e-12)
        assert np.allclose(got.nu[:, b], nat["nu"], rtol=1e-12)
        assert np.allclose(got.m[:, i], nat["m"], rtol=1e-10, atol=1e-12)
        assert np.allclose(got.Winv[:, i][:, :, i], nat["Winv"], rtol=1e-8, atol=1e-10)
    # cross-factor blocks of W^{-1} stay zero
    i, j = p.idx(0), p.idx(1)
    assert np.all(got.Winv[:, i][:, :, j] == 0) and np.all(got.Winv[:, j][:, :, i] == 0)


def test_uninformative_colour_factor_leaves_spatial_mixture():
    X, p, q = _problem(70, 5, 6, 3, seed=5)
    for name in ("kappa", "nu"):
        getattr(q, name)[:, 1] = getattr(q, name)[0, 1]
    q.m[:, 3:] = q.m[0, 3:]
    q.Winv[:, 3:, 3:] = q.Winv[0, 3:, 3:]
    qs = R.NW(alpha=q.alpha, kappa=q.kappa[:, 0], m=q.m[:, :3], Winv=q.Winv[:, :3, :3], nu=q.nu[:, 0])
    assert np.allclose(F.responsibilities(X, q), R.responsibilities(X[:, :3], qs), rtol=0, atol=1e-12)
    # the log-normaliser moves by the colour factor's own term, the same for every component
    Elnpi = digamma(q.alpha) - digamma(q.alpha.sum())
    colour = brute.rho(X[:, 3:], q.alpha, q.kappa[:, 1], q.m[:, 3:], q.Winv[:, 3:, 3:], q.nu[:, 1]) - Elnpi
    assert np.allclose(colour - colour[:, :1], 0, atol=1e-12)
    assert np.allclose(F.lse(X, q) - R.lse(X[:, :3], qs), colour[:, 0], rtol=0, atol=1e-10)


def test_cavi_bound_is_monotone():
    X, pr = scenes.random_problem(400, 12, 6, seed=99)
    p = F.NW2.from_prior(pr, 3)
    _, Fs = F.cavi(X.astype(np.float64), p, 8)
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(Fs, Fs[1:])), Fs


def test_prior_is_block_diagonal():
    X, pr = scenes.random_problem(30, 4, 5, seed=2)
    W0 = np.array(pr.W0, np.float64)
    W0[0, 4] = W0[4, 0] = 0.3 * W0[0, 0]        # a cross-factor entry the prior drops
    pr.W0 = W0
    p = F.NW2.from_prior(pr, 2)
    assert np.all(p.Winv[:, :2, 2:] == 0)
    assert np.allclose(p.Winv[0, :2, :2] @ W0[:2, :2], np.eye(2))
    assert np.allclose(p.Winv[0, 2:, 2:] @ W0[2:, 2:], np.eye(3))
