"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test reaches the oracle's result through an independent route: closed
forms, quadrature, a different decomposition of the same bound, invariants,
symmetries and limits. A plausible slip in the oracle (a dropped D/kappa term,
a sign in a KL, a transposed scatter, a wrong digamma argument) fails at least
one of them.
"""
import numpy as np
import pytest
from scipy.special import digamma

from oracle import brute
from oracle import vbgs_ref as R
from synth import scenes


def _prob(N, K, D, seed, **kw):
    X, pr = scenes.random_problem(N, K, D, seed, **kw)
    return X, pr, R.NW.from_prior(pr)


def _perturbed_posterior(q, seed):
    """A generic posterior (components differ in every parameter)."""
    g = np.random.default_rng(seed)
    K, D = q.m.shape
    A = g.normal(0, 0.3, (K, D, D))
    Winv = q.Winv * g.uniform(0.5, 2.0, (K, 1, 1)) + np.einsum("kij,klj->kil", A, A) * q.Winv[:, :1, :1]
    return R.NW(alpha=q.alpha * g.uniform(0.5, 5.0, K), kappa=q.kappa * g.uniform(0.5, 4.0, K),
                m=q.m + g.normal(0, 0.02, q.m.shape), Winv=Winv, nu=q.nu + g.uniform(0.0, 6.0, K))


@pytest.mark.parametrize("D", [1, 2, 5, 6])
def test_scores_match_explicit_inverse(D):
    X, pr, p = _prob(40, 5, D, 1)
    q = _perturbed_posterior(p, 2)
    e = R.expectations(q)
    Rb, lse_b = brute.responsibilities(X, q)
    lse = R.lse(X, q, e)
    assert np.allclose(lse, lse_b, rtol=1e-12, atol=1e-10)
    assert np.allclose(R.responsibilities(X, q, e), Rb, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("D,K", [(1, 3), (2, 4), (5, 5), (6, 3)])
def test_elbo_equals_bishop_seven_terms(D, K):
    """sum LSE - KL(q||p) must equal PRML's 10.70 assembled term by term at the same q."""
    X, pr, p = _prob(48, K, D, 3)
    p = _perturbed_posterior(p, 4)      # per-component frame prior
    q = _perturbed_posterior(p, 5)      # a different q
    e = R.expectations(q)
    F = R.elbo(R.lse(X, q, e).sum(), q, p, e)
    Fb = brute.elbo_bishop(X, q, p)
    assert abs(F - Fb) <= 1e-9 * max(1.0, abs(Fb))


@pytest.mark.parametrize("D", [1, 3, 6])
def test_k1_elbo_at_exact_posterior_is_log_marginal_likelihood(D):
    """K = 1: one update gives the conjugate posterior, at which F(q) = ln p(X) exactly."""
    X, pr, p = _prob(64, 1, D, 6)
    res = R.cavi(X, p, 2)
    lml = brute.log_marginal_k1(X, p.m[0], p.kappa[0], p.Winv[0], p.nu[0])
    F1 = res[1].elbo
    assert abs(F1 - lml) <= 1e-10 * abs(lml)
    assert res[0].elbo <= F1 + 1e-12 * abs(F1)


def test_update_matches_natural_parameters():
    X, pr, p = _prob(50, 4, 5, 7)
    p = _perturbed_posterior(p, 8)
    q = _perturbed_posterior(p, 9)
    Rr = R.responsibilities(X, q)
    st = R.stats(X, q, R.lse(X, q))
    qn = R.update(p, st)
    nat = brute.update_natural(p, Rr, X)
    for name in ("alpha", "kappa", "nu"):
        assert np.allclose(getattr(qn, name), nat[name], rtol=1e-12)
    assert np.allclose(qn.m, nat["m"], rtol=1e-10, atol=1e-12)
    assert np.allclose(qn.Winv, nat["Winv"], rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("a,b,c,d", [(1.0, 1.0, 2.0, 3.0), (0.7, 4.5, 1.0, 1.0), (12.0, 30.0, 3.0, 2.0)])
def test_kl_dirichlet_two_components_by_quadrature(a, b, c, d):
    kl = R.kl_dirichlet(np.array([a, b]), np.array([c, d]))
    assert abs(kl - brute.kl_beta_quad(a, b, c, d)) <= 1e-8 * max(1.0, kl)


@pytest.mark.parametrize("q,p", [((0.3, 4.0, 2.0, 5.0), (0.1, 1.0, 1.0, 3.0)),
                                 ((-0.2, 20.0, 0.5, 12.0), (0.0, 2.0, 3.0, 2.5))])
def test_kl_normal_wishart_d1_by_quadrature(q, p):
    mq, kq, Wq, nq = q
    mp, kp, Wp, np_ = p
    Q = R.NW(alpha=np.ones(1), kappa=np.array([kq]), m=np.array([[mq]]), Winv=np.array([[[1 / Wq]]]),
             nu=np.array([nq]))
    P = R.NW(alpha=np.ones(1), kappa=np.array([kp]), m=np.array([[mp]]), Winv=np.array([[[1 / Wp]]]),
             nu=np.array([np_]))
    kl = R.kl_nw(Q, P)[0]
    ref = brute.kl_normal_gamma_quad(mq, kq, Wq, nq, mp, kp, Wp, np_)
    assert abs(kl - ref) <= 1e-6 * max(1.0, abs(ref))


def test_expected_log_det_by_monte_carlo():
    """E[ln|Lambda|] under Wishart(W, nu) vs 200k samples (statistical pin, 5 sigma)."""
    from scipy.stats import wishart
    D, nu = 3, 6.5
    A = np.array([[2.0, 0.3, 0.1], [0.3, 1.0, -0.2], [0.1, -0.2, 0.5]])
    q = R.NW(alpha=np.ones(1), kappa=np.ones(1), m=np.zeros((1, D)), Winv=np.linalg.inv(A)[None], nu=np.array([nu]))
    e = R.expectations(q)
    s = wishart(df=nu, scale=A).rvs(size=200000, random_state=np.random.default_rng(0))
    ld = np.linalg.slogdet(s)[1]
    assert abs(e.ElnLam[0] - ld.mean()) <= 5 * ld.std() / np.sqrt(ld.size)


def test_digamma_special_values():
    """The digamma the oracle takes from SciPy: psi(1) = -gamma, psi(1/2) = -gamma - 2 ln 2, recurrence."""
    g = 0.57721566490153286061
    assert abs(digamma(1.0) + g) < 1e-15
    assert abs(digamma(0.5) + g + 2 * np.log(2)) < 1e-14
    x = np.linspace(0.1, 40, 97)
    assert np.allclose(digamma(x + 1), digamma(x) + 1 / x, rtol=1e-14, atol=1e-14)


def test_invariants_c1():
    X = scenes.c1_frame()
    pr = scenes.c1_prior(X)
    res = R.cavi(X, pr, 3)
    Xd = X.astype(np.float64)
    for r in res:
        st = r.stats
        assert abs(st.Nk.sum() - X.shape[0]) <= 1e-9 * X.shape[0]
        assert np.allclose(st.S1.sum(0), Xd.sum(0), rtol=1e-11)
        assert np.allclose(st.S2.sum(0), Xd.T @ Xd, rtol=1e-11)
    Rr = R.responsibilities(X[:300], res[-1].q_next)
    assert np.allclose(Rr.sum(1), 1.0, atol=1e-12)


def test_materialised_statistics_equal_the_fused_contraction():
    """Alg. 2 (materialise R, then reduce) and Alg. 3 / Eq. (fused_contr) (Delta S = R^T S_u with the
    per-point statistics S_u = [1, x, x x^T]) give the same N, S1, S2: here the N x K responsibilities
    from the explicit-inverse scores times the per-point statistics, against the oracle's sums."""
    X, pr, p = _prob(120, 7, 4, 17)
    q = _perturbed_posterior(p, 4)
    Xd = X.astype(np.float64)
    Rr, _ = brute.responsibilities(Xd, q)                 # materialised N x K
    D = Xd.shape[1]
    iu = np.triu_indices(D)
    Su = np.concatenate([np.ones((len(Xd), 1)), Xd, (Xd[:, :, None] * Xd[:, None, :])[:, iu[0], iu[1]]], 1)
    fused = Rr.T @ Su                                      # K x (1 + D + D(D+1)/2)
    got = R.stats(Xd, q, R.lse(Xd, q)).packed()
    assert np.allclose(got, fused, rtol=1e-10, atol=1e-12)


def test_elbo_monotone_c1():
    X = scenes.c1_frame()
    pr = scenes.c1_prior(X)
    F = [r.elbo for r in R.cavi(X, pr, 10)]
    for a, b in zip(F, F[1:]):
        assert b >= a - 1e-12 * abs(a)


def test_component_and_point_permutation():
    X, pr, p = _prob(120, 7, 6, 11)
    q = _perturbed_posterior(p, 12)
    st = R.stats(X, q, R.lse(X, q))
    g = np.random.default_rng(13)
    pk = g.permutation(q.K)
    pn = g.permutation(X.shape[0])
    qp = R.NW(alpha=q.alpha[pk], kappa=q.kappa[pk], m=q.m[pk], Winv=q.Winv[pk], nu=q.nu[pk])
    Xp = X[pn]
    st2 = R.stats(Xp, qp, R.lse(Xp, qp))
    assert np.allclose(st2.Nk, st.Nk[pk], rtol=1e-12, atol=1e-14)
    assert np.allclose(st2.S2, st.S2[pk], rtol=1e-12, atol=1e-14)
    assert np.allclose(np.sort(R.lse(Xp, qp)), np.sort(R.lse(X, q)), rtol=1e-13)


def test_affine_equivariance():
    """x -> A x + b with m -> A m + b and W^{-1} -> A W^{-1} A^T: r unchanged, F shifts by -N ln|det A|."""
    X, pr, p = _prob(90, 5, 3, 14)
    q = _perturbed_posterior(p, 15)
    A = np.array([[1.5, 0.2, 0.0], [0.1, 0.7, 0.3], [0.0, -0.4, 2.0]])
    b = np.array([0.3, -1.0, 2.0])

    def tr(nw):
        return R.NW(alpha=nw.alpha, kappa=nw.kappa, m=nw.m @ A.T + b,
                    Winv=np.einsum("ij,kjl,ml->kim", A, nw.Winv, A), nu=nw.nu)

    Xd = X.astype(np.float64)
    Xt = Xd @ A.T + b
    qt, pt = tr(q), tr(p)
    r0 = R.responsibilities(Xd, q)
    r1 = R.responsibilities(Xt, qt)
    assert np.allclose(r0, r1, atol=1e-11)
    F0 = R.elbo(R.lse(Xd, q).sum(), q, p)
    F1 = R.elbo(R.lse(Xt, qt).sum(), qt, pt)
    assert abs((F1 - F0) + X.shape[0] * np.log(abs(np.linalg.det(A)))) <= 1e-9 * abs(F0)
    s0 = R.stats(Xd, q, R.lse(Xd, q))
    s1 = R.stats(Xt, qt, R.lse(Xt, qt))
    assert np.allclose(s1.S1, s0.S1 @ A.T + s0.Nk[:, None] * b, rtol=1e-9, atol=1e-10)
    S2t = (np.einsum("ij,kjl,ml->kim", A, s0.S2, A) + np.einsum("ki,j->kij", s0.S1 @ A.T, b)
           + np.einsum("i,kj->kij", b, s0.S1 @ A.T) + s0.Nk[:, None, None] * np.outer(b, b))
    assert np.allclose(s1.S2, S2t, rtol=1e-9, atol=1e-9)


def test_separated_clusters_give_one_hot_statistics():
    g = np.random.default_rng(16)
    D, K, n_per = 3, 4, 30
    cen = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], float)
    X = np.concatenate([c + g.normal(0, 0.1, (n_per, D)) for c in cen]).astype(np.float32)
    pr = scenes.Prior(m0=cen.copy(), W0=np.eye(D) * 100.0, kappa0=1.0, nu0=D + 2.0, alpha0=1.0)
    p = R.NW.from_prior(pr)
    st = R.stats(X, p, R.lse(X, p))
    Xd = X.astype(np.float64)
    for k in range(K):
        xs = Xd[k * n_per:(k + 1) * n_per]
        assert abs(st.Nk[k] - n_per) < 1e-9
        assert np.allclose(st.S1[k], xs.sum(0), rtol=1e-10)
        assert np.allclose(st.S2[k], xs.T @ xs, rtol=1e-10)


def test_streaming_additivity():
    """With r held fixed, updating with A then (as new prior) B equals one update with A + B."""
    X, pr, p = _prob(100, 4, 4, 17)
    q = _perturbed_posterior(p, 18)
    XA, XB = X[:60], X[60:]
    sA = R.stats(XA, q, R.lse(XA, q), scatter=False)
    sB = R.stats(XB, q, R.lse(XB, q), scatter=False)
    two = R.update(R.update(p, sA), sB)
    sAB = R.Stats(Nk=sA.Nk + sB.Nk, S1=sA.S1 + sB.S1, S2=sA.S2 + sB.S2)
    one = R.update(p, sAB)
    for name in ("alpha", "kappa", "nu"):
        assert np.allclose(getattr(two, name), getattr(one, name), rtol=1e-12)
    assert np.allclose(two.m, one.m, rtol=1e-10, atol=1e-12)
    assert np.allclose(two.Winv, one.Winv, rtol=1e-8, atol=1e-10)


def test_empty_component_keeps_prior():
    X, pr, p = _prob(30, 3, 2, 19)
    p.m[2] = np.array([50.0, 50.0])      # far away: receives no mass
    st = R.stats(X, p, R.lse(X, p))
    assert st.Nk[2] < 1e-200
    q = R.update(p, st)
    assert np.allclose(q.m[2], p.m[2]) and np.allclose(q.Winv[2], p.Winv[2])


def test_relerr_definition():
    assert R.relerr([3.0, 4.0], [3.0, 4.0]) == 0.0
    assert abs(R.relerr([3.0, 4.0], [3.0, 5.0]) - 0.2) < 1e-15
    assert R.relerr([0.0], [1e-40]) == pytest.approx(1e-10)
