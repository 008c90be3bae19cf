"""Independent cross-checks for the oracle (tiny inputs only). Test infrastructure.

Each function reaches a quantity the oracle computes by a different route, so a
dropped term, a wrong sign or a transposed operand in the oracle shows up as a
disagreement:

* ``rho``: explicit matrix inverse of W^{-1} and ``slogdet`` instead of a
  Cholesky forward substitution.
* ``elbo_bishop``: the evidence lower bound assembled from the seven
  expectation terms of PRML eqs. 10.70-10.77 with the responsibilities written
  out, instead of sum_n LSE_n - KL(q||p).
* ``elbo_bishop_blocks``: the same seven terms for the two-factor (spatial / colour)
  model, with the responsibilities from explicit-inverse block scores.
* ``update_natural``: the posterior through natural parameters
  (kappa m, W^{-1} + kappa m m^T), instead of the centred scatter form.
* ``log_marginal_k1``: the closed-form Normal-Wishart marginal likelihood of a
  single Gaussian, ln p(X) (for K = 1 the ELBO at the exact posterior equals it).
* ``kl_beta_quad`` / ``kl_normal_gamma_quad``: KL divergences by numerical
  quadrature of q ln(q/p) (D = 1 and K = 2 special cases).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate
from scipy.special import digamma, gammaln, logsumexp, multigammaln
from scipy import stats as sst


def rho(X, alpha, kappa, m, Winv, nu):
    X = np.asarray(X, np.float64)
    N, D = X.shape
    K = m.shape[0]
    out = np.empty((N, K))
    Elnpi = digamma(alpha) - digamma(alpha.sum())
    for k in range(K):
        W = np.linalg.inv(Winv[k])
        sign, ld = np.linalg.slogdet(W)
        assert sign > 0
        ElnL = sum(digamma((nu[k] + 1 - i) / 2.0) for i in range(1, D + 1)) + D * np.log(2) + ld
        d = X - m[k]
        quad = np.einsum("ni,ij,nj->n", d, W, d)
        out[:, k] = Elnpi[k] + 0.5 * ElnL - 0.5 * D * np.log(2 * np.pi) - 0.5 * (D / kappa[k] + nu[k] * quad)
    return out


def responsibilities(X, q):
    r = rho(X, q.alpha, q.kappa, q.m, q.Winv, q.nu)
    return np.exp(r - logsumexp(r, axis=1, keepdims=True)), logsumexp(r, axis=1)


def _lnB(W, nu):
    D = W.shape[0]
    return -0.5 * nu * np.linalg.slogdet(W)[1] - 0.5 * nu * D * np.log(2) - multigammaln(nu / 2.0, D)


def _lnC(a):
    return gammaln(a.sum()) - gammaln(a).sum()


def _nw_terms(X, R, kq, mq, Winvq, nuq, kp, mp, Winvp, nup):
    """E[ln p(X|Z,mu,Lam)] + E[ln p(mu,Lam)] - E[ln q(mu,Lam)] of PRML 10.71, 10.74, 10.77 for one
    Normal-Wishart factor over the coordinates in X (per-component parameters, responsibilities R)."""
    N, D = X.shape
    K = mq.shape[0]
    Nk = R.sum(0)
    t_lik = t_pml = t_qml = 0.0
    for k in range(K):
        W = np.linalg.inv(Winvq[k])
        Wp = np.linalg.inv(Winvp[k])
        ElnL = sum(digamma((nuq[k] + 1 - i) / 2.0) for i in range(1, D + 1)) + D * np.log(2) \
            + np.linalg.slogdet(W)[1]
        if Nk[k] > 0:
            xb = (R[:, k:k + 1] * X).sum(0) / Nk[k]
            S = ((R[:, k:k + 1] * (X - xb)).T @ (X - xb)) / Nk[k]
        else:
            xb = np.zeros(D)
            S = np.zeros((D, D))
        dx = xb - mq[k]
        t_lik += 0.5 * Nk[k] * (ElnL - D / kq[k] - nuq[k] * np.trace(S @ W)
                                - nuq[k] * dx @ W @ dx - D * np.log(2 * np.pi))
        dm = mq[k] - mp[k]
        t_pml += 0.5 * (D * np.log(kp[k] / (2 * np.pi)) + ElnL - D * kp[k] / kq[k]
                        - kp[k] * nuq[k] * dm @ W @ dm) \
            + _lnB(Wp, nup[k]) + 0.5 * (nup[k] - D - 1) * ElnL - 0.5 * nuq[k] * np.trace(Winvp[k] @ W)
        H = -_lnB(W, nuq[k]) - 0.5 * (nuq[k] - D - 1) * ElnL + 0.5 * nuq[k] * D
        t_qml += 0.5 * ElnL + 0.5 * D * np.log(kq[k] / (2 * np.pi)) - 0.5 * D - H
    return t_lik + t_pml - t_qml


def _mix_terms(R, alpha_q, alpha_p):
    """E[ln p(Z|pi)] + E[ln p(pi)] - E[ln q(Z)] - E[ln q(pi)] of PRML 10.72, 10.73, 10.75, 10.76."""
    Elnpi = digamma(alpha_q) - digamma(alpha_q.sum())
    t_z = (R * Elnpi[None, :]).sum()
    t_ppi = _lnC(alpha_p) + ((alpha_p - 1) * Elnpi).sum()
    with np.errstate(divide="ignore", invalid="ignore"):
        t_qz = np.where(R > 0, R * np.log(R), 0.0).sum()
    t_qpi = ((alpha_q - 1) * Elnpi).sum() + _lnC(alpha_q)
    return t_z + t_ppi - t_qz - t_qpi


def elbo_bishop(X, q, p):
    """PRML 10.70: E[ln p(X|Z,mu,Lam)] + E[ln p(Z|pi)] + E[ln p(pi)] + E[ln p(mu,Lam)]
    - E[ln q(Z)] - E[ln q(pi)] - E[ln q(mu,Lam)], with per-component prior parameters."""
    X = np.asarray(X, np.float64)
    R, _ = responsibilities(X, q)
    return (_nw_terms(X, R, q.kappa, q.m, q.Winv, q.nu, p.kappa, p.m, p.Winv, p.nu)
            + _mix_terms(R, q.alpha, p.alpha))


def elbo_bishop_blocks(X, q, p, split):
    """The same seven-term bound for the two-factor model of Sec. 2.1.2: coordinates [0, split) and
    [split, D) each carry their own Normal-Wishart factor (kappa, nu of shape (K, 2)), the
    log-responsibility is the sum of the two factors' terms with E[ln pi] counted once, and the
    likelihood and parameter terms are summed over the factors."""
    X = np.asarray(X, np.float64)
    idx = [np.arange(0, split), np.arange(split, X.shape[1])]
    Elnpi = digamma(q.alpha) - digamma(q.alpha.sum())
    r = -Elnpi[None, :]
    for b, i in enumerate(idx):
        r = r + rho(X[:, i], q.alpha, q.kappa[:, b], q.m[:, i], q.Winv[:, i][:, :, i], q.nu[:, b])
    R = np.exp(r - logsumexp(r, axis=1, keepdims=True))
    t = _mix_terms(R, q.alpha, p.alpha)
    for b, i in enumerate(idx):
        t += _nw_terms(X[:, i], R, q.kappa[:, b], q.m[:, i], q.Winv[:, i][:, :, i], q.nu[:, b],
                       p.kappa[:, b], p.m[:, i], p.Winv[:, i][:, :, i], p.nu[:, b])
    return t


def update_natural(p, R, X):
    """Posterior through natural parameters: kappa, kappa m, W^{-1} + kappa m m^T, nu, alpha."""
    X = np.asarray(X, np.float64)
    Nk = R.sum(0)
    S1 = R.T @ X
    S2 = np.einsum("nk,ni,nj->kij", R, X, X)
    kappa = p.kappa + Nk
    km = p.kappa[:, None] * p.m + S1
    m = km / kappa[:, None]
    T3 = p.Winv + p.kappa[:, None, None] * p.m[:, :, None] * p.m[:, None, :] + S2
    Winv = T3 - kappa[:, None, None] * m[:, :, None] * m[:, None, :]
    return dict(alpha=p.alpha + Nk, kappa=kappa, m=m, Winv=Winv, nu=p.nu + Nk)


def log_marginal_k1(X, m0, kappa0, W0inv, nu0):
    """ln p(X) of a single Gaussian with a Normal-Wishart prior (conjugate closed form):
    -(N D / 2) ln pi + ln Gamma_D(nu_N/2) - ln Gamma_D(nu_0/2) + (nu_0/2) ln|W_0^{-1}|
    - (nu_N/2) ln|W_N^{-1}| + (D/2)(ln kappa_0 - ln kappa_N)."""
    X = np.asarray(X, np.float64)
    N, D = X.shape
    xb = X.mean(0)
    S = (X - xb).T @ (X - xb)
    kN = kappa0 + N
    nN = nu0 + N
    WNinv = W0inv + S + (kappa0 * N / kN) * np.outer(xb - m0, xb - m0)
    return (-0.5 * N * D * np.log(np.pi) + multigammaln(nN / 2.0, D) - multigammaln(nu0 / 2.0, D)
            + 0.5 * nu0 * np.linalg.slogdet(W0inv)[1] - 0.5 * nN * np.linalg.slogdet(WNinv)[1]
            + 0.5 * D * (np.log(kappa0) - np.log(kN)))


def kl_beta_quad(a, b, c, d):
    """KL(Beta(a,b) || Beta(c,d)) = int q ln(q/p) by adaptive quadrature."""
    q = sst.beta(a, b)
    p = sst.beta(c, d)
    f = lambda x: q.pdf(x) * (q.logpdf(x) - p.logpdf(x))
    v, _ = integrate.quad(f, 0.0, 1.0, limit=400, epsabs=1e-13, epsrel=1e-12)
    return v


def kl_normal_gamma_quad(mq, kq, Wq, nq, mp, kp, Wp, np_):
    """D = 1 Normal-Wishart KL by 2-D quadrature over (mu, lambda).

    lambda ~ Gamma(shape nu/2, scale 2W) (the 1-D Wishart), mu | lambda ~ N(m, 1/(kappa lambda))."""
    def logpdf(mu, lam, m, k, W, n):
        return sst.gamma.logpdf(lam, n / 2.0, scale=2.0 * W) + sst.norm.logpdf(mu, m, 1.0 / np.sqrt(k * lam))

    lam_q = sst.gamma(nq / 2.0, scale=2.0 * Wq)
    lo, hi = lam_q.ppf(1e-12), lam_q.ppf(1 - 1e-12)

    def inner(lam):
        sd = 1.0 / np.sqrt(kq * lam)
        f = lambda mu: np.exp(logpdf(mu, lam, mq, kq, Wq, nq)) * (
            logpdf(mu, lam, mq, kq, Wq, nq) - logpdf(mu, lam, mp, kp, Wp, np_))
        v, _ = integrate.quad(f, mq - 12 * sd, mq + 12 * sd, limit=200, epsabs=1e-14, epsrel=1e-11)
        return v

    v, _ = integrate.quad(inner, lo, hi, limit=400, epsabs=1e-12, epsrel=1e-10)
    return v
