"""FP64 CPU oracle for the VB Gaussian-mixture E-step, statistics, update and ELBO.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library. It shares no code
with the HIP path. Its per-pair loops live in ``vbgs_oracle.c`` (plain C, FP64,
direct non-expanded score); everything per component is NumPy / SciPy here.

Model (Sec. 2.1.2, Fig. 2): z ~ Cat(pi), pi ~ Dirichlet(alpha); each component k
has a Normal-Wishart prior on (mu_k, Lambda_k) -- the paper's NIW(m, kappa, V, n)
on (mu, Sigma) is the same distribution with Lambda = Sigma^{-1}, W = V^{-1},
nu = n. The per-frame fit of Alg. 1 (statistics S accumulated from the
responsibilities R and the per-point statistics S_u, then a closed-form
posterior) is the textbook coordinate-ascent VB for this model:

* expectations (Bishop, PRML eqs. 10.65-10.66):
    E[ln|Lambda_k|] = sum_{i=1..D} psi((nu_k + 1 - i)/2) + D ln 2 + ln|W_k|
    E[ln pi_k]      = psi(alpha_k) - psi(sum_j alpha_j)
* log-responsibility (PRML eqs. 10.46, 10.64):
    rho_nk = E[ln pi_k] + 1/2 E[ln|Lambda_k|] - D/2 ln(2 pi)
             - 1/2 (D / kappa_k + nu_k (x_n - m_k)^T W_k (x_n - m_k))
  r_nk = exp(rho_nk - LSE_n) (normalised over the K components)
* statistics (the Delta S of Alg. 1): N_k, S1_k = sum r x, S2_k = sum r x x^T
* update (PRML eqs. 10.58, 10.60-10.63), from the frame prior p:
    alpha = alpha_p + N,  kappa = kappa_p + N,  nu = nu_p + N,
    m = (kappa_p m_p + N xbar) / kappa,
    W^{-1} = W_p^{-1} + sum_n r (x - xbar)(x - xbar)^T
             + kappa_p N / (kappa_p + N) (xbar - m_p)(xbar - m_p)^T
* evidence lower bound at q (the ELBO returned by compute_elbo_delta, Sec. 2.1.2):
    F(q) = sum_n LSE_n - KL(Dir(alpha) || Dir(alpha_p)) - sum_k KL(NW_k || NW_p,k)

The readings where the paper is silent (joint D-dim Gaussian, KL against the
frame prior, when F is evaluated) are listed with the design notes.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np
from scipy.special import digamma, gammaln

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vbgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

LN2PI = float(np.log(2.0 * np.pi))


def build(force: bool = False) -> str:
    """Compile the C core with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        L.oracle_lse.argtypes = [i64, i64, ctypes.c_int, d, d, d, d, d, d]
        L.oracle_resp.argtypes = [i64, i64, ctypes.c_int, d, d, d, d, d, d, d]
        L.oracle_stats.argtypes = [i64, i64, i64, ctypes.c_int, d, d, d, d, d, d, d, d, d, d]
        L.oracle_pair_scores.argtypes = [i64, ctypes.c_int, d, i64p, i64p, d, d, d, d, d]
        L.oracle_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclasses.dataclass
class NW:
    """Per-component Dirichlet / Normal-Wishart parameters (prior or posterior)."""

    alpha: np.ndarray   # (K,)
    kappa: np.ndarray   # (K,)
    m: np.ndarray       # (K, D)
    Winv: np.ndarray    # (K, D, D)   inverse Wishart scale matrix
    nu: np.ndarray      # (K,)

    @property
    def K(self):
        return self.m.shape[0]

    @property
    def D(self):
        return self.m.shape[1]

    def copy(self):
        return NW(*(np.array(a, copy=True) for a in dataclasses.astuple(self)))

    @staticmethod
    def from_prior(prior) -> "NW":
        """Shared hyper-parameters broadcast to every component (prior q0 = p)."""
        K, D = prior.m0.shape
        W0inv = np.linalg.inv(np.asarray(prior.W0, np.float64))
        W0inv = 0.5 * (W0inv + W0inv.T)
        return NW(alpha=np.full(K, float(prior.alpha0)), kappa=np.full(K, float(prior.kappa0)),
                  m=np.array(prior.m0, np.float64, copy=True),
                  Winv=np.broadcast_to(W0inv, (K, D, D)).copy(), nu=np.full(K, float(prior.nu0)))


@dataclasses.dataclass
class Expect:
    L: np.ndarray        # (K, D, D) lower Cholesky factor of W^{-1}
    lndetW: np.ndarray   # (K,)
    ElnLam: np.ndarray   # (K,)
    Elnpi: np.ndarray    # (K,)
    g: np.ndarray        # (K,) score constant: Elnpi + ElnLam/2 - D/2 ln 2pi - D/(2 kappa)


def expectations(q: NW) -> Expect:
    """Cholesky of W^{-1}, ln|W|, E[ln|Lambda|] and E[ln pi] (PRML 10.65-10.66)."""
    D = q.D
    L = np.linalg.cholesky(q.Winv)  # raises LinAlgError if not positive definite
    lndetW = -2.0 * np.log(np.diagonal(L, axis1=1, axis2=2)).sum(axis=1)
    i = np.arange(1, D + 1)
    ElnLam = digamma((q.nu[:, None] + 1.0 - i[None, :]) / 2.0).sum(axis=1) + D * np.log(2.0) + lndetW
    Elnpi = digamma(q.alpha) - digamma(q.alpha.sum())
    g = Elnpi + 0.5 * ElnLam - 0.5 * D * LN2PI - 0.5 * D / q.kappa
    return Expect(L=L, lndetW=lndetW, ElnLam=ElnLam, Elnpi=Elnpi, g=g)


def _args(X, q: NW, e: Expect):
    return (_c(X), _c(q.m), _c(e.L), _c(e.g), _c(q.nu))


def lse(X, q: NW, e: Expect | None = None) -> np.ndarray:
    """LSE_n = ln sum_k exp(rho_nk) (max-shifted), FP64, direct form."""
    e = e or expectations(q)
    Xd, m, L, g, nu = _args(X, q, e)
    out = np.empty(Xd.shape[0])
    lib().oracle_lse(Xd.shape[0], q.K, q.D, _p(Xd), _p(m), _p(L), _p(g), _p(nu), _p(out))
    return out


def responsibilities(X, q: NW, e: Expect | None = None, lse_: np.ndarray | None = None):
    """Dense r (N x K); small problems only."""
    e = e or expectations(q)
    Xd, m, L, g, nu = _args(X, q, e)
    ls = _c(lse(X, q, e) if lse_ is None else lse_)
    R = np.empty((Xd.shape[0], q.K))
    lib().oracle_resp(Xd.shape[0], q.K, q.D, _p(Xd), _p(m), _p(L), _p(g), _p(nu), _p(ls), _p(R))
    return R


def pair_scores(X, q: NW, pn, pk, e: Expect | None = None):
    """rho for listed (point, component) pairs."""
    e = e or expectations(q)
    Xd, m, L, g, nu = _args(X, q, e)
    pn = _c(pn, np.int64)
    pk = _c(pk, np.int64)
    out = np.empty(pn.shape[0])
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib().oracle_pair_scores(pn.shape[0], q.D, _p(Xd), pn.ctypes.data_as(i64p), pk.ctypes.data_as(i64p),
                             _p(m), _p(L), _p(g), _p(nu), _p(out))
    return out


@dataclasses.dataclass
class Stats:
    Nk: np.ndarray     # (K,)
    S1: np.ndarray     # (K, D)
    S2: np.ndarray     # (K, D, D)
    scat: np.ndarray | None = None  # (K, D, D) centred scatter

    def packed(self) -> np.ndarray:
        """Feature order [N, S1 (D), upper(S2) row-major i <= j] -> (K, 1 + D + D(D+1)/2)."""
        D = self.S1.shape[1]
        iu = np.triu_indices(D)
        return np.concatenate([self.Nk[:, None], self.S1, self.S2[:, iu[0], iu[1]]], axis=1)


def stats(X, q: NW, lse_: np.ndarray, e: Expect | None = None, comps=None, scatter=True) -> Stats:
    """Sufficient statistics (raw coordinates, point-order FP64 sums) for all or a range of components."""
    e = e or expectations(q)
    Xd, m, L, g, nu = _args(X, q, e)
    ls = _c(lse_)
    k0, k1 = (0, q.K) if comps is None else comps
    n = k1 - k0
    D = q.D
    Nk = np.empty(n)
    S1 = np.empty((n, D))
    S2 = np.empty((n, D, D))
    sc = np.empty((n, D, D)) if scatter else None
    lib().oracle_stats(Xd.shape[0], k0, k1, D, _p(Xd), _p(m), _p(L), _p(g), _p(nu), _p(ls),
                       _p(Nk), _p(S1), _p(S2), _p(sc) if scatter else None)
    return Stats(Nk=Nk, S1=S1, S2=S2, scat=sc)


def update(p: NW, st: Stats) -> NW:
    """Conjugate posterior from the frame prior p and the statistics (PRML 10.58-10.63)."""
    Nk = st.Nk
    safe = np.where(Nk > 0, Nk, 1.0)
    xbar = np.where(Nk[:, None] > 0, st.S1 / safe[:, None], 0.0)
    kappa = p.kappa + Nk
    m = (p.kappa[:, None] * p.m + Nk[:, None] * xbar) / kappa[:, None]
    d = xbar - p.m
    corr = (p.kappa * Nk / (p.kappa + Nk))[:, None, None] * d[:, :, None] * d[:, None, :]
    scat = st.scat if st.scat is not None else (
        st.S2 - Nk[:, None, None] * xbar[:, :, None] * xbar[:, None, :])
    Winv = p.Winv + scat + corr
    Winv = 0.5 * (Winv + np.transpose(Winv, (0, 2, 1)))
    return NW(alpha=p.alpha + Nk, kappa=kappa, m=m, Winv=Winv, nu=p.nu + Nk)


def mvlgamma(a, D):
    """ln Gamma_D(a) = D(D-1)/4 ln pi + sum_{i=1..D} ln Gamma(a + (1 - i)/2)."""
    a = np.asarray(a, np.float64)
    i = np.arange(1, D + 1)
    return D * (D - 1) / 4.0 * np.log(np.pi) + gammaln(a[..., None] + (1.0 - i) / 2.0).sum(-1)


def lnB(lndetW, nu, D):
    """Log normaliser of the Wishart (PRML B.79)."""
    return -0.5 * nu * lndetW - 0.5 * nu * D * np.log(2.0) - mvlgamma(nu / 2.0, D)


def kl_dirichlet(alpha, alpha_p):
    a0, b0 = alpha.sum(), alpha_p.sum()
    return (gammaln(a0) - gammaln(alpha).sum() - gammaln(b0) + gammaln(alpha_p).sum()
            + ((alpha - alpha_p) * (digamma(alpha) - digamma(a0))).sum())


def kl_nw(q: NW, p: NW, eq: Expect | None = None, ep: Expect | None = None) -> np.ndarray:
    """Per-component KL(NW(q_k) || NW(p_k)), written from E_q[ln q] - E_q[ln p]."""
    eq = eq or expectations(q)
    ep = ep or expectations(p)
    D = q.D
    W = np.linalg.inv(q.Winv)
    d = q.m - p.m
    quad = np.einsum("ki,kij,kj->k", d, W, d)
    tr = np.einsum("kij,kji->k", p.Winv, W)
    gauss = 0.5 * (p.kappa * q.nu * quad + D * p.kappa / q.kappa - D + D * np.log(q.kappa / p.kappa))
    wish = (lnB(eq.lndetW, q.nu, D) - lnB(ep.lndetW, p.nu, D) + 0.5 * (q.nu - p.nu) * eq.ElnLam
            - 0.5 * q.nu * D + 0.5 * q.nu * tr)
    return gauss + wish


def elbo(sum_lse: float, q: NW, p: NW, eq: Expect | None = None) -> float:
    return float(sum_lse - kl_dirichlet(q.alpha, p.alpha) - kl_nw(q, p, eq).sum())


@dataclasses.dataclass
class StepResult:
    q_scored: NW      # posterior the E-step scored
    lse: np.ndarray
    elbo: float       # F at q_scored
    stats: Stats
    q_next: NW        # posterior after the update


def cavi_step(X, q: NW, p: NW) -> StepResult:
    """One coordinate-ascent step: E-step at q, F(q), statistics, update from p."""
    e = expectations(q)
    ls = lse(X, q, e)
    F = elbo(ls.sum(), q, p, e)
    st = stats(X, q, ls, e)
    return StepResult(q_scored=q, lse=ls, elbo=F, stats=st, q_next=update(p, st))


def cavi(X, prior_or_p, steps: int, q0: NW | None = None):
    """`steps` CAVI steps on one frame; returns the list of StepResult."""
    p = prior_or_p if isinstance(prior_or_p, NW) else NW.from_prior(prior_or_p)
    q = p.copy() if q0 is None else q0
    out = []
    for _ in range(steps):
        r = cavi_step(X, q, p)
        out.append(r)
        q = r.q_next
    return out


def relerr(ref, got, tau: float = 1e-30) -> float:
    """err = ||y_ref - y||_2 / max(||y_ref||_2, tau) (Eq. relerr)."""
    ref = np.asarray(ref, np.float64).ravel()
    got = np.asarray(got, np.float64).ravel()
    return float(np.linalg.norm(ref - got) / max(np.linalg.norm(ref), tau))
