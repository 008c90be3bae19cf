"""Two-modality mixture of Sec. 2.1.2 (test infrastructure only).

Each component k has two independent Normal-Wishart blocks over disjoint coordinate groups,
[0, s) (spatial) and [s, D) (colour), each with its own kappa, nu, m and W, and a Dirichlet weight:
  rho_nk = E[ln pi_k] + sum_b ( E[ln|Lambda_bk|]/2 - (D_b/2) ln 2 pi
                                - (D_b/kappa_bk + nu_bk (x_b - m_bk)^T W_bk (x_b - m_bk)) / 2 ).
The per-block expectations, updates and KL terms are those of vbgs_ref applied to each block;
the N x K passes reuse the FP64 C routines through the equivalent one-block form
L = blockdiag(L_b / sqrt(nu_b)), nu = 1, whose quadratic is sum_b nu_b d_b^T W_b d_b.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import digamma

from . import vbgs_ref as R


@dataclasses.dataclass
class NW2:
    alpha: np.ndarray   # (K,)
    kappa: np.ndarray   # (K, 2)
    m: np.ndarray       # (K, D)
    Winv: np.ndarray    # (K, D, D), zero across the blocks
    nu: np.ndarray      # (K, 2)
    split: int

    @property
    def K(self):
        return self.m.shape[0]

    @property
    def D(self):
        return self.m.shape[1]

    def idx(self, b):
        return np.arange(0, self.split) if b == 0 else np.arange(self.split, self.D)

    def block(self, b) -> R.NW:
        i = self.idx(b)
        return R.NW(alpha=self.alpha, kappa=self.kappa[:, b], m=self.m[:, i], Winv=self.Winv[:, i][:, :, i],
                    nu=self.nu[:, b])

    @staticmethod
    def from_prior(prior, split: int) -> "NW2":
        K, D = prior.m0.shape
        W0 = np.array(prior.W0, np.float64)
        Winv = np.zeros((D, D))
        for i in (np.arange(0, split), np.arange(split, D)):
            Wi = np.linalg.inv(W0[np.ix_(i, i)])
            Winv[np.ix_(i, i)] = 0.5 * (Wi + Wi.T)
        return NW2(alpha=np.full(K, float(prior.alpha0)), kappa=np.full((K, 2), float(prior.kappa0)),
                   m=np.array(prior.m0, np.float64, copy=True), Winv=np.broadcast_to(Winv, (K, D, D)).copy(),
                   nu=np.full((K, 2), float(prior.nu0)), split=split)


@dataclasses.dataclass
class Expect2:
    blocks: list          # per block: vbgs_ref.Expect of the block
    Elnpi: np.ndarray
    g: np.ndarray         # score constant
    joint_q: R.NW         # equivalent one-block parameters (nu = 1)
    joint_e: R.Expect


def expectations(q: NW2) -> Expect2:
    eb = [R.expectations(q.block(b)) for b in (0, 1)]
    Elnpi = digamma(q.alpha) - digamma(q.alpha.sum())
    g = Elnpi.copy()
    for b in (0, 1):
        Db = len(q.idx(b))
        g += 0.5 * eb[b].ElnLam - 0.5 * Db * R.LN2PI - 0.5 * Db / q.kappa[:, b]
    L = np.zeros((q.K, q.D, q.D))
    for b in (0, 1):
        i = q.idx(b)
        L[:, i[:, None], i[None, :]] = eb[b].L / np.sqrt(q.nu[:, b])[:, None, None]
    jq = R.NW(alpha=q.alpha, kappa=np.ones(q.K), m=q.m, Winv=np.einsum("kij,klj->kil", L, L), nu=np.ones(q.K))
    je = R.Expect(L=L, lndetW=np.zeros(q.K), ElnLam=np.zeros(q.K), Elnpi=Elnpi, g=g)
    return Expect2(blocks=eb, Elnpi=Elnpi, g=g, joint_q=jq, joint_e=je)


def lse(X, q: NW2, e: Expect2 | None = None):
    e = e or expectations(q)
    return R.lse(X, e.joint_q, e.joint_e)


def responsibilities(X, q: NW2, e: Expect2 | None = None):
    e = e or expectations(q)
    return R.responsibilities(X, e.joint_q, e.joint_e)


def stats(X, q: NW2, lse_, e: Expect2 | None = None, scatter=True) -> R.Stats:
    e = e or expectations(q)
    return R.stats(X, e.joint_q, lse_, e.joint_e, scatter=scatter)


def update(p: NW2, st: R.Stats) -> NW2:
    """Each block takes the conjugate update of its own coordinates; N_k is shared."""
    out = NW2(alpha=p.alpha + st.Nk, kappa=np.empty_like(p.kappa), m=np.empty_like(p.m),
              Winv=np.zeros_like(p.Winv), nu=np.empty_like(p.nu), split=p.split)
    for b in (0, 1):
        i = p.idx(b)
        sb = R.Stats(Nk=st.Nk, S1=st.S1[:, i], S2=st.S2[:, i][:, :, i],
                     scat=None if st.scat is None else st.scat[:, i][:, :, i])
        qb = R.update(p.block(b), sb)
        out.kappa[:, b], out.nu[:, b], out.m[:, i] = qb.kappa, qb.nu, qb.m
        out.Winv[:, i[:, None], i[None, :]] = qb.Winv
    return out


def elbo(sum_lse: float, q: NW2, p: NW2, e: Expect2 | None = None) -> float:
    """F = sum_n LSE_n - KL(Dir(alpha) || Dir(alpha_p)) - sum_k sum_b KL(NW_bk || NW_p,bk)."""
    kl = R.kl_dirichlet(q.alpha, p.alpha)
    for b in (0, 1):
        kl += R.kl_nw(q.block(b), p.block(b)).sum()
    return float(sum_lse - kl)


def cavi(X, p: NW2, steps: int):
    q, Fs = p, []
    for _ in range(steps):
        e = expectations(q)
        ls = lse(X, q, e)
        Fs.append(elbo(ls.sum(), q, p, e))
        q = update(p, stats(X, q, ls, e))
    return q, Fs
