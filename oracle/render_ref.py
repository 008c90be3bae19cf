"""Rendering of a fitted mixture and the PSNR of Sec. 5.1 (test infrastructure only).

The first s coordinates of a point are its position, the remaining Dc = D - s its colour. The
rendered colour at a position x is the colour the variational posterior expects there:

  c(x) = sum_k r_k(x) E_q[c | x, k],

* r_k(x): the responsibilities of the position marginal. Under Sigma ~ W^-1(Psi = W^-1, nu) the
  position block has Sigma_ss ~ W^-1(Psi_ss, nu - Dc), and mu_s | Sigma ~ N(m_s, Sigma_ss / kappa), so
  the marginal is the Normal-Wishart (m_s, kappa, (Psi_ss)^-1, nu - Dc) over s coordinates; r_k(x)
  are its E-step responsibilities (the one-factor oracle on those parameters). In the two-factor
  model (Sec. 2.1.2) the position factor itself is the marginal.
* E_q[c | x, k] = m_c + Psi_cs Psi_ss^-1 (x - m_s): given Sigma the colour's conditional mean is
  mu_c + Sigma_cs Sigma_ss^-1 (x - mu_s); its mean over mu | Sigma leaves m in place of mu, and the
  inverse-Wishart mean of Sigma_cs Sigma_ss^-1 is Psi_cs Psi_ss^-1. Two-factor model: m_c.

PSNR = 10 log10(255^2 / MSE), MSE over all pixels and channels of the 0..255-scaled difference
(colours in [0, 1], clamped, no 8-bit rounding).
"""
from __future__ import annotations

import numpy as np

from . import factorised_ref as FR
from . import vbgs_ref as R


def marginal(q: R.NW, s: int):
    """Position marginal (one-factor NW over [0, s)) and the regression (m_c, B) of every component."""
    D = q.D
    Dc = D - s
    Pss = q.Winv[:, :s, :s]
    Pcs = q.Winv[:, s:, :s]
    B = np.linalg.solve(Pss, np.transpose(Pcs, (0, 2, 1))).transpose(0, 2, 1)   # Pcs Pss^-1
    qs = R.NW(alpha=q.alpha.copy(), kappa=q.kappa.copy(), m=q.m[:, :s].copy(), Winv=Pss.copy(), nu=q.nu - Dc)
    return qs, q.m[:, s:].copy(), B


def marginal_factorised(q: FR.NW2):
    s = q.split
    qs = q.block(0)
    qs = R.NW(alpha=qs.alpha.copy(), kappa=qs.kappa.copy(), m=qs.m.copy(), Winv=qs.Winv.copy(), nu=qs.nu.copy())
    return qs, q.m[:, s:].copy(), np.zeros((q.K, q.D - s, s))


def render(Xq, qs: R.NW, mc, B):
    """Colour at the positions Xq (Nq x s): dense responsibilities, small problems only."""
    Xq = np.asarray(Xq, np.float64)
    Rr = R.responsibilities(Xq, qs)                                   # Nq x K
    d = Xq[:, None, :] - qs.m[None, :, :]                             # Nq x K x s
    ck = mc[None, :, :] + np.einsum("kcj,nkj->nkc", B, d)             # Nq x K x Dc
    return np.einsum("nk,nkc->nc", Rr, ck), R.lse(Xq, qs)


def render_points(Xq, qs: R.NW, mc, B, chunk=256):
    """The same colour for larger Nq, in chunks of points."""
    out = np.empty((len(Xq), mc.shape[1]))
    lse = np.empty(len(Xq))
    for i in range(0, len(Xq), chunk):
        out[i:i + chunk], lse[i:i + chunk] = render(Xq[i:i + chunk], qs, mc, B)
    return out, lse


def psnr(img, ref):
    a = 255.0 * np.clip(np.asarray(img, np.float64), 0.0, 1.0)
    b = 255.0 * np.clip(np.asarray(ref, np.float64), 0.0, 1.0)
    mse = float(np.mean((a - b) ** 2))
    return mse, (10.0 * np.log10(255.0 ** 2 / mse) if mse > 0 else np.inf)
