"""FP64 oracle for the learned candidate proposal (test infrastructure only).

The proposal is not part of the paper's method: it prunes which components each point is
scored against. What it computes here:

* MLP (ReLU): h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2), x' = (x - mu_in) * inv_s_in;
  logits z_nk = h2_n . E_k + beta_k (one embedding row E_k per component).
* top-C candidates per point under the total order (z descending, k ascending).
* pruned E-step: exact scores of the candidates only (the score of the mixture model of
  Sec. 2.1.2), LSE over the candidates, r~ = exp(s - LSE_C), statistics from r~.
* captured log-mass of point n: ln sum_{k in C_n} r_nk with the exact r over all K, which
  equals LSE_C(n) - LSE_all(n).
* training loss on exact responsibility targets (renormalised over the kept pairs):
  L = sum_n [ LSE_z(n) - sum_j rbar_nj z_{n, k_j} ] / B, its gradients, and one Adam step.

Parity unpinned: none. The network and logits are pinned by a hand-worked D = 3, H = 2, K = 3
example; the loss and its beta gradient by their closed form at zero embeddings (logits = beta);
the remaining gradients by central finite differences of that pinned loss; Adam by two
hand-computed steps with the default betas and by the constant-gradient identity (each step moves
lr sign(g)); top-C by a full argsort; captured mass by its definition through the dense
responsibilities.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import logsumexp

from . import vbgs_ref as R


@dataclasses.dataclass
class MLP:
    W1: np.ndarray    # (H, D)
    b1: np.ndarray    # (H,)
    W2: np.ndarray    # (H, H)
    b2: np.ndarray    # (H,)
    E: np.ndarray     # (K, H)
    beta: np.ndarray  # (K,)
    mu_in: np.ndarray     # (D,)
    inv_s_in: np.ndarray  # (D,)

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.E, self.beta]

    def copy(self):
        return MLP(*(np.array(a, copy=True) for a in dataclasses.astuple(self)))


def forward(m: MLP, X):
    x = (np.asarray(X, np.float64) - m.mu_in) * m.inv_s_in
    a1 = x @ m.W1.T + m.b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ m.W2.T + m.b2
    h2 = np.maximum(a2, 0.0)
    return x, h1, h2


def logits(m: MLP, X):
    return forward(m, X)[2] @ m.E.T + m.beta


def topc(z, C):
    """Indices of the C largest logits per row, ties broken by the smaller index."""
    N, K = z.shape
    C = min(C, K)
    out = np.empty((N, C), np.int64)
    for n in range(N):
        order = np.lexsort((np.arange(K), -z[n]))  # primary: -z ascending, secondary: k ascending
        out[n] = np.sort(order[:C])
    return out


def pruned_estep(X, q: R.NW, cand, e: R.Expect | None = None):
    """Exact scores of the candidates, LSE over them, r~ and the statistics (raw coordinates)."""
    e = e or R.expectations(q)
    N, C = cand.shape
    pn = np.repeat(np.arange(N), C)
    pk = cand.ravel()
    s = R.pair_scores(X, q, pn, pk, e).reshape(N, C)
    lse_c = logsumexp(s, axis=1)
    rr = np.exp(s - lse_c[:, None])
    Xd = np.asarray(X, np.float64)
    K, D = q.m.shape
    Nk = np.zeros(K)
    S1 = np.zeros((K, D))
    S2 = np.zeros((K, D, D))
    np.add.at(Nk, pk, rr.ravel())
    np.add.at(S1, pk, rr.ravel()[:, None] * Xd[pn])
    np.add.at(S2, pk, rr.ravel()[:, None, None] * Xd[pn][:, :, None] * Xd[pn][:, None, :])
    return lse_c, R.Stats(Nk=Nk, S1=S1, S2=S2)


def captured_log_mass(lse_c, lse_all):
    return np.asarray(lse_c) - np.asarray(lse_all)


def fallback_decision(cap, bound=np.log1p(-1e-4), frac=0.01):
    """Fall back when ln(mean_n exp(cap_n)) < bound or more than `frac` of the points lie below it."""
    cap = np.asarray(cap, np.float64)
    agg = logsumexp(cap) - np.log(cap.size)
    below = float(np.mean(cap < bound))
    return bool(agg < bound or below > frac), float(agg), below


def loss_and_grads(m: MLP, X, tk, tr):
    """Mean over the batch of LSE_z - sum_j rbar_j z_{k_j}; targets tk (B x M, -1 = empty), tr weights."""
    x, h1, h2 = forward(m, X)
    z = h2 @ m.E.T + m.beta
    B, K = z.shape
    valid = tk >= 0
    w = np.where(valid, tr, 0.0)
    ws = w.sum(axis=1, keepdims=True)
    w = np.where(ws > 0, w / np.where(ws > 0, ws, 1.0), 0.0)  # rows without targets: softmax term only
    kk = np.where(valid, tk, 0)
    lse = logsumexp(z, axis=1)
    zt = np.take_along_axis(z, kk, axis=1)
    L = float(np.mean(lse - (w * zt).sum(axis=1)))
    p = np.exp(z - lse[:, None])
    dz = p.copy()
    np.add.at(dz, (np.repeat(np.arange(B), tk.shape[1]), kk.ravel()), -w.ravel())
    dz /= B
    gE = dz.T @ h2
    gbeta = dz.sum(axis=0)
    dh2 = dz @ m.E
    da2 = dh2 * (h2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ m.W2
    da1 = dh1 * (h1 > 0)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0)
    return L, [gW1, gb1, gW2, gb2, gE, gbeta]


def loss_only(m: MLP, X, tk, tr):
    x, h1, h2 = forward(m, X)
    z = h2 @ m.E.T + m.beta
    valid = tk >= 0
    w = np.where(valid, tr, 0.0)
    ws = w.sum(axis=1, keepdims=True)
    w = np.where(ws > 0, w / np.where(ws > 0, ws, 1.0), 0.0)
    zt = np.take_along_axis(z, np.where(valid, tk, 0), axis=1)
    return float(np.mean(logsumexp(z, axis=1) - (w * zt).sum(axis=1)))


@dataclasses.dataclass
class Adam:
    lr: float = 1e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8


def adam_step(params, grads, m1, m2, t, opt: Adam):
    """In place: t is the 1-based step count after this update."""
    for p, g, a, b in zip(params, grads, m1, m2):
        a *= opt.b1
        a += (1 - opt.b1) * g
        b *= opt.b2
        b += (1 - opt.b2) * g * g
        ah = a / (1 - opt.b1 ** t)
        bh = b / (1 - opt.b2 ** t)
        p -= opt.lr * ah / (np.sqrt(bh) + opt.eps)
