"""Frame-stream driver over the C ABI (control flow and argument marshalling only).

Alg. 1 processes frames one after another: the E-step and statistics of a frame are folded
into the prior by the closed-form update, and the posterior is carried forward as the next
frame's prior (replay-free). With the learned proposal the first frames run the exact E-step
and provide training targets; later frames are pruned to the proposed candidates, audited,
and fall back to the exact E-step when the audit fails.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from .vbgs import VBGS


@dataclasses.dataclass
class FrameLog:
    frame: int
    mode: str              # "exact" or "pruned"
    elbo: float
    fallback: Optional[bool] = None
    captured: Optional[float] = None   # ln mean captured mass over the audit sample
    below: Optional[float] = None      # fraction of audited points below the bound


def train_on_targets(model: VBGS, data, steps: int, batch: int, lr: float, seed: int):
    """`steps` Adam steps; each picks one frame of `data` [(X, tk, tr)] and `batch` of its rows
    with targets, both drawn by a seeded host generator. Returns the loss history."""
    g = np.random.default_rng(seed)
    rows = []
    for X, tk, tr in data:
        has = (tk[:, 0] >= 0).nonzero().flatten().cpu().numpy()
        rows.append(has)
    losses = []
    for s in range(steps):
        f = int(g.integers(len(data)))
        r = rows[f]
        if r.size == 0:
            continue
        b = np.sort(g.choice(r, size=min(batch, r.size), replace=False)).astype(np.int32)
        X, tk, tr = data[f]
        loss, _ = model.train_step(X, tk, tr, b, lr=lr, apply=True)
        losses.append(loss)
    return [float(x.item()) for x in losses]


def run_stream(model: VBGS, frames: List[torch.Tensor], n_exact: int, train_steps: int = 0, batch: int = 4096,
               lr: float = 1e-3, audit: int = 4096, bound: float = float(np.log1p(-1e-4)), frac: float = 0.01,
               steps_per_frame: int = 1, seed: int = 0, retrain_steps: int = 0,
               reassign_n: int = 0) -> List[FrameLog]:
    """Process the frames in order. With reassign_n > 0 each frame starts with Alg. 1's `reassign`:
    the frame's per-point LSE under the current posterior, then the reassignment of reassign_n
    components (Gumbel draws from a generator seeded by (seed, frame)). Frames < n_exact: exact
    E-step, targets kept for training; after frame n_exact - 1 the proposal is trained for
    `train_steps`. Later frames: pruned E-step with an audit of `audit` seeded points; frames that
    fall back are added to the training data and trigger `retrain_steps` more steps."""
    logs, data = [], []
    for t, X in enumerate(frames):
        N = X.shape[0]
        if reassign_n > 0:
            lse, _ = model.estep_stats(X, stats=False)
            gm = np.random.default_rng([seed, t, 1]).gumbel(size=N)
            model.reassign(X, lse, gm, min(reassign_n, N, model.K))
        exact = t < n_exact or not model.params.proposal
        for s in range(steps_per_frame):
            last = s == steps_per_frame - 1
            if exact:
                model.estep_stats(X, lse=False, stats=False)
                F = model.elbo()
                if last and model.params.proposal:
                    tk, tr = model.export_targets(X)
                    data.append((X, tk, tr))
                model.update(commit=last)
                logs.append(FrameLog(t, "exact", float(F.item())))
            else:
                g = np.random.default_rng([seed, t, s])
                idx = np.sort(g.choice(N, size=min(audit, N), replace=False)).astype(np.int32)
                _, _, rep = model.estep_stats_pruned(X, audit_idx=idx, bound=bound, frac=frac, lse=False,
                                                     stats=False)
                F = model.elbo()
                model.update(commit=last)
                r = rep.cpu().numpy()
                logs.append(FrameLog(t, "pruned", float(F.item()), bool(r[0]), float(r[1]), float(r[2])))
                if last and r[0] and retrain_steps > 0:
                    model.estep_stats(X, lse=False, stats=False)  # exact targets of the failed frame
                    data.append((X, *model.export_targets(X)))
                    train_on_targets(model, data, retrain_steps, batch, lr, seed + t)
        if t == n_exact - 1 and model.params.proposal and train_steps > 0:
            train_on_targets(model, data, train_steps, batch, lr, seed)
    return logs
