"""Knob-level mixed-precision search for the E-step (Sec. 4.2, Eq. (mp_opt)).

The paper searches a per-operation precision map of a traced function. Here the operations are
the E-step's kernel knobs, each with levels ordered from highest to lowest precision:

- ``score``: fp64 (the FP64 direct-form path, which makes the other two knobs inert), or the
  precision of the MFMA score screen / GEMM: fp32, bf16x3 (split BF16), bf16;
- ``rescore``: FP64 exact rescoring of the screened pairs (on) or the GEMM result used as is (off);
- ``margin``: mass a point may lose to skipped pairs: 1e-12, 1e-6, 1e-3 (the screen margin is
  ln K + ln(1/mass) nats; it only matters with rescoring on).

The reference y^h is the all-highest configuration, the FP64 direct-form E-step. The error of a configuration is the relative
error of Eq. (relerr) (tau = 1e-30), taken over the per-point LSE and the three statistics blocks
(N_k; S1_k; S2_k), the largest of the four. The three passes follow Sec. 4.2:

1. precision-aware: the sensitivity of each knob at each lower level, measured by lowering that
   knob alone; start from all knobs at their lowest level and promote knobs to their highest
   level in decreasing order of sensitivity until the error is within eps; then try the promoted
   knobs together at each intermediate level, promoting again in the same order when that fails;
2. structure-aware: lower any knob by one level while the error stays within eps, until no such
   step is left;
3. latency-aware: a lowered knob whose next higher level runs no slower (by measured E-step time)
   is raised back.

Control flow and measurement only; every E-step runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
import torch

from .vbgs import VBGS

LEVELS = {
    "score": ["fp64", "fp32", "bf16x3", "bf16"],
    "rescore": [True, False],
    "margin": [1e-12, 1e-6, 1e-3],
}
KNOBS = ["score", "rescore", "margin"]
TAU = 1e-30


def relerr(ref: np.ndarray, x: np.ndarray) -> float:
    """Eq. (relerr): ||y_h - y||_2 / max(||y_h||_2, tau)."""
    ref = np.asarray(ref, np.float64).ravel()
    x = np.asarray(x, np.float64).ravel()
    return float(np.linalg.norm(ref - x) / max(np.linalg.norm(ref), TAU))


@dataclasses.dataclass
class Eval:
    config: Dict
    err: float
    ms: float


class Search:
    """One frame X and a state (frame prior and posterior) taken from `source` (a VBGS)."""

    def __init__(self, source: VBGS, X: torch.Tensor, reps: int = 3, n_max: Optional[int] = None):
        self.src, self.X, self.reps = source, X, reps
        self.n_max = n_max or X.shape[0]
        self.prior = source.get_params("prior")
        self.post = source.get_params("posterior")
        self.cache: Dict[Tuple, Eval] = {}
        self.log: List[Eval] = []
        ref = self._model(dict(score="fp64", rescore=True, margin=1e-12))
        lse, st = ref.estep_stats(X)
        torch.cuda.synchronize()
        self.ref = self._blocks(lse, st)
        self.ref_ms = self._time(ref)
        ref.close()

    # ---- evaluation -------------------------------------------------------------------------
    def _model(self, cfg: Dict) -> VBGS:
        s = self.src
        margin = math.log(s.K) + math.log(1.0 / cfg["margin"])
        m = VBGS(s.D, s.K, self.n_max, self.post["m"], np.eye(s.D), device=s.device, kappa0=s.params.kappa0,
                 nu0=s.params.nu0, alpha0=s.params.alpha0, score_prec=cfg["score"], exact=bool(cfg["rescore"]),
                 screen_margin=margin)
        for which, p in (("prior", self.prior), ("posterior", self.post)):
            m.set_params(which, p["alpha"], p["kappa"], p["m"], p["Winv"], p["nu"])
        return m

    def _blocks(self, lse, st):
        D = self.src.D
        st = st.cpu().numpy()
        return [lse.cpu().numpy(), st[:, :1], st[:, 1:1 + D], st[:, 1 + D:]]

    def _time(self, m: VBGS) -> float:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        m.estep_stats(self.X, lse=False, stats=False)
        e0.record()
        for _ in range(self.reps):
            m.estep_stats(self.X, lse=False, stats=False)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / self.reps

    @staticmethod
    def canonical(cfg: Dict) -> Dict:
        """The FP64 path ignores the screen knobs: they are reported at their highest level."""
        if cfg["score"] == "fp64":
            return {k: LEVELS[k][0] for k in KNOBS}
        return dict(cfg)

    def evaluate(self, cfg: Dict) -> Eval:
        cfg = self.canonical(cfg)
        key = tuple(cfg[k] for k in KNOBS)
        if key in self.cache:
            return self.cache[key]
        m = self._model(cfg)
        lse, st = m.estep_stats(self.X)
        torch.cuda.synchronize()
        got = self._blocks(lse, st)
        err = max(relerr(a, b) for a, b in zip(self.ref, got))
        ms = self._time(m)
        m.close()
        ev = Eval(dict(cfg), err, ms)
        self.cache[key] = ev
        self.log.append(ev)
        return ev

    # ---- the three passes -------------------------------------------------------------------
    def run(self, eps: float) -> Eval:
        high = {k: LEVELS[k][0] for k in KNOBS}
        low = {k: LEVELS[k][-1] for k in KNOBS}
        # 1. precision-aware: sensitivities of single-knob downcasts, then greedy promotion
        sens = {}
        for k in KNOBS:
            for lv in LEVELS[k][1:]:
                sens[(k, lv)] = self.evaluate({**high, k: lv}).err
        order = sorted(KNOBS, key=lambda k: -sens[(k, LEVELS[k][-1])])
        cfg = dict(low)
        promoted = []
        for k in order:
            if self.evaluate(cfg).err <= eps:
                break
            cfg[k] = high[k]
            promoted.append(k)
        for depth in range(len(max(LEVELS.values(), key=len)) - 2, 0, -1):  # intermediate levels
            trial = dict(cfg)
            for k in promoted:
                if depth < len(LEVELS[k]) - 1:
                    trial[k] = LEVELS[k][depth]
            if trial == cfg:
                continue
            for k in order:
                if self.evaluate(trial).err <= eps:
                    break
                if k in promoted:
                    trial[k] = high[k]
            if self.evaluate(trial).err <= eps:
                cfg = trial
        if self.evaluate(cfg).err > eps:
            cfg = dict(high)
        # 2. structure-aware: one-level downcasts while the constraint holds
        cfg = self.canonical(cfg)
        changed = True
        while changed:
            changed = False
            for k in KNOBS:
                if cfg["score"] == "fp64" and k != "score":
                    continue
                i = LEVELS[k].index(cfg[k])
                if i + 1 < len(LEVELS[k]):
                    trial = {**cfg, k: LEVELS[k][i + 1]}
                    if self.evaluate(trial).err <= eps:
                        cfg, changed = self.canonical(trial), True
        # 3. latency-aware: undo downcasts that do not pay
        changed = True
        while changed:
            changed = False
            for k in KNOBS:
                i = LEVELS[k].index(cfg[k])
                if i > 0:
                    up = self.canonical({**cfg, k: LEVELS[k][i - 1]})
                    if up != cfg and self.evaluate(up).ms <= self.evaluate(cfg).ms and self.evaluate(up).err <= eps:
                        cfg, changed = up, True
        return self.evaluate(cfg)
