"""Python binding of libvbgs: the same calls as the C ABI, over torch device tensors.

This module only marshals arguments (device pointers, sizes, the current HIP
stream); every step of the computation runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


class VBGSError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__("%s (%d)%s" % (_lib.STATUS.get(status, "?"), status, (": " + msg) if msg else ""))
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(s=None):
    s = torch.cuda.current_stream() if s is None else s
    return ctypes.c_void_p(s.cuda_stream)


def make_params(D, K, n_max, kappa0=1.0, nu0=None, alpha0=1.0, score_prec=None, exact=True,
                screen_margin=0.0, n_split=0, proposal=False, C=32, train_batch=4096, cull=True, modal_split=0,
                cull_dims=0, proposal_prec=0):
    p = _lib.Params()
    L = _lib.load()
    st = L.vbgs_default_params(ctypes.byref(p), int(D), int(K), int(n_max))
    if st:
        raise VBGSError(st)
    p.kappa0 = float(kappa0)
    p.nu0 = float(D + 2 if nu0 is None else nu0)
    p.alpha0 = float(alpha0)
    if score_prec is None:  # the automatic screen where it applies (exact mode, no proposal), else split BF16
        score_prec = "auto" if exact and not proposal and D <= 6 else ("bf16x3" if D <= 6 else "fp64")
    p.score_prec = _lib.PREC[score_prec] if isinstance(score_prec, str) else int(score_prec)
    p.exact = 1 if exact else 0
    p.screen_margin = float(screen_margin)
    p.n_split = int(n_split)
    p.proposal = 1 if proposal else 0
    p.C = int(C)
    p.train_batch = int(train_batch)
    p.cull = 1 if cull else 0
    p.modal_split = int(modal_split)
    p.cull_dims = int(cull_dims)
    p.proposal_prec = _lib.PREC[proposal_prec] if isinstance(proposal_prec, str) else int(proposal_prec)
    return p


def query_sizes(p):
    L = _lib.load()
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    st = L.vbgs_query_sizes(ctypes.byref(p), ctypes.byref(sb), ctypes.byref(wb))
    if st:
        raise VBGSError(st)
    return sb.value, wb.value


def psnr(a, b):
    """PSNR of Sec. 5.1 between two float32 device images in [0, 1] (any shape, same numel):
    returns a device tensor [MSE, PSNR] (FP64)."""
    L = _lib.load()
    if a.dtype != torch.float32 or b.dtype != torch.float32 or a.numel() != b.numel():
        raise ValueError("a and b must be float32 tensors of the same size")
    a, b = a.contiguous(), b.contiguous()
    out = torch.empty(2, dtype=torch.float64, device=a.device)
    st = L.vbgs_psnr(_ptr(a), _ptr(b), a.numel(), _ptr(out), _stream())
    if st:
        raise VBGSError(st)
    return out


class VBGS:
    """One mixture of K Normal-Wishart components over D-dimensional points.

    State (frame prior + posterior) and workspace are torch uint8 tensors owned
    by this object; the library never allocates device memory.
    """

    def __init__(self, D, K, n_max, m0, W0, device="cuda", state=None, **kw):
        self.lib = _lib.load()
        self.D, self.K, self.n_max = int(D), int(K), int(n_max)
        self.F = 1 + self.D + self.D * (self.D + 1) // 2
        self.device = torch.device(device)
        self.params = make_params(D, K, n_max, **kw)
        sb, wb = query_sizes(self.params)
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p()
        if state is not None:
            if state.numel() != sb or state.dtype != torch.uint8 or state.device != self.device:
                raise ValueError("state tensor does not match these params")
            self.state = state
            st = self.lib.vbgs_attach(ctypes.byref(self.ctx), ctypes.byref(self.params), _ptr(self.state),
                                      _ptr(self.workspace))
        else:
            self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
            m0 = torch.as_tensor(np.asarray(m0, np.float64) if not torch.is_tensor(m0) else m0,
                                 dtype=torch.float64).to(self.device).contiguous()
            if tuple(m0.shape) != (self.K, self.D):
                raise ValueError("m0 must be K x D")
            W0 = np.ascontiguousarray(np.asarray(W0, np.float64).reshape(self.D, self.D))
            self._m0 = m0
            st = self.lib.vbgs_init(ctypes.byref(self.ctx), ctypes.byref(self.params), _ptr(m0),
                                    W0.ctypes.data_as(ctypes.c_void_p), _ptr(self.state), _ptr(self.workspace),
                                    _stream())
        if st:
            raise VBGSError(st)

    def _check(self, st):
        if st:
            raise VBGSError(st, self.lib.vbgs_last_error(self.ctx).decode())

    def _points(self, X):
        if X.dtype != torch.float32 or X.device != self.device or not X.is_contiguous() or X.dim() != 2 \
                or X.shape[1] != self.D:
            raise ValueError("X must be a contiguous N x D float32 tensor on %s" % self.device)
        return X

    def estep_stats(self, X, lse=True, stats=True, lse_out=None, stats_out=None):
        X = self._points(X)
        N = X.shape[0]
        if lse and lse_out is None:
            lse_out = torch.empty(N, dtype=torch.float64, device=self.device)
        if stats and stats_out is None:
            stats_out = torch.empty((self.K, self.F), dtype=torch.float64, device=self.device)
        self._check(self.lib.vbgs_estep_stats(self.ctx, _ptr(X), N, _ptr(lse_out if lse else None),
                                              _ptr(stats_out if stats else None), _stream()))
        return (lse_out if lse else None), (stats_out if stats else None)

    def estep_stats_scratch(self, X, lse=True, stats=True, lse_out=None, stats_out=None):
        """estep_stats with the library's static scratch as the workspace (allocates nothing on the
        device when lse_out / stats_out are given); the context's own statistics are left unchanged."""
        X = self._points(X)
        N = X.shape[0]
        if lse and lse_out is None:
            lse_out = torch.empty(N, dtype=torch.float64, device=self.device)
        if stats and stats_out is None:
            stats_out = torch.empty((self.K, self.F), dtype=torch.float64, device=self.device)
        self._check(self.lib.vbgs_estep_stats_scratch(self.ctx, _ptr(X), N, _ptr(lse_out if lse else None),
                                                      _ptr(stats_out if stats else None), _stream()))
        return (lse_out if lse else None), (stats_out if stats else None)

    def update(self, commit=False):
        self._check(self.lib.vbgs_update(self.ctx, 1 if commit else 0, _stream()))

    def elbo(self, X=None, out=None):
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        if X is None:
            st = self.lib.vbgs_elbo(self.ctx, None, 0, _ptr(out), _stream())
        else:
            X = self._points(X)
            st = self.lib.vbgs_elbo(self.ctx, _ptr(X), X.shape[0], _ptr(out), _stream())
        self._check(st)
        return out

    def get_params(self, which="posterior"):
        w = 0 if which == "posterior" else 1
        K, D, dev = self.K, self.D, self.device
        kn = (K, 2) if self.params.modal_split > 0 else (K,)  # one kappa and nu per block
        o = dict(alpha=torch.empty(K, dtype=torch.float64, device=dev),
                 kappa=torch.empty(kn, dtype=torch.float64, device=dev),
                 m=torch.empty((K, D), dtype=torch.float64, device=dev),
                 Winv=torch.empty((K, D, D), dtype=torch.float64, device=dev),
                 nu=torch.empty(kn, dtype=torch.float64, device=dev))
        self._check(self.lib.vbgs_get_params(self.ctx, w, _ptr(o["alpha"]), _ptr(o["kappa"]), _ptr(o["m"]),
                                             _ptr(o["Winv"]), _ptr(o["nu"]), _stream()))
        return o

    def set_params(self, which, alpha, kappa, m, Winv, nu):
        w = 0 if which == "posterior" else 1
        t = [torch.as_tensor(np.asarray(a, np.float64) if not torch.is_tensor(a) else a, dtype=torch.float64)
             .to(self.device).contiguous() for a in (alpha, kappa, m, Winv, nu)]
        nb = 2 if self.params.modal_split > 0 else 1
        if t[1].numel() != self.K * nb or t[4].numel() != self.K * nb:
            raise ValueError("kappa and nu need %d value(s) per component" % nb)
        self._keep = t  # alive until the stream has consumed them
        self._check(self.lib.vbgs_set_params(self.ctx, w, *[_ptr(a) for a in t], _stream()))

    def sync_status(self):
        return self.lib.vbgs_sync_status(self.ctx, _stream())

    def clear_flags(self):
        self._check(self.lib.vbgs_clear_flags(self.ctx, _stream()))

    def counters(self):
        out = (ctypes.c_int64 * 11)()
        self._check(self.lib.vbgs_counters(self.ctx, out, _stream()))
        names = {v: k for k, v in _lib.PREC.items()}
        return dict(refined_pass1=out[0], refined_pass2=out[1], N=out[2], K=out[3], blocks=out[4],
                    blocks_dense=out[5], blocks_cum=out[6], n_over=out[7], screen=names.get(out[8], out[8]),
                    screen_bound_bf16x3=out[9] / 1000.0, seg_miss=out[10])

    def reassign(self, X, lse, gumbel, n):
        """Move the means of the n least-used components onto n points drawn with probabilities
        proportional to exp(-lse) (Gumbel-top-n with the given draws). lse: FP64 log normalisers
        in nats from estep_stats on X. Returns (points, comps) int32 device tensors."""
        X = self._points(X)
        N = X.shape[0]
        lse = torch.as_tensor(lse, dtype=torch.float64).to(self.device).contiguous()
        gumbel = torch.as_tensor(gumbel, dtype=torch.float64).to(self.device).contiguous()
        if lse.shape != (N,) or gumbel.shape != (N,):
            raise ValueError("lse and gumbel must have one FP64 value per point")
        pts = torch.empty(max(int(n), 0), dtype=torch.int32, device=self.device)
        comps = torch.empty_like(pts)
        self._check(self.lib.vbgs_reassign(self.ctx, _ptr(X), N, _ptr(lse), _ptr(gumbel), int(n),
                                           _ptr(pts) if n > 0 else None, _ptr(comps) if n > 0 else None, _stream()))
        return pts, comps

    # ---- rendering ------------------------------------------------------------------------
    def renderer(self, n_max, score_prec=None, exact=True, **kw):
        """The position context vbgs_render needs: D_s = modal_split (or 2 for D = 5 images, else 3),
        the model's K, n_max query positions. Its parameters are overwritten by every render."""
        s = self.params.modal_split or (2 if self.D == 5 else 3)
        return VBGS(s, self.K, n_max, np.zeros((self.K, s)), np.eye(s), device=self.device,
                    score_prec=score_prec, exact=exact, **kw)

    def render(self, position, Xq, lse=False, regress=None):
        """Colour expected at the query positions Xq (Nq x D_s FP32): the responsibilities of the
        position marginal times each component's colour given the position. Returns (colour Nq x Dc
        FP32, lse Nq FP64 or None)."""
        Xq = position._points(Xq)
        Nq, s = Xq.shape[0], position.D
        Dc = self.D - s
        if regress is None:
            regress = torch.empty((self.K, Dc * (1 + s)), dtype=torch.float64, device=self.device)
        colour = torch.empty((Nq, Dc), dtype=torch.float32, device=self.device)
        lse_out = torch.empty(Nq, dtype=torch.float64, device=self.device) if lse else None
        st = self.lib.vbgs_render(self.ctx, position.ctx, _ptr(Xq), Nq, _ptr(regress), _ptr(colour),
                                  _ptr(lse_out), _stream())
        if st:
            raise VBGSError(st, self.lib.vbgs_last_error(position.ctx).decode())
        return colour, lse_out

    # ---- learned candidate proposal -----------------------------------------------------
    def _f32(self, a):
        return torch.as_tensor(np.asarray(a, np.float32) if not torch.is_tensor(a) else a,
                               dtype=torch.float32).to(self.device).contiguous()

    def proposal_set(self, W1, b1, W2, b2, E, beta, mu_in, inv_s_in):
        t = [self._f32(a) for a in (W1, b1, W2, b2, E, beta, mu_in, inv_s_in)]
        self._keep = t
        self._check(self.lib.vbgs_proposal_set(self.ctx, *[_ptr(a) for a in t], _stream()))

    def proposal_get(self):
        H, D, K, dev = _lib.H, self.D, self.K, self.device
        o = dict(W1=torch.empty((H, D), device=dev), b1=torch.empty(H, device=dev),
                 W2=torch.empty((H, H), device=dev), b2=torch.empty(H, device=dev),
                 E=torch.empty((K, H), device=dev), beta=torch.empty(K, device=dev))
        self._check(self.lib.vbgs_proposal_get(self.ctx, *[_ptr(o[k]) for k in ("W1", "b1", "W2", "b2", "E", "beta")],
                                               _stream()))
        return o

    def estep_stats_pruned(self, X, audit_idx=None, bound=float(np.log1p(-1e-4)), frac=0.01, lse=True, stats=True,
                           audit_n=4096, audit_seed=0):
        """Pruned E-step. audit_idx: the audited points (int32, distinct); None draws min(audit_n, N)
        of them without replacement from a generator seeded by audit_seed; an empty sequence turns the
        audit off (the report's captured-mass fields then read NaN)."""
        X = self._points(X)
        N = X.shape[0]
        lse_out = torch.empty(N, dtype=torch.float64, device=self.device) if lse else None
        stats_out = torch.empty((self.K, self.F), dtype=torch.float64, device=self.device) if stats else None
        report = torch.zeros(4, dtype=torch.float64, device=self.device)
        if audit_idx is None:
            g = np.random.default_rng(audit_seed)
            audit_idx = np.sort(g.choice(N, size=min(int(audit_n), N), replace=False)).astype(np.int32)
        audit_idx = torch.as_tensor(audit_idx, dtype=torch.int32).to(self.device).contiguous()
        na = audit_idx.numel()
        if na == 0:
            audit_idx = None
        self._audit = audit_idx
        self._check(self.lib.vbgs_estep_stats_pruned(self.ctx, _ptr(X), N, _ptr(audit_idx), na, float(bound),
                                                     float(frac), _ptr(lse_out), _ptr(stats_out), _ptr(report),
                                                     _stream()))
        return lse_out, stats_out, report

    def proposal_candidates(self, X):
        X = self._points(X)
        C = self.params.C if self.params.C > 0 else 32
        out = torch.empty((X.shape[0], C), dtype=torch.int32, device=self.device)
        self._check(self.lib.vbgs_proposal_candidates(self.ctx, _ptr(X), X.shape[0], _ptr(out), _stream()))
        return out

    def export_targets(self, X):
        """Training targets of the last exact E-step, whose points X must be."""
        X = self._points(X)
        N = X.shape[0]
        tk = torch.empty((N, 64), dtype=torch.int32, device=self.device)
        tr = torch.empty((N, 64), dtype=torch.float32, device=self.device)
        self._check(self.lib.vbgs_export_targets(self.ctx, _ptr(X), int(N), _ptr(tk), _ptr(tr), _stream()))
        return tk, tr

    def n_train(self):
        H = _lib.H
        return H * self.D + H + H * H + H + self.K * H + self.K

    def train_step(self, X, tk, tr, batch_idx, lr=1e-3, apply=True, loss=True, grads=False):
        X = self._points(X)
        bidx = torch.as_tensor(batch_idx, dtype=torch.int32).to(self.device).contiguous()
        loss_out = torch.empty(1, dtype=torch.float64, device=self.device) if loss else None
        g = torch.empty(self.n_train(), dtype=torch.float32, device=self.device) if grads else None
        self._bidx = bidx
        self._check(self.lib.vbgs_proposal_train_step(self.ctx, _ptr(X), _ptr(tk), _ptr(tr), _ptr(bidx),
                                                      bidx.numel(), float(lr), 1 if apply else 0, _ptr(loss_out),
                                                      _ptr(g), _stream()))
        return loss_out, g

    def timing(self, enable=True, phases=None):
        """Per-phase HIP-event timing on (every phase, or only the named ones, e.g. ["pass1"]) or off."""
        if phases is None or not enable:
            self._check(self.lib.vbgs_timing(self.ctx, 1 if enable else 0))
        else:
            mask = 0
            for p in phases:
                mask |= 1 << _lib.PHASES.index(p)
            self._check(self.lib.vbgs_timing_phases(self.ctx, mask))

    def timing_read(self):
        ms = (ctypes.c_double * _lib.NPHASE)()
        cnt = (ctypes.c_int64 * _lib.NPHASE)()
        self._check(self.lib.vbgs_timing_read(self.ctx, ms, cnt, _stream()))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(_lib.PHASES)}

    def close(self):
        if self.ctx:
            self.lib.vbgs_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
