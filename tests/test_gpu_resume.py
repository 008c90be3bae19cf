"""Checkpoint and resume: a copy of the state buffer, attached to a new context (vbgs_attach) with a
workspace full of arbitrary bytes, continues the frame stream exactly as the uninterrupted context
does (bitwise: every reduction of the exact mode has a fixed order or is an integer sum), and the
sticky flags and counters of the new context start cleared."""
import numpy as np
import pytest
import torch

from synth import scenes

gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_08499_amd  # noqa: F401
    return torch.device("cuda:0")


def _frame_step(m, Xg):
    lse, st = m.estep_stats(Xg)
    F = m.elbo()
    m.update(commit=True)
    post = m.get_params("posterior")
    return [lse, st, F] + [post[k] for k in ("alpha", "kappa", "m", "Winv", "nu")]


@gpu
@pytest.mark.parametrize("prec", ["auto", "fp64"])
def test_resume_from_state_copy_is_bitwise_equal(dev, prec):
    import paper_2603_08499_amd as P
    scene = scenes.gauss_scene(2, 2000, 0.005, 0.05)
    frames = [scenes.c2_frame(t, N=30000, scene=scene) for t in range(6)]
    pr = scenes.c2_prior(frames[0], K=1500)
    kw = dict(kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0, score_prec=prec, exact=True)
    Xs = [torch.from_numpy(f).to(dev) for f in frames]
    a = P.VBGS(6, pr.K, 30000, pr.m0, pr.W0, device=dev, **kw)
    b = P.VBGS(6, pr.K, 30000, pr.m0, pr.W0, device=dev, **kw)
    for t in range(3):
        _frame_step(a, Xs[t])
        _frame_step(b, Xs[t])
    saved = b.state.clone()
    torch.cuda.synchronize()
    b.close()
    del b
    r = P.VBGS(6, pr.K, 30000, None, None, device=dev, state=saved, **kw)
    r.workspace.fill_(0xFF)  # stale flags and counters must not survive the attach
    for t in range(3, 6):
        want = _frame_step(a, Xs[t])
        got = _frame_step(r, Xs[t])
        for x, y in zip(want, got):
            assert torch.equal(x, y), t
    torch.cuda.synchronize()
    assert r.sync_status() == 0 and a.sync_status() == 0
    if prec == "auto":
        ca, cr = a.counters(), r.counters()
        # blocks screened since init (a) or since the attach (r): r saw frames 3..5 only
        assert 0 < cr["blocks_cum"] < ca["blocks_cum"]
        assert ca["blocks"] == cr["blocks"] and ca["refined_pass2"] == cr["refined_pass2"]
