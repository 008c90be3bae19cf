"""vbgs_estep_stats_scratch (the E-step that allocates nothing: a static device array of the library
is its workspace) against vbgs_estep_stats on the same context and points, through the C ABI: two
calls in a row, the second with fewer points, so that what the first call left in the shared array
cannot reach the second one's results. Both run the same kernels, so the results are compared
bitwise; the context's own statistics must be untouched by the scratch call."""
import ctypes

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


def _ctx(dev, pr, N, prec):
    import paper_2603_08499_amd as P
    m = P.VBGS(6, pr.K, N, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
               score_prec=prec, exact=True)
    return m


@gpu
@pytest.mark.parametrize("prec", ["auto", "bf16x3", "fp64"])
def test_scratch_estep_matches_workspace_estep(dev, prec):
    import paper_2603_08499_amd as P
    from paper_2603_08499_amd import _lib
    scene = scenes.gauss_scene(2, 2000, 0.005, 0.05)
    frames = [scenes.c2_frame(t, N=24000, scene=scene) for t in range(4)]
    pr = scenes.c2_prior(frames[0], K=3000)
    N = frames[0].shape[0]
    m = _ctx(dev, pr, N, prec)
    assert P.query_sizes(m.params)[1] <= _lib.SCRATCH_BYTES
    Xs = [torch.from_numpy(f).to(dev) for f in frames]
    for t in range(2):  # a committed posterior, not the prior
        m.estep_stats(Xs[t], lse=False, stats=False)
        m.update(commit=True)
    small = Xs[3][:7001].contiguous()
    for X in (Xs[2], small):  # two calls in a row, the second with fewer points
        print("scratch E-step: prec %s, N = %d, K = %d" % (prec, X.shape[0], pr.K), flush=True)
        lse_w, st_w = m.estep_stats(X)
        lse_s, st_s = m.estep_stats_scratch(X)
        torch.cuda.synchronize()
        assert torch.equal(lse_w, lse_s) and torch.equal(st_w, st_s)
        assert abs(st_s[:, 0].sum().item() - X.shape[0]) < 1e-9 * X.shape[0]
    assert m.sync_status() == 0
    # the scratch call leaves the context's statistics alone: the update after
    # [estep_stats(A), scratch(B)] equals the update after estep_stats(A)
    ref = _ctx(dev, pr, N, prec)
    ref.set_params("prior", **{k: v for k, v in m.get_params("prior").items()})
    ref.set_params("posterior", **{k: v for k, v in m.get_params("posterior").items()})
    for mm, extra in ((m, True), (ref, False)):
        mm.estep_stats(Xs[2], lse=False, stats=False)
        if extra:
            mm.estep_stats_scratch(small)
        mm.update(commit=False)
    a, b = m.get_params("posterior"), ref.get_params("posterior")
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k


@gpu
def test_scratch_rejects_params_beyond_its_size(dev):
    import paper_2603_08499_amd as P
    from paper_2603_08499_amd import _lib
    X, pr = scenes.random_problem(2000, 50, 6, seed=3)
    big = 400000  # n_max sizes the workspace beyond the scratch
    m = P.VBGS(6, pr.K, big, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0)
    assert P.query_sizes(m.params)[1] > _lib.SCRATCH_BYTES
    Xg = torch.from_numpy(X).to(dev)
    with pytest.raises(P.VBGSError) as e:
        m.estep_stats_scratch(Xg)
    assert e.value.status == -2 and "static scratch" in str(e.value)
    lse, st = m.estep_stats(Xg)  # the context still works
    torch.cuda.synchronize()
    assert m.sync_status() == 0 and abs(st[:, 0].sum().item() - 2000) < 1e-9 * 2000
