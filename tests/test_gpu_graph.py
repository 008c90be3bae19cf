"""One full update step (E-step with the culled sweep and the side-stream component preparation,
ELBO, committed update) captured once in a HIP graph and replayed: every replay must give what the
same step gives when its calls are made one by one. The step is deterministic (integer statistics
sums, fixed per-wave candidate order), so the comparison is bitwise. Eager work and host
synchronisations sit between the replays."""
import numpy as np
import pytest
import torch

from synth import scenes

gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_08499_amd  # noqa: F401  (fails loudly if libvbgs.so is missing)
    return torch.device("cuda:0")


def _model(dev, pr, n):
    import paper_2603_08499_amd as P
    return P.VBGS(pr.D, pr.K, n, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
                  score_prec="bf16x3", exact=True)


def _step(m, X, lse_out, st_out, F_out):
    m.estep_stats(X, lse_out=lse_out, stats_out=st_out)
    m.elbo(out=F_out)
    m.update(commit=True)


@gpu
def test_update_step_graph_replays_match_eager(dev):
    X, pr = scenes.random_problem(20000, 2000, 6, seed=77)
    Xd = torch.from_numpy(X).to(dev)
    N, K, F = X.shape[0], pr.K, 28
    eager, graphed = _model(dev, pr, N), _model(dev, pr, N)
    bufs = {name: (torch.empty(N, dtype=torch.float64, device=dev), torch.empty((K, F), dtype=torch.float64, device=dev),
                   torch.empty(1, dtype=torch.float64, device=dev)) for name in ("eager", "graph")}
    for m, name in ((eager, "eager"), (graphed, "graph")):  # one eager step each (measures the sweep's block costs)
        _step(m, Xd, *bufs[name])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _step(graphed, Xd, *bufs["graph"])
    for rep in range(4):
        g.replay()
        torch.cuda.synchronize()
        _step(eager, Xd, *bufs["eager"])
        torch.cuda.synchronize()
        assert graphed.sync_status() == 0 and eager.sync_status() == 0
        le, se, fe = (t.cpu().numpy() for t in bufs["eager"])
        lg, sg, fg = (t.cpu().numpy() for t in bufs["graph"])
        pe, pg = eager.get_params("posterior"), graphed.get_params("posterior")
        print("replay %d: ELBO %.10e vs %.10e" % (rep, fg[0], fe[0]), flush=True)
        assert np.array_equal(lg, le) and np.array_equal(sg, se) and np.array_equal(fg, fe)
        for k in pe:
            assert torch.equal(pe[k], pg[k]), k
    eager.close()
    graphed.close()
