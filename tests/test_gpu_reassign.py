"""GPU reassignment step (Alg. 1, `reassign`) against the oracle, on identical seeded inputs."""
import numpy as np
import pytest
import torch

from oracle import reassign_ref as RA
from oracle import vbgs_ref as R
from synth import scenes

gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_08499_amd  # noqa: F401
    return torch.device("cuda:0")


def _model(dev, pr, n_max, prec="bf16x3"):
    import paper_2603_08499_amd as P
    return P.VBGS(pr.D, pr.K, n_max, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
                  score_prec=prec, exact=True)


@gpu
@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
@pytest.mark.parametrize("N,K,n", [(3000, 500, 64), (777, 1000, 777), (5000, 37, 37)])
def test_reassign_matches_oracle(dev, prec, N, K, n):
    print("case", prec, N, K, n, flush=True)
    X, pr = scenes.random_problem(N, K, 6, seed=N + K)
    g = np.random.default_rng(N * 7 + K)
    p = R.NW.from_prior(pr)
    # posterior with usage counts that tie in places (integers) and differ in others
    alpha = pr.alpha0 + np.where(g.random(K) < 0.5, 0.0, g.integers(1, 30, K).astype(np.float64))
    q = R.NW(alpha=alpha, kappa=p.kappa, m=p.m, Winv=p.Winv, nu=p.nu)
    lse = g.normal(-4.0, 3.0, N)
    lse[::17] = lse[0]  # exact ties in the point values too
    gm = scenes.gumbel_noise(N, 0, cfg=97)
    gm[::17] = gm[0]
    m = _model(dev, pr, N, prec)
    m.set_params("posterior", q.alpha, q.kappa, q.m, q.Winv, q.nu)
    pts, comps = m.reassign(torch.from_numpy(X).to(dev), lse, gm, n)
    torch.cuda.synchronize()
    rp, rc = RA.reassign(X, lse, gm, alpha, n)
    assert np.array_equal(pts.cpu().numpy(), rp) and np.array_equal(comps.cpu().numpy(), rc)
    mp_ref, mq_ref = RA.apply(p.m, q.m, X, rp, rc)
    got_q, got_p = m.get_params("posterior"), m.get_params("prior")
    assert np.array_equal(got_q["m"].cpu().numpy(), mq_ref)
    assert np.array_equal(got_p["m"].cpu().numpy(), mp_ref)
    for key in ("alpha", "kappa", "nu", "Winv"):  # nothing else changes
        assert np.array_equal(got_q[key].cpu().numpy(), getattr(q, key))


@gpu
def test_reassign_after_estep_and_refit(dev):
    """The step in its place: E-step LSE -> reassign -> the next E-step scores the moved
    components; the selection is valid for the GPU's own LSE and usage."""
    X, pr = scenes.random_problem(4000, 300, 6, seed=11)
    m = _model(dev, pr, 4000)
    Xd = torch.from_numpy(X).to(dev)
    for _ in range(3):
        m.estep_stats(Xd, lse=False, stats=False)
        m.update(commit=True)
    lse, _ = m.estep_stats(Xd, stats=False)
    alpha = m.get_params("posterior")["alpha"].cpu().numpy()
    gm = scenes.gumbel_noise(4000, 3, cfg=96)
    n = 25
    pts, comps = m.reassign(Xd, lse, gm, n)
    pts, comps = pts.cpu().numpy(), comps.cpu().numpy()
    v = gm - lse.cpu().numpy()
    assert len(set(pts)) == n and len(set(comps)) == n
    assert v[pts].min() >= np.sort(v)[::-1][n - 1] - 1e-9 * max(1.0, abs(v).max())
    assert alpha[comps].max() <= np.sort(alpha)[n - 1] * (1 + 1e-7)
    assert np.array_equal(m.get_params("posterior")["m"].cpu().numpy()[comps], X[pts].astype(np.float64))
    with pytest.raises(Exception):
        m.elbo()  # the last E-step's bound no longer belongs to the posterior
    lse2, st = m.estep_stats(Xd)
    torch.cuda.synchronize()
    assert m.sync_status() == 0 and np.isfinite(lse2.cpu().numpy()).all()
    assert st[comps, 0].sum().item() > 0.0  # the moved components take responsibility


@gpu
def test_reassign_edge_cases(dev):
    X, pr = scenes.random_problem(100, 20, 3, seed=3)
    m = _model(dev, pr, 100)
    Xd = torch.from_numpy(X).to(dev)
    before = m.get_params("posterior")["m"].cpu().numpy()
    pts, comps = m.reassign(Xd, np.zeros(100), np.zeros(100), 0)
    assert pts.numel() == 0 and np.array_equal(m.get_params("posterior")["m"].cpu().numpy(), before)
    with pytest.raises(Exception):
        m.reassign(Xd, np.zeros(100), np.zeros(100), 21)
