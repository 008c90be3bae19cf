"""GPU parity of the two-factor (spatial / colour) likelihood of Sec. 2.1.2 against its FP64 oracle.

The library takes the factorised model when modal_split = s > 0: coordinates [0, s) and [s, D)
carry their own Normal-Wishart factor (own kappa, nu, W). Tolerances are those of the one-factor
parity tests: per-point LSE within 2e-6 nats, statistics relerr <= 1e-5, ELBO <= 1e-6 relative.
"""
import numpy as np
import pytest
import torch

from oracle import factorised_ref as F
from oracle import vbgs_ref as R
from synth import scenes

gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_08499_amd  # noqa: F401  (fails loudly if libvbgs.so is missing)
    return torch.device("cuda:0")


def _model(dev, pr, n_max, split, prec="bf16x3", **kw):
    import paper_2603_08499_amd as P
    return P.VBGS(pr.D, pr.K, n_max, pr.m0, pr.W0, device=dev, kappa0=pr.kappa0, nu0=pr.nu0, alpha0=pr.alpha0,
                  score_prec=prec, exact=True, modal_split=split, **kw)


def _stat_err(ref, got, D):
    cut = [0, 1, 1 + D, ref.shape[1]]
    return max(R.relerr(ref[:, a:b], got[:, a:b]) for a, b in zip(cut, cut[1:]))


def _perturbed(p: F.NW2, seed: int) -> F.NW2:
    g = np.random.default_rng(seed)
    K, D = p.m.shape
    Winv = np.zeros_like(p.Winv)
    for b in (0, 1):
        i = p.idx(b)
        A = g.normal(0, 0.25, (K, len(i), len(i)))
        base = p.Winv[:, i][:, :, i]
        Winv[:, i[:, None], i[None, :]] = (base * g.uniform(0.5, 2.0, (K, 1, 1))
                                           + np.einsum("kij,klj->kil", A, A) * base[:, :1, :1])
    return F.NW2(alpha=p.alpha * g.uniform(0.5, 5.0, K), kappa=p.kappa * g.uniform(0.5, 4.0, (K, 2)),
                 m=p.m + g.normal(0, 0.01, p.m.shape), Winv=Winv, nu=p.nu + g.uniform(0.0, 6.0, (K, 2)),
                 split=p.split)


def _set(m, which, q: F.NW2):
    m.set_params(which, q.alpha, q.kappa, q.m, q.Winv, q.nu)


@gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("N,K,D,split", [(3001, 301, 6, 3), (777, 90, 5, 2), (1500, 120, 2, 1), (1000, 1, 6, 3)])
def test_factorised_estep_parity(dev, prec, N, K, D, split):
    print("factorised case", prec, N, K, D, split, flush=True)
    X, pr = scenes.random_problem(N, K, D, seed=N + K + 1)
    p = F.NW2.from_prior(pr, split)
    q = _perturbed(p, 6)
    m = _model(dev, pr, N, split, prec)
    _set(m, "posterior", q)
    lse, st = m.estep_stats(torch.from_numpy(X).to(dev))
    Fg = m.elbo()
    m.update(commit=False)
    post = m.get_params("posterior")
    torch.cuda.synchronize()
    assert m.sync_status() == 0
    e = F.expectations(q)
    ls = F.lse(X, q, e)
    sr = F.stats(X, q, ls, e)
    Fr = F.elbo(ls.sum(), q, p, e)
    qn = F.update(p, sr)
    dl = np.abs(lse.cpu().numpy() - ls).max()
    es = _stat_err(sr.packed(), st.cpu().numpy(), D)
    eF = abs(Fg.item() - Fr) / abs(Fr)
    print("  max|dLSE| %.2e stats relerr %.2e ELBO relerr %.2e" % (dl, es, eF), m.counters())
    assert dl < 2e-6 and es < 1e-5 and eF < 1e-6
    assert R.relerr(qn.kappa, post["kappa"].cpu().numpy()) < 1e-5
    assert R.relerr(qn.nu, post["nu"].cpu().numpy()) < 1e-5
    assert R.relerr(qn.m, post["m"].cpu().numpy()) < 1e-5
    assert R.relerr(qn.Winv, post["Winv"].cpu().numpy()) < 1e-4


@gpu
@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_factorised_cavi_c1_trajectory(dev, prec):
    """Ten coordinate-ascent steps of the two-factor model on the 2-D image (x, y | r, g, b)."""
    X = scenes.c1_frame()
    pr = scenes.c1_prior(X)
    p = F.NW2.from_prior(pr, 2)
    q, Fr = F.cavi(X.astype(np.float64), p, 10)
    m = _model(dev, pr, X.shape[0], 2, prec)
    Xg = torch.from_numpy(X).to(dev)
    Fs = []
    for _ in range(10):
        m.estep_stats(Xg, lse=False)
        Fs.append(m.elbo().item())
        m.update(commit=False)
    post = m.get_params("posterior")
    torch.cuda.synchronize()
    rel = np.abs(np.array(Fs) - np.array(Fr)) / np.abs(np.array(Fr))
    print(prec, "ELBO relerr per step", rel.max())
    assert rel.max() < 1e-5
    assert all(b >= a - 1e-6 * abs(a) for a, b in zip(Fs, Fs[1:])), Fs
    assert R.relerr(q.m, post["m"].cpu().numpy()) < 1e-5
    assert R.relerr(q.Winv, post["Winv"].cpu().numpy()) < 1e-4
    assert R.relerr(q.kappa, post["kappa"].cpu().numpy()) < 1e-6


@gpu
def test_factorised_prior_and_roundtrip(dev):
    """The prior drops W0's cross-factor entries; parameters round-trip with two kappa / nu per row."""
    X, pr = scenes.random_problem(400, 30, 6, seed=4)
    W0 = np.array(pr.W0, np.float64)
    W0[0, 5] = W0[5, 0] = 0.2 * W0[0, 0]
    pr.W0 = W0
    m = _model(dev, pr, 400, 3)
    prior = m.get_params("prior")
    torch.cuda.synchronize()
    p = F.NW2.from_prior(pr, 3)
    for name in ("alpha", "kappa", "m", "Winv", "nu"):
        assert R.relerr(getattr(p, name), prior[name].cpu().numpy()) < 1e-13, name
    q = _perturbed(p, 8)
    _set(m, "posterior", q)
    post = m.get_params("posterior")
    torch.cuda.synchronize()
    assert tuple(post["kappa"].shape) == (30, 2)
    for name in ("alpha", "kappa", "m", "Winv", "nu"):
        assert R.relerr(getattr(q, name), post[name].cpu().numpy()) < 1e-13, name
    with pytest.raises(ValueError):
        m.set_params("posterior", q.alpha, q.kappa[:, 0], q.m, q.Winv, q.nu[:, 0])


@gpu
def test_factorised_culled_c3_slice(dev):
    """The culled sweep's per-tile bounds use the spatial factor's own nu: culled and unculled
    agree to FP64 rounding and both match the oracle on a slice of the c3 frame."""
    scene = scenes.gauss_scene(3, 10000, 0.003, 0.03)
    X0 = scenes.c3_frame(0, scene=scene)
    pr = scenes.c3_prior(X0, K=20000)
    X = np.ascontiguousarray(X0[100000:108192])
    p = F.NW2.from_prior(pr, 3)
    e = F.expectations(p)
    ls = F.lse(X, p, e)
    ref = F.stats(X, p, ls, e, scatter=False).packed()
    Xd = torch.from_numpy(X).to(dev)
    out = []
    for cull in (0, 1):
        m = _model(dev, pr, X.shape[0], 3, "bf16x3", cull=bool(cull))
        lse, st = m.estep_stats(Xd)
        torch.cuda.synchronize()
        assert m.sync_status() == 0
        l, s = lse.cpu().numpy(), st.cpu().numpy()
        print("  cull=%d max|dLSE| %.2e stats relerr %.2e" % (cull, np.abs(l - ls).max(), _stat_err(ref, s, 6)),
              m.counters())
        assert np.abs(l - ls).max() < 2e-6 and _stat_err(ref, s, 6) < 1e-5
        out.append((l, s))
        m.close()
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-9
    assert _stat_err(out[0][1], out[1][1], 6) < 1e-9
