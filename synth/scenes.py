"""Seeded synthetic scenes: the inputs shared by the oracle and the HIP path.

This module only draws data. It holds none of the method's arithmetic: no
expectations, scores, statistics or updates. Both the CPU oracle and the GPU
tests/benchmarks take their inputs from here so that they see identical bytes.

The paper trains on point clouds derived from posed RGB(-D) frames (Sec. 2.1.2,
the frame X_t of Alg. 1) of the Blender, Habitat and Replica datasets (Sec. 5.1).
Those datasets are not available, so every workload is a seeded synthetic
stand-in with the paper's scale: 1e5 components (Sec. 3, Sec. 5.2) and about one
camera frame of points.

Every draw uses ``numpy.random.Generator(PCG64(SeedSequence([2603, 8499, cfg,
frame, ...])))``; data are generated in float64 and handed out as float32 rows
(the GPU input type). Consumers widen the float32 values, never regenerate them.

Workloads (D = feature dimension, N = points per frame, K = components):

* ``c1`` 64x64 image, D=5 (u, v, r, g, b), 32 Gaussian blobs, K=256, unit prior.
* ``c2`` 3-D stream, D=6, 2000 anisotropic GT Gaussians, N=200000, K=10000,
  20 frames over a sliding x-window.
* ``c3`` orbiting pinhole camera over a 10000-Gaussian scene, D=6, N=307200
  (640x480), K=100000, 100 frames, depth noise sigma 0.005 along the view ray.
* ``c5`` 800x800 image, D=5, 20000 blobs and one background colour, K=50000.
* ``white`` c3's shapes with i.i.d. N(0.5, 0.15^2) coordinates.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_ROOT = (2603, 8499)


def rng(cfg: int, frame: int = 0, *extra: int) -> np.random.Generator:
    """Counter-style seeding: one independent stream per (config, frame, ...)."""
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence(list(SEED_ROOT) + [cfg, frame, *extra]))
    )


@dataclasses.dataclass
class Prior:
    """Shared Normal-Wishart / Dirichlet prior hyper-parameters.

    m0 is per component (K x D); W0 is the Wishart scale matrix (D x D, SPD),
    the same for every component; kappa0, nu0, alpha0 are scalars.
    """

    m0: np.ndarray
    W0: np.ndarray
    kappa0: float
    nu0: float
    alpha0: float

    @property
    def K(self) -> int:
        return self.m0.shape[0]

    @property
    def D(self) -> int:
        return self.m0.shape[1]


# ---------------------------------------------------------------------------
# small helpers (data drawing only)
# ---------------------------------------------------------------------------

def _haar_rotations(g: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed 3x3 rotations (QR of a Gaussian matrix, sign-fixed)."""
    A = g.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(A)
    s = np.sign(np.diagonal(R, axis1=1, axis2=2))
    s[s == 0] = 1.0
    Q = Q * s[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1.0
    return Q


def _log_uniform(g: np.random.Generator, lo: float, hi: float, size) -> np.ndarray:
    return np.exp(g.uniform(math.log(lo), math.log(hi), size))


def distinct_rows(g: np.random.Generator, X: np.ndarray, K: int) -> np.ndarray:
    """K distinct rows of X (by index), as float64: the initial prior means."""
    if K > X.shape[0]:
        raise ValueError("cannot draw %d distinct rows from %d points" % (K, X.shape[0]))
    idx = g.choice(X.shape[0], size=K, replace=False)
    return X[idx].astype(np.float64)


def r2_W0(D: int, K: int) -> np.ndarray:
    """Prior scale matrix matched to the component scale.

    Spatial dimensions get sigma_s^-2 with sigma_s = 0.5 K^(-1/3) (3-D) or
    0.5 K^(-1/2) (2-D images); colour dimensions get sigma_c^-2 = 400.
    """
    n_sp = 3 if D == 6 else 2
    sig_s = 0.5 * K ** (-1.0 / n_sp)
    d = np.full(D, 400.0)
    d[:n_sp] = sig_s ** -2
    return np.diag(d)


# ---------------------------------------------------------------------------
# c1 / c5: 2-D images built from Gaussian blobs
# ---------------------------------------------------------------------------

def _blob_image(g, H, W, n_blobs, s_lo, s_hi, background, beta=0.05, truncate=None):
    """rgb = (sum_j a_j c_j + beta b) / (sum_j a_j + beta), a_j = exp(-|uv-mu_j|^2 / (2 s_j^2))."""
    mu = g.uniform(0.0, 1.0, (n_blobs, 2))
    s = _log_uniform(g, s_lo, s_hi, n_blobs)
    col = g.uniform(0.0, 1.0, (n_blobs, 3))
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    num = np.zeros((H, W, 3))
    den = np.zeros((H, W))
    if truncate is None:
        uu, vv = np.meshgrid(u, v)  # (H, W): uu = column coordinate
        for j in range(n_blobs):
            a = np.exp(-0.5 * ((uu - mu[j, 0]) ** 2 + (vv - mu[j, 1]) ** 2) / s[j] ** 2)
            num += a[..., None] * col[j]
            den += a
    else:
        for j in range(n_blobs):
            r = truncate * s[j]
            c0 = max(0, int(math.floor((mu[j, 0] - r) * W)))
            c1 = min(W, int(math.ceil((mu[j, 0] + r) * W)) + 1)
            r0 = max(0, int(math.floor((mu[j, 1] - r) * H)))
            r1 = min(H, int(math.ceil((mu[j, 1] + r) * H)) + 1)
            if c0 >= c1 or r0 >= r1:
                continue
            uu, vv = np.meshgrid(u[c0:c1], v[r0:r1])
            a = np.exp(-0.5 * ((uu - mu[j, 0]) ** 2 + (vv - mu[j, 1]) ** 2) / s[j] ** 2)
            num[r0:r1, c0:c1] += a[..., None] * col[j]
            den[r0:r1, c0:c1] += a
    rgb = (num + beta * np.asarray(background)[None, None, :]) / (den + beta)[..., None]
    uu, vv = np.meshgrid(u, v)
    return uu, vv, rgb


def c1_frame():
    """c1: 64x64 pixels, D=5 rows (u, v, r, g, b) in raster order, N=4096."""
    g = rng(1, 0)
    uu, vv, rgb = _blob_image(g, 64, 64, 32, 0.02, 0.25, background=(0.0, 0.0, 0.0))
    rgb = rgb + g.normal(0.0, 0.01, rgb.shape)
    X = np.concatenate([uu[..., None], vv[..., None], rgb], axis=-1).reshape(-1, 5)
    return X.astype(np.float32)


def c1_prior(X: np.ndarray) -> Prior:
    g = rng(1, 0, 1)
    return Prior(m0=distinct_rows(g, X, 256), W0=np.eye(5), kappa0=1.0, nu0=7.0, alpha0=1.0)


def c5_frame(H: int = 800, W: int = 800, n_blobs: int = 20000):
    """c5: H x W pixels (default 800x800, N=640000), D=5, blobs over one background colour."""
    g = rng(5, 0)
    bg = g.uniform(0.0, 1.0, 3)
    uu, vv, rgb = _blob_image(g, H, W, n_blobs, 0.001, 0.02, background=bg, truncate=5.0)
    rgb = rgb + g.normal(0.0, 0.01, rgb.shape)
    X = np.concatenate([uu[..., None], vv[..., None], rgb], axis=-1).reshape(-1, 5)
    return X.astype(np.float32)


def c5_prior(X: np.ndarray, K: int = 50000) -> Prior:
    g = rng(5, 0, 1)
    return Prior(m0=distinct_rows(g, X, K), W0=r2_W0(5, K), kappa0=1.0, nu0=7.0, alpha0=1.0)


def c5_crop(X: np.ndarray, size: int = 160, H: int = 800, W: int = 800, K_full: int = 50000):
    """The top-left size x size pixels of a c5 frame with a prior of the full configuration's
    shape: K scaled by the crop's share of the pixels, means drawn from the crop, W0 of K_full."""
    Xc = np.ascontiguousarray(X.reshape(H, W, -1)[:size, :size].reshape(-1, X.shape[1]))
    K = max(1, round(K_full * size * size / (H * W)))
    g = rng(5, 0, 2)
    pr = Prior(m0=distinct_rows(g, Xc, K), W0=r2_W0(5, K_full), kappa0=1.0, nu0=7.0, alpha0=1.0)
    return Xc, pr


# ---------------------------------------------------------------------------
# c2 / c3: 3-D scenes of anisotropic Gaussians with a colour each
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class GaussScene:
    mu: np.ndarray     # (G, 3) centres
    L: np.ndarray      # (G, 3, 3) covariance factors: cov = L L^T
    col: np.ndarray    # (G, 3) colours


def gauss_scene(cfg: int, G: int, s_lo: float, s_hi: float) -> GaussScene:
    g = rng(cfg, 0, 7)
    mu = g.uniform(0.05, 0.95, (G, 3))
    sc = _log_uniform(g, s_lo, s_hi, (G, 3))
    Rt = _haar_rotations(g, G)
    L = Rt * sc[:, None, :]
    col = g.uniform(0.0, 1.0, (G, 3))
    return GaussScene(mu=mu, L=L, col=col)


def _sample_from(scene: GaussScene, g, idx, col_noise=0.01):
    z = g.standard_normal((idx.size, 3))
    xyz = scene.mu[idx] + np.einsum("nij,nj->ni", scene.L[idx], z)
    rgb = scene.col[idx] + g.normal(0.0, col_noise, (idx.size, 3))
    return xyz, rgb


def c2_frame(t: int, N: int = 200000, stationary: bool = False, scene: GaussScene | None = None):
    """c2 frame t: N points from GT Gaussians whose centre x lies in [0.03t, 0.03t+0.4]."""
    scene = scene or gauss_scene(2, 2000, 0.005, 0.05)
    g = rng(2, t)
    lo = 0.0 if stationary else 0.03 * t
    vis = np.nonzero((scene.mu[:, 0] >= lo) & (scene.mu[:, 0] <= lo + 0.4))[0]
    if vis.size == 0:
        vis = np.arange(scene.mu.shape[0])
    idx = vis[g.integers(0, vis.size, N)]
    xyz, rgb = _sample_from(scene, g, idx)
    xyz = np.clip(xyz, 0.0, 1.0)
    return np.concatenate([xyz, rgb], axis=1).astype(np.float32)


def c2_prior(X0: np.ndarray, K: int = 10000) -> Prior:
    g = rng(2, 0, 1)
    return Prior(m0=distinct_rows(g, X0, K), W0=r2_W0(6, K), kappa0=1.0, nu0=8.0, alpha0=1.0)


def _camera(t: int, radius: float = 1.5, elev: float = 0.35):
    ang = math.radians(3.6 * t)
    c = np.array([0.5, 0.5, 0.5])
    eye = c + np.array([radius * math.cos(ang), radius * math.sin(ang), elev])
    fwd = c - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return eye, fwd, right, down


def c3_frame(t: int, N: int = 307200, H: int = 480, W: int = 640, scene: GaussScene | None = None,
             depth_sigma: float = 0.005):
    """c3 frame t: N points sampled from the Gaussians visible to camera t.

    Pinhole camera, 60 degree vertical field of view, orbiting the cube centre
    at radius 1.5 (3.6 degrees per frame). Each point is drawn from a visible
    Gaussian (uniform over visible ones), moved along its view ray by
    N(0, depth_sigma^2), given its Gaussian's colour plus N(0, 0.01^2), and the
    points are sorted into the raster order of their projections.
    """
    scene = scene or gauss_scene(3, 10000, 0.003, 0.03)
    g = rng(3, t)
    eye, fwd, right, down = _camera(t)
    f = (H / 2) / math.tan(math.radians(30.0))
    rel = scene.mu - eye
    z = rel @ fwd
    u = f * (rel @ right) / np.maximum(z, 1e-9) + W / 2
    v = f * (rel @ down) / np.maximum(z, 1e-9) + H / 2
    vis = np.nonzero((z > 0.05) & (u >= 0) & (u < W) & (v >= 0) & (v < H))[0]
    if vis.size == 0:
        vis = np.arange(scene.mu.shape[0])
    idx = vis[g.integers(0, vis.size, N)]
    xyz, rgb = _sample_from(scene, g, idx)
    ray = xyz - eye
    ray /= np.linalg.norm(ray, axis=1, keepdims=True)
    xyz = xyz + ray * g.normal(0.0, depth_sigma, (N, 1))
    rel = xyz - eye
    zz = np.maximum(rel @ fwd, 1e-9)
    pu = np.clip(np.floor(f * (rel @ right) / zz + W / 2), 0, W - 1)
    pv = np.clip(np.floor(f * (rel @ down) / zz + H / 2), 0, H - 1)
    order = np.argsort(pv * W + pu, kind="stable")
    X = np.concatenate([xyz, rgb], axis=1)[order]
    return X.astype(np.float32)


def c3_prior(X0: np.ndarray, K: int = 100000) -> Prior:
    g = rng(3, 0, 1)
    return Prior(m0=distinct_rows(g, X0, K), W0=r2_W0(6, K), kappa0=1.0, nu0=8.0, alpha0=1.0)


def white_frame(t: int = 0, N: int = 307200, D: int = 6):
    """White-noise frame with c3's shapes: i.i.d. N(0.5, 0.15^2) coordinates."""
    g = rng(99, t)
    return g.normal(0.5, 0.15, (N, D)).astype(np.float32)


# ---------------------------------------------------------------------------
# small random problems for tests (tiny to medium shapes)
# ---------------------------------------------------------------------------

def random_problem(N: int, K: int, D: int, seed: int, spread: float = 0.08,
                   kappa0: float = 1.0, alpha0: float = 1.0, nu_extra: float = 2.0,
                   w_scale: float | None = None):
    """Clustered points in the unit cube plus a prior whose means are data rows.

    Points come from K_true = max(1, K // 2) isotropic clusters of std `spread`.
    Returns (X float32 N x D, Prior). The prior scale W0 = w_scale * I (default
    1 / spread^2, matched to the cluster size).
    """
    g = rng(1000 + D, seed, N, K)
    kt = max(1, K // 2)
    cen = g.uniform(0.1, 0.9, (kt, D))
    lab = g.integers(0, kt, N)
    X = cen[lab] + g.normal(0.0, spread, (N, D))
    X = X.astype(np.float32)
    m0 = X[g.choice(N, size=K, replace=K > N)].astype(np.float64)
    if K > N:
        m0 = m0 + g.normal(0.0, spread, m0.shape)
    ws = (1.0 / spread ** 2) if w_scale is None else w_scale
    pr = Prior(m0=m0, W0=np.eye(D) * ws, kappa0=kappa0, nu0=D + nu_extra, alpha0=alpha0)
    return X, pr


# ---------------------------------------------------------------------------
# proposal network initialisation (the random numbers the method draws, as inputs)
# ---------------------------------------------------------------------------

def mlp_init(D: int, H: int, K: int, seed: int, X0: np.ndarray | None = None):
    """He-initialised weights of the D -> H -> H -> K-embedding proposal network (float32).

    W1, W2 ~ N(0, 2 / fan_in); E ~ N(0, 1 / H); biases 0. The input normalisation
    (mu_in, inv_s_in) is the per-dimension mean and inverse standard deviation of X0
    (identity when X0 is None).
    """
    g = rng(77, seed, D, H, K)
    out = dict(W1=g.normal(0.0, np.sqrt(2.0 / D), (H, D)), b1=np.zeros(H),
               W2=g.normal(0.0, np.sqrt(2.0 / H), (H, H)), b2=np.zeros(H),
               E=g.normal(0.0, np.sqrt(1.0 / H), (K, H)), beta=np.zeros(K))
    if X0 is None:
        out["mu_in"], out["inv_s_in"] = np.zeros(D), np.ones(D)
    else:
        X0 = np.asarray(X0, np.float64)
        sd = X0.std(axis=0)
        out["mu_in"], out["inv_s_in"] = X0.mean(axis=0), 1.0 / np.where(sd > 0, sd, 1.0)
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in out.items()}


def audit_indices(N: int, n_audit: int, frame: int, cfg: int = 0) -> np.ndarray:
    """Seeded audit sample: n_audit distinct point indices of a frame of N points (sorted)."""
    g = rng(88, frame, cfg)
    n_audit = min(n_audit, N)
    return np.sort(g.choice(N, size=n_audit, replace=False)).astype(np.int32)


def gumbel_noise(N: int, frame: int, cfg: int = 0) -> np.ndarray:
    """Standard Gumbel draws -ln(-ln u), u ~ U(0, 1), FP64, for the biased point sampling of the
    reassignment step (one draw per point)."""
    u = rng(cfg, frame, 11).random(N)
    u = np.clip(u, 1e-300, 1.0 - 1e-16)
    return -np.log(-np.log(u))
