// Per-frame preparation and per-component FP64 kernels:
//   frame moments and quadratic point features (the per-point statistics S_u of Alg. 1),
//   posterior -> expectations -> score coefficients, and the KL terms of the ELBO,
//   conjugate update (Alg. 1: S <- S + Delta S, update_from_statistics), ELBO reduction.
#include "vbgs_internal.h"

namespace vbgs {

// ---------------------------------------------------------------------------
// state records: [alpha, kappa, nu, m (D), W^{-1} upper-packed row-major (i <= j)]
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tri_up(int i, int j, int D) {  // index of (i, j), i <= j
  return i * D - i * (i - 1) / 2 + (j - i);
}

__global__ void k_init_state(StateHeader* hdr, double* prior, double* post, const double* __restrict__ m0, Init0 in,
                             int D, int64_t K) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    hdr->magic = STATE_MAGIC;
    hdr->abi = VBGS_ABI_VERSION;
    hdr->D = D;
    hdr->K = K;
  }
  if (k >= K) return;
  double r[REC];
  for (int i = 0; i < REC; ++i) r[i] = 0.0;
  r[0] = in.alpha0;
  r[1] = in.kappa0;
  r[2] = in.nu0;
  if (in.split > 0) {  // second block: the same kappa0 and nu0
    r[rec_kc(D)] = in.kappa0;
    r[rec_kc(D) + 1] = in.nu0;
  }
  for (int i = 0; i < D; ++i) r[3 + i] = m0[k * D + i];
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j)
      r[3 + D + tri_up(i, j, D)] = coord_block(i, in.split) == coord_block(j, in.split) ? in.W0inv[i * D + j] : 0.0;
  for (int i = 0; i < REC; ++i) {
    prior[k * REC + i] = r[i];
    post[k * REC + i] = r[i];
  }
}

hipError_t launch_init_state(const DevPtrs& d, const double* m0, const Init0& init, hipStream_t s) {
  const int64_t K = d.K;
  hipLaunchKernelGGL(k_init_state, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<StateHeader*>(d.state), d.prior(), d.post(), m0, init, d.D, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// frame moments (deterministic two-level reduction) and features
// ---------------------------------------------------------------------------
// sum of v over a wave (xor butterfly: a fixed order)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// per j, the sum of v[j] over a workgroup of 256 threads: each wave's, then the four in order;
// thread t < 2 MAXD returns the sum for j = t
__device__ __forceinline__ double block_sums(const double (&v)[2 * MAXD], double (*sh)[2 * MAXD]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int j = 0; j < 2 * MAXD; ++j) {
    const double u = wave_sum(v[j]);
    if (lane == 0) sh[w][j] = u;
  }
  __syncthreads();
  return t < 2 * MAXD ? ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t] : 0.0;
}

// per workgroup of 256 threads, the sums of x and x^2 per coordinate over its range of points
__global__ __launch_bounds__(256) void k_moments_partial(const float* __restrict__ X, int64_t N, int D,
                                                         double* __restrict__ part) {
  __shared__ double sh[4][2 * MAXD];
  const int t = threadIdx.x;
  const int64_t per = (N + MOM_BLOCKS - 1) / MOM_BLOCKS;
  const int64_t a = (int64_t)blockIdx.x * per, b = min(N, a + per);
  double v[2 * MAXD];
#pragma unroll
  for (int j = 0; j < 2 * MAXD; ++j) v[j] = 0.0;
  for (int64_t n = a + t; n < b; n += 256)
#pragma unroll
    for (int i = 0; i < MAXD; ++i)
      if (i < D) {
        const double x = (double)X[n * D + i];
        if (isfinite(x)) {
          v[i] += x;
          v[MAXD + i] += x * x;
        }
      }
  const double r = block_sums(v, sh);
  if (t < 2 * MAXD) part[blockIdx.x * 2 * MAXD + t] = r;
}

__global__ __launch_bounds__(256) void k_moments_final(const double* __restrict__ part, int64_t N, int D,
                                                       FrameInfo* fr) {
  __shared__ double sh[4][2 * MAXD];
  __shared__ double tot[2 * MAXD];
  const int t = threadIdx.x;
  double v[2 * MAXD];
#pragma unroll
  for (int j = 0; j < 2 * MAXD; ++j) v[j] = 0.0;
  for (int b = t; b < MOM_BLOCKS; b += 256) {
    const f64x2* p2 = reinterpret_cast<const f64x2*>(part + b * 2 * MAXD);
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
      const f64x2 q = p2[j];
      v[2 * j] += q.x;
      v[2 * j + 1] += q.y;
    }
  }
  const double r = block_sums(v, sh);
  if (t < 2 * MAXD) tot[t] = r;
  __syncthreads();
  const int i = t;
  if (i >= MAXD) return;
  const double s1 = tot[i], s2 = tot[MAXD + i];
  float mu = 0.0f;
  double sc = 1.0;
  if (i < D && N > 0) {
    const double mean = s1 / (double)N;
    const double var = fmax(s2 / (double)N - mean * mean, 0.0);
    mu = (float)mean;
    const double sd = sqrt(var);
    if (sd > 0.0 && isfinite(sd)) sc = exp2(rint(log2(sd)));  // power of two: scaling is exact
  }
  fr->mu[i] = mu;
  fr->s[i] = sc;
  fr->inv_s[i] = (float)(1.0 / sc);
  if (i == 0) {
    fr->refined1 = 0;
    fr->refined2 = 0;
    fr->n_over = 0;
    fr->blocks = 0;
  }
}

// phi(x') = [1, x'_0..x'_{D-1}, x'_i x'_j (i <= j, row-major)], zero padded to 32 slots,
// with x' = (x - mu) / s computed in FP32. Stored as FP32 and as a bfloat16 hi/lo split,
// plus the Euclidean norm (rounded up) used by the screening bound.
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ X, int64_t N, int D,
                                                  const FrameInfo* __restrict__ fr, float* __restrict__ phi32,
                                                  uint16_t* __restrict__ phih, uint16_t* __restrict__ phil,
                                                  float* __restrict__ nphi, int* flags) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float xs[MAXD];
  bool fin = true;
  for (int i = 0; i < MAXD; ++i) {
    if (i < D) {
      const float v = X[n * D + i];
      fin = fin && isfinite(v);
      xs[i] = (v - fr->mu[i]) * fr->inv_s[i];
    }
  }
  if (!fin) {
    atomicOr(flags, FLAG_NONFINITE);
    for (int i = 0; i < D; ++i) xs[i] = 0.0f;
  }
  float f[FP];
  for (int i = 0; i < FP; ++i) f[i] = 0.0f;
  f[0] = 1.0f;
  int o = 1 + D;
  for (int i = 0; i < D; ++i) {
    f[1 + i] = xs[i];
    for (int j = i; j < D; ++j) f[o++] = xs[i] * xs[j];
  }
  double nn = 0.0;
  for (int i = 0; i < FP; ++i) nn += (double)f[i] * (double)f[i];
  if (phi32) {  // (null: no kernel of this context's precision reads the FP32 rows)
    f32x4* p32 = reinterpret_cast<f32x4*>(phi32 + n * FP);
    for (int q = 0; q < FP / 4; ++q) p32[q] = f32x4{f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]};
  }
  uint32_t hw[FP / 2], lw[FP / 2];
#pragma unroll
  for (int q = 0; q < FP / 2; ++q) {
    const uint16_t h0 = f2bf(f[2 * q]), h1 = f2bf(f[2 * q + 1]);
    const uint16_t l0 = f2bf(f[2 * q] - bf2f(h0)), l1 = f2bf(f[2 * q + 1] - bf2f(h1));
    hw[q] = (uint32_t)h0 | ((uint32_t)h1 << 16);
    lw[q] = (uint32_t)l0 | ((uint32_t)l1 << 16);
  }
  u32x4* ph = reinterpret_cast<u32x4*>(phih + n * FP);
  u32x4* pl = reinterpret_cast<u32x4*>(phil + n * FP);
#pragma unroll
  for (int q = 0; q < FP / 8; ++q) {
    ph[q] = u32x4{hw[4 * q], hw[4 * q + 1], hw[4 * q + 2], hw[4 * q + 3]};
    pl[q] = u32x4{lw[4 * q], lw[4 * q + 1], lw[4 * q + 2], lw[4 * q + 3]};
  }
  nphi[n] = (float)(sqrt(nn) * (1.0 + 1e-6));
}

// sum of alpha over the posterior and the frame prior: per-block partial sums over fixed ranges,
// then a fixed-order tree over the partials (deterministic)
constexpr int ALPHA_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_alpha_part(const double* __restrict__ prior, const double* __restrict__ post,
                                                    int64_t K, double* __restrict__ part) {
  __shared__ double sq[256], sp[256];
  const int t = threadIdx.x;
  const int64_t per = (K + ALPHA_BLOCKS - 1) / ALPHA_BLOCKS;
  const int64_t k0 = blockIdx.x * per, k1 = min(K, k0 + per);
  double a = 0.0, b = 0.0;
  for (int64_t k = k0 + t; k < k1; k += 256) {
    a += post[k * REC];
    b += prior[k * REC];
  }
  sq[t] = a;
  sp[t] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sq[t] += sq[t + w];
      sp[t] += sp[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = sq[0];
    part[2 * blockIdx.x + 1] = sp[0];
  }
}

__global__ __launch_bounds__(256) void k_alpha_final(const double* __restrict__ part, FrameInfo* fr) {
  __shared__ double sq[256], sp[256];
  const int t = threadIdx.x;
  sq[t] = part[2 * t];
  sp[t] = part[2 * t + 1];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sq[t] += sq[t + w];
      sp[t] += sp[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    fr->sum_alpha_q = sq[0];
    fr->sum_alpha_p = sp[0];
  }
}

// FP8 tier: rows of FP FP32 values -> OCP e4m3 bytes. Each row is scaled by the power of two 2^e that
// puts its largest magnitude in [224, 448] (the scaling is exact), rounded to nearest even by the
// hardware conversion; inv[r] = 2^-e undoes it on the scores.
__global__ __launch_bounds__(256) void k_fp8_rows(const float* __restrict__ src, int64_t nrows,
                                                  uint8_t* __restrict__ dst, float* __restrict__ inv) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nrows) return;
  float v[FP];
  const f32x4* s4 = reinterpret_cast<const f32x4*>(src + r * FP);
#pragma unroll
  for (int q = 0; q < FP / 4; ++q) {
    const f32x4 t = s4[q];
    v[4 * q] = t[0];
    v[4 * q + 1] = t[1];
    v[4 * q + 2] = t[2];
    v[4 * q + 3] = t[3];
  }
  float mx = 0.0f;
#pragma unroll
  for (int i = 0; i < FP; ++i) mx = fmaxf(mx, fabsf(v[i]));
  float sc = 1.0f, un = 1.0f;
  if (mx > 7.8886091e-31f && mx <= 3.4e38f) {  // 2^-100: rows below are left unscaled (they round to 0)
    int e;
    frexpf(448.0f / mx, &e);  // 448 / mx in [2^(e-1), 2^e)
    sc = ldexpf(1.0f, e - 1);
    un = ldexpf(1.0f, 1 - e);
  }
  uint32_t* d32 = reinterpret_cast<uint32_t*>(dst + r * FP);
#pragma unroll
  for (int q = 0; q < FP / 4; ++q) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q] * sc, v[4 * q + 1] * sc, 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * q + 2] * sc, v[4 * q + 3] * sc, w, true);
    d32[q] = (uint32_t)w;
  }
  inv[r] = un;
}

hipError_t launch_frame_prep(const DevPtrs& d, const float* X, int64_t N, hipStream_t s, int part_sel) {
  const Layout& L = *d.L;
  double* part = d.at<double>(L.mom_part);
  if (part_sel != 1) {
    hipLaunchKernelGGL(k_moments_partial, dim3(MOM_BLOCKS), dim3(256), 0, s, X, N, d.D, part);
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(256), 0, s, part, N, d.D, d.frame());
  }
  if (part_sel == 0) return hipGetLastError();
  if (N > 0 && d.D <= 6)  // quadratic features fill 1 + D + D(D+1)/2 <= 32 slots only for D <= 6
    hipLaunchKernelGGL(k_features, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, X, N, d.D, d.frame(),
                       L.f32rows || L.fp8 ? d.at<float>(L.phi32) : nullptr, d.at<uint16_t>(L.phih), d.at<uint16_t>(L.phil),
                       d.at<float>(L.nphi),
                       &d.frame()->flags);
  if (N > 0 && L.fp8)
    hipLaunchKernelGGL(k_fp8_rows, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, d.at<float>(L.phi32), N,
                       d.at<uint8_t>(L.phi8), d.at<float>(L.phis));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// posterior -> expectations -> coefficient rows (FP64, one thread per component)
// ---------------------------------------------------------------------------
template <int D>
__device__ bool cholesky(double A[D][D]) {  // in place, lower factor; false if not PD
  for (int j = 0; j < D; ++j) {
    double s = A[j][j];
    for (int t = 0; t < j; ++t) s -= A[j][t] * A[j][t];
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double l = sqrt(s);
    A[j][j] = l;
    for (int i = j + 1; i < D; ++i) {
      double v = A[i][j];
      for (int t = 0; t < j; ++t) v -= A[i][t] * A[j][t];
      A[i][j] = v / l;
    }
  }
  return true;
}

template <int D>
__device__ void load_winv(const double* r, double A[D][D]) {
  for (int i = 0; i < D; ++i)
    for (int j = i; j < D; ++j) A[i][j] = A[j][i] = r[3 + D + tri_up(i, j, D)];
}

struct CoefOut {  // rows in component order
  int64_t K;
  float* lam;           // lower bound on the score curvature in the first min(D, 3) coordinates
  double* direct;
  float* c32;  // (may be null: no FP32 rows)
  uint16_t* ch;
  uint16_t* cl;
  float* nc;
};

__device__ void write_dead_row(const CoefOut& o, int64_t k, int dts, bool expanded) {
  for (int i = 0; i < (expanded ? FP : 0); ++i) {
    const float v = i == 0 ? DEAD_C0 : 0.0f;
    if (o.c32) o.c32[k * FP + i] = v;
    const uint16_t h = f2bf(v);
    o.ch[k * FP + i] = h;
    o.cl[k * FP + i] = f2bf(v - bf2f(h));
  }
  if (expanded) o.nc[k] = 0.0f;
  for (int i = 0; i < dts; ++i) o.direct[k * dts + i] = i == 0 ? -1.0e300 : 0.0;
}

template <int D>
__global__ __launch_bounds__(128) void k_coeffs(const double* __restrict__ prior, const double* __restrict__ post,
                                                int64_t K, int64_t Kpad, const FrameInfo* __restrict__ fr,
                                                CoefOut o, int* flags, int split, int ns) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Kpad) return;
  constexpr int dts = D <= 6 ? 32 : 48;
  if (k >= K) {
    write_dead_row(o, k, dts, D <= 6);
    return;
  }
  const double* q = post + k * REC;
  // one block (split = 0) or two independent Normal-Wishart blocks (see coord_block)
  const int nb = split > 0 ? 2 : 1;
  const double alpha = q[0];
  double kap[2], nuv[2];
  int Db[2] = {split > 0 ? split : D, split > 0 ? D - split : 0};
  for (int b = 0; b < 2; ++b) {
    kap[b] = rec_kappa(q, D, b < nb ? b : 0);
    nuv[b] = rec_nu(q, D, b < nb ? b : 0);
  }
  const float lam = comp_lambda(q, D, split, ns);
  o.lam[k] = lam;
  double m[D];
  for (int i = 0; i < D; ++i) m[i] = q[3 + i];
  double L[D][D];
  load_winv<D>(q, L);
  if (!cholesky<D>(L)) {
    atomicOr(flags, FLAG_NOT_PD);
    write_dead_row(o, k, dts, D <= 6);
    o.lam[k] = 0.0f;
    return;
  }
  double lndet_b[2] = {0.0, 0.0};
  for (int i = 0; i < D; ++i) lndet_b[coord_block(i, split)] -= 2.0 * log(L[i][i]);
  // Linv = L^{-1} (lower triangular)
  double Li[D][D];
  for (int j = 0; j < D; ++j) {
    for (int i = 0; i < D; ++i) Li[i][j] = 0.0;
    Li[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < D; ++i) {
      double v = 0.0;
      for (int t = j; t < i; ++t) v += L[i][t] * Li[t][j];
      Li[i][j] = -v / L[i][i];
    }
  }
  // W = Linv^T Linv
  double W[D][D];
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b) {
      double v = 0.0;
      for (int t = b; t < D; ++t) v += Li[t][a] * Li[t][b];
      W[a][b] = W[b][a] = v;
    }
  double ElnLam_b[2] = {0.0, 0.0};
  for (int b = 0; b < nb; ++b) {
    ElnLam_b[b] = Db[b] * LN2 + lndet_b[b];
    for (int i = 1; i <= Db[b]; ++i) ElnLam_b[b] += vb_digamma(0.5 * (nuv[b] + 1.0 - i));
  }
  const double psi_sum = vb_digamma(fr->sum_alpha_q);
  const double psi_a = vb_digamma(alpha);
  const double Elnpi = psi_a - psi_sum;
  double g = Elnpi;
  for (int b = 0; b < nb; ++b) g += 0.5 * ElnLam_b[b] - 0.5 * Db[b] * LN2PI - 0.5 * Db[b] / kap[b];

  // direct-form row (raw coordinates, log2 units), built in registers and written 16 bytes at a
  // time (each thread writes a row of its own)
  double T[dts];
  T[0] = LOG2E * g;
  for (int i = 0; i < D; ++i) T[1 + i] = m[i];
  for (int i = 0; i < D; ++i) {
    const double us = sqrt(0.5 * nuv[coord_block(i, split)] * LOG2E);
    for (int j = 0; j <= i; ++j) T[1 + D + i * (i + 1) / 2 + j] = us * Li[i][j];
  }
  for (int i = 1 + D + D * (D + 1) / 2; i < dts; ++i) T[i] = 0.0;
  {
    f64x2* Tg = reinterpret_cast<f64x2*>(o.direct + k * dts);
#pragma unroll
    for (int i = 0; i < dts / 2; ++i) Tg[i] = f64x2{T[2 * i], T[2 * i + 1]};
  }

  // expanded coefficients in centred/scaled coordinates x' = (x - mu) / s (MFMA paths: D <= 6)
  if constexpr (D <= 6) {
  double ms[D], Wm[D];
  for (int i = 0; i < D; ++i) ms[i] = (m[i] - (double)fr->mu[i]) / fr->s[i];
  double mWm_b[2] = {0.0, 0.0};
  for (int a = 0; a < D; ++a) {
    double v = 0.0;
    for (int b = 0; b < D; ++b) v += W[a][b] * fr->s[a] * fr->s[b] * ms[b];
    Wm[a] = v;
    mWm_b[coord_block(a, split)] += ms[a] * v;
  }
  double c[FP];
  for (int i = 0; i < FP; ++i) c[i] = 0.0;
  double cq = 0.0;
  for (int b = 0; b < nb; ++b) cq += nuv[b] * mWm_b[b];
  c[0] = LOG2E * (g - 0.5 * cq);
  for (int a = 0; a < D; ++a) c[1 + a] = LOG2E * nuv[coord_block(a, split)] * Wm[a];
  int oo = 1 + D;
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b) {
      const double wab = W[a][b] * fr->s[a] * fr->s[b];  // zero across blocks
      c[oo++] = (a == b ? -0.5 : -1.0) * LOG2E * nuv[coord_block(a, split)] * wab;
    }
  double nn = 0.0;
  // the row's three formats, written 16 bytes at a time
  float v[FP];
  uint32_t hw[FP / 2], lw[FP / 2];
#pragma unroll
  for (int i = 0; i < FP; ++i) {
    v[i] = (float)c[i];
    nn += c[i] * c[i];
  }
#pragma unroll
  for (int i = 0; i < FP / 2; ++i) {
    const uint16_t h0 = f2bf(v[2 * i]), h1 = f2bf(v[2 * i + 1]);
    hw[i] = (uint32_t)h0 | ((uint32_t)h1 << 16);
    lw[i] = (uint32_t)f2bf(v[2 * i] - bf2f(h0)) | ((uint32_t)f2bf(v[2 * i + 1] - bf2f(h1)) << 16);
  }
  u32x4* chg = reinterpret_cast<u32x4*>(o.ch + k * FP);
  u32x4* clg = reinterpret_cast<u32x4*>(o.cl + k * FP);
  if (o.c32) {
    f32x4* c32g = reinterpret_cast<f32x4*>(o.c32 + k * FP);
#pragma unroll
    for (int i = 0; i < FP / 4; ++i) c32g[i] = f32x4{v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]};
  }
#pragma unroll
  for (int i = 0; i < FP / 8; ++i) {
    chg[i] = u32x4{hw[4 * i], hw[4 * i + 1], hw[4 * i + 2], hw[4 * i + 3]};
    clg[i] = u32x4{lw[4 * i], lw[4 * i + 1], lw[4 * i + 2], lw[4 * i + 3]};
  }
  o.nc[k] = (float)(sqrt(nn) * (1.0 + 1e-6));
  }

}


// KL(NW(q_k) || NW(p_k)) summed over the blocks, + the per-component part of KL(Dir(alpha) ||
// Dir(alpha_p)); only the ELBO needs it, so it runs apart from the coefficient rows (beside the
// sweep on the culled path). A non-positive-definite W^{-1} was flagged by k_coeffs; its KL is 0.
template <int D>
__global__ __launch_bounds__(128) void k_kl(const double* __restrict__ prior, const double* __restrict__ post,
                                            int64_t K, const FrameInfo* __restrict__ fr, double* __restrict__ kl,
                                            int* flags, int split) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double* q = post + k * REC;
  const double* p = prior + k * REC;
  const int nb = split > 0 ? 2 : 1;
  const double alpha = q[0];
  double kap[2], nuv[2];
  int Db[2] = {split > 0 ? split : D, split > 0 ? D - split : 0};
  for (int b = 0; b < 2; ++b) {
    kap[b] = rec_kappa(q, D, b < nb ? b : 0);
    nuv[b] = rec_nu(q, D, b < nb ? b : 0);
  }
  double m[D];
  for (int i = 0; i < D; ++i) m[i] = q[3 + i];
  double L[D][D];
  load_winv<D>(q, L);
  if (!cholesky<D>(L)) {
    kl[k] = 0.0;
    return;
  }
  double lndet_b[2] = {0.0, 0.0};
  for (int i = 0; i < D; ++i) lndet_b[coord_block(i, split)] -= 2.0 * log(L[i][i]);
  double Li[D][D];
  for (int j = 0; j < D; ++j) {
    for (int i = 0; i < D; ++i) Li[i][j] = 0.0;
    Li[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < D; ++i) {
      double v = 0.0;
      for (int t = j; t < i; ++t) v += L[i][t] * Li[t][j];
      Li[i][j] = -v / L[i][i];
    }
  }
  double W[D][D];
  for (int a = 0; a < D; ++a)
    for (int b = a; b < D; ++b) {
      double v = 0.0;
      for (int t = b; t < D; ++t) v += Li[t][a] * Li[t][b];
      W[a][b] = W[b][a] = v;
    }
  double ElnLam_b[2] = {0.0, 0.0};
  for (int b = 0; b < nb; ++b) {
    ElnLam_b[b] = Db[b] * LN2 + lndet_b[b];
    for (int i = 1; i <= Db[b]; ++i) ElnLam_b[b] += vb_digamma(0.5 * (nuv[b] + 1.0 - i));
  }
  const double psi_sum = vb_digamma(fr->sum_alpha_q);
  const double psi_a = vb_digamma(alpha);
  // the prior's factors, then the KL per block
  const double ap = p[0];
  double Lp[D][D];
  load_winv<D>(p, Lp);
  double Ap[D][D];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) Ap[a][b] = Lp[a][b];
  if (!cholesky<D>(Lp)) {
    atomicOr(flags, FLAG_NOT_PD);
    kl[k] = 0.0;
    return;
  }
  double lndetp_b[2] = {0.0, 0.0};
  for (int i = 0; i < D; ++i) lndetp_b[coord_block(i, split)] -= 2.0 * log(Lp[i][i]);
  double dm[D];
  for (int i = 0; i < D; ++i) dm[i] = m[i] - p[3 + i];
  double klnw = 0.0;
  for (int bb = 0; bb < nb; ++bb) {
    double quad = 0.0, tr = 0.0;
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b)
        if (coord_block(a, split) == bb && coord_block(b, split) == bb) {
          quad += dm[a] * W[a][b] * dm[b];
          tr += Ap[a][b] * W[b][a];
        }
    const double nu = nuv[bb], kappa = kap[bb], kp = rec_kappa(p, D, bb), np = rec_nu(p, D, bb);
    const int Dd = Db[bb];
    const double lnB_q = -0.5 * nu * lndet_b[bb] - 0.5 * nu * Dd * LN2 - vb_mvlgamma(0.5 * nu, Dd);
    const double lnB_p = -0.5 * np * lndetp_b[bb] - 0.5 * np * Dd * LN2 - vb_mvlgamma(0.5 * np, Dd);
    klnw += 0.5 * (kp * nu * quad + Dd * kp / kappa - Dd + Dd * log(kappa / kp)) + lnB_q - lnB_p +
            0.5 * (nu - np) * ElnLam_b[bb] - 0.5 * nu * Dd + 0.5 * nu * tr;
  }
  const double kd = -lgamma(alpha) + lgamma(ap) + (alpha - ap) * (psi_a - psi_sum);
  kl[k] = klnw + kd;
}

hipError_t launch_alpha(const DevPtrs& d, hipStream_t s) {
  double* apart = d.at<double>(d.L->mom_part);  // free again once the frame moments are final
  hipLaunchKernelGGL(k_alpha_part, dim3(ALPHA_BLOCKS), dim3(256), 0, s, d.prior(), d.post(), d.K, apart);
  hipLaunchKernelGGL(k_alpha_final, dim3(1), dim3(256), 0, s, apart, d.frame());
  return hipGetLastError();
}

hipError_t launch_coeffs(const DevPtrs& d, hipStream_t s, bool alpha, bool staged) {
  const Layout& L = *d.L;
  if (staged && L.fp8) return hipErrorInvalidValue;  // (the FP8 tier is never culled)
  if (alpha) {
    const hipError_t e = launch_alpha(d, s);
    if (e != hipSuccess) return e;
  }
  CoefOut o{d.K, d.at<float>(L.lam), d.at<double>(L.direct), d.at<float>(L.c32), d.at<uint16_t>(L.ch),
            d.at<uint16_t>(L.cl), d.at<float>(L.nc)};
  if (staged) {
    o.c32 = L.stage_c32 ? d.at<float>(L.c32u) : nullptr;
    o.ch = d.at<uint16_t>(L.chu);
    o.cl = d.at<uint16_t>(L.clu);
    o.nc = d.at<float>(L.ncu);
  }
  const dim3 grid((unsigned)((L.Kpad + 127) / 128)), blk(128);
  int* fl = &d.frame()->flags;
  switch (d.D) {
#define VB_CASE(DD) \
  case DD:          \
    hipLaunchKernelGGL(k_coeffs<DD>, grid, blk, 0, s, d.prior(), d.post(), d.K, L.Kpad, d.frame(), o, fl, d.split, d.nsp); \
    break;
    VB_CASE(1) VB_CASE(2) VB_CASE(3) VB_CASE(4) VB_CASE(5) VB_CASE(6) VB_CASE(7) VB_CASE(8)
#undef VB_CASE
    default:
      return hipErrorInvalidValue;
  }
  if (L.fp8)
    hipLaunchKernelGGL(k_fp8_rows, dim3((unsigned)((L.Kpad + 255) / 256)), dim3(256), 0, s, d.at<float>(L.c32),
                       L.Kpad, d.at<uint8_t>(L.c8), d.at<float>(L.cs8));
  return hipGetLastError();
}

// the sum of the KL terms over one contiguous range of components per workgroup (ELBO_BLOCKS
// workgroups of 256 threads, a fixed order)
constexpr int ELBO_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_kl_part(const double* __restrict__ kl, int64_t K, double* __restrict__ part) {
  __shared__ double b[256];
  const int t = threadIdx.x;
  const int64_t pk = (K + ELBO_BLOCKS - 1) / ELBO_BLOCKS, k0 = blockIdx.x * pk, k1 = min(k0 + pk, K);
  double u = 0.0;
  for (int64_t i = k0 + t; i < k1; i += 256) u += kl[i];
  b[t] = u;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) b[t] += b[t + w];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = b[0];
}

hipError_t launch_kl(const DevPtrs& d, hipStream_t s) {
  const Layout& L = *d.L;
  const dim3 grid((unsigned)((d.K + 127) / 128)), blk(128);
  switch (d.D) {
#define VB_CASE(DD) \
  case DD:          \
    hipLaunchKernelGGL(k_kl<DD>, grid, blk, 0, s, d.prior(), d.post(), d.K, d.frame(), d.at<double>(L.kl), \
                       &d.frame()->flags, d.split);                                                        \
    break;
    VB_CASE(1) VB_CASE(2) VB_CASE(3) VB_CASE(4) VB_CASE(5) VB_CASE(6) VB_CASE(7) VB_CASE(8)
#undef VB_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_kl_part, dim3(ELBO_BLOCKS), dim3(256), 0, s, d.at<double>(L.kl), d.K, d.at<double>(L.elbo_part));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// conjugate update through natural parameters (FP64, one thread per component)
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_update(double* prior, double* post, const double* __restrict__ st, int64_t K, int commit,
                         int split) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  constexpr int F = 1 + D + D * (D + 1) / 2;
  // records are REC = 48 doubles (384 bytes) apart: their loads and stores go 16 bytes at a time;
  // the prior record's doubles in use (through the second block's nu), rounded up to even
  constexpr int PU = ((rec_kc(D) + 3) & ~1) < REC ? ((rec_kc(D) + 3) & ~1) : REC;
  double p[PU + 2];
  p[PU] = p[PU + 1] = 0.0;  // (past the record: a second block's kappa and nu, which D = 8 never has)
  {
    const f64x2* pv = reinterpret_cast<const f64x2*>(prior + k * REC);
#pragma unroll
    for (int i = 0; i < PU / 2; ++i) {
      const f64x2 t = pv[i];
      p[2 * i] = t.x;
      p[2 * i + 1] = t.y;
    }
  }
  double S[F];
  if constexpr (F % 2 == 0) {
    const f64x2* sv = reinterpret_cast<const f64x2*>(st + k * F);
#pragma unroll
    for (int i = 0; i < F / 2; ++i) {
      const f64x2 t = sv[i];
      S[2 * i] = t.x;
      S[2 * i + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < F; ++i) S[i] = st[k * F + i];
  }
  const double Nk = S[0];
  double r[REC];
#pragma unroll
  for (int i = 0; i < REC; ++i) r[i] = 0.0;
  // per block: kappa = kappa_p + N, nu = nu_p + N (both blocks see the same N_k)
  double kp[2] = {1.0, 1.0}, kappa[2] = {1.0, 1.0};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (b == 1 && split == 0) break;
    kp[b] = rec_kappa(p, D, b);
    kappa[b] = kp[b] + Nk;
    r[b ? rec_kc(D) : 1] = kappa[b];
    r[b ? rec_kc(D) + 1 : 2] = rec_nu(p, D, b) + Nk;
  }
  r[0] = p[0] + Nk;
  double m[D], mp[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const int b = coord_block(i, split);
    mp[i] = p[3 + i];
    m[i] = (kp[b] * mp[i] + S[1 + i]) / kappa[b];
    r[3 + i] = m[i];
  }
  // W^{-1} + kappa m m^T is additive within a block: T3 = T3_prior + S2; zero across blocks
  constexpr int o = 1 + D;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      const int t = tri_up(i, j, D);
      const int b = coord_block(i, split);
      r[3 + D + t] = b == coord_block(j, split)
                         ? p[3 + D + t] + S[o + t] + kp[b] * mp[i] * mp[j] - kappa[b] * m[i] * m[j]
                         : 0.0;
    }
  f64x2* po = reinterpret_cast<f64x2*>(post + k * REC);
#pragma unroll
  for (int i = 0; i < REC / 2; ++i) po[i] = f64x2{r[2 * i], r[2 * i + 1]};
  if (commit) {
    f64x2* pp = reinterpret_cast<f64x2*>(prior + k * REC);
#pragma unroll
    for (int i = 0; i < REC / 2; ++i) pp[i] = f64x2{r[2 * i], r[2 * i + 1]};
  }
}

hipError_t launch_update(const DevPtrs& d, int commit, hipStream_t s) {
  const dim3 grid((unsigned)((d.K + 255) / 256));
  switch (d.D) {
#define VB_UP(DD)                                                                                          \
  case DD:                                                                                                 \
    hipLaunchKernelGGL(k_update<DD>, grid, dim3(256), 0, s, d.prior(), d.post(), d.at<double>(d.L->stats), d.K, \
                       commit, d.split);                                                                   \
    break;
    VB_UP(1) VB_UP(2) VB_UP(3) VB_UP(4) VB_UP(5) VB_UP(6) VB_UP(7) VB_UP(8)
#undef VB_UP
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ELBO: F = ln2 * sum LSE2 - [lnGamma(sum alpha) - lnGamma(sum alpha_p)] - sum_k kl_k
// ---------------------------------------------------------------------------
// In a fixed order (so the value does not depend on scheduling): the KL terms are summed in
// ELBO_BLOCKS contiguous ranges as soon as they are made (k_kl_part, with launch_kl), and one
// workgroup sums the LSE partials of the first pass and those range sums.
__global__ __launch_bounds__(256) void k_elbo(const double* __restrict__ lse_part, int64_t np,
                                              const double* __restrict__ klpart, const FrameInfo* __restrict__ fr,
                                              double* out) {
  __shared__ double a[256], b[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < np; i += 256) s += lse_part[i];
  a[t] = s;
  b[t] = klpart[t];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      a[t] += a[t + w];
      b[t] += b[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double kdir0 = lgamma(fr->sum_alpha_q) - lgamma(fr->sum_alpha_p);
    out[0] = LN2 * a[0] - kdir0 - b[0];
  }
}

hipError_t launch_elbo(const DevPtrs& d, int64_t n_lse_part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_elbo, dim3(1), dim3(256), 0, s, d.at<double>(d.L->lse_part), n_lse_part,
                     d.at<double>(d.L->elbo_part), d.frame(), out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// parameter get / set (full symmetric W^{-1} outside, upper-packed inside)
// ---------------------------------------------------------------------------
// kappa and nu hold one value per block (1 or 2 per component)
__global__ void k_get_set(double* rec, int set, int D, int64_t K, double* alpha, double* kappa, double* m,
                          double* Winv, double* nu, int split) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int nb = split > 0 ? 2 : 1;
  double* r = rec + k * REC;
  if (set) {
    r[0] = alpha[k];
    for (int b = 0; b < nb; ++b) {
      r[b ? rec_kc(D) : 1] = kappa[k * nb + b];
      r[b ? rec_kc(D) + 1 : 2] = nu[k * nb + b];
    }
    for (int i = 0; i < D; ++i) r[3 + i] = m[k * D + i];
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j)
        r[3 + D + tri_up(i, j, D)] = coord_block(i, split) == coord_block(j, split)
                                         ? 0.5 * (Winv[(k * D + i) * D + j] + Winv[(k * D + j) * D + i])
                                         : 0.0;
  } else {
    alpha[k] = r[0];
    for (int b = 0; b < nb; ++b) {
      kappa[k * nb + b] = r[b ? rec_kc(D) : 1];
      nu[k * nb + b] = r[b ? rec_kc(D) + 1 : 2];
    }
    for (int i = 0; i < D; ++i) m[k * D + i] = r[3 + i];
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j) {
        const double v = r[3 + D + tri_up(i, j, D)];
        Winv[(k * D + i) * D + j] = v;
        Winv[(k * D + j) * D + i] = v;
      }
  }
}

hipError_t launch_get_set(const DevPtrs& d, int which, int set, double* alpha, double* kappa, double* m,
                          double* Winv, double* nu, hipStream_t s) {
  double* rec = which == 0 ? d.post() : d.prior();
  hipLaunchKernelGGL(k_get_set, dim3((unsigned)((d.K + 255) / 256)), dim3(256), 0, s, rec, set, d.D, d.K, alpha,
                     kappa, m, Winv, nu, d.split);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// rendering: spatial marginal and colour regression of every component
// ---------------------------------------------------------------------------
// Coordinates [0, s) are the position, [s, D) the colour. With Sigma ~ W^-1(Psi = W^-1, nu) the
// marginal of the position block is Sigma_ss ~ W^-1(Psi_ss, nu - Dc) and mu_s | Sigma ~ N(m_s, Sigma_ss
// / kappa): a Normal-Wishart (m_s, kappa, W_s = Psi_ss^-1, nu - Dc) over s coordinates. The colour
// expected given the position and the component is m_c + B (x - m_s), B = Psi_cs Psi_ss^-1 (the mean
// of Sigma_cs Sigma_ss^-1 under the inverse Wishart). In the two-factor model the position factor is
// its own Normal-Wishart and B = 0. Writes the marginal as the record of an s-dimensional state
// (prior and posterior) and reg[k] = [m_c (Dc), B (Dc x s, row-major)].
__global__ void k_render_marginal(const double* __restrict__ post, int64_t K, int D, int split, int s,
                                  double* __restrict__ sp_prior, double* __restrict__ sp_post,
                                  double* __restrict__ reg, int* flags) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double* q = post + k * REC;
  const int Dc = D - s;
  double r[REC];
  for (int i = 0; i < REC; ++i) r[i] = 0.0;
  r[0] = q[0];
  r[1] = rec_kappa(q, D, 0);
  r[2] = split > 0 ? rec_nu(q, D, 0) : q[2] - Dc;
  for (int i = 0; i < s; ++i) r[3 + i] = q[3 + i];
  for (int i = 0; i < s; ++i)
    for (int j = i; j < s; ++j) r[3 + s + tri_up(i, j, s)] = q[3 + D + tri_up(i, j, D)];
  // Cholesky of Psi_ss (lower, row-major s x s)
  double Lc[MAXD * MAXD];
  bool pd = true;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = q[3 + D + tri_up(j, i, D)];
      for (int t = 0; t < j; ++t) v -= Lc[i * MAXD + t] * Lc[j * MAXD + t];
      if (i == j) {
        pd = pd && v > 0.0;
        Lc[i * MAXD + i] = v > 0.0 ? sqrt(v) : 1.0;
      } else {
        Lc[i * MAXD + j] = v / Lc[j * MAXD + j];
      }
    }
  if (!pd) atomicOr(flags, FLAG_NOT_PD);
  double* o = reg + k * (int64_t)(Dc * (1 + s));
  for (int c = 0; c < Dc; ++c) {
    o[c] = q[3 + s + c];
    // row c of B: Psi_ss b = Psi_s,c (forward then back substitution)
    double y[MAXD];
    for (int i = 0; i < s; ++i) {
      double v = split > 0 ? 0.0 : q[3 + D + tri_up(i, s + c, D)];
      for (int t = 0; t < i; ++t) v -= Lc[i * MAXD + t] * y[t];
      y[i] = v / Lc[i * MAXD + i];
    }
    for (int i = s - 1; i >= 0; --i) {
      double v = y[i];
      for (int t = i + 1; t < s; ++t) v -= Lc[t * MAXD + i] * y[t];
      y[i] = v / Lc[i * MAXD + i];
    }
    for (int j = 0; j < s; ++j) o[Dc + c * s + j] = pd ? y[j] : 0.0;
  }
  for (int i = 0; i < REC; ++i) {
    sp_prior[k * REC + i] = r[i];
    sp_post[k * REC + i] = r[i];
  }
}

hipError_t launch_render_marginal(const DevPtrs& model, const DevPtrs& sp, double* reg, hipStream_t s) {
  hipLaunchKernelGGL(k_render_marginal, dim3((unsigned)((model.K + 127) / 128)), dim3(128), 0, s, model.post(),
                     model.K, model.D, model.split, sp.D, sp.prior(), sp.post(), reg, &sp.frame()->flags);
  return hipGetLastError();
}

// mean squared error of two images in [0, 1] on the 0..255 scale (values clamped to [0, 1]) and
// the PSNR 10 log10(255^2 / MSE) of Sec. 5.1; one workgroup: each thread sums a fixed set of
// values in a fixed order, then a fixed tree (deterministic)
__global__ __launch_bounds__(1024) void k_psnr(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                               double* __restrict__ out) {
  __shared__ double red[1024];
  auto sq = [](float x, float y) {
    const double d = 255.0 * ((double)fminf(fmaxf(x, 0.0f), 1.0f) - (double)fminf(fmaxf(y, 0.0f), 1.0f));
    return d * d;
  };
  double acc = 0.0;
  int64_t i0 = 0;  // values before i0 are taken four at a time (16-byte loads, eight in flight)
  if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0) {
    const float4* a4 = reinterpret_cast<const float4*>(a);
    const float4* b4 = reinterpret_cast<const float4*>(b);
    const int64_t n4 = n / 4;
    int64_t j = threadIdx.x;
    for (; j + 3 * 1024 < n4; j += 4 * 1024) {
      float4 x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = a4[j + u * 1024];
        y[u] = b4[j + u * 1024];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += sq(x[u].x, y[u].x) + sq(x[u].y, y[u].y) + sq(x[u].z, y[u].z) + sq(x[u].w, y[u].w);
    }
    for (; j < n4; j += 1024) {
      const float4 x = a4[j], y = b4[j];
      acc += sq(x.x, y.x) + sq(x.y, y.y) + sq(x.z, y.z) + sq(x.w, y.w);
    }
    i0 = 4 * n4;
  }
  for (int64_t i = i0 + threadIdx.x; i < n; i += 1024) acc += sq(a[i], b[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mse = n > 0 ? red[0] / (double)n : 0.0;
    out[0] = mse;
    out[1] = mse > 0.0 ? 10.0 * log10(255.0 * 255.0 / mse) : INFINITY;
  }
}

hipError_t launch_psnr(const float* a, const float* b, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_psnr, dim3(1), dim3(1024), 0, s, a, b, n, out);
  return hipGetLastError();
}

__global__ void k_clear_flags(FrameInfo* fr) {
  fr->flags = 0;
  fr->refined1 = 0;
  fr->refined2 = 0;
  fr->blocks = 0;
  fr->blocks_cum = 0;
}

hipError_t launch_clear_flags(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(1), 0, s, d.frame());
  return hipGetLastError();
}

__global__ void k_merge_flags(const FrameInfo* src, FrameInfo* dst) { dst->flags |= src->flags; }

hipError_t launch_merge_flags(const FrameInfo* src, FrameInfo* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_flags, dim3(1), dim3(1), 0, s, src, dst);
  return hipGetLastError();
}

}  // namespace vbgs
