/*
 * Oracle core: plain, slow, FP64 CPU implementation of the per-pair work of the
 * variational-Bayes Gaussian-mixture E-step and its sufficient statistics.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code with
 * the HIP library (no headers, no helpers, no tables).
 *
 * What it computes (mixture model of Sec. 2.1.2, Fig. 2; per-frame fit of
 * Alg. 1; the weighted reduction Delta S = R^T S_u of Eq. (fused_contr)):
 *
 *   rho[n,k] = g[k] - 0.5 * nu[k] * || Linv_k (x_n - m_k) ||^2
 *
 * where L_k is the lower Cholesky factor of W_k^{-1}, so that
 * (x-m)^T W_k (x-m) = || L_k^{-1} (x-m) ||^2 (forward substitution), and g[k]
 * already holds E[ln pi_k] + 0.5 E[ln|Lambda_k|] - (D/2) ln(2 pi) - D/(2 kappa_k).
 * The score is evaluated directly in this non-expanded form, never as a dot
 * product of quadratic features.
 *
 *   LSE[n]  = ln sum_k exp(rho[n,k])              (max-shifted)
 *   r[n,k]  = exp(rho[n,k] - LSE[n])
 *   Nk[k]   = sum_n r[n,k]
 *   S1[k]   = sum_n r[n,k] x_n
 *   S2[k]   = sum_n r[n,k] x_n x_n^T             (raw coordinates, full D x D)
 *   scat[k] = sum_n r[n,k] (x_n - xbar_k)(x_n - xbar_k)^T,  xbar_k = S1[k] / Nk[k]
 *
 * Sums over n run in point order. Parallelism (OpenMP) is over points for LSE
 * and over components for the statistics, so every output element is summed
 * in the same fixed order regardless of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* forward substitution: y = L^{-1} v for lower-triangular L (row-major D x D) */
static double mahal(int D, const double *L, const double *x, const double *m) {
  double y[16];
  double q = 0.0;
  for (int i = 0; i < D; ++i) {
    double s = x[i] - m[i];
    for (int j = 0; j < i; ++j) s -= L[i * D + j] * y[j];
    y[i] = s / L[i * D + i];
    q += y[i] * y[i];
  }
  return q;
}

static double score(int D, const double *x, int64_t k, const double *m, const double *L,
                    const double *g, const double *nu) {
  return g[k] - 0.5 * nu[k] * mahal(D, L + k * D * D, x, m + k * D);
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* LSE[n] for n in [0, N). */
void oracle_lse(int64_t N, int64_t K, int D, const double *X, const double *m, const double *L,
                const double *g, const double *nu, double *lse) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t n = 0; n < N; ++n) {
    const double *x = X + n * D;
    double mx = -INFINITY;
    for (int64_t k = 0; k < K; ++k) {
      double s = score(D, x, k, m, L, g, nu);
      if (s > mx) mx = s;
    }
    double acc = 0.0;
    for (int64_t k = 0; k < K; ++k) acc += exp(score(D, x, k, m, L, g, nu) - mx);
    lse[n] = mx + log(acc);
  }
}

/* Responsibilities of a dense N x K block (small problems only). */
void oracle_resp(int64_t N, int64_t K, int D, const double *X, const double *m, const double *L,
                 const double *g, const double *nu, const double *lse, double *R) {
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int64_t k = 0; k < K; ++k)
      R[n * K + k] = exp(score(D, X + n * D, k, m, L, g, nu) - lse[n]);
}

/* Statistics for components [k0, k1) given LSE of all N points.
 * Nk: (k1-k0); S1: (k1-k0) x D; S2, scat: (k1-k0) x D x D. scat may be NULL. */
void oracle_stats(int64_t N, int64_t k0, int64_t k1, int D, const double *X, const double *m,
                  const double *L, const double *g, const double *nu, const double *lse,
                  double *Nk, double *S1, double *S2, double *scat) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = k0; k < k1; ++k) {
    int64_t o = k - k0;
    double n0 = 0.0, s1[16], s2[256];
    memset(s1, 0, sizeof(s1));
    memset(s2, 0, sizeof(s2));
    for (int64_t n = 0; n < N; ++n) {
      const double *x = X + n * D;
      double r = exp(score(D, x, k, m, L, g, nu) - lse[n]);
      n0 += r;
      for (int i = 0; i < D; ++i) {
        s1[i] += r * x[i];
        for (int j = 0; j < D; ++j) s2[i * D + j] += r * x[i] * x[j];
      }
    }
    Nk[o] = n0;
    for (int i = 0; i < D; ++i) S1[o * D + i] = s1[i];
    for (int i = 0; i < D * D; ++i) S2[o * D * D + i] = s2[i];
    if (scat) {
      double xb[16], sc[256];
      memset(sc, 0, sizeof(sc));
      for (int i = 0; i < D; ++i) xb[i] = n0 > 0.0 ? s1[i] / n0 : 0.0;
      if (n0 > 0.0) {
        for (int64_t n = 0; n < N; ++n) {
          const double *x = X + n * D;
          double r = exp(score(D, x, k, m, L, g, nu) - lse[n]);
          for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) sc[i * D + j] += r * (x[i] - xb[i]) * (x[j] - xb[j]);
        }
      }
      for (int i = 0; i < D * D; ++i) scat[o * D * D + i] = sc[i];
    }
  }
}

/* Scores of listed (point, component) pairs: out[i] = rho[pn[i], pk[i]]. */
void oracle_pair_scores(int64_t P, int D, const double *X, const int64_t *pn, const int64_t *pk,
                        const double *m, const double *L, const double *g, const double *nu,
                        double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < P; ++i) out[i] = score(D, X + pn[i] * D, pk[i], m, L, g, nu);
}
