// E-step + sufficient statistics on MFMA (gfx950).
//
// The quadratic form of the score is expanded, s_nk = c_k . phi(x_n) with quadratic point
// features phi = [1, x', upper(x' x'^T)] (x' centred and scaled per frame) and one
// coefficient row c_k per component, so scoring a tile is a GEMM on the matrix cores.
//
// pass 1 (point-tile parallel): stream LDS-staged tiles of coefficient rows past a register-
//   resident block of points; keep an online log-sum-exp per point -> LSE_n.
// pass 2 (component-tile parallel): stream LDS-staged tiles of points past a register-
//   resident block of components; recompute the scores, r = exp(s - LSE), and contract
//   r^T phi on the matrix cores (the fused Delta S = R^T S_u of Eq. (fused_contr)); FP32
//   accumulation per 64-point tile, folded into FP64 registers.
// The N x K responsibility matrix is never stored.
//
// exact = 1: the low-precision GEMM is a *screen*. Its error is bounded by
//   |s~ - s| <= eps_prec * ||c_k|| * ||phi_n||  (rounding of features, coefficients,
//   products and accumulation; Cauchy-Schwarz on sum_f |c_f phi_f|).
// A pair is rescored exactly (FP64, direct form) unless its upper bound lies more than the
// margin T below the point's running lower bound on max_k s (pass 1) or its LSE (pass 2);
// every skipped pair carries < 2^-T of the point's mass.
//
// MFMA operand layouts used (64 lanes, lane = 16 g + c, g = lane / 16, c = lane % 16):
//   v_mfma_f32_16x16x4_f32 : lane supplies A[c][g], B[g][c]; result lane holds D[4g + i][c].
//   v_mfma_f32_16x16x32_bf16: lane supplies A[c][8g .. 8g+7], B[8g .. 8g+7][c]; same result.
// Contraction slot 8g + j is the same feature index for both operands (j = MFMA step for FP32),
// so every lane loads 8 contiguous slots of one row.
#include "vbgs_internal.h"

namespace vbgs {

// screening bound factors (relative to ||c|| ||phi||), with a safety margin of >= 4x over the
// worst-case rounding analysis of each precision
__host__ __device__ constexpr float screen_eps(int prec) {
  return prec == VBGS_FP32 ? 1.52587890625e-05f     /* 2^-16 */
         : prec == VBGS_BF16 ? 1.5625e-02f          /* 2^-6  */
                             : 2.44140625e-04f;     /* 2^-12, split bf16 */
}

template <int P>
struct Opnd;
template <>
struct Opnd<VBGS_FP32> {
  f32x4 a, b;
};
template <>
struct Opnd<VBGS_BF16> {
  bf16x8 h;
};
template <>
struct Opnd<VBGS_BF16X3> {
  bf16x8 h, l;
};

template <int P>
__device__ __forceinline__ Opnd<P> load_op(const float* f32row, const uint16_t* hrow, const uint16_t* lrow,
                                           int g) {
  Opnd<P> o;
  if constexpr (P == VBGS_FP32) {
    o.a = *reinterpret_cast<const f32x4*>(f32row + 8 * g);
    o.b = *reinterpret_cast<const f32x4*>(f32row + 8 * g + 4);
  } else if constexpr (P == VBGS_BF16) {
    o.h = *reinterpret_cast<const bf16x8*>(hrow + 8 * g);
  } else {
    o.h = *reinterpret_cast<const bf16x8*>(hrow + 8 * g);
    o.l = *reinterpret_cast<const bf16x8*>(lrow + 8 * g);
  }
  return o;
}

template <int P>
__device__ __forceinline__ Opnd<P> zero_op() {
  Opnd<P> o;
  if constexpr (P == VBGS_FP32) {
    o.a = f32x4{0.f, 0.f, 0.f, 0.f};
    o.b = o.a;
  } else {
    for (int i = 0; i < 8; ++i) o.h[i] = (__bf16)0.0f;
    if constexpr (P == VBGS_BF16X3) o.l = o.h;
  }
  return o;
}

// 16 x 16 tile of scores: D[m][n] = sum_slots A_row(m) . B_row(n)
template <int P>
__device__ __forceinline__ f32x4 mfma_scores(const Opnd<P>& A, const Opnd<P>& B) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (P == VBGS_FP32) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[0], B.a[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[1], B.a[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[2], B.a[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[3], B.a[3], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[0], B.b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[1], B.b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[2], B.b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.b[3], B.b[3], acc, 0, 0, 0);
  } else if constexpr (P == VBGS_BF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, B.h, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, B.l, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l, B.h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, B.h, acc, 0, 0, 0);
  }
  return acc;
}

struct EArgs {
  const float* X;             // raw points N x D (FP32)
  const float* phi32;         // N x 32
  const uint16_t* phih;       // N x 32
  const uint16_t* phil;       // N x 32
  const float* nphi;          // N
  const double* direct;       // Kpad x dts
  const float* c32;           // Kpad x 32
  const uint16_t* ch;         // Kpad x 32
  const uint16_t* cl;         // Kpad x 32
  const float* nc;            // Kpad
  double* lse2;               // N (log2 units)
  double* lse_part;           // pass-1 workgroups
  double* lse_out;            // N (nats) or null
  double* spart;              // nsplit x Kpad x 32
  FrameInfo* frame;
  int64_t N, K, Kpad;
  int D, dts, nsplit;
  float T2, eps;
};

// online log-sum-exp (log2 units) of exactly rescored pairs, FP64
__device__ __forceinline__ void online_add(double& m, double& l, double s) {
  if (s > m) {
    l = l * exp2(m - s) + 1.0;
    m = s;
  } else {
    l += exp2(s - m);
  }
}

__device__ __forceinline__ void lse_merge(double& m, double& l, double om, double ol) {
  const double mn = fmax(m, om);
  if (mn == -INFINITY) return;
  const double a = (m == -INFINITY) ? 0.0 : l * exp2(m - mn);
  const double b = (om == -INFINITY) ? 0.0 : ol * exp2(om - mn);
  m = mn;
  l = a + b;
}

__device__ __forceinline__ void count_refined(unsigned long long* ctr, unsigned v) {
  // wave-level sum then one integer atomic per wave
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, (unsigned long long)v);
}

// ---------------------------------------------------------------------------
// pass 1: point-tile parallel online LSE
// ---------------------------------------------------------------------------
template <int P>
struct __attribute__((aligned(16))) CTile {
  float c32[P == VBGS_FP32 ? CT : 1][FP];
  uint16_t h[P == VBGS_FP32 ? 1 : CT][FP];
  uint16_t l[P == VBGS_BF16X3 ? CT : 1][FP];
  float nc[CT];
};

template <int P>
__device__ __forceinline__ void load_ctile(CTile<P>& T, const EArgs& a, int64_t k0) {
  const int t = threadIdx.x;  // 256 threads, 16 B each per sweep
  if constexpr (P == VBGS_FP32) {
    const uint4* src = reinterpret_cast<const uint4*>(a.c32 + k0 * FP);
    uint4* dst = reinterpret_cast<uint4*>(&T.c32[0][0]);
    dst[t] = src[t];
    dst[t + 256] = src[t + 256];
  } else {
    reinterpret_cast<uint4*>(&T.h[0][0])[t] = reinterpret_cast<const uint4*>(a.ch + k0 * FP)[t];
    if constexpr (P == VBGS_BF16X3)
      reinterpret_cast<uint4*>(&T.l[0][0])[t] = reinterpret_cast<const uint4*>(a.cl + k0 * FP)[t];
  }
  if (t < CT / 4) reinterpret_cast<uint4*>(T.nc)[t] = reinterpret_cast<const uint4*>(a.nc + k0)[t];
}

template <int P, bool EXACT>
__global__ __launch_bounds__(256) void k_pass1(const EArgs a) {
  __shared__ CTile<P> T;
  __shared__ double red[256];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * P1_PTS + w * (P1_PB * 16);

  Opnd<P> B[P1_PB];
  float nph[P1_PB], M[P1_PB], ls[P1_PB];
  double mref[P1_PB], lsd[P1_PB];
  bool val[P1_PB];
#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < a.N;
    if (val[b]) {
      B[b] = load_op<P>(a.phi32 + p * FP, a.phih + p * FP, a.phil + p * FP, g);
      nph[b] = a.nphi[p];
    } else {
      B[b] = zero_op<P>();
      nph[b] = 0.0f;
    }
    M[b] = -INFINITY;
    ls[b] = 0.0f;
    mref[b] = -INFINITY;
    lsd[b] = 0.0;
  }
  unsigned nref = 0;

  for (int64_t k0 = 0; k0 < a.Kpad; k0 += CT) {
    __syncthreads();
    load_ctile<P>(T, a, k0);
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const int r = cb * 16 + c;
      const Opnd<P> A = load_op<P>(&T.c32[P == VBGS_FP32 ? r : 0][0], &T.h[P == VBGS_FP32 ? 0 : r][0],
                                   &T.l[P == VBGS_BF16X3 ? r : 0][0], g);
      const f32x4 nc4 = *reinterpret_cast<const f32x4*>(&T.nc[cb * 16 + 4 * g]);
      const int64_t kb = k0 + cb * 16 + 4 * g;
#pragma unroll
      for (int b = 0; b < P1_PB; ++b) {
        const f32x4 s = mfma_scores<P>(A, B[b]);
        if constexpr (EXACT) {
          const float en = a.eps * nph[b];
          const float e0 = en * nc4[0], e1 = en * nc4[1], e2 = en * nc4[2], e3 = en * nc4[3];
          const float lo = fmaxf(fmaxf(s[0] - e0, s[1] - e1), fmaxf(s[2] - e2, s[3] - e3));
          M[b] = fmaxf(M[b], lo);
          const float thr = M[b] - a.T2;
          int need = (s[0] + e0 >= thr ? 1 : 0) | (s[1] + e1 >= thr ? 2 : 0) | (s[2] + e2 >= thr ? 4 : 0) |
                     (s[3] + e3 >= thr ? 8 : 0);
          if (!val[b]) need = 0;
          if (__builtin_amdgcn_ballot_w64(need != 0)) {
            if (need) {
              const int64_t p = p0 + 16 * b + c;
              const float* x = a.X + p * a.D;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int64_t k = kb + i;
                if (((need >> i) & 1) && k < a.K) {
                  online_add(mref[b], lsd[b], direct_score2(a.direct + k * a.dts, x, a.D));
                  ++nref;
                }
              }
            }
          }
        } else {
          const float mx = fmaxf(fmaxf(s[0], s[1]), fmaxf(s[2], s[3]));
          if (mx > M[b]) {
            ls[b] *= exp2f(M[b] - mx);
            M[b] = mx;
          }
          ls[b] += exp2f(s[0] - M[b]) + exp2f(s[1] - M[b]) + exp2f(s[2] - M[b]) + exp2f(s[3] - M[b]);
        }
      }
    }
    if constexpr (EXACT) {
#pragma unroll
      for (int b = 0; b < P1_PB; ++b) {
        M[b] = fmaxf(M[b], __shfl_xor(M[b], 16));
        M[b] = fmaxf(M[b], __shfl_xor(M[b], 32));
      }
    }
  }

#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    double m = EXACT ? mref[b] : (double)M[b];
    double l = EXACT ? lsd[b] : (double)ls[b];
    for (int off = 16; off <= 32; off <<= 1) {
      const double om = __shfl_xor(m, off);
      const double ol = __shfl_xor(l, off);
      lse_merge(m, l, om, ol);
    }
    const double L2 = m + log2(l);
    const int64_t p = p0 + 16 * b + c;
    if (g == 0) {
      red[w * 64 + b * 16 + c] = val[b] ? L2 : 0.0;
      if (val[b]) {
        a.lse2[p] = L2;
        if (a.lse_out) a.lse_out[p] = L2 * LN2;
      }
    }
  }
  if constexpr (EXACT) count_refined(&a.frame->refined1, nref);
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += red[i];
    a.lse_part[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// pass 2: component-tile parallel recompute + r^T phi on MFMA
// ---------------------------------------------------------------------------
template <int P, bool EXACT>
struct __attribute__((aligned(16))) PTile {
  float f32[(P == VBGS_FP32 || !EXACT) ? PT : 1][FP];
  uint16_t h[P == VBGS_FP32 ? 1 : PT][FP];
  uint16_t l[P == VBGS_BF16X3 ? PT : 1][FP];
  float nph[PT];
  double lse[PT];
};

template <int P, bool EXACT>
__device__ __forceinline__ void load_ptile(PTile<P, EXACT>& T, const EArgs& a, int64_t n0) {
  const int t = threadIdx.x;
  const int64_t nvalid = a.N - n0;  // > 0
  if constexpr (P == VBGS_FP32 || !EXACT) {
    // 64 rows x 128 B = 512 x 16 B
    for (int q = t; q < PT * FP / 4; q += 256) {
      const int row = q / (FP / 4);
      uint4 v = {0, 0, 0, 0};
      if (row < nvalid) v = reinterpret_cast<const uint4*>(a.phi32 + n0 * FP)[q];
      reinterpret_cast<uint4*>(&T.f32[0][0])[q] = v;
    }
  }
  if constexpr (P != VBGS_FP32) {
    const int row = t / (FP / 8);  // 64 rows x 64 B = 256 x 16 B
    uint4 v = {0, 0, 0, 0};
    if (row < nvalid) v = reinterpret_cast<const uint4*>(a.phih + n0 * FP)[t];
    reinterpret_cast<uint4*>(&T.h[0][0])[t] = v;
    if constexpr (P == VBGS_BF16X3) {
      uint4 u = {0, 0, 0, 0};
      if (row < nvalid) u = reinterpret_cast<const uint4*>(a.phil + n0 * FP)[t];
      reinterpret_cast<uint4*>(&T.l[0][0])[t] = u;
    }
  }
  if (t < PT) {
    const bool v = t < nvalid;
    T.nph[t] = v ? a.nphi[n0 + t] : 0.0f;
    T.lse[t] = v ? a.lse2[n0 + t] : INFINITY;
  }
}

template <int P, bool EXACT, int DT>  // DT: compile-time D for the exact variant (0 for the plain tiers)
__global__ __launch_bounds__(256) void k_pass2(const EArgs a) {
  __shared__ PTile<P, EXACT> T;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t kb = (int64_t)blockIdx.x * CT + w * 16;
  const int64_t kc = kb + c;
  const bool kval = kc < a.K;
  const Opnd<P> Bc = load_op<P>(a.c32 + kc * FP, a.ch + kc * FP, a.cl + kc * FP, g);
  const float ncv = a.nc[kc];
  const double* drow = a.direct + kc * a.dts;
  const int64_t ntile = (a.N + PT - 1) / PT;
  const int64_t t0 = ntile * blockIdx.y / a.nsplit, t1 = ntile * (blockIdx.y + 1) / a.nsplit;
  // plain tiers: FP64 fold of the MFMA r^T phi tiles (lane: comps kb + 4g + j, slots c, 16 + c);
  // exact tier: FP64 sums of the rescored pairs of component kc, centred at its mean m_kc
  constexpr int NACC = EXACT ? 1 + DT + DT * (DT + 1) / 2 : 8;
  double acc[NACC];
#pragma unroll
  for (int j = 0; j < NACC; ++j) acc[j] = 0.0;
  unsigned nref = 0;

  for (int64_t t = t0; t < t1; ++t) {
    const int64_t n0 = t * PT;
    __syncthreads();
    load_ptile<P, EXACT>(T, a, n0);
    __syncthreads();
    f32x4 sa = {0.f, 0.f, 0.f, 0.f}, sb = sa;
    bool used = false;
#pragma unroll
    for (int pb = 0; pb < PT / 16; ++pb) {
      const int r = pb * 16 + c;
      const Opnd<P> A = load_op<P>(&T.f32[(P == VBGS_FP32 || !EXACT) ? r : 0][0], &T.h[P == VBGS_FP32 ? 0 : r][0],
                                   &T.l[P == VBGS_BF16X3 ? r : 0][0], g);
      const f32x4 s = mfma_scores<P>(A, Bc);  // lane: points pb*16 + 4g + i, component kc
      const int rb = pb * 16 + 4 * g;
      float rr[4];
      if constexpr (EXACT) {
        const float en = a.eps * ncv;
        int need = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float thr = (float)(T.lse[rb + i] - (double)a.T2);
          if (kval && s[i] + en * T.nph[rb + i] >= thr) need |= 1 << i;
        }
        if (__builtin_amdgcn_ballot_w64(need != 0) != 0 && need) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if ((need >> i) & 1) {
              const int64_t p = n0 + rb + i;
              double dv[DT > 0 ? DT : 1];
              const double s2 = direct_score2_dt<DT>(drow, a.X + p * DT, dv);
              const double rv = exp2(s2 - T.lse[rb + i]);
              acc[0] += rv;
              int o = 1 + DT;
#pragma unroll
              for (int u = 0; u < DT; ++u) {
                const double rd = rv * dv[u];
                acc[1 + u] += rd;
#pragma unroll
                for (int v = u; v < DT; ++v) acc[o++] += rd * dv[v];
              }
              ++nref;
            }
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) rr[i] = kval ? exp2f(s[i] - (float)T.lse[rb + i]) : 0.0f;
        used = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float fa = T.f32[rb + i][c];
          const float fb = T.f32[rb + i][16 + c];
          sa = __builtin_amdgcn_mfma_f32_16x16x4f32(rr[i], fa, sa, 0, 0, 0);
          sb = __builtin_amdgcn_mfma_f32_16x16x4f32(rr[i], fb, sb, 0, 0, 0);
        }
      }
    }
    if constexpr (!EXACT) {
      if (used) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[j] += (double)sa[j];
          acc[4 + j] += (double)sb[j];
        }
      }
    }
  }
  if constexpr (EXACT) {
    // the four lane groups hold partial sums of the same component: combine (commutative pairs,
    // so every lane ends with bitwise the same total)
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
      acc[j] += __shfl_xor(acc[j], 16);
      acc[j] += __shfl_xor(acc[j], 32);
    }
    if (g == 0) {
      double* out = a.spart + ((int64_t)blockIdx.y * a.Kpad + kc) * FP;
#pragma unroll
      for (int j = 0; j < 1 + DT + DT * (DT + 1) / 2; ++j) out[j] = acc[j];
    }
    count_refined(&a.frame->refined2, nref);
  } else {
    // lane holds components kb + 4g + j at slots c and 16 + c
    double* out = a.spart + ((int64_t)blockIdx.y * a.Kpad + kb) * FP;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      out[(4 * g + j) * FP + c] = acc[j];
      out[(4 * g + j) * FP + 16 + c] = acc[4 + j];
    }
  }
}

// ---------------------------------------------------------------------------
// plain FP64 direct-form path (no GEMM): the comparator the mixed path is measured against
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_pass1_direct(const EArgs a) {
  constexpr int dts = D <= 6 ? 32 : 48;
  __shared__ double Tt[CT * dts];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * 256 + tid;
  const bool val = p < a.N;
  double x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = val ? (double)a.X[p * D + i] : 0.0;
  double m = -INFINITY, l = 0.0;
  for (int64_t k0 = 0; k0 < a.Kpad; k0 += CT) {
    __syncthreads();
    for (int q = tid; q < CT * dts; q += 256) Tt[q] = a.direct[k0 * dts + q];
    __syncthreads();
    const int kend = (int)min((int64_t)CT, a.K - k0);
    for (int kk = 0; kk < kend; ++kk) {
      const double s = direct_score2_t<D>(Tt + kk * dts, x);
      if (s > m) {
        l = l * exp2(m - s) + 1.0;
        m = s;
      } else {
        l += exp2(s - m);
      }
    }
  }
  const double L2 = m + log2(l);
  red[tid] = val ? L2 : 0.0;
  if (val) {
    a.lse2[p] = L2;
    if (a.lse_out) a.lse_out[p] = L2 * LN2;
  }
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += red[i];
    a.lse_part[blockIdx.x] = s;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_pass2_direct(const EArgs a) {
  constexpr int dts = D <= 6 ? 32 : 48;
  constexpr int F = 1 + D + D * (D + 1) / 2;
  __shared__ double xs[256][D + 1];
  const int tid = threadIdx.x;
  const int64_t k = (int64_t)blockIdx.x * 256 + tid;
  const bool kval = k < a.K;
  double Tk[1 + D + D * (D + 1) / 2];
#pragma unroll
  for (int i = 0; i < 1 + D + D * (D + 1) / 2; ++i) Tk[i] = kval ? a.direct[k * dts + i] : 0.0;
  if (!kval) Tk[0] = -1.0e300;
  double acc[F];
#pragma unroll
  for (int i = 0; i < F; ++i) acc[i] = 0.0;
  const int64_t nblk = (a.N + 255) / 256;
  const int64_t b0 = nblk * blockIdx.y / a.nsplit, b1 = nblk * (blockIdx.y + 1) / a.nsplit;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t n0 = b * 256;
    __syncthreads();
    {
      const int64_t p = n0 + tid;
      const bool v = p < a.N;
#pragma unroll
      for (int i = 0; i < D; ++i) xs[tid][i] = v ? (double)a.X[p * D + i] : 0.0;
      xs[tid][D] = v ? a.lse2[p] : INFINITY;
    }
    __syncthreads();
    const int nn = (int)min((int64_t)256, a.N - n0);
    for (int j = 0; j < nn; ++j) {
      const double r = exp2(direct_score2_t<D>(Tk, &xs[j][0]) - xs[j][D]);
      acc[0] += r;
      int o = 1 + D;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const double rx = r * xs[j][i];
        acc[1 + i] += rx;
#pragma unroll
        for (int jj = i; jj < D; ++jj) acc[o++] += rx * xs[j][jj];
      }
    }
  }
  if (kval) {
    double* out = a.spart + ((int64_t)blockIdx.y * a.Kpad + k) * (D <= 6 ? 32 : 48);
#pragma unroll
    for (int i = 0; i < F; ++i) out[i] = acc[i];
  }
}

// ---------------------------------------------------------------------------
// fold: fixed-order sum over splits, un-centre to raw coordinates
// ---------------------------------------------------------------------------
__global__ void k_fold(const double* __restrict__ spart, int nsplit, int64_t Kpad, int64_t K, int D,
                       const FrameInfo* __restrict__ fr, const double* __restrict__ direct, int dts, int mode,
                       double* __restrict__ stats, double* __restrict__ stats_out) {
  // mode 0: partials are raw; 1: centred/scaled frame coordinates x' = (x - mu) / s;
  // 2: raw coordinates centred at the component's own mean m_k
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int F = nfeat(D), SS = stat_stride(D);
  double v[48];
  for (int i = 0; i < F; ++i) {
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += spart[((int64_t)q * Kpad + k) * SS + i];
    v[i] = s;
  }
  double o[48];
  if (mode == 0) {
    for (int i = 0; i < F; ++i) o[i] = v[i];
  } else {
    // x = mu + s x':  S1 = mu N + s S1',  S2_ij = mu_i mu_j N + mu_i s_j S1'_j + s_i mu_j S1'_i + s_i s_j S2'_ij
    double mu[MAXD], sc[MAXD];
    for (int i = 0; i < D; ++i) {
      mu[i] = mode == 1 ? (double)fr->mu[i] : direct[k * dts + 1 + i];
      sc[i] = mode == 1 ? fr->s[i] : 1.0;
    }
    const double Nk = v[0];
    o[0] = Nk;
    for (int i = 0; i < D; ++i) o[1 + i] = mu[i] * Nk + sc[i] * v[1 + i];
    int t = 1 + D;
    for (int i = 0; i < D; ++i)
      for (int j = i; j < D; ++j, ++t)
        o[t] = mu[i] * mu[j] * Nk + mu[i] * sc[j] * v[1 + j] + sc[i] * mu[j] * v[1 + i] + sc[i] * sc[j] * v[t];
  }
  for (int i = 0; i < F; ++i) {
    stats[k * F + i] = o[i];
    if (stats_out) stats_out[k * F + i] = o[i];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static EArgs make_args(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out) {
  const Layout& L = *d.L;
  EArgs a;
  a.X = X;
  a.phi32 = d.at<float>(L.phi32);
  a.phih = d.at<uint16_t>(L.phih);
  a.phil = d.at<uint16_t>(L.phil);
  a.nphi = d.at<float>(L.nphi);
  a.direct = d.at<double>(L.direct);
  a.c32 = d.at<float>(L.c32);
  a.ch = d.at<uint16_t>(L.ch);
  a.cl = d.at<uint16_t>(L.cl);
  a.nc = d.at<float>(L.nc);
  a.lse2 = d.at<double>(L.lse2);
  a.lse_part = d.at<double>(L.lse_part);
  a.lse_out = lse_out;
  a.spart = d.at<double>(L.spart);
  a.frame = d.frame();
  a.N = N;
  a.K = d.K;
  a.Kpad = L.Kpad;
  a.D = d.D;
  a.dts = direct_stride(d.D);
  a.nsplit = c.nsplit;
  a.T2 = c.T2;
  a.eps = screen_eps(c.prec);
  return a;
}

hipError_t launch_pass1(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out,
                        hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const EArgs a = make_args(d, c, X, N, lse_out);
  if (c.prec == VBGS_FP64) {
    const dim3 grid((unsigned)((N + 255) / 256));
    switch (d.D) {
#define VB_CASE(DD) \
  case DD:          \
    hipLaunchKernelGGL(k_pass1_direct<DD>, grid, dim3(256), 0, s, a); break;
      VB_CASE(1) VB_CASE(2) VB_CASE(3) VB_CASE(4) VB_CASE(5) VB_CASE(6) VB_CASE(7) VB_CASE(8)
#undef VB_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((N + P1_PTS - 1) / P1_PTS));
#define VB_P1(PP, EE) hipLaunchKernelGGL((k_pass1<PP, EE>), grid, dim3(256), 0, s, a)
  if (c.prec == VBGS_FP32) {
    if (c.exact) VB_P1(VBGS_FP32, true); else VB_P1(VBGS_FP32, false);
  } else if (c.prec == VBGS_BF16) {
    if (c.exact) VB_P1(VBGS_BF16, true); else VB_P1(VBGS_BF16, false);
  } else {
    if (c.exact) VB_P1(VBGS_BF16X3, true); else VB_P1(VBGS_BF16X3, false);
  }
#undef VB_P1
  return hipGetLastError();
}

hipError_t launch_pass2(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, hipStream_t s) {
  const EArgs a = make_args(d, c, X, N, nullptr);
  if (c.prec == VBGS_FP64) {
    const dim3 grid((unsigned)((d.K + 255) / 256), (unsigned)c.nsplit);
    switch (d.D) {
#define VB_CASE(DD) \
  case DD:          \
    hipLaunchKernelGGL(k_pass2_direct<DD>, grid, dim3(256), 0, s, a); break;
      VB_CASE(1) VB_CASE(2) VB_CASE(3) VB_CASE(4) VB_CASE(5) VB_CASE(6) VB_CASE(7) VB_CASE(8)
#undef VB_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)(d.L->Kpad / CT), (unsigned)c.nsplit);
#define VB_P2(PP, EE, DD) hipLaunchKernelGGL((k_pass2<PP, EE, DD>), grid, dim3(256), 0, s, a)
#define VB_P2X(PP)                  \
  switch (d.D) {                    \
    case 1: VB_P2(PP, true, 1); break; \
    case 2: VB_P2(PP, true, 2); break; \
    case 3: VB_P2(PP, true, 3); break; \
    case 4: VB_P2(PP, true, 4); break; \
    case 5: VB_P2(PP, true, 5); break; \
    case 6: VB_P2(PP, true, 6); break; \
    default: return hipErrorInvalidValue; \
  }
  if (c.prec == VBGS_FP32) {
    if (c.exact) { VB_P2X(VBGS_FP32) } else VB_P2(VBGS_FP32, false, 0);
  } else if (c.prec == VBGS_BF16) {
    if (c.exact) { VB_P2X(VBGS_BF16) } else VB_P2(VBGS_BF16, false, 0);
  } else {
    if (c.exact) { VB_P2X(VBGS_BF16X3) } else VB_P2(VBGS_BF16X3, false, 0);
  }
#undef VB_P2X
#undef VB_P2
  return hipGetLastError();
}

hipError_t launch_fold(const DevPtrs& d, const EstepCfg& c, double* stats_out, hipStream_t s) {
  const int mode = c.prec == VBGS_FP64 ? 0 : (c.exact ? 2 : 1);
  hipLaunchKernelGGL(k_fold, dim3((unsigned)((d.K + 255) / 256)), dim3(256), 0, s, d.at<double>(d.L->spart),
                     c.nsplit, d.L->Kpad, d.K, d.D, d.frame(), d.at<double>(d.L->direct), direct_stride(d.D), mode,
                     d.at<double>(d.L->stats), stats_out);
  return hipGetLastError();
}

}  // namespace vbgs
