// E-step + sufficient statistics on MFMA (gfx950).
//
// The quadratic form of the score is expanded, s_nk = c_k . phi(x_n) with quadratic point
// features phi = [1, x', upper(x' x'^T)] (x' centred and scaled per frame) and one
// coefficient row c_k per component, so scoring a tile is a GEMM on the matrix cores.
//
// pass 1 (point-tile parallel): stream LDS-staged tiles of coefficient rows past a register-
//   resident block of points; keep an online log-sum-exp per point -> LSE_n.
// pass 2, plain precisions (exact = 0; component-tile parallel): stream LDS-staged tiles of
//   points past a register-resident block of components; recompute the scores,
//   r = exp(s - LSE), and contract r^T phi on the matrix cores (the fused Delta S = R^T S_u of
//   Eq. (fused_contr)); FP32 accumulation per 64-point tile, folded into FP64 registers.
// The N x K responsibility matrix is never stored.
//
// exact = 1: the low-precision GEMM of pass 1 is a *screen*. Its error is bounded by
//   |s~ - s| <= eps_prec * ||c_k|| * ||phi_n||  (rounding of features, coefficients,
//   products and accumulation; Cauchy-Schwarz on sum_f |c_f phi_f|).
// A pair is rescored exactly (FP64, direct form) unless its upper bound lies more than the
// margin T below a running lower bound on max_k s; every skipped pair carries < 2^-T of the
// point's mass. The rescored pairs that may still carry mass are recorded per point, so the
// statistics need no second sweep: r = 2^(s - LSE) of the recorded pairs is accumulated
// exactly (128-bit fixed point, integer atomics: order-independent and deterministic).
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
template <>
struct Opnd<VBGS_FP8> {
  long q;  // eight e4m3 bytes, slots 8 g .. 8 g + 7
};
template <>
struct Opnd<VBGS_FP64_CULLED> {};  // the FP64 comparator's sweep scores directly, without MFMA operands

// FP8 tier: this lane's eight e4m3 slots of a row
__device__ __forceinline__ Opnd<VBGS_FP8> load_op8(const uint8_t* row, int g) {
  Opnd<VBGS_FP8> o;
  o.q = *reinterpret_cast<const long*>(row + 8 * g);
  return o;
}

template <int P>
__device__ __forceinline__ Opnd<P> load_op(const float* f32row, const uint16_t* hrow, const uint16_t* lrow,
                                           int g) {
  Opnd<P> o;
  if constexpr (P == VBGS_FP64_CULLED) {
  } else if constexpr (P == VBGS_FP32) {
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
  if constexpr (P == VBGS_FP64_CULLED) {
  } else if constexpr (P == VBGS_FP32) {
    o.a = f32x4{0.f, 0.f, 0.f, 0.f};
    o.b = o.a;
  } else if constexpr (P == VBGS_FP8) {
    o.q = 0;
  } else {
    for (int i = 0; i < 8; ++i) o.h[i] = (__bf16)0.0f;
    if constexpr (P == VBGS_BF16X3) o.l = o.h;
  }
  return o;
}

// Empty asm that reads the operand registers: it makes the compiler wait for their loads at this
// point, so loads issued together stay together instead of being sunk next to each use.
template <int P>
__device__ __forceinline__ void operands_ready(const Opnd<P>& o) {
  if constexpr (P == VBGS_FP32) {
    asm volatile("" ::"v"(__builtin_bit_cast(u32x4, o.a)), "v"(__builtin_bit_cast(u32x4, o.b)));
  } else if constexpr (P == VBGS_BF16) {
    asm volatile("" ::"v"(__builtin_bit_cast(u32x4, o.h)));
  } else {
    asm volatile("" ::"v"(__builtin_bit_cast(u32x4, o.h)), "v"(__builtin_bit_cast(u32x4, o.l)));
  }
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
  } else if constexpr (P == VBGS_FP8) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(A.q, B.q, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, B.l, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l, B.h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h, B.h, acc, 0, 0, 0);
  }
  return acc;
}



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

// Drop candidates that can no longer carry mass (score below the exact running maximum minus
// the margin); FP32 rounding is monotone, so fl(s) < fl(thr) implies s < thr.
__device__ __noinline__ int evict_candidates(int32_t* __restrict__ ck, float* __restrict__ cs, float thr) {
  int w = 0;
  for (int j = 0; j < CS; ++j) {
    const float v = cs[j];
    const int32_t k = ck[j];
    if (v >= thr) {
      cs[w] = v;
      ck[w] = k;
      ++w;
    }
  }
  return w;
}

// ---------------------------------------------------------------------------
// pass 1: point-tile parallel online LSE (exact mode: the only sweep over all pairs; every pair
// that pass 2 would need has s >= LSE - T >= max - T, so it is rescored and recorded here)
// ---------------------------------------------------------------------------
template <int P>
struct __attribute__((aligned(16))) CTile {
  float c32[P == VBGS_FP32 ? CT : 1][FP];
  uint16_t h[P == VBGS_FP32 || P == VBGS_FP8 ? 1 : CT][FP];
  uint16_t l[P == VBGS_BF16X3 ? CT : 1][FP];
  uint8_t q8[P == VBGS_FP8 ? CT : 1][FP];
  float cs8[P == VBGS_FP8 ? CT : 4];
  float nc[CT];
};

// one thread's share of a coefficient tile (16 B pieces), staged in registers so the global
// loads of tile t + 1 overlap the MFMA work on tile t (native vectors: a struct of HIP's uint4 was
// kept in per-lane scratch memory)
template <int P>
struct TileRegs {
  u32x4 v[P == VBGS_FP32 ? 2 : (P == VBGS_BF16X3 ? 2 : 1)];
  u32x4 nc, s8;
};

template <int P>
__device__ __forceinline__ void tile_fetch(TileRegs<P>& R, const EArgs& a, int64_t k0) {
  const int t = threadIdx.x;  // 256 threads
  if constexpr (P == VBGS_FP32) {
    const u32x4* src = reinterpret_cast<const u32x4*>(a.c32 + k0 * FP);
    R.v[0] = src[t];
    R.v[1] = src[t + 256];
  } else if constexpr (P == VBGS_FP8) {  // 64 rows x 32 B = 128 x 16 B, scales 16 x 16 B
    R.v[0] = t < CT * FP / 16 ? reinterpret_cast<const u32x4*>(a.c8 + k0 * FP)[t] : u32x4{0u, 0u, 0u, 0u};
    R.s8 = t < CT / 4 ? reinterpret_cast<const u32x4*>(a.cs8 + k0)[t] : u32x4{0u, 0u, 0u, 0u};
  } else {
    R.v[0] = reinterpret_cast<const u32x4*>(a.ch + k0 * FP)[t];
    if constexpr (P == VBGS_BF16X3) R.v[1] = reinterpret_cast<const u32x4*>(a.cl + k0 * FP)[t];
  }
  R.nc = t < CT / 4 ? reinterpret_cast<const u32x4*>(a.nc + k0)[t] : u32x4{0u, 0u, 0u, 0u};
}

template <int P>
__device__ __forceinline__ void tile_store(CTile<P>& T, const TileRegs<P>& R) {
  const int t = threadIdx.x;
  if constexpr (P == VBGS_FP32) {
    reinterpret_cast<u32x4*>(&T.c32[0][0])[t] = R.v[0];
    reinterpret_cast<u32x4*>(&T.c32[0][0])[t + 256] = R.v[1];
  } else if constexpr (P == VBGS_FP8) {
    if (t < CT * FP / 16) reinterpret_cast<u32x4*>(&T.q8[0][0])[t] = R.v[0];
    if (t < CT / 4) reinterpret_cast<u32x4*>(T.cs8)[t] = R.s8;
  } else {
    reinterpret_cast<u32x4*>(&T.h[0][0])[t] = R.v[0];
    if constexpr (P == VBGS_BF16X3) reinterpret_cast<u32x4*>(&T.l[0][0])[t] = R.v[1];
  }
  if (t < CT / 4) reinterpret_cast<u32x4*>(T.nc)[t] = R.nc;
}

// Record a screened pair (its score upper bound hi) in the point's list for this lane group.
// A full list first drops entries whose upper bound fell below the running lower bound on the
// point's maximum minus the margin; if it is still full the point is marked overflowed.
__device__ __forceinline__ void record_candidate(const EArgs& a, int64_t p, int g, int64_t k, float hi, float dead,
                                                 int& cn, bool& ovf) {
  int32_t* ck = a.cand_k + (p * 4 + g) * CS;
  float* cs = a.cand_s + (p * 4 + g) * CS;
  if (cn == CS) cn = evict_candidates(ck, cs, dead);
  if (cn < CS) {
    ck[cn] = (int32_t)k;
    cs[cn] = hi;
    ++cn;
  } else {
    ovf = true;
  }
}

// The pairs of one candidate list (of point p) that can carry mass (score >= thr) are counted per
// component; the count before this pair's increment, its rank among the component's pairs,
// replaces its score (cs, as the bits of an int32) and places it in the transpose. With segments
// (a.seg) the pair goes there at once, at seg[k].x + rank, if that is inside the component's
// segment (else a.seg_miss is set and the transpose is redone by k_scatter_pairs). The others
// leave the list (ck = -1). Eight at a time, so that the loads and the atomics of a chunk are in
// flight together.
__device__ __forceinline__ void keep_pairs(const EArgs& a, int32_t p, int32_t* __restrict__ ck, float* __restrict__ cs,
                                           int cn, float thr, unsigned& kept) {
  for (int j0 = 0; j0 < cn; j0 += 8) {
    float sv[8];
    int32_t kv[8], rk[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = j0 + u < cn;
      sv[u] = in ? cs[j0 + u] : -INFINITY;
      kv[u] = in ? ck[j0 + u] : -1;
    }
    int2 sg[8];  // the segments, loaded with the atomics in flight
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool want = kv[u] >= 0 && sv[u] >= thr;
      rk[u] = want ? atomicAdd(&a.ccount[kv[u]], 1) : -1;
      sg[u] = want && a.seg ? a.seg[kv[u]] : int2{0, 0};
    }
    if (a.seg) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (rk[u] >= 0) {
          if (rk[u] < sg[u].y - sg[u].x)
            a.ent_n[sg[u].x + rk[u]] = p;
          else
            atomicOr(a.seg_miss, 1);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (j0 + u < cn) {
        if (rk[u] >= 0) {
          cs[j0 + u] = __int_as_float(rk[u]);
          ++kept;
        } else {
          ck[j0 + u] = -1;
        }
      }
    }
  }
}

// the pair range of component k in ent_n: its segment, or (no segments, or a pair missed its
// segment) the exclusive scan of the counts
__device__ __forceinline__ void pair_range(const EArgs& a, int64_t k, int32_t& e0, int32_t& e1) {
  if (a.seg && *a.seg_miss == 0) {
    e0 = a.seg[k].x;
    e1 = e0 + a.ccount[k];
  } else {
    e0 = a.coffset[k];
    e1 = a.coffset[k + 1];
  }
}

template <int P, bool EXACT>
__global__ __launch_bounds__(256) void k_pass1(const EArgs a) {
  __shared__ CTile<P> T[2];
  __shared__ double red[256];
  if (EXACT && a.gate && a.gate[0] == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * P1_PTS + w * (P1_PB * 16);

  Opnd<P> B[P1_PB];
  float nphE[P1_PB], M[P1_PB], ls[P1_PB];
  float psc[P1_PB];  // FP8 tier: factor undoing the point row's scaling
  int cn[P1_PB];
  bool val[P1_PB], ovf[P1_PB];
#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < a.N;
    psc[b] = 1.0f;
    if (val[b]) {
      if constexpr (P == VBGS_FP8) {
        B[b] = load_op8(a.phi8 + p * FP, g);
        psc[b] = a.phis[p];
      } else {
        B[b] = load_op<P>(a.phi32 + p * FP, a.phih + p * FP, a.phil + p * FP, g);
      }
      nphE[b] = a.eps * a.nphi[p];
    } else {
      B[b] = zero_op<P>();
      nphE[b] = 0.0f;
    }
    M[b] = -INFINITY;
    ls[b] = 0.0f;
    cn[b] = 0;
    ovf[b] = false;
  }
  unsigned nref = 0;

  TileRegs<P> R;
  tile_fetch<P>(R, a, 0);
  tile_store<P>(T[0], R);
  __syncthreads();
  const int64_t ntiles = a.Kpad / CT;
  for (int64_t it = 0; it < ntiles; ++it) {
    const int cur = (int)(it & 1);
    if (it + 1 < ntiles) tile_fetch<P>(R, a, (it + 1) * CT);
    const CTile<P>& Tc = T[cur];
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const int r = cb * 16 + c;
      Opnd<P> A;
      f32x4 csc = {1.f, 1.f, 1.f, 1.f};  // FP8 tier: factors undoing rows cb * 16 + 4 g + i
      if constexpr (P == VBGS_FP8) {
        A = load_op8(&Tc.q8[r][0], g);
        csc = *reinterpret_cast<const f32x4*>(&Tc.cs8[cb * 16 + 4 * g]);
      } else {
        A = load_op<P>(&Tc.c32[P == VBGS_FP32 ? r : 0][0], &Tc.h[P == VBGS_FP32 ? 0 : r][0],
                       &Tc.l[P == VBGS_BF16X3 ? r : 0][0], g);
      }
      const f32x4 nc4 = *reinterpret_cast<const f32x4*>(&Tc.nc[cb * 16 + 4 * g]);
      const float ncm = fmaxf(fmaxf(nc4[0], nc4[1]), fmaxf(nc4[2], nc4[3]));
#pragma unroll
      for (int b = 0; b < P1_PB; ++b) {
        f32x4 s = mfma_scores<P>(A, B[b]);
        if constexpr (P == VBGS_FP8) {
#pragma unroll
          for (int i = 0; i < 4; ++i) s[i] = s[i] * csc[i] * psc[b];
        }
        const float mx = fmaxf(fmaxf(s[0], s[1]), fmaxf(s[2], s[3]));
        if constexpr (EXACT) {
          // one bound for the lane's four pairs: |s~ - s| <= e = eps ||phi|| max_i ||c_i||;
          // M is a running lower bound on max_k s, so a pair whose upper bound s~ + e is below
          // M - T carries < 2^-T of the point's mass and is skipped
          const float e = nphE[b] * ncm;
          M[b] = fmaxf(M[b], mx - e);
          const float thr = M[b] - a.T2 - e;
          if (val[b] && mx >= thr) {
            const int64_t p = p0 + 16 * b + c;
            const int64_t kb = it * CT + cb * 16 + 4 * g;
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (s[i] >= thr && kb + i < a.K) {
                record_candidate(a, p, g, kb + i, s[i] + e, M[b] - a.T2, cn[b], ovf[b]);
                ++nref;
              }
          }
        } else {
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
    if (it + 1 < ntiles) tile_store<P>(T[cur ^ 1], R);
    __syncthreads();
  }

  if constexpr (EXACT) {
    // publish the lists: the four lane groups of a point agree on whether it overflowed
#pragma unroll
    for (int b = 0; b < P1_PB; ++b) {
      const int64_t p = p0 + 16 * b + c;
      int o = ovf[b] ? 1 : 0;
      o |= __shfl_xor(o, 16);
      o |= __shfl_xor(o, 32);
      if (val[b]) {
        a.cand_n[p * 4 + g] = o ? -1 : cn[b];
        if (o && g == 0) a.over_list[atomicAdd(&a.frame->n_over, 1)] = (int32_t)p;
      }
    }
    count_refined(&a.frame->refined1, nref);
    if (lane == 0) {
      atomicAdd(&a.frame->blocks, (unsigned long long)(ntiles * (CT / 16)));
      atomicAdd(&a.frame->blocks_cum, (unsigned long long)(ntiles * (CT / 16)));
    }
  } else {
#pragma unroll
    for (int b = 0; b < P1_PB; ++b) {
      double m = (double)M[b];
      double l = (double)ls[b];
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
    __syncthreads();
    if (tid == 0) {
      double sacc = 0.0;
      for (int i = 0; i < 256; ++i) sacc += red[i];
      a.lse_part[blockIdx.x] = sacc;
    }
  }
}

// ---------------------------------------------------------------------------
// exact mode, culled sweep over spatially sorted points and components
// ---------------------------------------------------------------------------
// Points are taken in curve order (a wave holds 64 spatially close points) and the coefficient
// rows in the order of (curvature class, Hilbert code of the mean), 64 rows per tile. Bounds on
// the score of a pair with a point x (first min(D, 3) raw coordinates S):
//   tile t:  G_t - Lam_t dist^2(x_S, box_t)       (TileInfo: max G, min lambda, box of the means)
//   row k:   G_k - lambda_k |x_S - m_k,S|^2       (RowBound)
// A pair whose bound lies below the point's running lower bound M minus the margin T is one the
// per-pair screen would drop, so it is never screened. Each wave works on its own:
//   1. pilot: the centre tiles (in each curvature class, the tiles at the Hilbert positions of its
//      first and last point) are screened without recording, which brings every M close to its
//      final value;
//   2. the seed tiles (the centres and their two neighbours), now recording candidates;
//   3. every other tile, 64 at a time (one per lane): a tile is screened when its bound reaches
//      M - T for at least one point of the wave; within it, a 16-row block is screened when one
//      of its row bounds, taken over the wave's box, reaches the wave's smallest M - T.
// Each wave stages its own tiles in LDS (the rows stay resident in the caches, being read by
// every wave), so waves never wait for one another.
__device__ __forceinline__ float box_d2(const TileInfo& t, const float* lo, const float* hi) {
  float d2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float gap = fmaxf(fmaxf(t.lo[i] - hi[i], lo[i] - t.hi[i]), 0.0f);
    d2 = fmaf(gap, gap, d2);
  }
  return d2;
}

// Eight searches at once, one per group of eight lanes (lane >> 3 = q): the last tile whose
// first code is <= code_q (0 when there is none), eight probes per group and step.
__device__ __forceinline__ int64_t find_tiles8(const TileInfo* __restrict__ ti, int64_t ntiles, uint32_t code,
                                               int lane) {
  const int q = lane >> 3, r = lane & 7;
  int64_t L = 0, R = ntiles - 1;
  for (;;) {
    const bool active = L < R;
    if (__ballot(active) == 0ull) break;
    const int64_t span = R - L + 1;
    const int64_t pos = L + span * r / 8;
    const bool le = active && ti[pos].code <= code;
    const unsigned gm = (unsigned)(__ballot(le) >> (8 * q)) & 0xFFu;
    if (active) {
      if (gm == 0u) {
        R = L;  // only when L = 0 and code is below the first tile's
      } else {
        const int last = 31 - __clz(gm);
        const int64_t nl = L + span * last / 8;
        const int64_t nr = last == 7 ? R : L + span * (last + 1) / 8 - 1;
        L = nl;
        R = nr > nl ? nr : nl;
      }
    }
  }
  return L;
}

// tiles that at most this many of a wave's points reach are scored directly (direct_tile)
constexpr int DIRECT_MAX = 2;

// Workgroups are dealt to the eight XCDs in turn; renumber them so that each XCD takes one
// contiguous range of the curve order, whose component tiles then stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % 8, q = b / 8, per = nb / 8, rem = nb % 8;
  return x * per + (x < rem ? x : rem) + q;
}

// One tile's operands staged in LDS by asynchronous global -> LDS copies (lane L's 16 bytes at
// 16 L of each piece), so that the copy of the next tile overlaps the work on the current one.
typedef __attribute__((address_space(3))) void lds_void;

template <int P>
struct TileStage {
  static constexpr int NB = P == VBGS_FP64_CULLED ? 1 : CT / 16;  // (the FP64 comparator stages nothing)
  u32x4 a[NB][2][64];  // coefficient rows: [16-row block][hi / lo (FP32: first / second half)][lane]
  u32x4 rb[2][64];          // RowBound of row `lane`, two 16-byte halves
  int32_t krow[64];         // component of row `lane`
};

__device__ __forceinline__ void dma16(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (lds_void*)dst, 16, 0, 0);
}

// start copying tile t into st (after the reads of its previous contents have completed)
template <int P>
__device__ __forceinline__ void stage_tile(const EArgs& a, int64_t t, int lane, TileStage<P>& st) {
  const int g = lane >> 4, c = lane & 15;
  const int64_t r0 = t * CT;
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
  for (int cb = 0; cb < CT / 16; ++cb) {
    const int64_t r = r0 + cb * 16 + c;
    if constexpr (P == VBGS_FP32) {
      dma16(a.c32 + r * FP + 8 * g, &st.a[cb][0][0]);
      dma16(a.c32 + r * FP + 8 * g + 4, &st.a[cb][1][0]);
    } else {
      dma16(a.ch + r * FP + 8 * g, &st.a[cb][0][0]);
      if constexpr (P == VBGS_BF16X3) dma16(a.cl + r * FP + 8 * g, &st.a[cb][1][0]);
    }
  }
  const char* rbp = reinterpret_cast<const char*>(a.rowb + r0 + lane);
  dma16(rbp, &st.rb[0][0]);
  dma16(rbp + 16, &st.rb[1][0]);
  __builtin_amdgcn_global_load_lds(a.corder + r0 + lane, (lds_void*)&st.krow[0], 4, 0, 0);
}

// wait for the copies of the staged tile and read this lane's pieces
template <int P>
__device__ __forceinline__ void read_stage(const TileStage<P>& st, int lane, Opnd<P>* A, RowBound& rb,
                                           int32_t& krow) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
  for (int cb = 0; cb < CT / 16; ++cb) {
    if constexpr (P == VBGS_FP32) {
      A[cb].a = __builtin_bit_cast(f32x4, st.a[cb][0][lane]);
      A[cb].b = __builtin_bit_cast(f32x4, st.a[cb][1][lane]);
    } else {
      A[cb].h = __builtin_bit_cast(bf16x8, st.a[cb][0][lane]);
      if constexpr (P == VBGS_BF16X3) A[cb].l = __builtin_bit_cast(bf16x8, st.a[cb][1][lane]);
    }
  }
  const u32x4 h0 = st.rb[0][lane], h1 = st.rb[1][lane];  // RowBound {G, Lam, m[3], nc, pad[2]}
  rb.G = __uint_as_float(h0.x);
  rb.Lam = __uint_as_float(h0.y);
  rb.m[0] = __uint_as_float(h0.z);
  rb.m[1] = __uint_as_float(h0.w);
  rb.m[2] = __uint_as_float(h1.x);
  rb.nc = __uint_as_float(h1.y);
  krow = st.krow[lane];
}

template <int P>
struct SweepWave {
  Opnd<P> B[P1_PB];
  float nphE[P1_PB], M[P1_PB];
  int cn[P1_PB];
  bool val[P1_PB], ovf[P1_PB];
  float lo[3], hi[3];
  unsigned nref, nblk;
  float mw;  // the wave's smallest M when last taken (seeds: -inf)
};

// screen tile t for the wave's points (see above); rec: record candidates. st holds tile t when
// staged is set (else it is copied here); t_next >= 0 starts the copy of the next tile.
// tk: the wave's LDS slot for the tile's component indices (lane = row)
template <int P>
__device__ __forceinline__ void screen_tile(const EArgs& a, SweepWave<P>& S, int64_t t, int64_t t_next, bool staged,
                                            bool rec, int lane, unsigned bm, float* __restrict__ mv,
                                            const int32_t* __restrict__ pid, int32_t* __restrict__ tk,
                                            TileStage<P>& st) {
  const int g = lane >> 4, c = lane & 15;
  const int64_t r0 = t * CT;
  if (!staged) stage_tile<P>(a, t, lane, st);
  Opnd<P> A[CT / 16];
  RowBound rb;
  int32_t krow;  // rows past K hold no component (never recorded)
  read_stage<P>(st, lane, A, rb, krow);
  if (t_next >= 0) stage_tile<P>(a, t_next, lane, st);
  // largest coefficient norm of this lane's four rows 16 cb + 4 g + i (i < 4), per block cb
  float nc4 = fmaxf(rb.nc, __shfl_xor(rb.nc, 1));
  nc4 = fmaxf(nc4, __shfl_xor(nc4, 2));
  const float mw = S.mw;  // stale lower bound on the wave's smallest M (M only grows)
  const float margin = a.T2 + 1.0f;
  float d2 = 0.0f;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    // the mean is rounded to FP32: shrink the gap by a bound on that rounding
    const float gap =
        fmaxf(fmaxf(rb.m[q] - S.hi[q], S.lo[q] - rb.m[q]) - fabsf(rb.m[q]) * 2.384185791015625e-7f, 0.0f);
    d2 = fmaf(gap, gap, d2);
  }
  const unsigned long long rmask = __ballot(rb.G - rb.Lam * d2 >= mw - margin);
  tk[lane] = krow;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int cb = 0; cb < CT / 16; ++cb) {
    if (((rmask >> (16 * cb)) & 0xFFFFull) == 0ull) continue;  // wave-uniform
    ++S.nblk;
    const float ncm = __shfl(nc4, 16 * cb + 4 * g);  // rows 16 cb + 4 g + i, i < 4
    // the four point blocks' products first (independent MFMA chains), then their screens
    f32x4 svb[P1_PB];
#pragma unroll
    for (int b = 0; b < P1_PB; ++b)
      if (bm & (1u << b)) svb[b] = mfma_scores<P>(A[cb], S.B[b]);
#pragma unroll
    for (int b = 0; b < P1_PB; ++b) {
      if (!(bm & (1u << b))) continue;  // no point of this block within reach (wave-uniform)
      const f32x4 sv = svb[b];
      const float mx = fmaxf(fmaxf(sv[0], sv[1]), fmaxf(sv[2], sv[3]));
      const float e = S.nphE[b] * ncm;
      S.M[b] = fmaxf(S.M[b], mx - e);
      const float thr = S.M[b] - a.T2 - e;
      if (rec && S.val[b] && mx >= thr) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t r = r0 + cb * 16 + 4 * g + q;
          if (sv[q] >= thr && r < a.K) {
            record_candidate(a, pid[16 * b + c], g, tk[cb * 16 + 4 * g + q], sv[q] + e, S.M[b] - a.T2, S.cn[b],
                             S.ovf[b]);
            ++S.nref;
          }
        }
      }
    }
  }
}

// Tiles that only a few of the wave's points reach (points far from every component, whose
// bounds reach many tiles that the rest of the wave never needs) are not staged for the MFMA
// screen: lane = row, each reaching point in turn is tested against the row bounds and the pairs
// that pass are scored exactly in FP64 (the same score the exact LSE gives them later), raise the
// point's M and are recorded like screened pairs (error bound 0). pm: the wave's points (lane
// index = point slot) that reach the tile; buf: 64 LDS entries for the recorded pairs.
// a lane's row of a tile for direct scoring: its bound and component (rows past K: no component)
struct DirectRow {
  float G, Lam, m[3];
  int32_t k;
};

__device__ __forceinline__ DirectRow load_direct_row(const EArgs& a, int64_t t, int lane) {
  DirectRow d{-INFINITY, 0.0f, {0.0f, 0.0f, 0.0f}, -1};
  const int64_t r = t * CT + lane;
  if (r < a.K) {
    const RowBound rb = a.rowb[r];
    d.G = rb.G;
    d.Lam = rb.Lam;
    d.m[0] = rb.m[0];
    d.m[1] = rb.m[1];
    d.m[2] = rb.m[2];
    d.k = a.corder[r];
  }
  return d;
}

template <int P>
__device__ __forceinline__ void direct_tile(const EArgs& a, SweepWave<P>& S, const DirectRow& dr, unsigned long long pm,
                                            bool rec, int lane, float* __restrict__ mv, const int32_t* __restrict__ pid,
                                            const float4* __restrict__ pts, float2* __restrict__ buf) {
  const int g = lane >> 4, c = lane & 15;
  const bool rv = dr.k >= 0;
  const float rg = dr.G, rl = dr.Lam, rm[3] = {dr.m[0], dr.m[1], dr.m[2]};
  const int32_t k = rv ? dr.k : 0;
  const double* row = a.direct + (int64_t)k * a.dts;
  const float margin = a.T2 + 1.0f;
  while (pm) {
    const int p = __ffsll((long long)pm) - 1;  // wave-uniform
    pm &= pm - 1ull;
    const float4 xp = pts[p];
    const float xq[3] = {xp.x, xp.y, xp.z};
    float d2 = 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float gap = fmaxf(fabsf(xq[q] - rm[q]) - fabsf(rm[q]) * 2.384185791015625e-7f, 0.0f);
      d2 = fmaf(gap, gap, d2);
    }
    const float Mp = mv[p];
    const bool pass = rv && rg - rl * d2 >= Mp - margin;
    double s2 = -INFINITY;
    if (pass) s2 = direct_score2_rt(row, a.X + (int64_t)pid[p] * a.D, a.D);
    // the largest exact score is a lower bound on the point's maximum (rounded down)
    float smax = pass ? __double2float_rd(s2) : -INFINITY;
    for (int o = 1; o < 64; o <<= 1) smax = fmaxf(smax, __shfl_xor(smax, o));
    const float Mn = fmaxf(Mp, smax);
    const int pb = p >> 4;
#pragma unroll
    for (int b = 0; b < P1_PB; ++b)
      if (b == pb && c == (p & 15)) S.M[b] = fmaxf(S.M[b], Mn);
    if (lane == 0) mv[p] = Mn;
    if (rec) {
      const float hi = pass ? __double2float_ru(s2) : -INFINITY;
      const unsigned long long km = __ballot(pass && hi >= Mn - a.T2);
      if (km) {
        if (pass && hi >= Mn - a.T2) {
          const int idx = __builtin_amdgcn_mbcnt_hi((unsigned)(km >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u));
          buf[idx] = make_float2(__int_as_float(k), hi);
        }
        __builtin_amdgcn_wave_barrier();
        const int cnt = __popcll(km);
        if (c == (p & 15)) {  // the point's four lane groups take every fourth pair
#pragma unroll
          for (int b = 0; b < P1_PB; ++b)
            if (b == pb && S.val[b])
              for (int i = g; i < cnt; i += 4) {
                const float2 e = buf[i];
                record_candidate(a, pid[p], g, __float_as_int(e.x), e.y, S.M[b] - a.T2, S.cn[b], S.ovf[b]);
                ++S.nref;
              }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
}

// make each point's M the largest over its four lane groups and publish it for the tile tests
template <int P>
__device__ __forceinline__ void share_m(SweepWave<P>& S, int lane, float* __restrict__ mv) {
  const int g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    S.M[b] = fmaxf(S.M[b], __shfl_xor(S.M[b], 16));
    S.M[b] = fmaxf(S.M[b], __shfl_xor(S.M[b], 32));
    if (g == 0 && S.val[b]) mv[16 * b + c] = S.M[b];
  }
  __builtin_amdgcn_wave_barrier();
}

template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_sweep(const EArgs a) {
  // one wave per workgroup, so that a finished wave frees its slot at once
  if (a.gate && a.gate[0] == 0) return;
  __shared__ float4 pts[1][64];   // first three raw coordinates of the wave's points
  __shared__ float mvs[1][64];    // their current lower bounds M (+inf for empty slots)
  __shared__ int32_t pids[1][64]; // their original indices
  __shared__ int32_t seeds[1][24];
  __shared__ uint8_t bms[1][64];  // per tile of the current chunk: the 16-point blocks it reaches
  __shared__ int32_t tks[1][64];  // component indices of the tile being screened
  __shared__ TileStage<P> stg;    // operands of the tile being screened or the next one
  // pairs of a directly scored tile: component (bits), score. Direct tiles are scored only while no
  // tile is staged (the FP64 comparator stages none), so they share the stage's memory, which keeps
  // the workgroup within the LDS that twelve of them per CU may hold.
  float2* const dbuf = reinterpret_cast<float2*>(&stg.a[0][0][0]);
  static_assert(sizeof(stg.a) >= 64 * sizeof(float2), "direct-tile buffer");
  const uint64_t t_start = wall_clock64();
  const int lane = threadIdx.x, w = 0, g = lane >> 4, c = lane & 15;
  if (blockIdx.x == 0 && lane == 0) a.bprev[0] = gridDim.x;  // read by the next launch's k_block_order
  const int64_t jb = a.border[xcd_block(blockIdx.x, gridDim.x)];
  const int64_t j0 = jb * (P1_PB * 16);  // sorted positions
  const int ns = a.nsp;
  float* mv = mvs[w];
  const int32_t* pid = pids[w];

  SweepWave<P> S;
  S.mw = -INFINITY;
  S.nref = 0;
  S.nblk = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    S.lo[i] = INFINITY;
    S.hi[i] = -INFINITY;
  }
#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    const int64_t j = j0 + 16 * b + c;
    S.val[b] = j < a.N;
    const int64_t p = S.val[b] ? a.porder[j] : 0;
    float v[3] = {0.0f, 0.0f, 0.0f};
    if (S.val[b]) {
      S.B[b] = load_op<P>(a.phi32 + p * FP, a.phih + p * FP, a.phil + p * FP, g);
      S.nphE[b] = a.eps * a.nphi[p];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        v[i] = i < ns ? a.X[p * a.D + i] : 0.0f;
        S.lo[i] = fminf(S.lo[i], v[i]);
        S.hi[i] = fmaxf(S.hi[i], v[i]);
      }
    } else {
      S.B[b] = zero_op<P>();
      S.nphE[b] = 0.0f;
    }
    if (g == 0) {
      pts[w][16 * b + c] = make_float4(v[0], v[1], v[2], 0.0f);
      mvs[w][16 * b + c] = S.val[b] ? -INFINITY : INFINITY;
      pids[w][16 * b + c] = (int32_t)p;
    }
    S.M[b] = -INFINITY;
    S.cn[b] = 0;
    S.ovf[b] = false;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    for (int off = 1; off < 64; off <<= 1) {
      S.lo[i] = fminf(S.lo[i], __shfl_xor(S.lo[i], off));
      S.hi[i] = fmaxf(S.hi[i], __shfl_xor(S.hi[i], off));
    }
  __builtin_amdgcn_wave_barrier();
  if (j0 < a.N) {
    const int64_t ntiles = a.Kpad / CT;
    // seeds: in each curvature class, the tiles around the Hilbert positions of the wave's first
    // and last point (eight centres c_q, q = 2 class + end)
    const int64_t jl = min(j0 + 63, a.N - 1);
    const int qq = lane >> 3;
    const uint32_t pc = a.pcode[(qq & 1) ? jl : j0] & 0x3FFFFFFFu;
    const int32_t cen = (int32_t)find_tiles8(a.tinfo, ntiles, ((uint32_t)(qq >> 1) << 30) | pc, lane);
    int32_t cq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) cq[q] = __builtin_amdgcn_readfirstlane(__shfl(cen, 8 * q));
    auto near_centre = [&](int64_t t, int upto) {
      bool r = false;
#pragma unroll
      for (int q = 0; q < 8; ++q) r |= q < upto && t >= cq[q] - 1 && t <= cq[q] + 1;
      return r;
    };
    // the distinct centres first, then their neighbours c_q +- 1 (all distinct, inside the table)
    int nseed = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      bool dup = false;
#pragma unroll
      for (int r = 0; r < 8; ++r) dup |= r < q && cq[r] == cq[q];
      if (!dup) {
        if (lane == 0) seeds[w][nseed] = cq[q];
        ++nseed;
      }
    }
    const int ncen = nseed;
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int d = -1; d <= 1; d += 2) {
        const int64_t t = (int64_t)cq[q] + d;
        bool centre = false;
#pragma unroll
        for (int r = 0; r < 8; ++r) centre |= t == cq[r];
        if (t >= 0 && t < ntiles && !centre && !near_centre(t, q)) {
          if (lane == 0) seeds[w][nseed] = (int32_t)t;
          ++nseed;
        }
      }
    __builtin_amdgcn_wave_barrier();
    // a pilot over the centres raises M without recording; then every seed is screened, recording
    const int npil = ncen, nst = npil + nseed;
    auto seed_at = [&](int i) { return (int64_t)__builtin_amdgcn_readfirstlane(seeds[w][i < npil ? i : i - npil]); };
    for (int i = 0; i < nst; ++i) {
      if constexpr (P == VBGS_FP64_CULLED) {
        const unsigned long long all = __ballot(mv[lane] < INFINITY);  // the wave's valid points
        direct_tile<P>(a, S, load_direct_row(a, seed_at(i), lane), all, i >= npil, lane, mv, pid, pts[w], dbuf);
      } else {
        const int64_t tn = i + 1 < nst ? seed_at(i + 1) : -1;
        screen_tile<P>(a, S, seed_at(i), tn, i > 0, i >= npil, lane, 0xFu, mv, pid, tks[w], stg);
      }
      share_m<P>(S, lane, mv);
    }
    const float margin = a.T2 + 1.0f;
    const float4 xme = pts[w][lane];  // this lane's point (lane = point of the wave)
    uint32_t* slist = a.slist + jb * ntiles;  // the block's directly scored tiles
    int64_t nsl = 0;
    for (int64_t base = 0; base < ntiles; base += 64) {
      share_m<P>(S, lane, mv);
      // lane = tile: the wave's box against the tile bound
      const int64_t t = base + lane;
      float mw = INFINITY;
#pragma unroll
      for (int b = 0; b < P1_PB; ++b)
        if (S.val[b]) mw = fminf(mw, S.M[b]);
      for (int o = 1; o < 64; o <<= 1) mw = fminf(mw, __shfl_xor(mw, o));
      S.mw = mw;
      TileInfo ti{};
      bool cand = false;
      if (t < ntiles && !near_centre(t, 8)) {
        ti = a.tinfo[t];
        cand = ti.G - ti.Lam * box_d2(ti, S.lo, S.hi) >= mw - margin;
      }
      // lane = point: each candidate tile against every point's own bound and M
      const float thr_me = mv[lane] - margin;
      unsigned long long cm = __ballot(cand), m = 0ull, msp = 0ull;
      while (cm) {
        const int i = __ffsll((long long)cm) - 1;
        cm &= cm - 1ull;
        const float tG = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ti.G), i));
        const float tL = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ti.Lam), i));
        const float xq[3] = {xme.x, xme.y, xme.z};
        float d2 = 0.0f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const float tlo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ti.lo[q]), i));
          const float thi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ti.hi[q]), i));
          const float gap = fmaxf(fmaxf(tlo - xq[q], xq[q] - thi), 0.0f);
          d2 = fmaf(gap, gap, d2);
        }
        const unsigned long long pm = __ballot(tG - tL * d2 >= thr_me);
        if (pm != 0ull && (P == VBGS_FP64_CULLED || __popcll(pm) <= DIRECT_MAX)) {
          msp |= 1ull << i;  // few points reach it: direct FP64 scoring after the screened tiles
        } else if (pm != 0ull) {
          m |= 1ull << i;
          // which 16-point blocks (lane = point, block = lane / 16) reach the tile
          const unsigned bmi = ((pm & 0xFFFFull) ? 1u : 0u) | ((pm & 0xFFFF0000ull) ? 2u : 0u) |
                               ((pm & 0xFFFF00000000ull) ? 4u : 0u) | ((pm >> 48) ? 8u : 0u);
          if (lane == 0) bms[w][i] = (uint8_t)bmi;
        }
      }
      __builtin_amdgcn_wave_barrier();
      if constexpr (P != VBGS_FP64_CULLED) {
        bool staged = false;
        while (m) {
          const int i = __ffsll((long long)m) - 1;
          m &= m - 1ull;
          const int64_t tn = m ? base + (__ffsll((long long)m) - 1) : -1;
          screen_tile<P>(a, S, base + i, tn, staged, true, lane, __builtin_amdgcn_readfirstlane(bms[w][i]), mv, pid,
                         tks[w], stg);
          staged = tn >= 0;
        }
      }
      // the tiles that few points reach wait in the block's list until every screened tile has
      // raised the points' M (fewer pairs pass then, and the screen's registers are free)
      while (msp) {
        const int i = __ffsll((long long)msp) - 1;
        msp &= msp - 1ull;
        if (lane == 0) slist[nsl] = (uint32_t)(base + i);
        ++nsl;
      }
    }
    share_m<P>(S, lane, mv);
    // The listed tiles, 64 at a time: lane = tile loads its bound, then (lane = point) each tile in
    // turn is tested against every point with the point's current M, as in the chunk scan. M only
    // grows, so the tiles that no point reaches at the start of the batch are dropped at once; the
    // others are tested again when their turn comes, with the rows of the next one in flight.
    auto reach = [&](const TileInfo& tb, int i) {
      const float tG = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tb.G), i));
      const float tL = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tb.Lam), i));
      const float xq[3] = {xme.x, xme.y, xme.z};
      float d2 = 0.0f;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float tlo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tb.lo[q]), i));
        const float thi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tb.hi[q]), i));
        const float gap = fmaxf(fmaxf(tlo - xq[q], xq[q] - thi), 0.0f);
        d2 = fmaf(gap, gap, d2);
      }
      return __ballot(tG - tL * d2 >= mv[lane] - margin);
    };
    for (int64_t base = 0; base < nsl; base += 64) {
      const int64_t q = base + lane;
      TileInfo tb{};
      int32_t tl = 0;
      if (q < nsl) {
        tl = (int32_t)slist[q];
        tb = a.tinfo[tl];
      }
      const int nq = (int)min((int64_t)64, nsl - base);
      unsigned long long keep = 0ull;
      for (int i = 0; i < nq; ++i)
        if (reach(tb, i)) keep |= 1ull << i;
      DirectRow drn{};
      if (keep) drn = load_direct_row(a, __builtin_amdgcn_readlane(tl, __ffsll((long long)keep) - 1), lane);
      while (keep) {
        const int i = __ffsll((long long)keep) - 1;
        keep &= keep - 1ull;
        const DirectRow dr = drn;
        if (keep) drn = load_direct_row(a, __builtin_amdgcn_readlane(tl, __ffsll((long long)keep) - 1), lane);
        const unsigned long long pm = reach(tb, i);
        if (pm) direct_tile<P>(a, S, dr, pm, true, lane, mv, pid, pts[w], dbuf);
      }
    }
    share_m<P>(S, lane, mv);
  }
  unsigned kept = 0;
#pragma unroll
  for (int b = 0; b < P1_PB; ++b) {
    int o = S.ovf[b] ? 1 : 0;
    o |= __shfl_xor(o, 16);
    o |= __shfl_xor(o, 32);
    const int32_t p = pid[16 * b + c];
    if (S.val[b]) {
      a.cand_n[(int64_t)p * 4 + g] = o ? -1 : S.cn[b];
      if (o && g == 0) {
        a.over_list[atomicAdd(&a.frame->n_over, 1)] = p;
        a.lse2[p] = (double)S.M[b];  // lower bound on the point's largest score, for the rescan's culling
      }
    }
    // The exact LSE of the wave's points, here rather than in a pass of its own: the block's
    // pairs are rescored while it still holds its slot, which fills the GPU during the sweep's
    // tail. Each lane rescores the list it wrote (list g of point 16 b + c) in FP64, the point's
    // four lists merge by shuffles, and the pairs within the margin of the LSE are kept and
    // counted per component for the statistics (overflowed points: the rescan does all of it).
    const bool live = S.val[b] && !o;
    double mm = -INFINITY, ll = 0.0;
    int32_t* ck = a.cand_k + ((int64_t)p * 4 + g) * CS;
    float* cs = a.cand_s + ((int64_t)p * 4 + g) * CS;
    if (live) {
      const float* xp = a.X + (int64_t)p * a.D;
      for (int j = 0; j < S.cn[b]; ++j) {
        const double sc = direct_score2_rt(a.direct + (int64_t)ck[j] * a.dts, xp, a.D);
        online_add(mm, ll, sc);
        cs[j] = (float)sc;
      }
    }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const double m2 = __shfl_xor(mm, off), l2 = __shfl_xor(ll, off);
      const double mn = fmax(mm, m2);
      if (mn > -INFINITY) {
        ll = (mm == -INFINITY ? 0.0 : ll * exp2(mm - mn)) + (m2 == -INFINITY ? 0.0 : l2 * exp2(m2 - mn));
        mm = mn;
      }
    }
    if (live) {
      const double L2 = mm + log2(ll);
      if (g == 0) a.lse2[p] = L2;
      const float thr = (float)(L2 - (double)a.T2);  // FP32 rounding is monotone (see evict_candidates)
      keep_pairs(a, p, ck, cs, S.cn[b], thr, kept);
    }
  }
  count_refined(&a.frame->refined2, kept);
  count_refined(&a.frame->refined1, S.nref);
  if (lane == 0) {
    a.bcost[jb] = (float)(wall_clock64() - t_start);
    a.bcode[jb] = a.pcode[j0];
  }
  if (lane == 0 && S.nblk) {
    atomicAdd(&a.frame->blocks, (unsigned long long)S.nblk);
    atomicAdd(&a.frame->blocks_cum, (unsigned long long)S.nblk);
  }
}

// ---------------------------------------------------------------------------
// pass 2 (plain GEMM precisions): component-tile parallel recompute + r^T phi on MFMA
// ---------------------------------------------------------------------------
template <int P>
struct __attribute__((aligned(16))) PTile {
  float f32[PT][FP];
  uint16_t h[P == VBGS_FP32 || P == VBGS_FP8 ? 1 : PT][FP];
  uint16_t l[P == VBGS_BF16X3 ? PT : 1][FP];
  uint8_t q8[P == VBGS_FP8 ? PT : 1][FP];
  float ps8[PT];
  float nph[PT];
  double lse[PT];
};

template <int P>
__device__ __forceinline__ void load_ptile(PTile<P>& T, const EArgs& a, int64_t n0) {
  const int t = threadIdx.x;
  const int64_t nvalid = a.N - n0;  // > 0
  for (int q = t; q < PT * FP / 4; q += 256) {  // 64 rows x 128 B = 512 x 16 B
    const int row = q / (FP / 4);
    uint4 v = {0, 0, 0, 0};
    if (row < nvalid) v = reinterpret_cast<const uint4*>(a.phi32 + n0 * FP)[q];
    reinterpret_cast<uint4*>(&T.f32[0][0])[q] = v;
  }
  if constexpr (P == VBGS_FP8) {
    const int row = t / (FP / 16);  // 64 rows x 32 B = 128 x 16 B
    if (t < PT * FP / 16) {
      uint4 v = {0, 0, 0, 0};
      if (row < nvalid) v = reinterpret_cast<const uint4*>(a.phi8 + n0 * FP)[t];
      reinterpret_cast<uint4*>(&T.q8[0][0])[t] = v;
    }
  } else if constexpr (P != VBGS_FP32) {
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
    if constexpr (P == VBGS_FP8) T.ps8[t] = v ? a.phis[n0 + t] : 0.0f;
    T.nph[t] = v ? a.nphi[n0 + t] : 0.0f;
    T.lse[t] = v ? a.lse2[n0 + t] : INFINITY;
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_pass2(const EArgs a) {
  __shared__ PTile<P> T;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t kb = (int64_t)blockIdx.x * CT + w * 16;
  const int64_t kc = kb + c;
  const bool kval = kc < a.K;
  Opnd<P> Bc;
  float csc = 1.0f;  // FP8 tier: factor undoing the component row's scaling
  if constexpr (P == VBGS_FP8) {
    Bc = load_op8(a.c8 + kc * FP, g);
    csc = a.cs8[kc];
  } else {
    Bc = load_op<P>(a.c32 + kc * FP, a.ch + kc * FP, a.cl + kc * FP, g);
  }
  const int64_t ntile = (a.N + PT - 1) / PT;
  const int64_t t0 = ntile * blockIdx.y / a.nsplit, t1 = ntile * (blockIdx.y + 1) / a.nsplit;
  // FP64 fold of the FP32 MFMA r^T phi tiles; lane holds comps kb + 4g + j at slots c and 16 + c
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;

  for (int64_t t = t0; t < t1; ++t) {
    const int64_t n0 = t * PT;
    __syncthreads();
    load_ptile<P>(T, a, n0);
    __syncthreads();
    f32x4 sa = {0.f, 0.f, 0.f, 0.f}, sb = sa;
#pragma unroll
    for (int pb = 0; pb < PT / 16; ++pb) {
      const int r = pb * 16 + c;
      Opnd<P> A;
      if constexpr (P == VBGS_FP8) {
        A = load_op8(&T.q8[r][0], g);
      } else {
        A = load_op<P>(&T.f32[r][0], &T.h[P == VBGS_FP32 ? 0 : r][0], &T.l[P == VBGS_BF16X3 ? r : 0][0], g);
      }
      f32x4 s = mfma_scores<P>(A, Bc);  // lane: points pb*16 + 4g + i, component kc
      const int rb = pb * 16 + 4 * g;
      if constexpr (P == VBGS_FP8) {
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = s[i] * T.ps8[rb + i] * csc;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float rr = kval ? exp2f(s[i] - (float)T.lse[rb + i]) : 0.0f;
        sa = __builtin_amdgcn_mfma_f32_16x16x4f32(rr, T.f32[rb + i][c], sa, 0, 0, 0);
        sb = __builtin_amdgcn_mfma_f32_16x16x4f32(rr, T.f32[rb + i][16 + c], sb, 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[j] += (double)sa[j];
      acc[4 + j] += (double)sb[j];
    }
  }
  double* out = a.spart + ((int64_t)blockIdx.y * a.Kpad + kb) * FP;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    out[(4 * g + j) * FP + c] = acc[j];
    out[(4 * g + j) * FP + 16 + c] = acc[4 + j];
  }
}

// ---------------------------------------------------------------------------
// exact mode, statistics from the recorded candidates
// ---------------------------------------------------------------------------
// v * 2^64 as a two's-complement 128-bit integer {lo, hi} added with integer atomics: the sum is
// exact (to 2^-64 per term) and independent of the order of the additions, so the statistics
// are bitwise reproducible without sorting the contributions by component.
// The 128-bit fixed-point image of v: v = hi + lo 2^-64 up to the bits below 2^-64, which are
// dropped (hi = floor(v), returned as an integer-valued double; 0 <= lo < 2^64). Every step is
// exact in FP64 (a power-of-two scaling, the difference of a number and its floor), and the
// fraction's two 32-bit halves are converted separately.
__device__ __forceinline__ double fx_split(double v, unsigned long long& lo) {
  // no fusion of v - hi_d with the product that made v: every path converts the same rounded v
#pragma clang fp contract(off)
  double hi_d = floor(v);
  double frac = v - hi_d;  // exact, in [0, 1]
  if (frac >= 1.0) {  // (v a tiny negative number)
    frac = 0.0;
    hi_d += 1.0;
  }
  const double f1 = ldexp(frac, 32);     // [0, 2^32)
  const double a1 = floor(f1);
  const double f2 = ldexp(f1 - a1, 32);  // exact, [0, 2^32)
  lo = ((unsigned long long)(uint32_t)a1 << 32) | (unsigned long long)(uint32_t)f2;
  return hi_d;
}

__device__ __forceinline__ void fx_add(unsigned long long* cell, double v) {
  unsigned long long lo;
  const double hi_d = fx_split(v, lo);
  const unsigned long long old = atomicAdd(&cell[0], lo);
  const long long h = (long long)hi_d + ((old + lo < old) ? 1 : 0);
  if (h != 0) atomicAdd(&cell[1], (unsigned long long)h);
}

// contributions of one pair to the statistics of component k, in coordinates centred at m_k
// and scaled by the frame's power-of-two scales (so the fixed point keeps its resolution)
template <int DT>
__device__ __forceinline__ void fx_pair(unsigned long long* __restrict__ fx, int64_t k, double r,
                                        const double* d, const double* is) {
  unsigned long long* row = fx + k * FP * 2;
  fx_add(row, r);
  double u[DT];
#pragma unroll
  for (int i = 0; i < DT; ++i) {
    u[i] = d[i] * is[i];
    fx_add(row + 2 * (1 + i), r * u[i]);
  }
  int o = 1 + DT;
#pragma unroll
  for (int i = 0; i < DT; ++i)
#pragma unroll
    for (int j = i; j < DT; ++j, ++o) fx_add(row + 2 * o, r * u[i] * u[j]);
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n, const int32_t* gate) {
  if (gate && gate[0] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ---- dispatch order of the culled sweep ------------------------------------------------------------
// Workgroups go to the eight XCDs in turn and each XCD takes one contiguous range of the point
// blocks (xcd_block). Within its range, an XCD starts the blocks predicted to take longest first
// (longest processing time first), so that the long blocks do not form the tail. A block's
// predicted cost is the longest time the previous launch on the same context measured for the
// blocks that covered the same stretch of the curve order: the previous blocks are in Hilbert
// order, so those from the one whose first code is the largest not above this block's first code
// to the one whose first code is the largest not above its last code (the same block when the
// points are the same, as in coordinate-ascent steps on one frame; its neighbours in space on a
// new frame, where a block that straddles a costly one is likely costly too). A range longer than
// BO_MAX, or a reset, keeps the curve order. Any order gives the same results.
constexpr int BO_SPAN = 32;  // previous blocks looked at per block
constexpr int BO_MAX = 4096;
constexpr int BO_LDS = 8192;  // previous blocks whose codes are searched in LDS

__global__ __launch_bounds__(1024) void k_block_order(float* __restrict__ bcost, const uint32_t* __restrict__ bcode,
                                                      const uint32_t* __restrict__ pcode, int64_t N, int64_t nb,
                                                      int64_t cap,
                                                      const int64_t* __restrict__ bprev,
                                                      int32_t* __restrict__ border, int reset) {
  __shared__ unsigned long long key[BO_MAX];
  const int tid = threadIdx.x, x = blockIdx.x;
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t start = x * per + (x < rem ? x : rem), len = per + (x < rem ? 1 : 0);
  if (reset) {
    for (int64_t i = (int64_t)x * 1024 + tid; i < cap; i += 8 * 1024) bcost[i] = 0.0f;
  }
  const int64_t np = reset ? 0 : bprev[0];
  if (reset || len > BO_MAX || np < 1 || np > cap) {
    for (int64_t i = tid; i < len; i += 1024) border[start + i] = (int32_t)(start + i);
    return;
  }
  // the previous launch's block codes in LDS for the searches below (when they fit)
  __shared__ uint32_t bcs[BO_LDS];
  const bool in_lds = np <= BO_LDS;
  if (in_lds)
    for (int64_t i = tid; i < np; i += 1024) bcs[i] = bcode[i];
  __syncthreads();
  int n2 = 1;
  while (n2 < len) n2 <<= 1;
  for (int i = tid; i < n2; i += 1024) {
    if (i < len) {
      // the previous blocks covering this block's first and last points: last code <= each (else
      // the first block)
      auto cover = [&](uint32_t code) {
        int64_t lo = 0, hi = np - 1;
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) >> 1;
          if ((in_lds ? bcs[mid] : bcode[mid]) <= code) lo = mid;
          else hi = mid - 1;
        }
        return lo;
      };
      const int64_t jf = (start + i) * 64, jl = min(jf + 63, N - 1);
      const int64_t b0 = cover(pcode[jf]), b1 = cover(pcode[jl]);
      float v = 0.0f;
      for (int64_t b = b0; b <= b1 && b < b0 + BO_SPAN; ++b) {
        const float c = bcost[b];
        v = c > v ? c : v;  // (NaN and negative costs count as 0)
      }
      key[i] = ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(v)) << 32) | (unsigned)i;
    } else {
      key[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < n2; i += 1024) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long u = key[i], v = key[ixj];
          if ((u > v) == ((i & k) == 0)) {
            key[i] = v;
            key[ixj] = u;
          }
        }
      }
      __syncthreads();
    }
  for (int i = tid; i < len; i += 1024) border[start + i] = (int32_t)(start + (int64_t)(key[i] & 0xFFFFFFFFull));
}

// ---- screen precision of the exact mode -------------------------------------------------------------
// The screen's error bound for a pair is eps |c_k| |phi_n| (log2 units). For the mean row and
// feature norms the split-BF16 bound (eps = 2^-12) is recorded in the frame; with VBGS_AUTO the FP32
// screen (eps = 2^-16) is taken when that bound exceeds AUTO_BUDGET (a loose screen records so
// many candidates that points overflow their lists). Two fixed-order stages (deterministic).
constexpr float AUTO_BUDGET = 32.0f;
constexpr int SCR_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_screen_part(const float* __restrict__ nc, int64_t nrow,
                                                     const float* __restrict__ nphi, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double a[256], b[256];
  const int t = threadIdx.x;
  const int64_t pr = (nrow + SCR_BLOCKS - 1) / SCR_BLOCKS, pn = (n + SCR_BLOCKS - 1) / SCR_BLOCKS;
  const int64_t r0 = blockIdx.x * pr, r1 = min(r0 + pr, nrow), n0 = blockIdx.x * pn, n1 = min(n0 + pn, n);
  double s = 0.0, u = 0.0;
  for (int64_t i = r0 + t; i < r1; i += 256) s += nc[i];
  for (int64_t i = n0 + t; i < n1; i += 256) u += nphi[i];
  a[t] = s;
  b[t] = u;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      a[t] += a[t + w];
      b[t] += b[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[blockIdx.x] = a[0];
    part[SCR_BLOCKS + blockIdx.x] = b[0];
  }
}

// force: the configured precision, or VBGS_AUTO to choose; gate[0] / gate[1]: run the split-BF16 /
// the FP32 screen
__global__ __launch_bounds__(256) void k_screen_pick(const double* __restrict__ part, int64_t K, int64_t n,
                                                     int force, FrameInfo* __restrict__ fr,
                                                     int32_t* __restrict__ gate) {
  __shared__ double a[256], b[256];
  const int t = threadIdx.x;
  a[t] = part[t];
  b[t] = part[SCR_BLOCKS + t];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      a[t] += a[t + w];
      b[t] += b[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const float slack = (float)((double)screen_eps(VBGS_BF16X3) * (a[0] / (double)K) * (b[0] / (double)n));
    const int prec = force != VBGS_AUTO ? force : (slack > AUTO_BUDGET ? VBGS_FP32 : VBGS_BF16X3);
    fr->screen_slack = slack;
    fr->screen_prec = prec;
    gate[0] = prec == VBGS_BF16X3 ? 1 : 0;
    gate[1] = prec == VBGS_FP32 ? 1 : 0;
  }
}

// ---- exact LSE of the recorded candidates, one thread per point ---------------------------------
template <int DT>
__global__ __launch_bounds__(256) void k_point_lse(const EArgs a) {
  __shared__ double red[256];
  if (a.gate && a.gate[0] == 0) return;
  const int tid = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * 256 + tid;
  double L2 = 0.0;
  unsigned kept = 0;
  if (p < a.N) {
    if (a.cand_n[p * 4] < 0) {
      L2 = a.lse2[p];  // overflowed point: full rescan by k_over_lse
    } else {
      const float* x = a.X + p * DT;
      double m = -INFINITY, l = 0.0;
      for (int g = 0; g < 4; ++g) {
        const int cnt = a.cand_n[p * 4 + g];
        const int64_t e0 = (p * 4 + g) * CS;
        // eight candidates at a time, so that their rows are fetched together
        for (int j = 0; j < cnt; j += 8) {
          int32_t kk[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) kk[u] = j + u < cnt ? a.cand_k[e0 + j + u] : -1;
          double sc[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            double d[DT];
            sc[u] = kk[u] >= 0 ? direct_score2_dt<DT>(a.direct + (int64_t)kk[u] * a.dts, x, d) : -INFINITY;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (kk[u] >= 0) {
              online_add(m, l, sc[u]);
              a.cand_s[e0 + j + u] = (float)sc[u];
            }
        }
      }
      L2 = m + log2(l);
      a.lse2[p] = L2;
      // keep the pairs that can carry mass (FP32 rounding is monotone, see evict_candidates)
      const float thr = (float)(L2 - (double)a.T2);
      for (int g = 0; g < 4; ++g)
        keep_pairs(a, (int32_t)p, a.cand_k + (p * 4 + g) * CS, a.cand_s + (p * 4 + g) * CS, a.cand_n[p * 4 + g], thr,
                   kept);
    }
    if (a.lse_out) a.lse_out[p] = L2 * LN2;
  }
  red[tid] = L2;
  count_refined(&a.frame->refined2, kept);
  __syncthreads();
  if (tid == 0) {
    double sacc = 0.0;
    for (int i = 0; i < 256; ++i) sacc += red[i];
    a.lse_part[blockIdx.x] = sacc;
  }
}

// After the culled sweep (which computed the LSE of its points) and the overflow rescan: per 256
// points the fixed-order partial sum of the LSEs for the ELBO, and the LSEs in nats if requested.
__global__ __launch_bounds__(256) void k_lse_finish(const EArgs a) {
  __shared__ double red[256];
  if (a.gate && a.gate[0] == 0) return;
  const int tid = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * 256 + tid;
  const double L2 = p < a.N ? a.lse2[p] : 0.0;
  if (p < a.N && a.lse_out) a.lse_out[p] = L2 * LN2;
  red[tid] = L2;
  __syncthreads();
  if (tid == 0) {
    double sacc = 0.0;
    for (int i = 0; i < 256; ++i) sacc += red[i];
    a.lse_part[blockIdx.x] = sacc;
  }
}

// ---- overflowed points: exact LSE over all K (one workgroup per point) --------------------------
// After the culled sweep the rescan visits only the rows whose bound reaches thr (the sweep's
// lower bound on the point's largest score minus the margin; tiles first, then rows); without
// culling it scores every component.
__device__ __forceinline__ float point_tile_d2(const TileInfo& t, const float* x3) {
  float d2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float gap = fmaxf(fmaxf(t.lo[i] - x3[i], x3[i] - t.hi[i]), 0.0f);
    d2 = fmaf(gap, gap, d2);
  }
  return d2;
}

__device__ __forceinline__ float point_row_d2(const RowBound& r, const float* x3) {
  float d2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float gap = fmaxf(fabsf(x3[i] - r.m[i]) - fabsf(r.m[i]) * 2.384185791015625e-7f, 0.0f);
    d2 = fmaf(gap, gap, d2);
  }
  return d2;
}

// call f(k) for every component whose bound with x reaches thr (culled) or for every component.
// Culled: each wave tests 64 tiles at a time (lane = tile), then the rows of the tiles that pass,
// two tiles at a time (lane = row), so that the row-bound loads of a tile are issued together.
// Needs a workgroup of whole waves.
template <int DT, typename F>
__device__ __forceinline__ void over_rows(const EArgs& a, const float* x, float thr, F&& f) {
  static_assert(CT == 64, "a tile's rows are one wave's lanes");
  if (a.cull) {
    float x3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) x3[i] = i < DT && i < a.nsp ? x[i] : 0.0f;
    const int64_t ntiles = a.Kpad / CT;
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    auto row_test = [&](int64_t row, const RowBound& rb) {
      if (row < a.K && rb.G - rb.Lam * point_row_d2(rb, x3) >= thr) f((int64_t)a.corder[row]);
    };
    for (int64_t base = (int64_t)(threadIdx.x >> 6) * 64; base < ntiles; base += (int64_t)nw * 64) {
      const int64_t t = base + lane;
      bool pass = false;
      if (t < ntiles) {
        const TileInfo ti = a.tinfo[t];
        pass = ti.G - ti.Lam * point_tile_d2(ti, x3) >= thr;
      }
      unsigned long long pm = __ballot(pass);
      while (pm) {
        const int i1 = __ffsll((long long)pm) - 1;
        pm &= pm - 1ull;
        const int i2 = pm ? __ffsll((long long)pm) - 1 : -1;
        if (pm) pm &= pm - 1ull;
        const int64_t r1 = (base + i1) * CT + lane;
        const int64_t r2 = i2 >= 0 ? (base + i2) * CT + lane : -1;
        RowBound b1{}, b2{};
        if (r1 < a.K) b1 = a.rowb[r1];
        if (r2 >= 0 && r2 < a.K) b2 = a.rowb[r2];
        row_test(r1, b1);
        if (r2 >= 0) row_test(r2, b2);
      }
    }
  } else {
    for (int64_t k = threadIdx.x; k < a.K; k += blockDim.x) f(k);
  }
}

template <int DT>
__global__ __launch_bounds__(256) void k_over_lse(const EArgs a) {
  __shared__ double sm[256], sl[256];
  if (a.gate && a.gate[0] == 0) return;
  const int n_over = a.frame->n_over;
  for (int i = blockIdx.x; i < n_over; i += gridDim.x) {
    const int64_t p = a.over_list[i];
    const float* x = a.X + p * DT;
    double m = -INFINITY, l = 0.0;
    const float thr = a.cull ? (float)a.lse2[p] - a.T2 - 1.0f : 0.0f;
    over_rows<DT>(a, x, thr, [&](int64_t k) {
      double d[DT];
      online_add(m, l, direct_score2_dt<DT>(a.direct + k * a.dts, x, d));
    });
    sm[threadIdx.x] = m;
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        double mm = sm[threadIdx.x], ll = sl[threadIdx.x];
        lse_merge(mm, ll, sm[threadIdx.x + w], sl[threadIdx.x + w]);
        sm[threadIdx.x] = mm;
        sl[threadIdx.x] = ll;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) a.lse2[p] = sm[0] + log2(sl[0]);
    __syncthreads();
  }
}

// ---- rendering: colour expected at each query position ------------------------------------------
// sum_k r_k(x) (m_c,k + B_k (x - m_s,k)) with r_k(x) = exp2(s2_k(x) - LSE2(x)) the responsibilities of
// the position marginal; reg[k] = [m_c (Dc), B (Dc x DT)]. One thread per point over its kept
// candidates (exact MFMA mode) or over every component (FP64 mode); overflowed points are left to
// k_render_over.
constexpr int RMAX = MAXD;

template <int DT>
__device__ __forceinline__ void render_add(double* acc, int Dc, const double* __restrict__ g, const double* d,
                                           double r) {
#pragma unroll
  for (int c = 0; c < RMAX; ++c)
    if (c < Dc) {
      double v = g[c];
#pragma unroll
      for (int j = 0; j < DT; ++j) v = fma(g[Dc + c * DT + j], d[j], v);
      acc[c] = fma(r, v, acc[c]);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_render_points(const EArgs a, const double* __restrict__ reg, int Dc,
                                                       int dense, float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= a.N) return;
  if (!dense && a.cand_n[p * 4] < 0) return;
  const int rs = Dc * (1 + DT);
  const double L2 = a.lse2[p];
  const float* x = a.X + p * DT;
  double acc[RMAX];
#pragma unroll
  for (int c = 0; c < RMAX; ++c) acc[c] = 0.0;
  double d[DT];
  if (dense) {
    for (int64_t k = 0; k < a.K; ++k) {
      const double s2 = direct_score2_dt<DT>(a.direct + k * a.dts, x, d);
      render_add<DT>(acc, Dc, reg + k * rs, d, exp2(s2 - L2));
    }
  } else {
    for (int g = 0; g < 4; ++g) {
      const int cnt = a.cand_n[p * 4 + g];
      for (int j = 0; j < cnt; ++j) {
        const int32_t k = a.cand_k[(p * 4 + g) * CS + j];
        if (k < 0) continue;
        const double s2 = direct_score2_dt<DT>(a.direct + (int64_t)k * a.dts, x, d);
        render_add<DT>(acc, Dc, reg + (int64_t)k * rs, d, exp2(s2 - L2));
      }
    }
  }
#pragma unroll
  for (int c = 0; c < RMAX; ++c)
    if (c < Dc) out[p * Dc + c] = (float)acc[c];
}

// overflowed points: one workgroup per point over the rows its bound reaches (or every component)
template <int DT>
__global__ __launch_bounds__(256) void k_render_over(const EArgs a, const double* __restrict__ reg, int Dc,
                                                     float* __restrict__ out) {
  __shared__ double red[RMAX][256];
  const int n_over = a.frame->n_over;
  const int rs = Dc * (1 + DT);
  for (int i = blockIdx.x; i < n_over; i += gridDim.x) {
    const int64_t p = a.over_list[i];
    const double L2 = a.lse2[p];
    const float* x = a.X + p * DT;
    double acc[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) acc[c] = 0.0;
    over_rows<DT>(a, x, (float)L2 - a.T2 - 1.0f, [&](int64_t k) {
      double d[DT];
      const double s2 = direct_score2_dt<DT>(a.direct + k * a.dts, x, d);
      render_add<DT>(acc, Dc, reg + k * rs, d, exp2(s2 - L2));
    });
#pragma unroll
    for (int c = 0; c < RMAX; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
#pragma unroll
        for (int c = 0; c < RMAX; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
      }
      __syncthreads();
    }
    if ((int)threadIdx.x < Dc) out[p * Dc + threadIdx.x] = (float)red[threadIdx.x][0];
    __syncthreads();
  }
}

// ---- overflowed points: statistics of every pair within the margin (fixed-point atomics) --------
template <int DT>
__global__ __launch_bounds__(256) void k_over_stats(const EArgs a) {
  const int n_over = a.frame->n_over;
  double is[DT];
#pragma unroll
  for (int i = 0; i < DT; ++i) is[i] = 1.0 / a.frame->s[i];
  for (int i = blockIdx.x; i < n_over; i += gridDim.x) {
    const int64_t p = a.over_list[i];
    const double L2 = a.lse2[p];
    const float* x = a.X + p * DT;
    over_rows<DT>(a, x, (float)L2 - a.T2 - 1.0f, [&](int64_t k) {
      double d[DT];
      const double s2 = direct_score2_dt<DT>(a.direct + k * a.dts, x, d);
      if (s2 >= L2 - (double)a.T2) fx_pair<DT>(a.fx, k, exp2(s2 - L2), d, is);
    });
  }
}

// ---- transpose of the kept pairs: exclusive scan of the per-component counts (one workgroup) ----
// exclusive scan of the per-component pair counts (off[K] = total) in two coalesced steps: block
// sums, then the local scans, each block adding the sums of the blocks before it
constexpr int SCAN_B = 1024;
// (gate: when set, the scan runs only if gate[0] != 0)
__global__ __launch_bounds__(256) void k_scan_blocks(const int32_t* __restrict__ cnt, int64_t K,
                                                     int32_t* __restrict__ bsum, const int32_t* gate) {
  if (gate && gate[0] == 0) return;
  __shared__ int32_t red[256];
  const int t = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * SCAN_B + 4 * t;
  int32_t v = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) v += k0 + i < K ? cnt[k0 + i] : 0;
  red[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) bsum[blockIdx.x] = red[0];
}

__device__ __forceinline__ int32_t block_excl_scan256(int32_t v, int32_t* sh, int32_t& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = 1; w < 256; w <<= 1) {
    const int32_t u = t >= w ? sh[t - w] : 0;
    __syncthreads();
    sh[t] += u;
    __syncthreads();
  }
  total = sh[255];
  const int32_t r = sh[t] - v;
  __syncthreads();
  return r;
}

// each block starts from the sum of the block sums before it (a strided sum and a tree in LDS);
// the last block also writes the total
__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ cnt, int64_t K,
                                                    const int32_t* __restrict__ bsum, int32_t* __restrict__ off,
                                                    const int32_t* gate) {
  if (gate && gate[0] == 0) return;
  __shared__ int32_t sh[256];
  const int t = threadIdx.x;
  int32_t pre = 0;
  for (int64_t b = t; b < (int64_t)blockIdx.x; b += 256) pre += bsum[b];
  sh[t] = pre;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const int32_t base = sh[0];
  __syncthreads();
  const int64_t k0 = (int64_t)blockIdx.x * SCAN_B + 4 * t;
  int32_t c[4], v = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c[i] = k0 + i < K ? cnt[k0 + i] : 0;
    v += c[i];
  }
  int32_t total;
  int32_t run = base + block_excl_scan256(v, sh, total);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (k0 + i < K) off[k0 + i] = run;
    run += c[i];
  }
  if (blockIdx.x == gridDim.x - 1 && t == 255) off[K] = run;
}

// Segments of the kept pairs for the next culled sweep, from the counts of the last one (read
// before they are cleared): component k gets 3 c_k + 32 slots (c_k clamped to [0, 2^24]), in
// component order, the starts clamped to the capacity of ent_n, so that the segments never overlap
// whatever the counts hold (a pair that finds no room sets the miss flag). Clears the flag. One
// workgroup, each thread a contiguous range of components.
constexpr int SEG_T = 1024;
__device__ __forceinline__ long long seg_slots(int32_t c) { return 3ll * min(max(c, 0), 1 << 24) + 32; }

// (cnt holds Kpad + 1 >= K + 1 entries and seg Kpad, Kpad a multiple of 64, so the 16-byte
// accesses of a range that starts at a multiple of 4 below K stay inside them)
__global__ __launch_bounds__(SEG_T) void k_seg_layout(const int32_t* __restrict__ cnt, int64_t K, int64_t cap,
                                                      int2* __restrict__ seg, int32_t* __restrict__ miss) {
  __shared__ long long wsum[SEG_T / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t per = ((K + SEG_T - 1) / SEG_T + 3) / 4 * 4;
  const int64_t k0 = min(K, (int64_t)t * per), k1 = min(K, k0 + per);
  long long s = 0;
#pragma unroll 4
  for (int64_t k = k0; k < k1; k += 4) {
    const int4 v = *reinterpret_cast<const int4*>(cnt + k);
    s += seg_slots(v.x) + (k + 1 < k1 ? seg_slots(v.y) : 0) + (k + 2 < k1 ? seg_slots(v.z) : 0) +
         (k + 3 < k1 ? seg_slots(v.w) : 0);
  }
  long long x = s;  // inclusive scan over the workgroup
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  long long off = x - s;
  for (int q = 0; q < w; ++q) off += wsum[q];
  // (the entries past K - 1 in the last group are written too and never read)
#pragma unroll 4
  for (int64_t k = k0; k < k1; k += 4) {
    const int4 v = *reinterpret_cast<const int4*>(cnt + k);
    int32_t o[5];
    o[0] = (int32_t)min(off, (long long)cap);
    off += seg_slots(v.x);
    o[1] = (int32_t)min(off, (long long)cap);
    off += seg_slots(v.y);
    o[2] = (int32_t)min(off, (long long)cap);
    off += seg_slots(v.z);
    o[3] = (int32_t)min(off, (long long)cap);
    off += seg_slots(v.w);
    o[4] = (int32_t)min(off, (long long)cap);
    int4* s4 = reinterpret_cast<int4*>(seg + k);
    s4[0] = int4{o[0], o[1], o[1], o[2]};
    s4[1] = int4{o[2], o[3], o[3], o[4]};
  }
  if (t == 0) miss[0] = 0;
}

hipError_t launch_seg_layout(const DevPtrs& d, hipStream_t s) {
  const Layout& L = *d.L;
  const int64_t cap = L.ent_cap < INT32_MAX ? L.ent_cap : INT32_MAX;
  hipLaunchKernelGGL(k_seg_layout, dim3(1), dim3(SEG_T), 0, s, d.at<int32_t>(L.ccount), d.K, cap,
                     d.at<int2>(L.segoff), d.at<int32_t>(L.seg_miss));
  return hipGetLastError();
}

// exclusive scan of n counts: off[i] = sum_{j < i} cnt[j], off[n] = total; part: ceil(n / SCAN_B) + 1
hipError_t launch_excl_scan(const int32_t* cnt, int64_t n, int32_t* off, int32_t* part, hipStream_t s) {
  const int64_t nsb = (n + SCAN_B - 1) / SCAN_B;
  if (nsb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nsb), dim3(256), 0, s, cnt, n, part, (const int32_t*)nullptr);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nsb), dim3(256), 0, s, cnt, n, part, off, (const int32_t*)nullptr);
  return hipGetLastError();
}

// one thread per candidate list (point i / 4, list i % 4): each kept pair goes to its component's
// segment at the rank it drew when it was kept (keep_pairs)
// (a grid of at most SCATTER_BLOCKS workgroups, each list taken by the thread i = list mod stride:
// with segments and no miss the launch is a few workgroups that exit at once)
constexpr int SCATTER_BLOCKS = 2048;
__global__ __launch_bounds__(256) void k_scatter_pairs(const EArgs a) {
  if (a.seg && *a.seg_miss == 0) return;  // every pair is in its segment already
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.N * 4; i += (int64_t)gridDim.x * 256) {
    const int64_t p = i >> 2;
    const int cnt = a.cand_n[i];
    if (cnt <= 0 || a.cand_n[p * 4] < 0) continue;  // (an overflowed point: the rescan's statistics)
    const int32_t* ck = a.cand_k + i * CS;
    const float* cs = a.cand_s + i * CS;
    for (int j0 = 0; j0 < cnt; j0 += 8) {
      int32_t k[8], r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        k[u] = j0 + u < cnt ? ck[j0 + u] : -1;
        r[u] = j0 + u < cnt ? __float_as_int(cs[j0 + u]) : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k[u] >= 0) a.ent_n[a.coffset[k[u]] + r[u]] = (int32_t)p;
    }
  }
}

// ---- per-component exact statistics: 128-bit fixed-point sums in registers ----------------------
// The sum of integers does not depend on the order of the pairs, so the scatter order above does
// not affect the result (bitwise reproducible).
struct Fx128 {
  unsigned long long lo;
  long long hi;
  double hd;  // more of hi, summed in FP64 by fx_acc_small
};

__device__ __forceinline__ void fx_acc(Fx128& a, double v) {
  unsigned long long lo;
  const double hi_d = fx_split(v, lo);
  a.lo += lo;
  a.hi += (long long)hi_d + (a.lo < lo ? 1 : 0);
}

// fx_acc for |v| < 2^26: the integer parts are summed in FP64, exactly (fewer than 2^25 terms per
// sum, since N < 2^25, so every partial sum stays below 2^52)
__device__ __forceinline__ void fx_acc_small(Fx128& a, double v) {
  unsigned long long lo;
  const double hi_d = fx_split(v, lo);
  a.lo += lo;
  a.hd += hi_d + (a.lo < lo ? 1.0 : 0.0);
}

// hi with the FP64 part folded in
__device__ __forceinline__ void fx_fold(Fx128& a) {
  a.hi += (long long)a.hd;
  a.hd = 0.0;
}

// the record of one pair keeps every product r u_i u_j below 2^26 (r <= 1): all |u_i| < 2^13
template <int DT>
__device__ __forceinline__ bool small_offsets(const double* u) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < DT; ++i) ok = ok && fabs(u[i]) < 8192.0;
  return ok;
}

// A component with more than HEAVY kept pairs is summed by a whole workgroup (k_comp_stats_heavy),
// so that no lane group walks a long list; 128-bit integer sums do not depend on how the pairs are
// split among lanes.
constexpr int HEAVY = 4096;
constexpr int SG = 32;  // lanes per component group in the statistics kernels

// The statistics of component k in raw coordinates: lane f of a group of SG lanes starting at lane
// gb holds sum f centred at the component's mean m_k (v); the group's N_k and first moments come
// by shuffles, and x = m_k + d gives N, S1 = m N + S1', S2_ij = m_i m_j N + m_i S1'_j + m_j S1'_i + S2'_ij.
// Every lane of the wave takes part in the shuffles; `own` lanes write.
template <int DT>
__device__ __forceinline__ void comp_stats_emit(const EArgs& a, int64_t k, int f, int fi, int fj, double v, int gb,
                                                bool own) {
  constexpr int F = 1 + DT + DT * (DT + 1) / 2;
  const double Nk = __shfl(v, gb);
  const double ai = __shfl(v, gb + 1 + (fi >= 0 ? fi : 0));
  const double aj = __shfl(v, gb + 1 + (fj >= 0 ? fj : 0));
  if (!own) return;
  double o = v;
  if (fi >= 0) {
    const double mi = a.direct[k * a.dts + 1 + fi];
    if (fj < 0) {
      o = mi * Nk + v;
    } else {
      const double mj = a.direct[k * a.dts + 1 + fj];
      o = mi * mj * Nk + mi * aj + mj * ai + v;
    }
  }
  a.stats[k * F + f] = o;
  if (a.stats_out) a.stats_out[k * F + f] = o;
}

// Components with more than HEAVY pairs, one workgroup of 256 lanes per component (the workgroup
// of components [64 b, 64 b + 64) takes its heavy ones in turn). Each chunk of 256 pairs is scored
// one pair per lane into LDS; then group j of SG lanes takes pairs [SG j, SG j + SG) of the chunk,
// lane f adding feature f into its 128-bit sum; the groups' sums of each feature are added last.
template <int DT>
__global__ __launch_bounds__(256) void k_comp_stats_heavy(const EArgs a) {
  constexpr int F = 1 + DT + DT * (DT + 1) / 2;
  constexpr int R = 2 + DT, NG = 256 / SG;  // per pair: r, u[DT], 1
  __shared__ double buf[256 * R];
  __shared__ Fx128 part[NG][SG];
  __shared__ int32_t heavy[64];
  __shared__ int nheavy;
  const int tid = threadIdx.x, grp = tid / SG, l = tid % SG;
  if (tid == 0) nheavy = 0;
  __syncthreads();
  if (tid < 64) {
    const int64_t k = (int64_t)blockIdx.x * 64 + tid;
    int32_t e0 = 0, e1 = 0;
    if (k < a.K) pair_range(a, k, e0, e1);
    if (e1 - e0 > HEAVY) heavy[atomicAdd(&nheavy, 1)] = (int32_t)k;
  }
  __syncthreads();
  const int nh = nheavy;
  if (nh == 0) return;
  int fi = l >= 1 && l <= DT ? l - 1 : -1, fj = -1;
  {
    int o = 1 + DT;
#pragma unroll
    for (int i = 0; i < DT; ++i)
#pragma unroll
      for (int j = i; j < DT; ++j, ++o)
        if (o == l) {
          fi = i;
          fj = j;
        }
  }
  // the slots this lane multiplies: r u_i u_j as (r u_i) u_j, an absent factor reading the 1
  const int ia = fi >= 0 ? 1 + fi : R - 1, ib = fj >= 0 ? 1 + fj : R - 1;
  double is[DT];
#pragma unroll
  for (int i = 0; i < DT; ++i) is[i] = 1.0 / a.frame->s[i];
  for (int h = 0; h < nh; ++h) {
    const int64_t k = heavy[h];
    Fx128 acc;  // group 0 starts from the overflowed points' contributions
    acc.lo = grp == 0 && l < F ? a.fx[(k * FP + l) * 2] : 0ull;
    acc.hi = grp == 0 && l < F ? (long long)a.fx[(k * FP + l) * 2 + 1] : 0ll;
    acc.hd = 0.0;
    const double* row = a.direct + k * a.dts;
    int32_t e0, e1;
    pair_range(a, k, e0, e1);
    for (int32_t c0 = e0; c0 < e1; c0 += 256) {
      const int m = min(256, e1 - c0);
      bool small = true;
      if (tid < m) {
        const int64_t n = a.ent_n[c0 + tid];
        double d[DT];
        const double s2 = direct_score2_dt<DT>(row, a.X + n * DT, d);
        buf[tid * R] = exp2(s2 - a.lse2[n]);
#pragma unroll
        for (int i = 0; i < DT; ++i) buf[tid * R + 1 + i] = d[i] * is[i];
        buf[tid * R + R - 1] = 1.0;
        small = small_offsets<DT>(buf + tid * R + 1);
      }
      const bool all_small = __syncthreads_and(small ? 1 : 0);
      if (l < F) {
        const int q1 = min(m, grp * SG + SG);
        if (all_small) {
          for (int q = grp * SG; q < q1; ++q) {
            const double* rq = buf + q * R;
            fx_acc_small(acc, (rq[0] * rq[ia]) * rq[ib]);
          }
        } else {
          for (int q = grp * SG; q < q1; ++q) {
            const double* rq = buf + q * R;
            fx_acc(acc, (rq[0] * rq[ia]) * rq[ib]);
          }
        }
      }
      __syncthreads();
    }
    fx_fold(acc);
    part[grp][l] = acc;
    __syncthreads();
    const bool own = grp == 0 && l < F;
    double v = 0.0;
    if (own) {
#pragma unroll
      for (int j = 1; j < NG; ++j) {
        const Fx128 o = part[j][l];
        const unsigned long long lo = acc.lo + o.lo;
        acc.hi += o.hi + (lo < o.lo ? 1 : 0);
        acc.lo = lo;
      }
      v = (double)acc.hi + (double)acc.lo * 5.42101086242752217e-20;
      if (fi >= 0) v = v * a.frame->s[fi];
      if (fj >= 0) v = v * a.frame->s[fj];
    }
    comp_stats_emit<DT>(a, k, l, fi, fj, v, (threadIdx.x & 63) & ~(SG - 1), own);
    __syncthreads();
  }
}

// One group of SG lanes per component with at most HEAVY pairs (the others: k_comp_stats_heavy).
// The pairs are taken SG at a time: each lane scores one pair (its responsibility r and scaled
// offset u) into LDS, then lane f < F adds feature f (r, r u_i or r u_i u_j) of every pair of the
// chunk into its own 128-bit sum, so no lane holds more than one sum.
template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_comp_stats(const EArgs a) {
  constexpr int F = 1 + DT + DT * (DT + 1) / 2;
  constexpr int R = 2 + DT;  // per pair: r, u[DT], 1
  __shared__ double buf[256 / SG][SG * R];
  __shared__ f64x2 rows[256 / SG][16];  // each group's component row (direct form, 32 doubles)
  const int grp = threadIdx.x / SG, l = threadIdx.x % SG;
  const int64_t k = (int64_t)blockIdx.x * (256 / SG) + grp;
  int32_t e0 = 0, e1 = 0;
  if (k < a.K) pair_range(a, k, e0, e1);
  const bool val = k < a.K && e1 - e0 <= HEAVY;  // uniform over the group
  // the feature this lane sums: r (l = 0), r u_i (l = 1 + i), r u_i u_j (i <= j, row-major)
  int fi = l >= 1 && l <= DT ? l - 1 : -1, fj = -1;
  {
    int o = 1 + DT;
#pragma unroll
    for (int i = 0; i < DT; ++i)
#pragma unroll
      for (int j = i; j < DT; ++j, ++o)
        if (o == l) {
          fi = i;
          fj = j;
        }
  }
  // the slots this lane multiplies: r u_i u_j as (r u_i) u_j, an absent factor reading the 1
  const int ia = fi >= 0 ? 1 + fi : R - 1, ib = fj >= 0 ? 1 + fj : R - 1;
  const bool mine = val && l < F;
  Fx128 acc;  // starts from the overflowed points' contributions
  acc.lo = mine ? a.fx[(k * FP + l) * 2] : 0ull;
  acc.hi = mine ? (long long)a.fx[(k * FP + l) * 2 + 1] : 0ll;
  acc.hd = 0.0;
  if (val) {
    double is[DT];
#pragma unroll
    for (int i = 0; i < DT; ++i) is[i] = 1.0 / a.frame->s[i];
    // the row once per group in LDS, read by every pair's score (instead of 28 registers per lane)
    static_assert(SG >= 16, "row copy");
    if (l < 16) rows[grp][l] = reinterpret_cast<const f64x2*>(a.direct + k * a.dts)[l];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double* row = reinterpret_cast<const double*>(rows[grp]);
    double* rec = buf[grp];
    for (int32_t c0 = e0; c0 < e1; c0 += SG) {
      const int m = min(SG, e1 - c0);
      bool small = true;
      if (l < m) {
        const int64_t n = a.ent_n[c0 + l];
        double d[DT];
        const double s2 = direct_score2_dt<DT>(row, a.X + n * DT, d);
        rec[l * R] = exp2(s2 - a.lse2[n]);
#pragma unroll
        for (int i = 0; i < DT; ++i) rec[l * R + 1 + i] = d[i] * is[i];
        rec[l * R + R - 1] = 1.0;
        small = small_offsets<DT>(rec + l * R + 1);
      }
      const bool all_small = __ballot(!small) == 0ull;  // (both groups of the wave)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (l < F) {
        if (all_small) {
#pragma unroll 2
          for (int q = 0; q < m; ++q) {
            const double* rq = rec + q * R;
            fx_acc_small(acc, (rq[0] * rq[ia]) * rq[ib]);
          }
        } else {
#pragma unroll 2
          for (int q = 0; q < m; ++q) {
            const double* rq = rec + q * R;
            fx_acc(acc, (rq[0] * rq[ia]) * rq[ib]);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  double v = 0.0;
  if (mine) {  // fixed point -> FP64, undo the scaling; raw coordinates centred at m_k
    fx_fold(acc);
    v = (double)acc.hi + (double)acc.lo * 5.42101086242752217e-20;
    if (fi >= 0) v = v * a.frame->s[fi];
    if (fj >= 0) v = v * a.frame->s[fj];
  }
  comp_stats_emit<DT>(a, k, l, fi, fj, v, (threadIdx.x & 63) & ~(SG - 1), mine);
}

__global__ void k_zero_i32(int32_t* p, int64_t n, const int32_t* gate) {
  if (gate && gate[0] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
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
template <int D>
__global__ void k_fold(const double* __restrict__ spart, int nsplit, int64_t Kpad, int64_t K,
                       const FrameInfo* __restrict__ fr, const double* __restrict__ direct, int dts, int mode,
                       double* __restrict__ stats, double* __restrict__ stats_out) {
  // mode 0: partials are raw; 1: centred/scaled frame coordinates x' = (x - mu) / s;
  // 2: raw coordinates centred at the component's own mean m_k
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  constexpr int F = 1 + D + D * (D + 1) / 2, SS = D <= 6 ? 32 : 48;
  double v[F];
#pragma unroll
  for (int i = 0; i < F; ++i) {
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += spart[((int64_t)q * Kpad + k) * SS + i];
    v[i] = s;
  }
  double o[F];
  if (mode == 0) {
#pragma unroll
    for (int i = 0; i < F; ++i) o[i] = v[i];
  } else {
    // x = mu + s x':  S1 = mu N + s S1',  S2_ij = mu_i mu_j N + mu_i s_j S1'_j + s_i mu_j S1'_i + s_i s_j S2'_ij
    double mu[D], sc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      mu[i] = mode == 1 ? (double)fr->mu[i] : direct[k * dts + 1 + i];
      sc[i] = mode == 1 ? fr->s[i] : 1.0;
    }
    const double Nk = v[0];
    o[0] = Nk;
#pragma unroll
    for (int i = 0; i < D; ++i) o[1 + i] = mu[i] * Nk + sc[i] * v[1 + i];
    int t = 1 + D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i; j < D; ++j, ++t)
        o[t] = mu[i] * mu[j] * Nk + mu[i] * sc[j] * v[1 + j] + sc[i] * mu[j] * v[1 + i] + sc[i] * sc[j] * v[t];
  }
#pragma unroll
  for (int i = 0; i < F; ++i) {
    stats[k * F + i] = o[i];
    if (stats_out) stats_out[k * F + i] = o[i];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// exact mode: screen sweep recording candidates, then the exact LSE (overflowed points first);
// every kernel honours a.gate
// the three stages of the exact E-step over all pairs: clear the transpose counters, screen
// (sweep), exact per-point LSE from the candidate lists
static hipError_t exact_stage(const EArgs& a, int prec, int D, int64_t N, hipStream_t s, int cull, int stage) {
  if (N <= 0) return hipSuccess;
  if (stage == 0) {
    const int64_t Kp1 = a.Kpad + 1;
    hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, a.ccount, Kp1, a.gate);
    hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, s, a.fx, a.Kpad * FP * 2, a.gate);
  } else if (stage == 1) {  // the screen's choice (needs the component rows)
    hipLaunchKernelGGL(k_screen_part, dim3(SCR_BLOCKS), dim3(256), 0, s, a.nc, a.Kpad, a.nphi, N, a.scr_part);
    hipLaunchKernelGGL(k_screen_pick, dim3(1), dim3(256), 0, s, a.scr_part, a.K, N, prec, a.frame, a.scr_gate);
  } else if (stage == 4) {  // with culling, the blocks' dispatch order (needs the point order only)
    if (cull)
      hipLaunchKernelGGL(k_block_order, dim3(8), dim3(1024), 0, s, a.bcost, a.bcode, a.pcode, N, (int64_t)((N + 63) / 64),
                         a.nb_cap, a.bprev, a.border, a.order_reset);
  } else if (stage == 3) {  // the screening sweep
    const dim3 grid((unsigned)((N + P1_PTS - 1) / P1_PTS));
    // VBGS_AUTO: both screens are enqueued, each gated by the choice (the other exits at once)
    EArgs ab = a, af = a;
    if (prec == VBGS_AUTO) {
      ab.gate = a.scr_gate;
      ab.eps = screen_eps(VBGS_BF16X3);
      af.gate = a.scr_gate + 1;
      af.eps = screen_eps(VBGS_FP32);
    }
    const bool run_bf3 = prec == VBGS_BF16X3 || prec == VBGS_AUTO, run_f32 = prec == VBGS_FP32 || prec == VBGS_AUTO;
    if (cull) {
      const dim3 gw((unsigned)((N + 63) / 64));  // one 64-point wave per workgroup
      if (run_f32) hipLaunchKernelGGL((k_sweep<VBGS_FP32>), gw, dim3(64), 0, s, af);
      if (prec == VBGS_BF16) hipLaunchKernelGGL((k_sweep<VBGS_BF16>), gw, dim3(64), 0, s, a);
      if (run_bf3) hipLaunchKernelGGL((k_sweep<VBGS_BF16X3>), gw, dim3(64), 0, s, ab);
      if (prec == VBGS_FP64_CULLED) hipLaunchKernelGGL((k_sweep<VBGS_FP64_CULLED>), gw, dim3(64), 0, s, a);
    } else {
      if (run_f32) hipLaunchKernelGGL((k_pass1<VBGS_FP32, true>), grid, dim3(256), 0, s, af);
      if (prec == VBGS_BF16) hipLaunchKernelGGL((k_pass1<VBGS_BF16, true>), grid, dim3(256), 0, s, a);
      if (run_bf3) hipLaunchKernelGGL((k_pass1<VBGS_BF16X3, true>), grid, dim3(256), 0, s, ab);
    }
  } else {
    const dim3 gp((unsigned)((N + 255) / 256));
    switch (D) {
#define VB_LSE(DD)                                                                   \
  case DD:                                                                           \
    hipLaunchKernelGGL(k_over_lse<DD>, dim3(256), dim3(256), 0, s, a);                \
    if (cull) hipLaunchKernelGGL(k_lse_finish, gp, dim3(256), 0, s, a); /* LSE: sweep */ \
    else hipLaunchKernelGGL(k_point_lse<DD>, gp, dim3(256), 0, s, a);                \
    break;
      VB_LSE(1) VB_LSE(2) VB_LSE(3) VB_LSE(4) VB_LSE(5) VB_LSE(6)
#undef VB_LSE
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_exact_sweep(const EArgs& a, int prec, int D, int64_t N, hipStream_t s, int cull) {
  hipError_t e = hipSuccess;
  for (const int stage : {0, 4, 1, 3, 2})
    if (e == hipSuccess) e = exact_stage(a, prec, D, N, s, cull, stage);
  return e;
}

// exact LSE of externally provided candidate lists (counts are zeroed here, ungated)
hipError_t launch_point_lse(const EArgs& a, int D, int64_t N, hipStream_t s) {
  const int64_t Kp1 = a.Kpad + 1;
  hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, a.ccount, Kp1, nullptr);
  hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, s, a.fx, a.Kpad * FP * 2, nullptr);
  if (N <= 0) return hipGetLastError();
  EArgs u = a;
  u.gate = nullptr;
  const dim3 gp((unsigned)((N + 255) / 256));
  switch (D) {
#define VB_PL(DD) \
  case DD:        \
    hipLaunchKernelGGL(k_point_lse<DD>, gp, dim3(256), 0, s, u); break;
    VB_PL(1) VB_PL(2) VB_PL(3) VB_PL(4) VB_PL(5) VB_PL(6)
#undef VB_PL
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// statistics of the kept candidates: overflowed points (atomics), transpose, per-component sums
hipError_t launch_sparse_stats(const EArgs& a, int D, int64_t N, hipStream_t s) {
  if (N > 0) {
    const int64_t ng = (4 * N + 255) / 256;
    const dim3 gp((unsigned)(ng < SCATTER_BLOCKS ? ng : SCATTER_BLOCKS));  // k_scatter_pairs
    const int64_t nsb = (a.K + SCAN_B - 1) / SCAN_B;
    const int32_t* miss = a.seg ? a.seg_miss : nullptr;  // with segments, the scan only after a miss
    switch (D) {
#define VB_ST(DD)                                                                         \
  case DD:                                                                                \
    hipLaunchKernelGGL(k_over_stats<DD>, dim3(256), dim3(256), 0, s, a);                  \
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nsb), dim3(256), 0, s, a.ccount, a.K, a.scan_part, miss); \
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nsb), dim3(256), 0, s, a.ccount, a.K, a.scan_part,         \
                       a.coffset, miss);                                                                       \
    hipLaunchKernelGGL(k_scatter_pairs, gp, dim3(256), 0, s, a);                          \
    hipLaunchKernelGGL(k_comp_stats<DD>, dim3((unsigned)((a.K + 256 / SG - 1) / (256 / SG))), dim3(256), 0, s, a); \
    hipLaunchKernelGGL(k_comp_stats_heavy<DD>, dim3((unsigned)((a.K + 63) / 64)), dim3(256), 0, s, a); \
    break;
      VB_ST(1) VB_ST(2) VB_ST(3) VB_ST(4) VB_ST(5) VB_ST(6)
#undef VB_ST
      default:
        return hipErrorInvalidValue;
    }
  } else {  // no points: zero statistics
    const int64_t nst = a.K * (1 + D + D * (D + 1) / 2);
    hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(a.stats), nst,
                       nullptr);
    if (a.stats_out)
      hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(a.stats_out),
                         nst, nullptr);
  }
  return hipGetLastError();
}

EArgs make_eargs(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out) {
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
  a.phi8 = d.at<uint8_t>(L.phi8);
  a.phis = d.at<float>(L.phis);
  a.c8 = d.at<uint8_t>(L.c8);
  a.cs8 = d.at<float>(L.cs8);
  a.lse2 = d.at<double>(L.lse2);
  a.lse_part = d.at<double>(L.lse_part);
  a.lse_out = lse_out;
  a.spart = d.at<double>(L.spart);
  a.stats = d.at<double>(L.stats);
  a.stats_out = nullptr;
  a.cand_k = d.at<int32_t>(L.cand_k);
  a.cand_s = d.at<float>(L.cand_s);
  a.cand_n = d.at<int32_t>(L.cand_n);
  a.over_list = d.at<int32_t>(L.over_list);
  a.fx = d.at<unsigned long long>(L.fx);
  a.ccount = d.at<int32_t>(L.ccount);
  a.coffset = d.at<int32_t>(L.coffset);
  a.seg = c.seg ? d.at<int2>(L.segoff) : nullptr;
  a.seg_miss = d.at<int32_t>(L.seg_miss);
  a.ent_n = d.at<int32_t>(L.ent_n);
  a.frame = d.frame();
  a.gate = c.gate;
  a.porder = d.at<int32_t>(L.porder);
  a.pcode = d.at<uint32_t>(L.pcode);
  a.corder = d.at<int32_t>(L.corder);
  a.tinfo = d.at<TileInfo>(L.tinfo);
  a.rowb = d.at<RowBound>(L.rowb);
  a.ncg = d.at<f32x4>(L.ncg);
  a.scan_part = d.at<int32_t>(L.scan_part);
  a.N = N;
  a.K = d.K;
  a.Kpad = L.Kpad;
  a.D = d.D;
  a.dts = direct_stride(d.D);
  a.nsplit = c.nsplit;
  a.T2 = c.T2;
  a.cull = c.cull;
  a.nsp = d.nsp;
  a.slist = d.at<uint32_t>(L.slist);
  a.bcost = d.at<float>(L.bcost);
  a.bcode = d.at<uint32_t>(L.bcode);
  a.border = d.at<int32_t>(L.border);
  a.bprev = d.at<int64_t>(L.bprev);
  a.nb_cap = (L.bcode - L.bcost) / 4;
  a.scr_part = d.at<double>(L.scr_part);
  a.scr_gate = d.at<int32_t>(L.scr_gate);
  a.order_reset = c.order_reset;
  a.eps = screen_eps(c.prec);
  return a;
}

hipError_t launch_render(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, const double* reg, int Dc,
                         float* out, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const EArgs a = make_eargs(d, c, X, N, nullptr);
  const int dense = c.prec == VBGS_FP64 ? 1 : 0;
  const dim3 gp((unsigned)((N + 255) / 256));
  switch (d.D) {
#define VB_RD(DD)                                                                              \
  case DD:                                                                                     \
    if (!dense) hipLaunchKernelGGL(k_render_over<DD>, dim3(256), dim3(256), 0, s, a, reg, Dc, out); \
    hipLaunchKernelGGL(k_render_points<DD>, gp, dim3(256), 0, s, a, reg, Dc, dense, out);     \
    break;
    VB_RD(1) VB_RD(2) VB_RD(3) VB_RD(4) VB_RD(5) VB_RD(6)
#undef VB_RD
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass1(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out,
                        hipStream_t s, int stage) {
  if (N <= 0) return hipSuccess;
  const EArgs a = make_eargs(d, c, X, N, lse_out);
  if (c.prec != VBGS_FP64 && c.exact) {
    if (stage >= 0) return exact_stage(a, c.prec, d.D, N, s, c.cull, stage);
    return launch_exact_sweep(a, c.prec, d.D, N, s, c.cull);
  }
  if (stage == 0 || stage == 1 || stage == 2 || stage == 4) return hipSuccess;  // the whole pass is stage 3 (or -1)
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
  if (!c.exact) {
    if (c.prec == VBGS_FP32) VB_P1(VBGS_FP32, false);
    else if (c.prec == VBGS_BF16) VB_P1(VBGS_BF16, false);
    else if (c.prec == VBGS_FP8) VB_P1(VBGS_FP8, false);
    else VB_P1(VBGS_BF16X3, false);
  }
#undef VB_P1
  return hipGetLastError();
}

hipError_t launch_pass2(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, hipStream_t s,
                        double* stats_out) {
  EArgs a = make_eargs(d, c, X, N, nullptr);
  a.stats_out = stats_out;  // the exact mode writes the final statistics here and in a.stats
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
  if (c.exact) return launch_sparse_stats(a, d.D, N, s);
  const dim3 grid((unsigned)(d.L->Kpad / CT), (unsigned)c.nsplit);
#define VB_P2(PP) hipLaunchKernelGGL((k_pass2<PP>), grid, dim3(256), 0, s, a)
  if (c.prec == VBGS_FP32) {
    VB_P2(VBGS_FP32);
  } else if (c.prec == VBGS_BF16) {
    VB_P2(VBGS_BF16);
  } else if (c.prec == VBGS_FP8) {
    VB_P2(VBGS_FP8);
  } else {
    VB_P2(VBGS_BF16X3);
  }
#undef VB_P2
  return hipGetLastError();
}

hipError_t launch_fold(const DevPtrs& d, const EstepCfg& c, double* stats_out, hipStream_t s) {
  const int mode = c.prec == VBGS_FP64 ? 0 : (c.exact ? 2 : 1);
  if (mode == 2) return hipSuccess;  // the exact statistics kernels wrote the final values
  const int nsplit = mode == 2 ? 1 : c.nsplit;
  const dim3 grid((unsigned)((d.K + 255) / 256));
  switch (d.D) {
#define VB_FD(DD)                                                                                           \
  case DD:                                                                                                  \
    hipLaunchKernelGGL(k_fold<DD>, grid, dim3(256), 0, s, d.at<double>(d.L->spart), nsplit, d.L->Kpad, d.K,  \
                       d.frame(), d.at<double>(d.L->direct), direct_stride(d.D), mode, d.at<double>(d.L->stats), \
                       stats_out);                                                                          \
    break;
    VB_FD(1) VB_FD(2) VB_FD(3) VB_FD(4) VB_FD(5) VB_FD(6) VB_FD(7) VB_FD(8)
#undef VB_FD
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vbgs
