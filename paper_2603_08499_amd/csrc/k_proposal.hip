// Learned candidate proposal: network forward, BF16-MFMA logits with a streaming exact top-C,
// audit of the captured mass with a device-side fallback decision, and the training kernels.
//
// Network: x' = (x - mu_in) * inv_s_in, h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2) (H = 128),
// logits z_nk = h2_n . E_k + beta_k. The logits contraction has depth 128 = 4 steps of
// v_mfma_f32_16x16x32_bf16 (lane layout as in k_estep.hip: contraction slot 32q + 8g + j).
//
// Products over the components with the softmax weights p (training) contract a 32-wide group
// of components (or points) held by one lane as two 16-blocks: contraction slot 8g + j of the
// group maps to member (j < 4 ? 4g + j : 16 + 4g + j - 4), which is what a lane holds after the
// logits MFMA. The second operand is stored transposed in that permuted order so that each lane
// reads 8 contiguous values.
#include "prop_internal.h"

namespace vbgs {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int perm_slot(int kk) {  // member of a 32-group -> contraction slot
  return kk < 16 ? 8 * (kk >> 2) + (kk & 3) : 8 * ((kk - 16) >> 2) + 4 + ((kk - 16) & 3);
}

// total order used by the top-C selection: larger z first, then the smaller index
__device__ __forceinline__ bool better(float za, int ka, float zb, int kb) {
  return za > zb || (za == zb && ka < kb);
}

// Rearrange v[0..n) (with indices k) so that its first c entries are the c best in the total
// order (quickselect, Lomuto partition around the middle element). Thread-private memory.
__device__ __noinline__ void select_best(float* v, int32_t* k, int n, int c) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    float pv = v[mid];
    int32_t pk = k[mid];
    v[mid] = v[hi];
    k[mid] = k[hi];
    v[hi] = pv;
    k[hi] = pk;
    int st = lo;
    for (int i = lo; i < hi; ++i) {
      if (better(v[i], k[i], pv, pk)) {
        const float tv = v[i];
        const int32_t tk = k[i];
        v[i] = v[st];
        k[i] = k[st];
        v[st] = tv;
        k[st] = tk;
        ++st;
      }
    }
    v[hi] = v[st];
    k[hi] = k[st];
    v[st] = pv;
    k[st] = pk;
    // entries [lo, st) are better than the pivot, st is the pivot
    if (st == c || st == c - 1) return;
    if (st > c) hi = st - 1;
    else lo = st + 1;
  }
}

// worst (in the total order) of v[0..n)
__device__ __forceinline__ void worst_of(const float* v, const int32_t* k, int n, float& wz, int32_t& wk) {
  wz = v[0];
  wk = k[0];
  for (int i = 1; i < n; ++i)
    if (better(wz, wk, v[i], k[i])) {
      wz = v[i];
      wk = k[i];
    }
}

// ---------------------------------------------------------------------------
// weights -> MFMA operand copies: E (bf16 rows), E^T (bf16, permuted per 32 components),
// beta padded with -inf, W2^T (FP32)
// ---------------------------------------------------------------------------
__global__ void k_prop_prepare(const PArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = t / VBGS_H;
  const int f = (int)(t % VBGS_H);
  if (k < a.Kpad) {
    const float e = k < a.K ? a.E[k * VBGS_H + f] : 0.0f;
    const uint16_t h = f2bf(e);
    a.Ebf[k * VBGS_H + f] = h;
    const int64_t G = k / 32;
    a.EbfT[(G * VBGS_H + f) * 32 + perm_slot((int)(k % 32))] = h;
    if (f == 0) a.betap[k] = k < a.K ? a.beta[k] : -INFINITY;
  }
  if (t < (int64_t)VBGS_H * VBGS_H) {
    const int i = (int)(t / VBGS_H), j = (int)(t % VBGS_H);
    a.W2T[i * VBGS_H + j] = a.W2[j * VBGS_H + i];
  }
}

// ---------------------------------------------------------------------------
// network forward: 128 threads (one per hidden unit) x 32 points per workgroup
// ---------------------------------------------------------------------------
constexpr int MLP_PTS = 32;

__global__ __launch_bounds__(128) void k_mlp_fwd(const PArgs a, const float* __restrict__ X,
                                                 const int32_t* __restrict__ idx, int64_t n, MlpOut o) {
  __shared__ float xs[MLP_PTS][MAXD];
  __shared__ float h1s[MLP_PTS][VBGS_H];
  const int j = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * MLP_PTS;
  for (int q = j; q < MLP_PTS * a.D; q += VBGS_H) {
    const int p = q / a.D, d = q % a.D;
    float v = 0.0f;
    if (n0 + p < n) {
      const int64_t row = idx ? (int64_t)idx[n0 + p] : n0 + p;
      v = (X[row * a.D + d] - a.mu_in[d]) * a.inv_s_in[d];
    }
    xs[p][d] = v;
  }
  __syncthreads();
  float w1[MAXD];
  for (int d = 0; d < a.D; ++d) w1[d] = a.W1[j * a.D + d];
  const float bj1 = a.b1[j];
  for (int p = 0; p < MLP_PTS; ++p) {
    float s = bj1;
    for (int d = 0; d < a.D; ++d) s = fmaf(w1[d], xs[p][d], s);
    h1s[p][j] = fmaxf(s, 0.0f);
  }
  __syncthreads();
  float acc[MLP_PTS];
  const float bj2 = a.b2[j];
#pragma unroll
  for (int p = 0; p < MLP_PTS; ++p) acc[p] = bj2;
  for (int i = 0; i < VBGS_H; ++i) {
    const float w = a.W2T[i * VBGS_H + j];
#pragma unroll
    for (int p = 0; p < MLP_PTS; ++p) acc[p] = fmaf(w, h1s[p][i], acc[p]);
  }
#pragma unroll
  for (int p = 0; p < MLP_PTS; ++p) {
    const int64_t r = n0 + p;
    if (r >= o.npad) continue;
    const bool v = r < n;
    const float h2 = v ? fmaxf(acc[p], 0.0f) : 0.0f;
    if (o.h2b) o.h2b[r * VBGS_H + j] = f2bf(h2);
    if (o.h2T) o.h2T[((r / 32) * VBGS_H + j) * 32 + perm_slot((int)(r % 32))] = f2bf(h2);
    if (v) {
      if (o.h2) o.h2[r * VBGS_H + j] = h2;
      if (o.h1) o.h1[r * VBGS_H + j] = h1s[p][j];
      if (o.xs && j < a.D) o.xs[r * MAXD + j] = xs[p][j];
    }
  }
}

// ---------------------------------------------------------------------------
// logits tiles
// ---------------------------------------------------------------------------
struct __attribute__((aligned(16))) ETile {
  uint16_t e[CT][VBGS_H];  // 16 KB
  float beta[CT];
};

// native vectors: the staging registers of a tile stay in VGPRs (a struct of HIP's uint4 was kept
// in per-lane scratch memory, a store and a reload of 80 B per lane per tile)
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

struct ETileRegs {
  u32x4_t v[4];
  u32x4_t b;
};

__device__ __forceinline__ void etile_fetch(ETileRegs& R, const PArgs& a, int64_t k0) {
  const int t = threadIdx.x;  // 256 threads x 4 x 16 B = 16 KB
  const u32x4_t* src = reinterpret_cast<const u32x4_t*>(a.Ebf + k0 * VBGS_H);
#pragma unroll
  for (int q = 0; q < 4; ++q) R.v[q] = src[t + 256 * q];
  R.b = t < CT / 4 ? reinterpret_cast<const u32x4_t*>(a.betap + k0)[t] : u32x4_t{0u, 0u, 0u, 0u};
}

__device__ __forceinline__ void etile_store(ETile& T, const ETileRegs& R) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) reinterpret_cast<u32x4_t*>(&T.e[0][0])[t + 256 * q] = R.v[q];
  if (t < CT / 4) reinterpret_cast<u32x4_t*>(T.beta)[t] = R.b;
}

struct HOp {
  bf16x8_t q[4];
};

__device__ __forceinline__ HOp load_h(const uint16_t* row, int g) {
  HOp o;
#pragma unroll
  for (int q = 0; q < 4; ++q) o.q[q] = *reinterpret_cast<const bf16x8_t*>(row + 32 * q + 8 * g);
  return o;
}

__device__ __forceinline__ HOp zero_h() {
  HOp o;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int i = 0; i < 8; ++i) o.q[q][i] = (__bf16)0.0f;
  return o;
}

__device__ __forceinline__ f32x4 mfma_h(const HOp& A, const HOp& B) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.q[q], B.q[q], acc, 0, 0, 0);
  return acc;
}

// ---- FP8 logits: OCP e4m3 operands, the whole depth 128 in one v_mfma_scale_f32_16x16x128_f8f6f4 ----
// Each embedding row and each point's h2 row is scaled by the power of two that puts its largest
// magnitude in [224, 448] (k_rows128_fp8); the MFMA's block scales stay 1 (E8M0 127) and the two row
// factors are undone on the FP32 products: z = acc * sh_n * se_k + beta_k. Lane group g holds
// contraction slots [32 g, 32 g + 32) of both operands (the same slots on both sides, so the
// unit's order of the 32 bytes within a lane does not matter).
typedef int v8i_t __attribute__((ext_vector_type(8)));

struct __attribute__((aligned(16))) ETile8 {
  uint8_t e[CT][VBGS_H];  // 8 KB
  float beta[CT];
  float se[CT];  // factors undoing each row's scaling
};

struct ETile8Regs {
  u32x4_t v[2];
  u32x4_t b;  // threads 0..15: beta, 16..31: se
};

__device__ __forceinline__ void etile8_fetch(ETile8Regs& R, const PArgs& a, int64_t k0) {
  const int t = threadIdx.x;  // 256 threads x 2 x 16 B = 8 KB
  const u32x4_t* src = reinterpret_cast<const u32x4_t*>(a.E8 + k0 * VBGS_H);
#pragma unroll
  for (int q = 0; q < 2; ++q) R.v[q] = src[t + 256 * q];
  R.b = t < CT / 4 ? reinterpret_cast<const u32x4_t*>(a.betap + k0)[t]
                   : (t < CT / 2 ? reinterpret_cast<const u32x4_t*>(a.sE + k0)[t - CT / 4] : u32x4_t{0u, 0u, 0u, 0u});
}

__device__ __forceinline__ void etile8_store(ETile8& T, const ETile8Regs& R) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) reinterpret_cast<u32x4_t*>(&T.e[0][0])[t + 256 * q] = R.v[q];
  if (t < CT / 4) reinterpret_cast<u32x4_t*>(T.beta)[t] = R.b;
  else if (t < CT / 2) reinterpret_cast<u32x4_t*>(T.se)[t - CT / 4] = R.b;
}

__device__ __forceinline__ v8i_t load_h8(const uint8_t* row, int g) {
  return *reinterpret_cast<const v8i_t*>(row + 32 * g);
}

__device__ __forceinline__ f32x4 mfma_h8(const v8i_t& A, const v8i_t& B) {
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(A, B, zero, 0, 0, 0, 127, 0, 127);
}

// the logits passes over either operand precision
template <bool F8>
struct Logits;

template <>
struct Logits<false> {
  typedef ETile Tile;
  typedef ETileRegs Regs;
  typedef HOp Op;
  static __device__ __forceinline__ void fetch(Regs& R, const PArgs& a, int64_t k0) { etile_fetch(R, a, k0); }
  static __device__ __forceinline__ void store(Tile& T, const Regs& R) { etile_store(T, R); }
  static __device__ __forceinline__ Op point(const PArgs& a, int64_t p, int g) { return load_h(a.h2b + p * VBGS_H, g); }
  static __device__ __forceinline__ Op zero() { return zero_h(); }
  static __device__ __forceinline__ float pscale(const PArgs&, int64_t) { return 1.0f; }
  static __device__ __forceinline__ Op row(const Tile& T, int r, int g) { return load_h(&T.e[r][0], g); }
  // logits of rows 16 cb + 4 g + i (i < 4) of the tile for the lane's point
  static __device__ __forceinline__ void logits(const Tile& T, int cb, int g, const Op& A, const Op& B, float,
                                                float* z) {
    const f32x4 zz = mfma_h(A, B);
    const f32x4 bt = *reinterpret_cast<const f32x4*>(&T.beta[cb * 16 + 4 * g]);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = zz[i] + bt[i];
  }
};

template <>
struct Logits<true> {
  typedef ETile8 Tile;
  typedef ETile8Regs Regs;
  typedef v8i_t Op;
  static __device__ __forceinline__ void fetch(Regs& R, const PArgs& a, int64_t k0) { etile8_fetch(R, a, k0); }
  static __device__ __forceinline__ void store(Tile& T, const Regs& R) { etile8_store(T, R); }
  static __device__ __forceinline__ Op point(const PArgs& a, int64_t p, int g) { return load_h8(a.h8 + p * VBGS_H, g); }
  static __device__ __forceinline__ Op zero() { return v8i_t{0, 0, 0, 0, 0, 0, 0, 0}; }
  static __device__ __forceinline__ float pscale(const PArgs& a, int64_t p) { return a.sh[p]; }
  static __device__ __forceinline__ Op row(const Tile& T, int r, int g) { return load_h8(&T.e[r][0], g); }
  static __device__ __forceinline__ void logits(const Tile& T, int cb, int g, const Op& A, const Op& B, float sh,
                                                float* z) {
    const f32x4 zz = mfma_h8(A, B);
    const f32x4 bt = *reinterpret_cast<const f32x4*>(&T.beta[cb * 16 + 4 * g]);
    const f32x4 se = *reinterpret_cast<const f32x4*>(&T.se[cb * 16 + 4 * g]);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = fmaf(zz[i], sh * se[i], bt[i]);
  }
};

// rows of 128 values -> OCP e4m3 bytes, each row scaled by the power of two that puts its largest
// magnitude in [224, 448] (exact), rounded to nearest even by the hardware conversion; inv[r] undoes
// the scaling. Rows r >= nvalid (padding) are zero with factor 1. Input FP32 or BF16 (uint16).
template <typename T>
__global__ __launch_bounds__(256) void k_rows128_fp8(const T* __restrict__ src, int64_t nrows, int64_t nvalid,
                                                     uint8_t* __restrict__ dst, float* __restrict__ inv) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nrows) return;
  auto val = [&](int f) -> float {
    if constexpr (sizeof(T) == 2) return __uint_as_float((uint32_t)src[r * VBGS_H + f] << 16);
    else return src[r * VBGS_H + f];
  };
  float mx = 0.0f;
  if (r < nvalid)
    for (int f = 0; f < VBGS_H; ++f) mx = fmaxf(mx, fabsf(val(f)));
  float sc = 1.0f, un = 1.0f;
  if (mx > 7.8886091e-31f && mx <= 3.4e38f) {  // 2^-100: rows below are left unscaled (they round to 0)
    int e;
    frexpf(448.0f / mx, &e);  // 448 / mx in [2^(e-1), 2^e)
    sc = ldexpf(1.0f, e - 1);
    un = ldexpf(1.0f, 1 - e);
  }
  uint32_t* d32 = reinterpret_cast<uint32_t*>(dst + r * VBGS_H);
  for (int q = 0; q < VBGS_H / 4; ++q) {
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (r < nvalid)
      for (int i = 0; i < 4; ++i) v[i] = val(4 * q + i) * sc;
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
    d32[q] = (uint32_t)w;
  }
  inv[r] = un;
}

// ---------------------------------------------------------------------------
// streaming exact top-C per (point, lane group); 4 waves x 4 point blocks of 16
// ---------------------------------------------------------------------------
// A lower bound on each point's C-th best logit for C <= 4 NB: every lane group keeps its NB best
// logits in registers (a compare-exchange chain); the four groups' NB-th best values are each the
// smallest of NB distinct logits of the point, so their minimum is at or below its (4 NB)-th best.
// k_logits_topc starts its thresholds there, so that its candidate buffers fill (and are
// reselected) far less often than from -inf. NB = 8 serves C <= 32, NB = 16 serves C <= 64.
template <int NB, bool F8>
__global__ __launch_bounds__(256) void k_topc_thresh(const PArgs a, int64_t N) {
  typedef Logits<F8> LG;
  __shared__ typename LG::Tile T[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 256 + w * 64;
  typename LG::Op B[4];
  float shp[4];
  float r[4][NB];
  bool val[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < N;
    B[b] = val[b] ? LG::point(a, p, g) : LG::zero();
    shp[b] = val[b] ? LG::pscale(a, p) : 1.0f;
#pragma unroll
    for (int j = 0; j < NB; ++j) r[b][j] = -INFINITY;
  }
  typename LG::Regs R;
  LG::fetch(R, a, 0);
  LG::store(T[0], R);
  __syncthreads();
  const int64_t ntiles = a.Kpad / CT;
  for (int64_t it = 0; it < ntiles; ++it) {
    const int cur = (int)(it & 1);
    if (it + 1 < ntiles) LG::fetch(R, a, (it + 1) * CT);
    const typename LG::Tile& Tc = T[cur];
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const typename LG::Op A = LG::row(Tc, cb * 16 + c, g);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        float z[4];
        LG::logits(Tc, cb, g, A, B[b], shp[b], z);
        const float mx = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
        if (mx > r[b][NB - 1]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = z[i];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              const float hi = fmaxf(r[b][j], v);
              v = fminf(r[b][j], v);
              r[b][j] = hi;
            }
          }
        }
      }
    }
    if (it + 1 < ntiles) LG::store(T[cur ^ 1], R);
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    float t = r[b][NB - 1];
    t = fminf(t, __shfl_xor(t, 16));
    t = fminf(t, __shfl_xor(t, 32));
    if (val[b] && g == 0) a.tthr[p0 + 16 * b + c] = t;
  }
}

template <bool F8>
__global__ __launch_bounds__(256) void k_logits_topc(const PArgs a, int64_t N) {
  typedef Logits<F8> LG;
  __shared__ typename LG::Tile T[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 256 + w * 64;
  const int C = a.C, CAP = 2 * a.C;
  typename LG::Op B[4];
  float shp[4];
  float zt[4];
  int cnt[4];
  bool val[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < N;
    B[b] = val[b] ? LG::point(a, p, g) : LG::zero();
    shp[b] = val[b] ? LG::pscale(a, p) : 1.0f;
    // just below the lower bound on the C-th best, so that a logit equal to it still enters
    const float t = a.tthr && val[b] ? a.tthr[p] : -INFINITY;
    zt[b] = t == -INFINITY ? t : nextafterf(t, -INFINITY);
    cnt[b] = 0;
  }
  typename LG::Regs R;
  LG::fetch(R, a, 0);
  LG::store(T[0], R);
  __syncthreads();
  const int64_t ntiles = a.Kpad / CT;
  for (int64_t it = 0; it < ntiles; ++it) {
    const int cur = (int)(it & 1);
    if (it + 1 < ntiles) LG::fetch(R, a, (it + 1) * CT);
    const typename LG::Tile& Tc = T[cur];
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const typename LG::Op A = LG::row(Tc, cb * 16 + c, g);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        float z[4];
        LG::logits(Tc, cb, g, A, B[b], shp[b], z);
        const float mx = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
        if (val[b] && mx > zt[b]) {
          const int64_t p = p0 + 16 * b + c;
          float* bz = a.tz + (p * 4 + g) * CAP;
          int32_t* bk = a.tk + (p * 4 + g) * CAP;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (z[i] > zt[b]) {  // components arrive in increasing index, so ties never qualify
              bz[cnt[b]] = z[i];
              bk[cnt[b]] = (int32_t)(it * CT + cb * 16 + 4 * g + i);
              if (++cnt[b] == CAP) {
                select_best(bz, bk, CAP, C);
                cnt[b] = C;
                int32_t wk;
                worst_of(bz, bk, C, zt[b], wk);
              }
            }
          }
        }
      }
    }
    if (it + 1 < ntiles) LG::store(T[cur ^ 1], R);
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    if (!val[b]) continue;
    const int64_t p = p0 + 16 * b + c;
    float* bz = a.tz + (p * 4 + g) * CAP;
    int32_t* bk = a.tk + (p * 4 + g) * CAP;
    if (cnt[b] > C) {
      select_best(bz, bk, cnt[b], C);
      cnt[b] = C;
    }
    a.tcnt[p * 4 + g] = cnt[b];
  }
}

// merge the four lane-group lists of a point into its top-C and publish them as candidate lists
__global__ __launch_bounds__(256) void k_topc_merge(const PArgs a, const EArgs e, int64_t N) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const int C = a.C, CAP = 2 * a.C;
  float* bz = a.tz + p * 4 * CAP;
  int32_t* bk = a.tk + p * 4 * CAP;
  int n = 0;
  for (int g = 0; g < 4; ++g) {
    const int c = a.tcnt[p * 4 + g];
    for (int j = 0; j < c; ++j) {
      bz[n + j] = bz[g * CAP + j];
      bk[n + j] = bk[g * CAP + j];
    }
    n += c;
  }
  const int m = min(n, C);
  if (n > C) select_best(bz, bk, n, C);
  for (int g = 0; g < 4; ++g) e.cand_n[p * 4 + g] = max(0, min(CS, m - g * CS));
  for (int j = 0; j < m; ++j) e.cand_k[(p * 4 + j / CS) * CS + (j % CS)] = bk[j];
}

// candidates of each point, ascending index, padded with -1
__global__ __launch_bounds__(256) void k_topc_export(const EArgs e, int64_t N, int C, int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  int32_t v[64];
  int m = 0;
  for (int g = 0; g < 4; ++g)
    for (int j = 0; j < e.cand_n[p * 4 + g]; ++j) v[m++] = e.cand_k[(p * 4 + g) * CS + j];
  for (int i = 1; i < m; ++i) {  // insertion sort, m <= 64
    const int32_t x = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > x) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = x;
  }
  for (int j = 0; j < C; ++j) out[p * C + j] = j < m ? v[j] : -1;
}

// ---------------------------------------------------------------------------
// audit: dense exact LSE of the audited points, captured mass, fallback decision
// ---------------------------------------------------------------------------
// exact FP64 LSE of the audited points over all K: AP points per workgroup, so that each
// coefficient row is read once for all of them; per point an online (max, sum) per thread, then a
// fixed-order merge over lanes and waves
constexpr int AP = 8;

template <int DT>
__global__ __launch_bounds__(256) void k_audit_lse(const EArgsLite e, const int32_t* __restrict__ idx, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ float xs[AP][DT];
  __shared__ double wm[4][AP], wl[4][AP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * AP;
  const int np = (int)(n - i0 < AP ? n - i0 : AP);
  if (tid < AP * DT) {
    const int j = tid / DT, q = tid % DT;
    xs[j][q] = j < np ? e.X[(int64_t)idx[i0 + j] * DT + q] : 0.0f;
  }
  __syncthreads();
  double m[AP], l[AP];
#pragma unroll
  for (int j = 0; j < AP; ++j) {
    m[j] = -INFINITY;
    l[j] = 0.0;
  }
  for (int64_t k = tid; k < e.K; k += 256) {
    const double* row = e.direct + k * e.dts;
#pragma unroll
    for (int j = 0; j < AP; ++j) {
      if (j >= np) break;
      double d[DT];
      const double sc = direct_score2_dt<DT>(row, &xs[j][0], d);
      if (sc > m[j]) {
        l[j] = l[j] * exp2(m[j] - sc) + 1.0;
        m[j] = sc;
      } else {
        l[j] += exp2(sc - m[j]);
      }
    }
  }
  auto merge = [](double& ma, double& la, double mb, double lb) {
    const double mn = fmax(ma, mb);
    if (mn == -INFINITY) return;
    la = (ma == -INFINITY ? 0.0 : la * exp2(ma - mn)) + (mb == -INFINITY ? 0.0 : lb * exp2(mb - mn));
    ma = mn;
  };
#pragma unroll
  for (int j = 0; j < AP; ++j) {
    for (int off = 32; off > 0; off >>= 1) merge(m[j], l[j], __shfl_xor(m[j], off), __shfl_xor(l[j], off));
    if (lane == 0) {
      wm[w][j] = m[j];
      wl[w][j] = l[j];
    }
  }
  __syncthreads();
  if (tid < np) {
    double mm = wm[0][tid], ll = wl[0][tid];
    for (int q = 1; q < 4; ++q) merge(mm, ll, wm[q][tid], wl[q][tid]);
    out[i0 + tid] = mm + log2(ll);
  }
}

__global__ __launch_bounds__(256) void k_audit_decide(const double* __restrict__ lse2_c, const int32_t* __restrict__ idx,
                                                      const double* __restrict__ lse2_all, int64_t n, double bound,
                                                      double frac, int32_t* gate, double* report) {
  __shared__ double smax[256], ssum[256], smin[256];
  __shared__ int sbel[256];
  const int t = threadIdx.x;
  double mx = -INFINITY, mn = INFINITY;
  int bel = 0;
  for (int64_t i = t; i < n; i += 256) {
    const double cap = (lse2_c[idx[i]] - lse2_all[i]) * LN2;
    mx = fmax(mx, cap);
    mn = fmin(mn, cap);
    bel += cap < bound ? 1 : 0;
  }
  smax[t] = mx;
  smin[t] = mn;
  sbel[t] = bel;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      smax[t] = fmax(smax[t], smax[t + w]);
      smin[t] = fmin(smin[t], smin[t + w]);
      sbel[t] += sbel[t + w];
    }
    __syncthreads();
  }
  const double M = smax[0];
  double s = 0.0;
  for (int64_t i = t; i < n; i += 256) s += exp((lse2_c[idx[i]] - lse2_all[i]) * LN2 - M);
  ssum[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) ssum[t] += ssum[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double agg = n > 0 ? M + log(ssum[0]) - log((double)n) : 0.0;
    const double fb = n > 0 ? (double)sbel[0] / (double)n : 0.0;
    const int fall = (n > 0 && (agg < bound || fb > frac)) ? 1 : 0;
    gate[0] = fall;
    if (report) {
      report[0] = fall;
      report[1] = agg;
      report[2] = fb;
      report[3] = n > 0 ? smin[0] : 0.0;
    }
  }
}

// no audit: the pruned statistics stand (gate 0); the report's captured-mass fields read NaN so
// that an unaudited frame cannot pass for one whose candidates captured all of the mass
__global__ void k_no_audit(int32_t* gate, double* report) {
  gate[0] = 0;
  if (report) {
    report[0] = 0.0;
    report[1] = report[2] = report[3] = __builtin_nan("");
  }
}

// ---------------------------------------------------------------------------
// training targets from an exact E-step: the kept pairs with r = 2^(s - LSE)
// ---------------------------------------------------------------------------
// FP64 score (log2 units) of one pair in direct form, any supported D
__device__ double score2_anyd(const double* __restrict__ row, const float* __restrict__ x, int D) {
  double d[MAXD];
  switch (D) {
    case 1: return direct_score2_dt<1>(row, x, d);
    case 2: return direct_score2_dt<2>(row, x, d);
    case 3: return direct_score2_dt<3>(row, x, d);
    case 4: return direct_score2_dt<4>(row, x, d);
    case 5: return direct_score2_dt<5>(row, x, d);
    case 6: return direct_score2_dt<6>(row, x, d);
    case 7: return direct_score2_dt<7>(row, x, d);
    default: return direct_score2_dt<8>(row, x, d);
  }
}

__global__ __launch_bounds__(256) void k_export_targets(const EArgsLite e, int64_t N, int32_t* __restrict__ tk,
                                                        float* __restrict__ tr) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  int m = 0;
  if (e.cand_n[p * 4] >= 0) {
    const double L2 = e.lse2[p];
    for (int g = 0; g < 4; ++g) {
      const int cnt = e.cand_n[p * 4 + g];
      for (int j = 0; j < cnt; ++j) {
        const int64_t q = (p * 4 + g) * CS + j;
        const int32_t k = e.cand_k[q];
        if (k < 0) continue;
        // (the E-step keeps a kept pair's rank in its score slot: the score is computed again)
        const double s2 = score2_anyd(e.direct + (int64_t)k * e.dts, e.X + p * e.D, e.D);
        tk[p * 64 + m] = k;
        tr[p * 64 + m] = (float)exp2(s2 - L2);
        ++m;
      }
    }
  }
  for (; m < 64; ++m) {
    tk[p * 64 + m] = -1;
    tr[p * 64 + m] = 0.0f;
  }
}

// ---------------------------------------------------------------------------
// training: logits LSE per batch point (natural units)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_train_lse(const PArgs a, int64_t B) {
  __shared__ ETile T[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 256 + w * 64;
  // component slice blockIdx.y of gridDim.y: tiles [t0, t1)
  const int64_t ntiles = a.Kpad / CT;
  const int64_t t0 = ntiles * blockIdx.y / gridDim.y, t1 = ntiles * (blockIdx.y + 1) / gridDim.y;
  HOp Bh[4];
  float M[4], L[4];
  bool val[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < B;
    Bh[b] = val[b] ? load_h(a.th2b + p * VBGS_H, g) : zero_h();
    M[b] = -INFINITY;
    L[b] = 0.0f;
  }
  ETileRegs R;
  if (t0 < t1) {
    etile_fetch(R, a, t0 * CT);
    etile_store(T[0], R);
  }
  __syncthreads();
  const float l2e = (float)LOG2E;
  for (int64_t it = t0; it < t1; ++it) {
    const int cur = (int)((it - t0) & 1);
    if (it + 1 < t1) etile_fetch(R, a, (it + 1) * CT);
    const ETile& Tc = T[cur];
#pragma unroll
    for (int cb = 0; cb < CT / 16; ++cb) {
      const HOp A = load_h(&Tc.e[cb * 16 + c][0], g);
      const f32x4 bt = *reinterpret_cast<const f32x4*>(&Tc.beta[cb * 16 + 4 * g]);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const f32x4 zz = mfma_h(A, Bh[b]);
        float z[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] = (zz[i] + bt[i]) * l2e;  // log2 units; -inf for padding
        const float mx = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
        if (mx > M[b]) {
          L[b] *= exp2f(M[b] - mx);
          M[b] = mx;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) L[b] += exp2f(z[i] - M[b]);
      }
    }
    if (it + 1 < t1) etile_store(T[cur ^ 1], R);
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    float m = M[b], l = L[b];
    for (int off = 16; off <= 32; off <<= 1) {
      const float om = __shfl_xor(m, off), ol = __shfl_xor(l, off);
      const float mn = fmaxf(m, om);
      l = (m == -INFINITY ? 0.0f : l * exp2f(m - mn)) + (om == -INFINITY ? 0.0f : ol * exp2f(om - mn));
      m = mn;
    }
    const int64_t p = p0 + 16 * b + c;
    if (g == 0 && val[b]) {
      float* o = a.tlpart + ((int64_t)blockIdx.y * B + p) * 2;
      o[0] = m;
      o[1] = l;
    }
  }
}

// the slices' (max, sum) of each point merged in slice order: LSE in nats
__global__ __launch_bounds__(256) void k_train_lse_merge(const PArgs a, int64_t B, int S) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= B) return;
  float m = -INFINITY, l = 0.0f;
  for (int s = 0; s < S; ++s) {
    const float om = a.tlpart[((int64_t)s * B + p) * 2], ol = a.tlpart[((int64_t)s * B + p) * 2 + 1];
    const float mn = fmaxf(m, om);
    if (mn == -INFINITY) continue;
    l = (m == -INFINITY ? 0.0f : l * exp2f(m - mn)) + (om == -INFINITY ? 0.0f : ol * exp2f(om - mn));
    m = mn;
  }
  a.tlse[p] = (m + log2f(l)) * (float)LN2;
}

// ---------------------------------------------------------------------------
// training: dh2_n = (1/B) sum_k p_nk E_k (dense part), point parallel, 2 point blocks per wave
// ---------------------------------------------------------------------------
struct __attribute__((aligned(16))) ETileT {
  uint16_t e[CT][VBGS_H];                   // rows (logits operand)
  uint16_t t[CT / 32][VBGS_H][32];          // transposed, permuted per 32 (product operand)
  float beta[CT];
};

__global__ __launch_bounds__(256) void k_train_dh(const PArgs a, int64_t B) {
  __shared__ ETileT T;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 128 + w * 32;
  HOp Bh[2];
  float lse2[2];
  bool val[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int64_t p = p0 + 16 * b + c;
    val[b] = p < B;
    Bh[b] = val[b] ? load_h(a.th2b + p * VBGS_H, g) : zero_h();
    lse2[b] = val[b] ? a.tlse[p] * (float)LOG2E : INFINITY;
  }
  f32x4 acc[2][8];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int f = 0; f < 8; ++f) acc[b][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float l2e = (float)LOG2E, invB = 1.0f / (float)B;
  const int64_t ntiles = a.Kpad / CT;  // component slice blockIdx.y: tiles [t0, t1)
  const int64_t t0 = ntiles * blockIdx.y / gridDim.y, t1 = ntiles * (blockIdx.y + 1) / gridDim.y;
  for (int64_t k0 = t0 * CT; k0 < t1 * CT; k0 += CT) {
    __syncthreads();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.Ebf + k0 * VBGS_H);
      const uint4* srt = reinterpret_cast<const uint4*>(a.EbfT + k0 * VBGS_H);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        reinterpret_cast<uint4*>(&T.e[0][0])[tid + 256 * q] = src[tid + 256 * q];
        reinterpret_cast<uint4*>(&T.t[0][0][0])[tid + 256 * q] = srt[tid + 256 * q];
      }
      if (tid < CT / 4) reinterpret_cast<uint4*>(T.beta)[tid] = reinterpret_cast<const uint4*>(a.betap + k0)[tid];
    }
    __syncthreads();
#pragma unroll
    for (int grp = 0; grp < CT / 32; ++grp) {
      const HOp A0 = load_h(&T.e[grp * 32 + c][0], g);
      const HOp A1 = load_h(&T.e[grp * 32 + 16 + c][0], g);
      const f32x4 b0 = *reinterpret_cast<const f32x4*>(&T.beta[grp * 32 + 4 * g]);
      const f32x4 b1 = *reinterpret_cast<const f32x4*>(&T.beta[grp * 32 + 16 + 4 * g]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const f32x4 z0 = mfma_h(A0, Bh[b]);
        const f32x4 z1 = mfma_h(A1, Bh[b]);
        bf16x8_t P;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          P[i] = (__bf16)(exp2f((z0[i] + b0[i]) * l2e - lse2[b]) * invB);
          P[4 + i] = (__bf16)(exp2f((z1[i] + b1[i]) * l2e - lse2[b]) * invB);
        }
#pragma unroll
        for (int f = 0; f < 8; ++f) {
          const bf16x8_t Et = *reinterpret_cast<const bf16x8_t*>(&T.t[grp][16 * f + c][8 * g]);
          acc[b][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P, Et, acc[b][f], 0, 0, 0);
        }
      }
    }
  }
  // lane holds dh2(point 16 b + 4g + i, feature 16 f + c)
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = p0 + 16 * b + 4 * g + i;
      if (p < B)
#pragma unroll
        for (int f = 0; f < 8; ++f) a.tdpart[((int64_t)blockIdx.y * B + p) * VBGS_H + 16 * f + c] = acc[b][f][i];
    }
}

// dh2 = the slices' partial rows added in slice order
__global__ __launch_bounds__(256) void k_train_dh_sum(const PArgs a, int64_t B, int S) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= B * VBGS_H) return;
  float v = 0.0f;
  for (int s = 0; s < S; ++s) v += a.tdpart[(int64_t)s * B * VBGS_H + q];
  a.tdh2[q] = v;
}

// ---------------------------------------------------------------------------
// training: dE_k = (1/B) sum_n p_nk h2_n and dbeta_k = (1/B) sum_n p_nk (dense parts),
// component parallel: 4 waves x 16 components, streaming 32-point groups of the batch
// ---------------------------------------------------------------------------
struct __attribute__((aligned(16))) HTile {
  uint16_t h[64][VBGS_H];           // rows
  uint16_t t[2][VBGS_H][32];        // transposed, permuted per 32 points
  float lse2[64];
};

__global__ __launch_bounds__(256) void k_train_de(const PArgs a, int64_t B) {
  __shared__ HTile T;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int64_t kb = (int64_t)blockIdx.x * 64 + w * 16;
  const int64_t kc = kb + c;  // < Kpad
  const HOp Bc = load_h(a.Ebf + kc * VBGS_H, g);
  const float bc = a.betap[kc];
  const float l2e = (float)LOG2E, invB = 1.0f / (float)B;
  f32x4 acc[8];
#pragma unroll
  for (int f = 0; f < 8; ++f) acc[f] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbeta = 0.0f;
  for (int64_t n0 = 0; n0 < a.Bpad; n0 += 64) {
    __syncthreads();
    {
      const uint4* src = reinterpret_cast<const uint4*>(a.th2b + n0 * VBGS_H);
      const uint4* srt = reinterpret_cast<const uint4*>(a.th2T + n0 * VBGS_H);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        reinterpret_cast<uint4*>(&T.h[0][0])[tid + 256 * q] = src[tid + 256 * q];
        reinterpret_cast<uint4*>(&T.t[0][0][0])[tid + 256 * q] = srt[tid + 256 * q];
      }
      if (tid < 64) T.lse2[tid] = (n0 + tid < B) ? a.tlse[n0 + tid] * (float)LOG2E : INFINITY;
    }
    __syncthreads();
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
      const HOp A0 = load_h(&T.h[grp * 32 + c][0], g);
      const HOp A1 = load_h(&T.h[grp * 32 + 16 + c][0], g);
      const f32x4 z0 = mfma_h(A0, Bc);  // lane: points grp*32 + 4g + i, component kc
      const f32x4 z1 = mfma_h(A1, Bc);
      bf16x8_t P;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float q0 = exp2f((z0[i] + bc) * l2e - T.lse2[grp * 32 + 4 * g + i]) * invB;
        const float q1 = exp2f((z1[i] + bc) * l2e - T.lse2[grp * 32 + 16 + 4 * g + i]) * invB;
        dbeta += q0 + q1;
        P[i] = (__bf16)q0;
        P[4 + i] = (__bf16)q1;
      }
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        const bf16x8_t Ht = *reinterpret_cast<const bf16x8_t*>(&T.t[grp][16 * f + c][8 * g]);
        acc[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(P, Ht, acc[f], 0, 0, 0);
      }
    }
  }
  dbeta += __shfl_xor(dbeta, 16);
  dbeta += __shfl_xor(dbeta, 32);
  // lane holds dE(component kb + 4g + i, feature 16 f + c)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t k = kb + 4 * g + i;
    if (k < a.K)
#pragma unroll
      for (int f = 0; f < 8; ++f) a.gE[k * VBGS_H + 16 * f + c] = acc[f][i];
  }
  if (g == 0 && kc < a.K) a.gbeta[kc] = dbeta;
}

// ---------------------------------------------------------------------------
// training: sparse target term and per-point loss (thread per batch point)
// ---------------------------------------------------------------------------
// one wave per batch point, lane l taking features l and 64 + l
__global__ __launch_bounds__(256) void k_train_sparse(const PArgs a, const int32_t* __restrict__ tk,
                                                      const float* __restrict__ tr, const int32_t* __restrict__ bidx,
                                                      int64_t B) {
  static_assert(VBGS_H == 128, "two features per lane");
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= B) return;  // whole waves
  const int64_t row = bidx[n];
  const int32_t kl = tk[row * 64 + lane];  // lane j holds target j
  const float rl = kl >= 0 ? tr[row * 64 + lane] : 0.0f;
  float wsum = rl;
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off);
  if (!(wsum > 0.0f)) {  // no targets: only the softmax term (dense kernels) contributes
    if (lane == 0) a.tloss[n] = (double)a.tlse[n];
    return;
  }
  const float invB = 1.0f / (float)B;
  const float h0 = a.th2[n * VBGS_H + lane], h1 = a.th2[n * VBGS_H + 64 + lane];
  float d0 = 0.0f, d1 = 0.0f;
  double zt = 0.0;
  unsigned long long live = __ballot(kl >= 0);
  while (live) {
    const int j = __ffsll((long long)live) - 1;
    live &= live - 1ull;
    const int32_t k = __shfl(kl, j);
    const float wv = __shfl(rl, j) / wsum;
    const float* Ek = a.E + (int64_t)k * VBGS_H;
    const float e0 = Ek[lane], e1 = Ek[64 + lane];
    float z = fmaf(h0, e0, h1 * e1);
    for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off);
    z += a.beta[k];
    d0 -= invB * wv * e0;
    d1 -= invB * wv * e1;
    atomicAdd(&a.gE[(int64_t)k * VBGS_H + lane], -invB * wv * h0);
    atomicAdd(&a.gE[(int64_t)k * VBGS_H + 64 + lane], -invB * wv * h1);
    if (lane == 0) atomicAdd(&a.gbeta[k], -invB * wv);
    zt += (double)wv * (double)z;
  }
  a.tdh2[n * VBGS_H + lane] += d0;
  a.tdh2[n * VBGS_H + 64 + lane] += d1;
  if (lane == 0) a.tloss[n] = (double)a.tlse[n] - zt;
}

// ---------------------------------------------------------------------------
// training: backward through the hidden layers, deterministic reductions over the batch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_train_dh1(const PArgs a, int64_t B) {
  const int64_t t = (int64_t)blockIdx.x * 128 + threadIdx.x;
  const int64_t n = t / VBGS_H;
  const int i = (int)(t % VBGS_H);
  if (n >= B) return;
  float s = 0.0f;
  for (int j = 0; j < VBGS_H; ++j) {
    const float d2 = a.th2[n * VBGS_H + j] > 0.0f ? a.tdh2[n * VBGS_H + j] : 0.0f;
    s = fmaf(d2, a.W2[j * VBGS_H + i], s);
  }
  a.tdp1[n * VBGS_H + i] = a.th1[n * VBGS_H + i] > 0.0f ? s : 0.0f;
}

// hidden-layer weight gradients, index t over [gW2 (H x H), gb2 (H), gW1 (H x D), gb1 (H)]; the
// batch is split into TRAIN_W_SPLIT slices (blockIdx.y), whose partial sums k_train_wgrad_sum adds
// in slice order
__device__ __forceinline__ float* wgrad_dst(const PArgs& a, int64_t t) {
  const int H = VBGS_H;
  const int64_t nW2 = (int64_t)H * H, nW1 = (int64_t)H * a.D;
  if (t < nW2) return a.gW2 + t;
  if (t < nW2 + H) return a.gb2 + (t - nW2);
  if (t < nW2 + H + nW1) return a.gW1 + (t - nW2 - H);
  return a.gb1 + (t - nW2 - H - nW1);
}

__global__ __launch_bounds__(256) void k_train_wgrad(const PArgs a, int64_t B) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int H = VBGS_H, D = a.D;
  const int64_t nW2 = (int64_t)H * H, nW1 = (int64_t)H * D, nw = nW2 + H + nW1 + H;
  const int64_t n0 = B * blockIdx.y / gridDim.y, n1 = B * (blockIdx.y + 1) / gridDim.y;
  if (t >= nw) return;
  float s = 0.0f;
  if (t < nW2) {  // gW2[j][i] = sum_n dpre2[n][j] h1[n][i]
    const int j = (int)(t / H), i = (int)(t % H);
    for (int64_t n = n0; n < n1; ++n) {
      const float d2 = a.th2[n * H + j] > 0.0f ? a.tdh2[n * H + j] : 0.0f;
      s = fmaf(d2, a.th1[n * H + i], s);
    }
  } else if (t < nW2 + H) {  // gb2
    const int j = (int)(t - nW2);
    for (int64_t n = n0; n < n1; ++n) s += a.th2[n * H + j] > 0.0f ? a.tdh2[n * H + j] : 0.0f;
  } else if (t < nW2 + H + nW1) {  // gW1[j][d] = sum_n dpre1[n][j] x'[n][d]
    const int64_t u = t - nW2 - H;
    const int j = (int)(u / D), d = (int)(u % D);
    for (int64_t n = n0; n < n1; ++n) s = fmaf(a.tdp1[n * H + j], a.txs[n * MAXD + d], s);
  } else {  // gb1
    const int j = (int)(t - nW2 - H - nW1);
    for (int64_t n = n0; n < n1; ++n) s += a.tdp1[n * H + j];
  }
  a.twpart[(int64_t)blockIdx.y * nw + t] = s;
}

__global__ __launch_bounds__(256) void k_train_wgrad_sum(const PArgs a, int64_t nw, int S) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nw) return;
  float s = 0.0f;
  for (int q = 0; q < S; ++q) s += a.twpart[(int64_t)q * nw + t];
  *wgrad_dst(a, t) = s;
}

__global__ __launch_bounds__(256) void k_train_loss(const double* __restrict__ lp, int64_t B, double* out) {
  __shared__ double s[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < B; i += 256) v += lp[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0] / (double)B;
}

// Adam on the flat trainable array (W1, b1, W2, b2, E, beta); the step count lives in the state
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ gr,
                                              float* __restrict__ m1, float* __restrict__ m2, const double* step,
                                              int64_t n, float lr) {
  const double t = step[0] + 1.0;
  const float c1 = (float)(1.0 / (1.0 - pow(0.9, t))), c2 = (float)(1.0 / (1.0 - pow(0.999, t)));
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float g = gr[i];
    const float a = 0.9f * m1[i] + 0.1f * g;
    const float b = 0.999f * m2[i] + 0.001f * g * g;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a * c1) / (sqrtf(b * c2) + 1e-8f);
  }
}

__global__ void k_step_inc(double* step) { step[0] += 1.0; }

__global__ void k_zero_f32(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_prop_prepare(const PArgs& a, hipStream_t s) {
  const int64_t n = std::max<int64_t>(a.Kpad * VBGS_H, (int64_t)VBGS_H * VBGS_H);
  hipLaunchKernelGGL(k_prop_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  if (a.f8)  // embedding rows as scaled e4m3 for the FP8 logits
    hipLaunchKernelGGL(k_rows128_fp8<float>, dim3((unsigned)((a.Kpad + 255) / 256)), dim3(256), 0, s, a.E, a.Kpad,
                       a.K, a.E8, a.sE);
  return hipGetLastError();
}

hipError_t launch_mlp_fwd(const PArgs& a, const float* X, const int32_t* idx, int64_t n, const MlpOut& o,
                          hipStream_t s) {
  if (o.npad <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((o.npad + MLP_PTS - 1) / MLP_PTS)), dim3(128), 0, s, a, X, idx, n, o);
  return hipGetLastError();
}

hipError_t launch_topc(const PArgs& a, const EArgsLite& e, int64_t N, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const dim3 grid((unsigned)((N + 255) / 256));
  if (a.f8) {  // the points' h2 rows as scaled e4m3
    hipLaunchKernelGGL(k_rows128_fp8<uint16_t>, grid, dim3(256), 0, s, a.h2b, N, N, a.h8, a.sh);
    if (a.C <= 32) hipLaunchKernelGGL((k_topc_thresh<8, true>), grid, dim3(256), 0, s, a, N);
    else hipLaunchKernelGGL((k_topc_thresh<16, true>), grid, dim3(256), 0, s, a, N);
    hipLaunchKernelGGL(k_logits_topc<true>, grid, dim3(256), 0, s, a, N);
  } else {
    if (a.C <= 32) hipLaunchKernelGGL((k_topc_thresh<8, false>), grid, dim3(256), 0, s, a, N);
    else hipLaunchKernelGGL((k_topc_thresh<16, false>), grid, dim3(256), 0, s, a, N);
    hipLaunchKernelGGL(k_logits_topc<false>, grid, dim3(256), 0, s, a, N);
  }
  hipLaunchKernelGGL(k_topc_merge, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, e, N);
  return hipGetLastError();
}

hipError_t launch_topc_export(const EArgsLite& e, int64_t N, int C, int32_t* out, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_topc_export, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, e, N, C, out);
  return hipGetLastError();
}

hipError_t launch_audit(const EArgsLite& e, int D, const int32_t* idx, int64_t n, double* aud, const double* lse2,
                        double bound, double frac, int32_t* gate, double* report, hipStream_t s) {
  if (n > 0) {
    switch (D) {
#define VB_AU(DD) \
  case DD:        \
    hipLaunchKernelGGL(k_audit_lse<DD>, dim3((unsigned)((n + AP - 1) / AP)), dim3(256), 0, s, e, idx, n, aud); \
    break;
      VB_AU(1) VB_AU(2) VB_AU(3) VB_AU(4) VB_AU(5) VB_AU(6)
#undef VB_AU
      default:
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_audit_decide, dim3(1), dim3(256), 0, s, lse2, idx, aud, n, bound, frac, gate, report);
  } else {
    hipLaunchKernelGGL(k_no_audit, dim3(1), dim3(1), 0, s, gate, report);
  }
  return hipGetLastError();
}

hipError_t launch_export_targets(const EArgsLite& e, int64_t N, int32_t* tk, float* tr, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_export_targets, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, e, N, tk, tr);
  return hipGetLastError();
}

hipError_t launch_train(const PArgs& a, const float* X, const int32_t* tk, const float* tr, const int32_t* bidx,
                        int64_t B, float lr, int apply, double* loss_out, float* grads_out, hipStream_t s) {
  MlpOut o{};
  o.npad = a.Bpad;
  o.h1 = a.th1;
  o.h2 = a.th2;
  o.h2b = a.th2b;
  o.h2T = a.th2T;
  o.xs = a.txs;
  hipError_t e = launch_mlp_fwd(a, X, bidx, B, o, s);
  if (e != hipSuccess) return e;
  const int sl = train_lse_split(B), sd = train_dh_split(B);
  hipLaunchKernelGGL(k_train_lse, dim3((unsigned)((B + 255) / 256), (unsigned)sl), dim3(256), 0, s, a, B);
  hipLaunchKernelGGL(k_train_lse_merge, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, a, B, sl);
  hipLaunchKernelGGL(k_train_dh, dim3((unsigned)((B + 127) / 128), (unsigned)sd), dim3(256), 0, s, a, B);
  hipLaunchKernelGGL(k_train_dh_sum, dim3((unsigned)((B * VBGS_H + 255) / 256)), dim3(256), 0, s, a, B, sd);
  hipLaunchKernelGGL(k_train_de, dim3((unsigned)(a.Kpad / 64)), dim3(256), 0, s, a, B);
  hipLaunchKernelGGL(k_train_sparse, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, a, tk, tr, bidx, B);
  hipLaunchKernelGGL(k_train_dh1, dim3((unsigned)((B * VBGS_H + 127) / 128)), dim3(128), 0, s, a, B);
  const int64_t nw = (int64_t)VBGS_H * VBGS_H + VBGS_H + (int64_t)VBGS_H * a.D + VBGS_H;
  hipLaunchKernelGGL(k_train_wgrad, dim3((unsigned)((nw + 255) / 256), TRAIN_W_SPLIT), dim3(256), 0, s, a, B);
  hipLaunchKernelGGL(k_train_wgrad_sum, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, a, nw, TRAIN_W_SPLIT);
  if (loss_out) hipLaunchKernelGGL(k_train_loss, dim3(1), dim3(256), 0, s, a.tloss, B, loss_out);
  if (grads_out) {
    e = hipMemcpyAsync(grads_out, a.grads, (size_t)a.n_train * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  if (apply) {
    hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, s, a.W, a.grads, a.m1, a.m2, a.step, a.n_train, lr);
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, s, a.step);
    e = launch_prop_prepare(a, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3(1024), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace vbgs
