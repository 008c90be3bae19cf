// Internal definitions shared by the HIP translation units of libvbgs.
// gfx950 (CDNA4) only: 64-lane wavefronts, MFMA matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cfloat>

#include "../../include/vbgs.h"

namespace vbgs {

constexpr double LOG2E = 1.4426950408889634074;
constexpr double LN2 = 0.69314718055994530942;
constexpr double LN2PI = 1.8378770664093454836;
constexpr double LNPI = 1.1447298858494001741;

constexpr int MAXD = VBGS_MAX_D;
constexpr int FP = 32;        // padded feature / coefficient slots per row
constexpr int REC = 48;       // doubles per component record in the state
constexpr int CT = 64;        // components per LDS tile (pass 1) and per pass-2 workgroup
constexpr int PT = 64;        // points per LDS tile (pass 2)
constexpr int P1_PB = 4;      // 16-point blocks per wave in pass 1
constexpr int P1_PTS = 4 * P1_PB * 16;  // points per pass-1 workgroup (4 waves)
constexpr int MOM_BLOCKS = 1024;
constexpr int CS = 32;        // candidate slots per (point, lane group) in the exact sweep
constexpr float DEAD_C0 = -1.0e30f;     // constant slot of padding components

// device flag bits
constexpr int FLAG_NOT_PD = 1;
constexpr int FLAG_NONFINITE = 2;

inline __host__ __device__ int nfeat(int D) { return 1 + D + D * (D + 1) / 2; }
inline __host__ __device__ int ntri(int D) { return D * (D + 1) / 2; }
inline __host__ __device__ int direct_stride(int D) { return D <= 6 ? 32 : 48; }
// doubles per component row of the statistics partials (F = 45 at D = 8)
inline __host__ __device__ int stat_stride(int D) { return D <= 6 ? 32 : 48; }

// Per-frame data written by the moment kernels, read by every later kernel.
struct FrameInfo {
  float mu[MAXD];        // centring offsets (FP32 values, used exactly)
  float inv_s[MAXD];     // 1 / s, s a power of two (exact)
  double s[MAXD];
  double sum_alpha_q, sum_alpha_p;
  int32_t flags;
  int32_t pad0;
  unsigned long long refined1, refined2;
  int32_t n_over;        // points whose candidate lists overflowed in the sweep
  int32_t lam_anchor;    // curvature class anchor of the component sort (bin of lambda, see lam_bin)
  unsigned long long blocks;      // 64-point x 64-component blocks screened by the exact sweep
  unsigned long long blocks_cum;  // the same, summed since the last clear of the flags
  float screen_slack;    // split-BF16 screen bound for the mean |c| and |phi| (log2 units)
  int32_t screen_prec;   // screen precision the last sweep used
};

// Bound of a 64-row tile of the spatially sorted component table (culled exact sweep).
struct TileInfo {
  float G;          // max over the tile of the score constant g2 (log2 units)
  float Lam;        // min over the tile of lambda_k: s2 <= g2 - lambda_k |x_S - m_k,S|^2
  float lo[3], hi[3];  // box of the means in the culling coordinates (the others read 0)
  uint32_t code;    // Hilbert code of the tile's first row
  uint32_t pad;
};

// Bound of one row of the sorted component table: s2 <= G - Lam |x_S - m_S|^2 (m rounded to
// nearest), and the norm of the row's expanded coefficients (the screen's error scale)
struct RowBound {
  float G, Lam;
  float m[3];
  float nc;
  float pad[2];
};

// float roundings of a double that stay below / above it
__device__ __forceinline__ float f_down(double v) {
  float f = (float)v;
  return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float f_up(double v) {
  float f = (float)v;
  return (double)f < v ? nextafterf(f, INFINITY) : f;
}

// Coordinate blocks. With a modal split s (0 < s < D) a component is two independent
// Normal-Wishart blocks (Sec. 2.1.2): coordinates [0, s) and [s, D), each with its own kappa, nu
// and W (cross-block entries of W^-1 are zero). The record keeps block 0's kappa and nu at slots
// 1 and 2 and block 1's at KC and KC + 1. With s = 0 all coordinates form one block.
__host__ __device__ __forceinline__ int coord_block(int i, int split) { return (split > 0 && i >= split) ? 1 : 0; }
__host__ __device__ constexpr int rec_kc(int D) { return 3 + D + D * (D + 1) / 2; }
__device__ __forceinline__ double rec_kappa(const double* q, int D, int b) { return b ? q[rec_kc(D)] : q[1]; }
__device__ __forceinline__ double rec_nu(const double* q, int D, int b) { return b ? q[rec_kc(D) + 1] : q[2]; }

// lambda_k, a lower bound on the curvature of the score (log2 units) in the first ns (<= 3)
// raw coordinates S: s2 = g2 - (log2e / 2) d^T A d with A = blockdiag(nu_b W_b) and, with d
// restricted to S, d^T A d >= d_S^T ((A^-1)_SS)^-1 d_S >= |d_S|^2 / tr (A^-1)_SS, where
// (A^-1)_ii = (W^-1)_ii / nu_b(i). Slightly reduced so that its FP32 rounding stays below the bound.
// q: the component's record. Returns 0 when the trace is not positive.
__device__ __forceinline__ float comp_lambda(const double* q, int D, int split, int ns) {
  double tr = 0.0;
  for (int i = 0; i < ns; ++i) tr += q[3 + D + i * D - i * (i - 1) / 2] / rec_nu(q, D, coord_block(i, split));
  return tr > 0.0 ? (float)(0.5 * LOG2E / tr * (1.0 - 1e-6)) : 0.0f;
}

// histogram bin of lambda in half-octaves, 0..127 (lambda <= 0 maps to bin 0)
constexpr int LAM_BINS = 128;
__device__ __forceinline__ int lam_bin(float lam) {
  if (!(lam > 0.0f)) return 0;
  const int b = (int)floorf(2.0f * log2f(lam)) + 64;
  return b < 0 ? 0 : (b > LAM_BINS - 1 ? LAM_BINS - 1 : b);
}

// Offsets (bytes) into the caller's workspace.
struct Layout {
  size_t phi8, phis, c8, cs8;  // FP8 tier: e4m3 rows and the factors that undo their scaling
  int fp8;
  int f32rows;  // the points' FP32 feature rows are read (FP32, automatic and FP8 screens; plain tiers)
  size_t frame, mom_part, phi32, phih, phil, nphi, lse2, lse_part, direct, c32, ch, cl, nc, kl,
      spart, stats, cand_k, cand_s, cand_n, over_list, fx, ccount, coffset, ent_n, segoff, seg_miss, total;
  int64_t Kpad, n_lse_part;
  int64_t ent_cap;  // entries of ent_n
  int nsplit_max;
  // spatial ordering (culled exact sweep)
  size_t pkeys, porder, pcode, ckeys, corder, cinv, ccode, lam, tinfo, rowb, ncg, lhist, scan_part;
  // the coefficient rows in component order (FP32, BF16 hi / lo, norms), written while the
  // components are sorted and gathered into the sorted tables with the tile bounds; c32u only
  // where a screen of the context's precision reads FP32 rows (stage_c32)
  size_t c32u, chu, clu, ncu;
  int stage_c32;
  size_t bcost, bcode, border;  // per 64-point block of the culled sweep: measured time, Hilbert code
                                // of its first point, dispatch order
  size_t bprev;                 // number of blocks of the last sweep (int64)
  size_t slist;                 // per block, the tiles it scores directly (uint32, Kpad / 64 per block)
  size_t elbo_part;  // 2 x 256 partial sums of the ELBO reduction
  size_t scr_part, scr_gate;  // screen choice: 2 x 256 partial norm sums, two gate flags
  size_t rx_tmp, rx_hist, rx_off, rx_part;  // radix sort: ping-pong keys, digit histograms, scan
  size_t rx2_tmp, rx2_hist, rx2_off, rx2_part;  // the same for the component sort (runs concurrently)
  // learned proposal (workspace)
  size_t p_tthr;  // per point: lower bound on its C-th best logit
  size_t p_E8, p_sE, p_h8, p_sh;  // FP8 logits: e4m3 embedding and point rows, their scale factors
  size_t p_tlpart, p_tdpart, p_twpart;  // training: per-slice partial LSE, dh2 rows, weight gradients
  size_t p_Ebf, p_EbfT, p_betap, p_W2T, p_h2b, p_tz, p_tk, p_tcnt, p_aud, p_gate, p_th1, p_th2, p_txs, p_tlse,
      p_tdh2, p_tdp1, p_th2b, p_th2T, p_tloss, p_grads;
  int64_t Bpad_max;
  // learned proposal (state, byte offsets from the start of the state buffer)
  size_t s_W, s_mu, s_is, s_m1, s_m2, s_step, state_total;
};

// State buffer: a header followed by the frame-prior and posterior records.
struct StateHeader {
  int64_t magic, abi, D, K;
  int64_t pad[28];
};
constexpr int64_t STATE_MAGIC = 0x5342474256ll;  // "VBGBS"

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Digamma for x > 0: upward recurrence psi(x) = psi(x+1) - 1/x until x >= 10,
// then the asymptotic series of Abramowitz & Stegun 6.3.18 (Bernoulli numbers
// B_2..B_14); the first omitted term is below 1e-16 at x = 10.
__device__ inline double vb_digamma(double x) {
  double acc = 0.0;
  while (x < 10.0) {
    acc -= 1.0 / x;
    x += 1.0;
  }
  const double r = 1.0 / x, r2 = r * r;
  const double t =
      r2 * (1.0 / 12 -
            r2 * (1.0 / 120 -
                  r2 * (1.0 / 252 - r2 * (1.0 / 240 - r2 * (1.0 / 132 - r2 * (691.0 / 32760 - r2 / 12))))));
  return acc + log(x) - 0.5 * r - t;
}

// ln Gamma_D(a) = D(D-1)/4 ln pi + sum_{i=1..D} ln Gamma(a + (1-i)/2)
__device__ inline double vb_mvlgamma(double a, int D) {
  double s = 0.25 * D * (D - 1) * LNPI;
  for (int i = 1; i <= D; ++i) s += lgamma(a + 0.5 * (1 - i));
  return s;
}

// Exact score of one (point, component) pair in log2 units, FP64, direct
// (non-expanded) form: s2 = g2 - || U (x - m) ||^2 with U = sqrt(nu log2(e) / 2) L^{-1},
// L L^T = W^{-1}. Row layout: [g2, m_0..m_{D-1}, U lower-packed row-major].
__device__ __forceinline__ double direct_score2(const double* __restrict__ T, const float* __restrict__ x,
                                                int D) {
  double d[MAXD];
#pragma unroll
  for (int i = 0; i < MAXD; ++i)
    if (i < D) d[i] = (double)x[i] - T[1 + i];
  double q = 0.0;
  const double* U = T + 1 + D;
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    if (i < D) {
      double y = 0.0;
#pragma unroll
      for (int j = 0; j <= i; ++j) y = fma(U[i * (i + 1) / 2 + j], d[j], y);
      q = fma(y, y, q);
    }
  }
  return T[0] - q;
}

// Same score, also returning the difference vector d = x - m (raw coordinates, FP64).
__device__ __forceinline__ double direct_score2_d(const double* __restrict__ T, const float* __restrict__ x, int D,
                                                  double* d) {
#pragma unroll
  for (int i = 0; i < MAXD; ++i) d[i] = (i < D) ? (double)x[i] - T[1 + i] : 0.0;
  double q = 0.0;
  const double* U = T + 1 + D;
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    if (i < D) {
      double y = 0.0;
#pragma unroll
      for (int j = 0; j <= i; ++j) y = fma(U[i * (i + 1) / 2 + j], d[j], y);
      q = fma(y, y, q);
    }
  }
  return T[0] - q;
}

template <int D>
__device__ __forceinline__ double direct_score2_dt(const double* __restrict__ T, const float* __restrict__ x,
                                                   double* d) {
#pragma unroll
  for (int i = 0; i < D; ++i) d[i] = (double)x[i] - T[1 + i];
  double q = 0.0;
  const double* U = T + 1 + D;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double y = 0.0;
#pragma unroll
    for (int j = 0; j <= i; ++j) y = fma(U[i * (i + 1) / 2 + j], d[j], y);
    q = fma(y, y, q);
  }
  return T[0] - q;
}

// FP64 score (log2 units) of one pair in direct form, for a run-time D <= 6 (the MFMA paths)
__device__ __forceinline__ double direct_score2_rt(const double* __restrict__ row, const float* __restrict__ x, int D) {
  double d[MAXD];
  switch (D) {
    case 1: return direct_score2_dt<1>(row, x, d);
    case 2: return direct_score2_dt<2>(row, x, d);
    case 3: return direct_score2_dt<3>(row, x, d);
    case 4: return direct_score2_dt<4>(row, x, d);
    case 5: return direct_score2_dt<5>(row, x, d);
    default: return direct_score2_dt<6>(row, x, d);
  }
}

template <int D>
__device__ __forceinline__ double direct_score2_t(const double* __restrict__ T, const double* __restrict__ x) {
  double d[D];
#pragma unroll
  for (int i = 0; i < D; ++i) d[i] = x[i] - T[1 + i];
  double q = 0.0;
  const double* U = T + 1 + D;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double y = 0.0;
#pragma unroll
    for (int j = 0; j <= i; ++j) y = fma(U[i * (i + 1) / 2 + j], d[j], y);
    q = fma(y, y, q);
  }
  return T[0] - q;
}

// ---------------------------------------------------------------------------
// host-side launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
Layout make_layout(const vbgs_params& p);

struct DevPtrs {
  char* ws;
  double* state;
  const Layout* L;
  int D;
  int64_t K;
  int split;  // modal split (0: one block)
  int nsp;    // leading coordinates the culling bounds use (1..3)
  template <class T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  FrameInfo* frame() const { return at<FrameInfo>(L->frame); }
  double* prior() const { return state + sizeof(StateHeader) / 8; }
  double* post() const { return prior() + (size_t)K * REC; }
};

struct Init0 {
  double W0inv[MAXD * MAXD];
  double alpha0, kappa0, nu0;
  int split;
};

hipError_t launch_init_state(const DevPtrs& d, const double* m0, const Init0& init, hipStream_t s);
// part: 0 frame moments, 1 features, 2 both
hipError_t launch_frame_prep(const DevPtrs& d, const float* X, int64_t N, hipStream_t s, int part = 2);
// the sum of alpha over the posterior (FrameInfo::sum_alpha_q), which the coefficient rows need
hipError_t launch_alpha(const DevPtrs& d, hipStream_t s);
// alpha = false: launch_alpha has already run on this stream or one it waited for; staged = true
// (culled path): the expanded rows go to the component-order staging tables (launch_tile_info
// gathers them into the sorted order), else straight into the tables in component order
hipError_t launch_coeffs(const DevPtrs& d, hipStream_t s, bool alpha = true, bool staged = false);
// per-component KL terms of the ELBO (after launch_coeffs: it reads the frame's alpha sum)
hipError_t launch_kl(const DevPtrs& d, hipStream_t s);
hipError_t launch_update(const DevPtrs& d, int commit, hipStream_t s);
hipError_t launch_elbo(const DevPtrs& d, int64_t n_lse_part, double* out, hipStream_t s);
hipError_t launch_get_set(const DevPtrs& d, int which, int set, double* alpha, double* kappa, double* m,
                          double* Winv, double* nu, hipStream_t s);
hipError_t launch_clear_flags(const DevPtrs& d, hipStream_t s);
// dst->flags |= src->flags (sticky device flags of one workspace added to another's)
hipError_t launch_merge_flags(const FrameInfo* src, FrameInfo* dst, hipStream_t s);
// rendering: the position marginal of the model's posterior written into the s-dimensional state
// of sp, and reg[k] = [m_c, B]; the colour at query positions from sp's first pass
hipError_t launch_render_marginal(const DevPtrs& model, const DevPtrs& sp, double* reg, hipStream_t s);
hipError_t launch_psnr(const float* a, const float* b, int64_t n, double* out, hipStream_t s);
hipError_t launch_sort_points(const DevPtrs& d, const float* X, int64_t N, hipStream_t s);
hipError_t launch_excl_scan(const int32_t* cnt, int64_t n, int32_t* off, int32_t* part, hipStream_t s);
constexpr int RX_B = 1024;  // keys per workgroup of the radix sort
hipError_t launch_sort_comps(const DevPtrs& d, hipStream_t s);
hipError_t launch_tile_info(const DevPtrs& d, hipStream_t s);
hipError_t launch_reassign(const DevPtrs& d, const float* X, int64_t N, const double* lse, const double* gumbel,
                           int64_t n, int32_t* out_pts, int32_t* out_comps, hipStream_t s);

struct EstepCfg {
  int prec;      // vbgs_prec
  int exact;     // 1: screen + exact rescoring
  float T2;      // screen margin in log2 units
  int nsplit;    // pass-2 point splits
  const int32_t* gate = nullptr;  // device flag gating the exact dense kernels (proposal fallback)
  int cull = 0;                   // culled sweep over spatially sorted points and components
  int seg = 0;                    // kept pairs written straight into per-component segments
  int order_reset = 0;            // forget the measured block costs (first sweep of a context)
};

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
  const uint8_t* phi8;        // FP8 tier: N x 32 e4m3 features
  const float* phis;          // N: factor undoing each feature row's scaling
  const uint8_t* c8;          // Kpad x 32 e4m3 coefficients
  const float* cs8;           // Kpad: factor undoing each coefficient row's scaling
  double* lse2;               // N (log2 units)
  double* lse_part;           // pass-1 workgroups
  double* lse_out;            // N (nats) or null
  double* spart;              // nsplit x Kpad x 32
  double* stats;              // K x F statistics (exact mode: written by the statistics kernels)
  double* stats_out;          // the caller's copy of them, or null
  int32_t* cand_k;            // exact sweep: N x 4 x CS component indices
  float* cand_s;              // N x 4 x CS exact scores (log2 units, rounded to FP32)
  int32_t* cand_n;            // N x 4 list lengths, -1 = overflowed point
  int32_t* over_list;         // overflowed points
  unsigned long long* fx;     // Kpad x 32 x {lo, hi}: 128-bit fixed-point statistics (overflowed points)
  int32_t* ccount;            // Kpad + 1: kept pairs per component (their ranks: keep_pairs)
  int32_t* coffset;           // Kpad + 1: exclusive scan of ccount
  int32_t* ent_n;             // kept pairs grouped by component: point index
  const int2* seg;            // or null: per component, its segment [x, y) of ent_n sized from the
                              // last counts; keep_pairs writes each pair at x + rank when it fits
  int32_t* seg_miss;          // set when a pair did not fit: the statistics take the scan + transpose
  FrameInfo* frame;
  const int32_t* gate;        // when set, the exact dense kernels run only if gate[0] != 0
  const int32_t* porder;      // culled sweep: sorted position -> point index
  const uint32_t* pcode;      // Hilbert codes of the sorted points
  const int32_t* corder;      // sorted row -> component index
  const TileInfo* tinfo;      // per-tile bounds of the sorted component table
  const RowBound* rowb;       // per-row bounds of the sorted component table
  const f32x4* ncg;           // per tile and lane group g: for each 16-row block cb, the largest
                              // coefficient norm of rows 16 cb + 4 g .. 16 cb + 4 g + 3
  int32_t* scan_part;         // block sums of the pair-count scan
  float* bcost;               // culled sweep: per 64-point block, the duration of its last sweep
  uint32_t* bcode;            // and the Hilbert code of its first point then
  int32_t* border;            // culled sweep: dispatch position -> block (costliest first per XCD)
  int64_t* bprev;             // culled sweep: blocks of the last launch (their bcost / bcode entries)
  uint32_t* slist;            // culled sweep: per 64-point block, its tiles scored directly (Kpad / 64 each)
  int64_t nb_cap;             // capacity of bcost / border
  double* scr_part;           // screen choice: partial sums of the row and feature norms
  int32_t* scr_gate;          // screen choice: [run split BF16, run FP32]
  int order_reset;
  int64_t N, K, Kpad;
  int D, dts, nsplit;
  float T2, eps;
  int cull;                   // the culled sweep ran: sorted tables and bounds are valid
  int nsp;                    // leading coordinates of the culling bounds (1..3); the others read 0
};
EArgs make_eargs(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out);
// stage -1: the whole first pass; exact MFMA mode in stages 0 (clear the transpose counters),
// 4 (with culling, the blocks' dispatch order), 1 (screen choice), 3 (the screening sweep) and 2
// (exact per-point LSE), in that order (0 and 4 need no component work); other modes run the
// whole pass in stage 3
hipError_t launch_pass1(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, double* lse_out,
                        hipStream_t s, int stage = -1);
// stats_out (or null): the caller's statistics; the exact mode writes them in pass 2 (fold is then empty)
hipError_t launch_pass2(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, hipStream_t s,
                        double* stats_out);
hipError_t launch_fold(const DevPtrs& d, const EstepCfg& c, double* stats_out, hipStream_t s);
// exact statistics from candidate lists (transpose + per-component sums) and exact per-point LSE
hipError_t launch_exact_sweep(const EArgs& a, int prec, int D, int64_t N, hipStream_t s, int cull = 0);
hipError_t launch_point_lse(const EArgs& a, int D, int64_t N, hipStream_t s);
hipError_t launch_sparse_stats(const EArgs& a, int D, int64_t N, hipStream_t s);
// the kept pairs' segments (EArgs::seg) for the next culled sweep, from the counts of the last one;
// before the counts are cleared
hipError_t launch_seg_layout(const DevPtrs& d, hipStream_t s);
hipError_t launch_render(const DevPtrs& d, const EstepCfg& c, const float* X, int64_t N, const double* reg, int Dc,
                         float* out, hipStream_t s);

}  // namespace vbgs
