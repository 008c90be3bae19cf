// Spatial ordering for the culled exact sweep: 3-D Hilbert-curve keys of points and component means,
// a stable radix sort of 64-bit keys on their code (key = code << 32 | index, so every key is
// unique and the order is deterministic; the reassignment step sorts with a bitonic network), and
// per-tile bounds of the sorted component rows.
#include "vbgs_internal.h"

namespace vbgs {

// spread the low 10 bits of v so that bit i moves to bit 3i
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Hilbert-curve code of the first ns (<= 3) coordinates, each quantised to 10 bits over the
// frame's window mu +- 4 s (clamped): the same map for points and component means. Unlike the
// Morton order, consecutive cells of the Hilbert order are always neighbours, so a run of
// consecutive points (a sweep block) or components (a tile) has a tighter box. The index comes
// from Skilling's transform of the coordinates ("Programming the Hilbert curve", 2004): undo the
// per-level reflections and exchanges, Gray-encode, and interleave the bits, most significant
// level first, coordinate 0 first within a level.
__device__ __forceinline__ uint32_t curve_code(const float* x, const double* xd, int ns, const FrameInfo* fr) {
  uint32_t q[3] = {0u, 0u, 0u};
  for (int i = 0; i < ns; ++i) {
    const double v = x ? (double)x[i] : xd[i];
    double u = (v - (double)fr->mu[i]) / (8.0 * fr->s[i]) + 0.5;
    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    q[i] = (uint32_t)(u * 1023.0);
  }
  if (ns > 1) {
    for (uint32_t b = 1u << 9; b > 1u; b >>= 1) {
      const uint32_t low = b - 1u;
      for (int i = 0; i < ns; ++i) {
        if (q[i] & b) {
          q[0] ^= low;
        } else {
          const uint32_t t = (q[0] ^ q[i]) & low;
          q[0] ^= t;
          q[i] ^= t;
        }
      }
    }
    for (int i = 1; i < ns; ++i) q[i] ^= q[i - 1];
    uint32_t t = 0u;
    for (uint32_t b = 1u << 9; b > 1u; b >>= 1)
      if (q[ns - 1] & b) t ^= b - 1u;
    for (int i = 0; i < ns; ++i) q[i] ^= t;
  }
  uint32_t code = 0;
  for (int i = 0; i < ns; ++i) code |= spread3(q[i]) << (ns - 1 - i);
  return code;
}

__global__ void k_point_keys(const float* __restrict__ X, int64_t N, int64_t Npow, int D, int ns, const FrameInfo* fr,
                             unsigned long long* __restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Npow) return;
  keys[n] = n < N ? ((unsigned long long)curve_code(X + n * D, nullptr, ns, fr) << 32) | (unsigned long long)n
                  : ~0ull;
}

// Components are sorted by (curvature class, Hilbert code of the mean): a tile bound uses the
// smallest curvature lambda of its rows, so rows of very different lambda are kept apart. The
// classes are octave pairs (factor 4 in lambda) below an anchor, the half-octave bin of the 90th
// percentile of lambda over the components: class 0 holds lambda >= anchor / 4, class 3 the
// broadest components (and degenerate ones).
__global__ void k_lam_hist(const double* __restrict__ post, int64_t K, int D, int split, int ns,
                           int* __restrict__ hist) {
  __shared__ int h[LAM_BINS];
  for (int i = threadIdx.x; i < LAM_BINS; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[lam_bin(comp_lambda(post + k * REC, D, split, ns))], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < LAM_BINS; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

__global__ void k_lam_anchor(int* __restrict__ hist, int64_t K, FrameInfo* fr) {
  if (threadIdx.x != 0) return;
  int64_t above = 0;
  int b = LAM_BINS - 1;
  for (; b > 0; --b) {
    above += hist[b];
    if (above * 10 >= K) break;
  }
  fr->lam_anchor = b;
}

__global__ void k_zero_hist(int* hist) {
  if (threadIdx.x < LAM_BINS) hist[threadIdx.x] = 0;
}

__global__ void k_comp_keys(const double* __restrict__ post, int64_t K, int64_t Kpow, int D, int split, int ns,
                            const FrameInfo* fr, unsigned long long* __restrict__ keys) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Kpow) return;
  if (k >= K) {
    keys[k] = ~0ull;
    return;
  }
  const double* q = post + k * REC;
  const int b = lam_bin(comp_lambda(q, D, split, ns));
  const int gap = fr->lam_anchor - b;
  const uint32_t cls = b == 0 ? 3u : (gap < 4 ? 0u : (uint32_t)min(gap / 4, 3));
  const uint32_t code = (cls << 30) | curve_code(nullptr, q + 3, ns, fr);
  keys[k] = ((unsigned long long)code << 32) | (unsigned long long)k;
}

// ---- bitonic sort ---------------------------------------------------------------------------
constexpr int BS_LOCAL = 2048;  // elements per workgroup in the LDS stages (1024 threads)

__device__ __forceinline__ void cmp_swap(unsigned long long& a, unsigned long long& b, bool up) {
  if ((a > b) == up) {
    const unsigned long long t = a;
    a = b;
    b = t;
  }
}

// all stages k <= BS_LOCAL (full sort of each 2048-chunk, alternating directions like the global network)
__global__ __launch_bounds__(1024) void k_bitonic_local_sort(unsigned long long* keys) {
  __shared__ unsigned long long s[BS_LOCAL];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * BS_LOCAL;
  s[t] = keys[base + t];
  s[t + 1024] = keys[base + t + 1024];
  __syncthreads();
  for (int k = 2; k <= BS_LOCAL; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int i = 2 * t - (t & (j - 1));  // lower index of this thread's pair
      const int64_t gi = base + i;
      const bool up = (gi & k) == 0;
      cmp_swap(s[i], s[i + j], up);
      __syncthreads();
    }
  }
  keys[base + t] = s[t];
  keys[base + t + 1024] = s[t + 1024];
}

// stage k > BS_LOCAL, the passes with j < BS_LOCAL inside each chunk
__global__ __launch_bounds__(1024) void k_bitonic_local_merge(unsigned long long* keys, int64_t k) {
  __shared__ unsigned long long s[BS_LOCAL];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * BS_LOCAL;
  s[t] = keys[base + t];
  s[t + 1024] = keys[base + t + 1024];
  __syncthreads();
  for (int j = BS_LOCAL >> 1; j > 0; j >>= 1) {
    const int i = 2 * t - (t & (j - 1));
    const bool up = ((base + i) & k) == 0;
    cmp_swap(s[i], s[i + j], up);
    __syncthreads();
  }
  keys[base + t] = s[t];
  keys[base + t + 1024] = s[t + 1024];
}

// one global pass (stage k, distance j >= BS_LOCAL): one thread per pair
__global__ __launch_bounds__(256) void k_bitonic_global(unsigned long long* keys, int64_t n, int64_t k, int64_t j) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n / 2) return;
  const int64_t i = 2 * t - (t & (j - 1));
  const bool up = (i & k) == 0;
  unsigned long long a = keys[i], b = keys[i + j];
  if ((a > b) == up) {
    keys[i] = b;
    keys[i + j] = a;
  }
}

hipError_t launch_sort_keys(unsigned long long* keys, int64_t npow, hipStream_t s) {
  // npow: a power of two >= BS_LOCAL
  hipLaunchKernelGGL(k_bitonic_local_sort, dim3((unsigned)(npow / BS_LOCAL)), dim3(1024), 0, s, keys);
  for (int64_t k = 2 * BS_LOCAL; k <= npow; k <<= 1) {
    for (int64_t j = k >> 1; j >= BS_LOCAL; j >>= 1)
      hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((npow / 2 + 255) / 256)), dim3(256), 0, s, keys, npow, k,
                         j);
    hipLaunchKernelGGL(k_bitonic_local_merge, dim3((unsigned)(npow / BS_LOCAL)), dim3(1024), 0, s, keys, k);
  }
  return hipGetLastError();
}

// sorted keys -> order (sorted position -> index), inverse (index -> sorted position), codes
__global__ void k_unpack_order(const unsigned long long* __restrict__ keys, int64_t n, int32_t* __restrict__ order,
                               int32_t* __restrict__ inverse, uint32_t* __restrict__ codes) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const unsigned long long v = keys[j];
  const int32_t idx = (int32_t)(v & 0xFFFFFFFFull);
  order[j] = idx;
  if (inverse) inverse[idx] = (int32_t)j;
  if (codes) codes[j] = (uint32_t)(v >> 32);
}

// 16-byte chunks of the tile's rows from the component-order table (consecutive lanes on
// consecutive chunks of a row, so reads and writes are whole rows); k: the component of row `lane`
template <int C>
__device__ __forceinline__ void gather_rows(const void* __restrict__ src, void* __restrict__ dst, int64_t t, int k,
                                            int lane) {
  const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
  u32x4* d4 = reinterpret_cast<u32x4*>(dst);
#pragma unroll
  for (int q = 0; q < C; ++q) {
    const int i = q * 64 + lane, r = i / C, c = i % C;
    const int kr = __shfl(k, r);
    d4[(t * CT + r) * C + c] = s4[(int64_t)kr * C + c];
  }
}

struct TileRows {  // component-order rows (c32u may be null) -> their sorted tables
  const float* c32u;
  const uint16_t* chu;
  const uint16_t* clu;
  const float* ncu;
  float* c32;
  uint16_t* ch;
  uint16_t* cl;
  float* nc;
  RowBound* rowb;
};

// Per 64-row tile of the sorted component table: the rows gathered from component order, each
// row's bound record (G = g2 rounded up, its lambda, the first three coordinates of its mean, its
// norm), and the tile's G = max g2, Lambda = min lambda (a lower bound on the curvature of the
// score in the first three raw coordinates), box of those coordinates of the means, and the
// Hilbert code of the first row. G and the box are rounded outward, so the bound formed from them
// in FP32 stays above every score of the tile. Empty (padding) tiles get G = -inf. Dead rows
// (padding, and components whose W^-1 is not positive definite) get G = -FLT_MAX.
__global__ __launch_bounds__(256) void k_tile_info(const int32_t* __restrict__ corder,
                                                   const uint32_t* __restrict__ ccode, int64_t K, int64_t ntiles,
                                                   int D, int ns, const double* __restrict__ direct, int dts,
                                                   const float* __restrict__ lam, TileRows g,
                                                   TileInfo* __restrict__ info, float* __restrict__ ncg) {
  // one wave per tile, lane = row
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const int64_t j = t * CT + lane;
  const int k = j < K ? corder[j] : (int)j;  // padding rows: their own (dead) rows
  if (g.c32u) gather_rows<FP * 4 / 16>(g.c32u, g.c32, t, k, lane);
  gather_rows<FP * 2 / 16>(g.chu, g.ch, t, k, lane);
  gather_rows<FP * 2 / 16>(g.clu, g.cl, t, k, lane);
  const float nc_row = g.ncu[k];
  g.nc[j] = nc_row;
  float G = -INFINITY, Lm = INFINITY, lo[3], hi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lo[i] = INFINITY;
    hi[i] = -INFINITY;
  }
  RowBound rb{};
  rb.G = -FLT_MAX;
  if (j < K) {
    const double* T = direct + (int64_t)k * dts;
    rb.G = f_up(T[0]);
    rb.Lam = lam[k];
    rb.nc = nc_row;
    G = rb.G;
    Lm = rb.Lam;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i < ns) {
        rb.m[i] = (float)T[1 + i];
        lo[i] = f_down(T[1 + i]);
        hi[i] = f_up(T[1 + i]);
      }
  }
  g.rowb[j] = rb;
  for (int o = 1; o < 64; o <<= 1) {
    G = fmaxf(G, __shfl_xor(G, o));
    Lm = fminf(Lm, __shfl_xor(Lm, o));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lo[i] = fminf(lo[i], __shfl_xor(lo[i], o));
      hi[i] = fmaxf(hi[i], __shfl_xor(hi[i], o));
    }
  }
  // norms of the four-row groups, stored [tile][g][cb] (row 16 cb + 4 g + i): each lane of the
  // sweep reads its four values with one 16-byte load
  float nc = nc_row;
  nc = fmaxf(nc, __shfl_xor(nc, 1));
  nc = fmaxf(nc, __shfl_xor(nc, 2));
  if ((lane & 3) == 0) {
    const int cb = lane >> 4, gq = (lane >> 2) & 3;
    ncg[t * CT / 4 + gq * 4 + cb] = nc;
  }
  if (lane == 0) {
    TileInfo ti;
    ti.G = G;
    ti.Lam = Lm;
    for (int i = 0; i < 3; ++i) {
      ti.lo[i] = i < ns ? lo[i] : 0.0f;
      ti.hi[i] = i < ns ? hi[i] : 0.0f;
    }
    ti.code = t * CT < K ? ccode[t * CT] : 0xFFFFFFFFu;
    ti.pad = 0;
    info[t] = ti;
  }
}

// ---- stable LSD radix sort of 64-bit keys on their upper 32 bits (four 8-bit digits) -------------
// The lower 32 bits (the element index) ride along; the input is in index order, so equal codes
// keep index order, as the full 64-bit order would. Per pass: digit histograms per workgroup of
// RX_B keys (digit-major), their exclusive scan, and a stable scatter that ranks keys of equal digit
// within each wave by ballots on the digit's bits.
__global__ __launch_bounds__(256) void k_radix_hist(const unsigned long long* __restrict__ keys, int64_t n, int shift,
                                                    int32_t* __restrict__ hist, int64_t nb) {
  __shared__ int32_t h[256];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RX_B;
#pragma unroll
  for (int i = 0; i < RX_B / 256; ++i) {
    const int64_t j = base + i * 256 + t;
    if (j < n) atomicAdd(&h[(int)((keys[j] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  hist[(int64_t)t * nb + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const unsigned long long* __restrict__ in,
                                                       unsigned long long* __restrict__ out, int64_t n, int shift,
                                                       const int32_t* __restrict__ off, int64_t nb) {
  __shared__ int32_t run[256];    // next output position per digit
  __shared__ int32_t wc[4][256];  // per wave: keys of each digit in the current chunk, then their base
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = off[(int64_t)t * nb + blockIdx.x];
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * RX_B;
  for (int ch = 0; ch < RX_B / 256; ++ch) {
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][t] = 0;
    __syncthreads();
    const int64_t j = base + ch * 256 + t;
    const bool valid = j < n;
    const unsigned long long key = valid ? in[j] : 0ull;
    const int dg = (int)((key >> shift) & 255ull);
    unsigned long long eq = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bal = __ballot(valid && ((dg >> b) & 1));
      eq &= ((dg >> b) & 1) ? bal : ~bal;
    }
    const int rank = __popcll(eq & below);
    if (valid && rank == 0) wc[w][dg] = __popcll(eq);
    __syncthreads();
    {  // thread t: digit t, bases of the four waves
      int acc = run[t];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = wc[q][t];
        wc[q][t] = acc;
        acc += v;
      }
      run[t] = acc;
    }
    __syncthreads();
    if (valid) out[wc[w][dg] + rank] = key;
    __syncthreads();
  }
}

// sorts keys[0, n) (tmp: n keys of scratch); four passes, so the result is back in keys. The
// component sort (comps) has scratch of its own, so that it can run beside the point sort.
// passes 8-bit digits from the top of the code (4: all 32 bits; 3: the top 24, equal keys there
// keeping index order); *sorted is the buffer that holds the result
static hipError_t radix_sort32(const DevPtrs& d, unsigned long long* keys, int64_t n, hipStream_t s, bool comps,
                               int passes, unsigned long long** sorted) {
  *sorted = keys;
  if (n <= 1) return hipSuccess;
  const Layout& L = *d.L;
  unsigned long long* tmp = d.at<unsigned long long>(comps ? L.rx2_tmp : L.rx_tmp);
  int32_t* hist = d.at<int32_t>(comps ? L.rx2_hist : L.rx_hist);
  int32_t* off = d.at<int32_t>(comps ? L.rx2_off : L.rx_off);
  int32_t* part = d.at<int32_t>(comps ? L.rx2_part : L.rx_part);
  const int64_t nb = (n + RX_B - 1) / RX_B;
  unsigned long long* src = keys;
  unsigned long long* dst = tmp;
  for (int pass = 4 - passes; pass < 4; ++pass) {
    const int shift = 32 + 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(256), 0, s, src, n, shift, hist, nb);
    hipError_t e = launch_excl_scan(hist, 256 * nb, off, part, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(256), 0, s, src, dst, n, shift, off, nb);
    unsigned long long* x = src;
    src = dst;
    dst = x;
  }
  *sorted = src;
  return hipGetLastError();
}

// the top 24 bits of the codes (cells of 1/256 of the frame extent per axis) order the tiles as well as
// all 32 do (same sweep time) with one pass fewer on each side of the fork
constexpr int POINT_SORT_PASSES = 3, COMP_SORT_PASSES = 3;

hipError_t launch_sort_points(const DevPtrs& d, const float* X, int64_t N, hipStream_t s) {
  const Layout& L = *d.L;
  if (N <= 0) return hipSuccess;
  unsigned long long* keys = d.at<unsigned long long>(L.pkeys);
  hipLaunchKernelGGL(k_point_keys, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, X, N, N, d.D, d.nsp,
                     d.frame(), keys);
  unsigned long long* sorted;
  hipError_t e = radix_sort32(d, keys, N, s, false, POINT_SORT_PASSES, &sorted);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_order, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, sorted, N,
                     d.at<int32_t>(L.porder), (int32_t*)nullptr, d.at<uint32_t>(L.pcode));
  return hipGetLastError();
}

hipError_t launch_sort_comps(const DevPtrs& d, hipStream_t s) {
  const Layout& L = *d.L;
  unsigned long long* keys = d.at<unsigned long long>(L.ckeys);
  int* hist = d.at<int>(L.lhist);
  hipLaunchKernelGGL(k_zero_hist, dim3(1), dim3(LAM_BINS), 0, s, hist);
  hipLaunchKernelGGL(k_lam_hist, dim3((unsigned)min((d.K + 255) / 256, (int64_t)1024)), dim3(256), 0, s, d.post(), d.K, d.D,
                     d.split, d.nsp, hist);
  hipLaunchKernelGGL(k_lam_anchor, dim3(1), dim3(64), 0, s, hist, d.K, d.frame());
  hipLaunchKernelGGL(k_comp_keys, dim3((unsigned)((d.K + 255) / 256)), dim3(256), 0, s, d.post(), d.K, d.K, d.D,
                     d.split, d.nsp, d.frame(), keys);
  unsigned long long* sorted;
  hipError_t e = radix_sort32(d, keys, d.K, s, true, COMP_SORT_PASSES, &sorted);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_order, dim3((unsigned)((d.K + 255) / 256)), dim3(256), 0, s, sorted, d.K,
                     d.at<int32_t>(L.corder), d.at<int32_t>(L.cinv), d.at<uint32_t>(L.ccode));
  return hipGetLastError();
}

hipError_t launch_tile_info(const DevPtrs& d, hipStream_t s) {
  const Layout& L = *d.L;
  const int64_t ntiles = L.Kpad / CT;
  if (d.D > 6) return hipErrorInvalidValue;  // (the MFMA rows exist for D <= 6 only)
  TileRows g{L.stage_c32 ? d.at<float>(L.c32u) : nullptr, d.at<uint16_t>(L.chu), d.at<uint16_t>(L.clu),
             d.at<float>(L.ncu), d.at<float>(L.c32), d.at<uint16_t>(L.ch), d.at<uint16_t>(L.cl), d.at<float>(L.nc),
             d.at<RowBound>(L.rowb)};
  hipLaunchKernelGGL(k_tile_info, dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s, d.at<int32_t>(L.corder),
                     d.at<uint32_t>(L.ccode), d.K, ntiles, d.D, d.nsp, d.at<double>(L.direct), direct_stride(d.D),
                     d.at<float>(L.lam), g, d.at<TileInfo>(L.tinfo), d.at<float>(L.ncg));
  return hipGetLastError();
}

// ---- reassignment of under-used components ---------------------------------------------------
// Sort keys: the order-preserving 64-bit image of an FP64 value (complemented for a descending
// order) with the low 25 bits replaced by the element's index; padding keys are all ones.
constexpr int RA_IDX_BITS = 25;
constexpr unsigned long long RA_IDX_MASK = (1ull << RA_IDX_BITS) - 1ull;

__device__ __forceinline__ unsigned long long ord64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

// points: value g_n - LSE_n (largest first)
__global__ void k_reassign_point_keys(const double* __restrict__ lse, const double* __restrict__ gumbel, int64_t N,
                                      int64_t Npow, unsigned long long* __restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= Npow) return;
  keys[n] = n < N ? ((~ord64(gumbel[n] - lse[n])) & ~RA_IDX_MASK) | (unsigned long long)n : ~0ull;
}

// components: posterior alpha (smallest first)
__global__ void k_reassign_comp_keys(const double* __restrict__ post, int64_t K, int64_t Kpow,
                                     unsigned long long* __restrict__ keys) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Kpow) return;
  keys[k] = k < K ? (ord64(post[k * REC]) & ~RA_IDX_MASK) | (unsigned long long)k : ~0ull;
}

// the i-th sampled point becomes the mean of the i-th least-used component (prior and posterior)
__global__ void k_reassign_apply(const unsigned long long* __restrict__ pkeys,
                                 const unsigned long long* __restrict__ ckeys, int64_t n, const float* __restrict__ X,
                                 int D, double* __restrict__ prior, double* __restrict__ post,
                                 int32_t* __restrict__ out_pts, int32_t* __restrict__ out_comps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = (int64_t)(pkeys[i] & RA_IDX_MASK), k = (int64_t)(ckeys[i] & RA_IDX_MASK);
  for (int d = 0; d < D; ++d) {
    const double x = (double)X[p * D + d];
    prior[k * REC + 3 + d] = x;
    post[k * REC + 3 + d] = x;
  }
  if (out_pts) out_pts[i] = (int32_t)p;
  if (out_comps) out_comps[i] = (int32_t)k;
}

hipError_t launch_reassign(const DevPtrs& d, const float* X, int64_t N, const double* lse, const double* gumbel,
                           int64_t n, int32_t* out_pts, int32_t* out_comps, hipStream_t s) {
  const Layout& L = *d.L;
  if (n <= 0) return hipSuccess;
  int64_t npow = BS_LOCAL, kpow = BS_LOCAL;
  while (npow < N) npow <<= 1;
  while (kpow < d.K) kpow <<= 1;
  unsigned long long* pk = d.at<unsigned long long>(L.pkeys);
  unsigned long long* ck = d.at<unsigned long long>(L.ckeys);
  hipLaunchKernelGGL(k_reassign_point_keys, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, s, lse, gumbel, N,
                     npow, pk);
  hipError_t e = launch_sort_keys(pk, npow, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reassign_comp_keys, dim3((unsigned)((kpow + 255) / 256)), dim3(256), 0, s, d.post(), d.K,
                     kpow, ck);
  e = launch_sort_keys(ck, kpow, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reassign_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pk, ck, n, X, d.D,
                     d.prior(), d.post(), out_pts, out_comps);
  return hipGetLastError();
}

}  // namespace vbgs
