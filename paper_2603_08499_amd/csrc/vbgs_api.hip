// C ABI of libvbgs: parameter validation, workspace layout, launch sequencing.
// Every entry point enqueues on the caller's stream; nothing here allocates device memory.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>

#include "prop_internal.h"

using namespace vbgs;

// Ring of event pairs per phase; a slot is harvested (its elapsed time added) when it is
// reused, long after its events completed, so recording never waits inside a timed loop.
struct PhaseTimer {
  static constexpr int RING = 64;
  hipEvent_t a[RING], b[RING];
  bool used[RING];
  int head;
  double ms;
  int64_t count;
};

struct vbgs_ctx {
  vbgs_params p;
  bool timing;
  uint32_t timing_mask;  // the phases recorded while timing is on
  bool timers_made;
  bool prop_ready;     // the state holds network weights
  bool prop_prepared;  // the workspace holds their MFMA operand copies
  PhaseTimer tm[VBGS_NPHASE];
  Layout L;
  void* state;
  void* ws;
  int64_t last_N;
  uint64_t post_version;
  uint64_t lse_version;
  bool have_stats;
  bool order_reset;  // the sweep's block costs are not measured yet
  bool seg_used;     // the last E-step wrote its kept pairs into segments (culled path)
  bool pending_clear;  // attached to a state: the workspace's flags and counters are not cleared yet
  // side streams (default priority) of the culled path: the component preparation, which overlaps
  // the point preparation, and the KL terms of the ELBO, which overlap both (not the sweep: their
  // waves hold most of a SIMD's registers and would keep the sweep's first blocks waiting)
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t begin = nullptr, fork = nullptr, join = nullptr, kl_done = nullptr, rows_done = nullptr,
             feat_done = nullptr;
  int nsplit;
  float T2;
  void* scratch = nullptr;  // device address of this device's static scratch (vbgs_estep_stats_scratch)
  std::string scratch_err;
  std::string err;
  DevPtrs dev() const { return DevPtrs{(char*)ws, (double*)state, &L, p.D, p.K, p.modal_split, cull_ns()}; }
  // leading coordinates of the culling bounds: the spatial block of the two-factor model, the pixel
  // position of an image (D = 5), else up to three
  int cull_ns() const {
    if (p.cull_dims > 0) return p.cull_dims;
    if (p.modal_split > 0 && p.modal_split <= 3) return p.modal_split;
    if (p.D == 5) return 2;
    return p.D < 3 ? p.D : 3;
  }
};

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int auto_split_mfma(int64_t Kpad) {
  const int64_t tiles = Kpad / CT;
  int64_t s = (1024 + tiles - 1) / tiles;
  return (int)(s < 1 ? 1 : (s > 32 ? 32 : s));
}
int auto_split_direct(int64_t K) {
  const int64_t tiles = (K + 255) / 256;
  int64_t s = (2048 + tiles - 1) / tiles;
  return (int)(s < 1 ? 1 : (s > 64 ? 64 : s));
}

vbgs_status check_params(const vbgs_params* p, std::string* why) {
  if (!p) {
    if (why) *why = "params is NULL";
    return VBGS_ERR_ARG;
  }
  if (p->abi_version != VBGS_ABI_VERSION) {
    if (why) *why = "abi_version mismatch";
    return VBGS_ERR_ARG;
  }
  if (p->D < 1 || p->D > VBGS_MAX_D) {
    if (why) *why = "D must be in 1..8";
    return VBGS_ERR_SHAPE;
  }
  if (p->K < 1 || p->K > (int64_t)1 << 30) {
    if (why) *why = "K must be in 1..2^30";
    return VBGS_ERR_SHAPE;
  }
  if (p->n_max < 0 || p->n_max > (int64_t)1 << 31) {
    if (why) *why = "n_max must be in 0..2^31";
    return VBGS_ERR_SHAPE;
  }
  if (!(p->kappa0 > 0) || !(p->alpha0 > 0) || !(p->nu0 > p->D - 1) || !isfinite(p->kappa0) ||
      !isfinite(p->alpha0) || !isfinite(p->nu0)) {
    if (why) *why = "prior scalars need kappa0 > 0, alpha0 > 0, nu0 > D - 1";
    return VBGS_ERR_ARG;
  }
  if (p->score_prec < VBGS_FP64 || p->score_prec > VBGS_FP64_CULLED) {
    if (why) *why = "unknown score_prec";
    return VBGS_ERR_ARG;
  }
  if (p->score_prec != VBGS_FP64 && p->D > 6) {
    if (why) *why = "MFMA precisions support D <= 6 (32 feature slots); use VBGS_FP64";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (p->score_prec != VBGS_FP64 && p->exact == 1 && p->n_max > ((int64_t)1 << 23)) {
    if (why) *why = "exact MFMA mode supports n_max <= 2^23 (the 128 candidate slots per point are indexed in int32)";
    return VBGS_ERR_SHAPE;
  }
  if (p->exact != 0 && p->exact != 1) {
    if (why) *why = "exact must be 0 or 1";
    return VBGS_ERR_ARG;
  }
  if (p->score_prec == VBGS_FP64_CULLED && (p->exact != 1 || p->cull != 1 || p->proposal || p->modal_split)) {
    if (why) *why = "VBGS_FP64_CULLED is the culled exact sweep with FP64 scores: exact = 1, cull = 1, no proposal, one block";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (p->score_prec == VBGS_FP8 && p->exact != 0) {
    if (why) *why = "VBGS_FP8 is a plain tier (exact = 0): as a screen its error bound would admit nearly every pair";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (p->score_prec == VBGS_AUTO && (p->exact != 1 || p->proposal)) {
    if (why) *why = "VBGS_AUTO chooses the screen of the exact mode: it needs exact = 1 and no proposal";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (!isfinite(p->screen_margin)) {
    if (why) *why = "screen_margin must be finite";
    return VBGS_ERR_ARG;
  }
  if (p->n_split < 0 || p->n_split > 64) {
    if (why) *why = "n_split must be in 0..64";
    return VBGS_ERR_ARG;
  }
  if (p->proposal != 0 && p->proposal != 1) {
    if (why) *why = "proposal must be 0 or 1";
    return VBGS_ERR_ARG;
  }
  if (p->proposal && (p->score_prec == VBGS_FP64 || p->exact != 1 || p->D > 6)) {
    if (why) *why = "the proposal needs an MFMA precision with exact = 1 and D <= 6";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (p->C < 0 || p->C > 64 || p->train_batch < 0 || p->train_batch > 65536) {
    if (why) *why = "C must be in 0..64 and train_batch in 0..65536 (0 = default)";
    return VBGS_ERR_ARG;
  }
  if (p->cull != 0 && p->cull != 1) {
    if (why) *why = "cull must be 0 or 1";
    return VBGS_ERR_ARG;
  }
  if (p->modal_split < 0 || p->modal_split >= p->D) {
    if (why) *why = "modal_split must be in 0..D-1";
    return VBGS_ERR_ARG;
  }
  if (p->modal_split > 0 && (rec_kc(p->D) + 2 > REC || p->proposal)) {
    if (why) *why = "the two-factor model needs D <= 7 (record room for the colour kappa, nu) and no proposal";
    return VBGS_ERR_UNSUPPORTED;
  }
  if (p->cull_dims < 0 || p->cull_dims > 3 || p->cull_dims > p->D) {
    if (why) *why = "cull_dims must be in 0..min(D, 3)";
    return VBGS_ERR_ARG;
  }
  if (p->proposal_prec != 0 && p->proposal_prec != VBGS_BF16 && p->proposal_prec != VBGS_FP8) {
    if (why) *why = "proposal_prec must be 0, VBGS_BF16 or VBGS_FP8";
    return VBGS_ERR_ARG;
  }
  for (int i = 0; i < 3; ++i)
    if (p->reserved[i] != 0) {
      if (why) *why = "reserved fields must be zero";
      return VBGS_ERR_ARG;
    }
  return VBGS_OK;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void harvest(PhaseTimer& t, int slot) {
  if (!t.used[slot]) return;
  float ms = 0.0f;
  if (hipEventSynchronize(t.b[slot]) == hipSuccess && hipEventElapsedTime(&ms, t.a[slot], t.b[slot]) == hipSuccess) {
    t.ms += ms;
    t.count++;
  }
  t.used[slot] = false;
}

// RAII recorder of one phase on one stream
struct Phase {
  vbgs_ctx* c;
  int ph;
  hipStream_t s;
  int slot;
  Phase(vbgs_ctx* c_, int ph_, hipStream_t s_);
  ~Phase();
};

vbgs_status fail(vbgs_ctx* c, vbgs_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

vbgs_status hipfail(vbgs_ctx* c, hipError_t e, const char* where) {
  if (e == hipSuccess) return VBGS_OK;
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  return fail(c, VBGS_ERR_HIP, buf);
}

bool aligned(const void* p) { return ((uintptr_t)p % ALIGN) == 0; }

}  // namespace

Phase::Phase(vbgs_ctx* c_, int ph_, hipStream_t s_) : c(c_), ph(ph_), s(s_), slot(-1) {
  if (!c->timing || !((c->timing_mask >> ph) & 1u)) return;
  PhaseTimer& t = c->tm[ph];
  slot = t.head;
  harvest(t, slot);
  hipEventRecord(t.a[slot], s);
}
Phase::~Phase() {
  if (slot < 0) return;
  PhaseTimer& t = c->tm[ph];
  hipEventRecord(t.b[slot], s);
  t.used[slot] = true;
  t.head = (t.head + 1) % PhaseTimer::RING;
}

namespace vbgs {
Layout make_layout(const vbgs_params& p) {
  Layout L{};
  const int64_t K = p.K, n = p.n_max;
  L.Kpad = (K + CT - 1) / CT * CT;
  L.n_lse_part = (n + 255) / 256;
  int ns = auto_split_mfma(L.Kpad);
  const int nd = auto_split_direct(K);
  if (nd > ns) ns = nd;
  if (p.n_split > ns) ns = p.n_split;
  L.nsplit_max = ns;
  const int dts = direct_stride(p.D);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = up(o + (bytes ? bytes : 1));
    return at;
  };
  L.frame = take(sizeof(FrameInfo));
  L.mom_part = take((size_t)MOM_BLOCKS * 2 * MAXD * 8);
  L.phi32 = take((size_t)n * FP * 4);
  L.phih = take((size_t)n * FP * 2);
  L.phil = take((size_t)n * FP * 2);
  L.nphi = take((size_t)n * 4);
  L.lse2 = take((size_t)n * 8);
  L.lse_part = take((size_t)(L.n_lse_part + 1) * 8);
  L.direct = take((size_t)L.Kpad * dts * 8);
  L.c32 = take((size_t)L.Kpad * FP * 4);
  L.ch = take((size_t)L.Kpad * FP * 2);
  L.cl = take((size_t)L.Kpad * FP * 2);
  L.nc = take((size_t)L.Kpad * 4);
  L.fp8 = p.score_prec == VBGS_FP8 ? 1 : 0;
  L.f32rows = (p.exact && (p.score_prec == VBGS_BF16X3 || p.score_prec == VBGS_BF16)) ? 0 : 1;
  L.phi8 = take(L.fp8 ? (size_t)n * FP : 0);
  L.phis = take(L.fp8 ? (size_t)n * 4 : 0);
  L.c8 = take(L.fp8 ? (size_t)L.Kpad * FP : 0);
  L.cs8 = take(L.fp8 ? (size_t)L.Kpad * 4 : 0);
  L.kl = take((size_t)K * 8);
  // pass-2 partials of the FP64 path and of the plain tiers (the exact MFMA mode sums in fixed point)
  const bool exact_mfma = p.score_prec != VBGS_FP64 && p.exact == 1;
  L.spart = take(exact_mfma ? 0 : (size_t)ns * L.Kpad * stat_stride(p.D) * 8);
  L.stats = take((size_t)K * nfeat(p.D) * 8);
  const bool sparse = p.score_prec != VBGS_FP64;  // exact MFMA mode: candidate lists + fixed-point sums
  {  // the culled path's staging rows
    const bool staged = sparse && p.exact == 1 && p.cull == 1;
    L.stage_c32 = staged && !(p.score_prec == VBGS_BF16X3 || p.score_prec == VBGS_BF16) ? 1 : 0;
    L.c32u = take(L.stage_c32 ? (size_t)L.Kpad * FP * 4 : 0);
    L.chu = take(staged ? (size_t)L.Kpad * FP * 2 : 0);
    L.clu = take(staged ? (size_t)L.Kpad * FP * 2 : 0);
    L.ncu = take(staged ? (size_t)L.Kpad * 4 : 0);
  }
  L.cand_k = take(sparse ? (size_t)n * 4 * CS * 4 : 0);
  L.cand_s = take(sparse ? (size_t)n * 4 * CS * 4 : 0);
  L.cand_n = take(sparse ? (size_t)n * 4 * 4 : 0);
  L.over_list = take(sparse ? (size_t)n * 4 : 0);
  L.fx = take(sparse ? (size_t)L.Kpad * FP * 16 : 0);
  L.ccount = take(sparse ? (size_t)(L.Kpad + 1) * 4 : 0);
  L.coffset = take(sparse ? (size_t)(L.Kpad + 1) * 4 : 0);
  L.segoff = take(sparse ? (size_t)L.Kpad * 8 : 0);
  L.seg_miss = take(sparse ? 4 : 0);
  L.ent_n = take(sparse ? (size_t)n * 4 * CS * 4 : 0);
  L.ent_cap = sparse ? n * 4 * CS : 0;
  int64_t npow = 2048, kpow = 2048;
  while (npow < n) npow <<= 1;
  while (kpow < K) kpow <<= 1;
  L.pkeys = take((size_t)npow * 8);  // also used by the reassignment step in every mode
  L.porder = take(sparse ? (size_t)n * 4 : 0);
  L.pcode = take(sparse ? (size_t)n * 4 : 0);
  L.ckeys = take((size_t)kpow * 8);
  {
    const int64_t nk = std::max<int64_t>(n, K), nbx = (nk + RX_B - 1) / RX_B, ne = 256 * nbx;
    L.rx_tmp = take(sparse ? (size_t)nk * 8 : 0);
    L.rx_hist = take(sparse ? (size_t)ne * 4 : 0);
    L.rx_off = take(sparse ? (size_t)(ne + 1) * 4 : 0);
    L.rx_part = take(sparse ? (size_t)((ne + 1023) / 1024 + 2) * 4 : 0);
    const int64_t nbk = (K + RX_B - 1) / RX_B, nek = 256 * nbk;
    L.rx2_tmp = take(sparse ? (size_t)K * 8 : 0);
    L.rx2_hist = take(sparse ? (size_t)nek * 4 : 0);
    L.rx2_off = take(sparse ? (size_t)(nek + 1) * 4 : 0);
    L.rx2_part = take(sparse ? (size_t)((nek + 1023) / 1024 + 2) * 4 : 0);
  }
  L.corder = take(sparse ? (size_t)L.Kpad * 4 : 0);
  L.cinv = take(sparse ? (size_t)L.Kpad * 4 : 0);
  L.ccode = take(sparse ? (size_t)L.Kpad * 4 : 0);
  L.lam = take((size_t)L.Kpad * 4);
  L.tinfo = take(sparse ? (size_t)(L.Kpad / CT) * sizeof(TileInfo) : 0);
  L.rowb = take(sparse ? (size_t)L.Kpad * sizeof(RowBound) : 0);
  L.ncg = take(sparse ? (size_t)L.Kpad / 4 * sizeof(float) : 0);
  L.lhist = take(sparse ? (size_t)LAM_BINS * 4 : 0);
  L.scan_part = take(sparse ? (size_t)((L.Kpad + 1023) / 1024 + 1) * 4 : 0);
  L.elbo_part = take(512 * 8);
  L.scr_part = take(512 * 8);
  L.scr_gate = take(2 * 4);
  L.bcost = take(sparse ? (size_t)((n + 63) / 64) * 4 : 0);
  L.bcode = take(sparse ? (size_t)((n + 63) / 64) * 4 : 0);
  L.border = take(sparse ? (size_t)((n + 63) / 64) * 4 : 0);
  L.bprev = take(8);
  L.slist = take(sparse ? (size_t)((n + 63) / 64) * (L.Kpad / CT) * 4 : 0);
  // learned proposal
  const bool pr = p.proposal == 1;
  const int C = p.C > 0 ? p.C : 32;
  const int64_t Bt = p.train_batch > 0 ? p.train_batch : 4096;
  L.Bpad_max = (Bt + 63) / 64 * 64;
  const size_t H = VBGS_H;
  L.p_Ebf = take(pr ? (size_t)L.Kpad * H * 2 : 0);
  L.p_EbfT = take(pr ? (size_t)L.Kpad * H * 2 : 0);
  L.p_betap = take(pr ? (size_t)L.Kpad * 4 : 0);
  L.p_W2T = take(pr ? H * H * 4 : 0);
  L.p_h2b = take(pr ? (size_t)n * H * 2 : 0);
  L.p_tz = take(pr ? (size_t)n * 4 * 2 * C * 4 : 0);
  L.p_tk = take(pr ? (size_t)n * 4 * 2 * C * 4 : 0);
  L.p_tcnt = take(pr ? (size_t)n * 4 * 4 : 0);
  L.p_tthr = take(pr ? (size_t)n * 4 : 0);
  const bool f8 = pr && p.proposal_prec == VBGS_FP8;
  L.p_E8 = take(f8 ? (size_t)L.Kpad * H : 0);
  L.p_sE = take(f8 ? (size_t)L.Kpad * 4 : 0);
  L.p_h8 = take(f8 ? (size_t)n * H : 0);
  L.p_sh = take(f8 ? (size_t)n * 4 : 0);
  L.p_aud = take(pr ? (size_t)n * 8 : 0);
  L.p_gate = take(pr ? 64 : 0);
  const size_t Bp = (size_t)L.Bpad_max;
  L.p_th1 = take(pr ? Bp * H * 4 : 0);
  L.p_th2 = take(pr ? Bp * H * 4 : 0);
  L.p_txs = take(pr ? Bp * MAXD * 4 : 0);
  L.p_tlse = take(pr ? Bp * 4 : 0);
  L.p_tdh2 = take(pr ? Bp * H * 4 : 0);
  L.p_tdp1 = take(pr ? Bp * H * 4 : 0);
  L.p_tlpart = take(pr ? (size_t)32 * Bp * 2 * 4 : 0);
  L.p_tdpart = take(pr ? std::min<size_t>((size_t)16 * Bp, 65536) * H * 4 : 0);
  L.p_twpart = take(pr ? (size_t)TRAIN_W_SPLIT * (H * H + 2 * H + H * MAXD) * 4 : 0);
  L.p_th2b = take(pr ? Bp * H * 2 : 0);
  L.p_th2T = take(pr ? Bp * H * 2 : 0);
  L.p_tloss = take(pr ? Bp * 8 : 0);
  const PropOffsets po(p.D, p.K);
  L.p_grads = take(pr ? (size_t)po.n * 4 : 0);
  L.total = o;
  // state: header, frame prior, posterior, then the proposal block
  size_t so = sizeof(StateHeader) + (size_t)2 * p.K * REC * 8;
  L.s_W = so;
  L.s_mu = so + (size_t)po.n * 4;
  L.s_is = L.s_mu + MAXD * 4;
  L.s_m1 = up(L.s_is + MAXD * 4);
  L.s_m2 = up(L.s_m1 + (size_t)po.n * 4);
  L.s_step = up(L.s_m2 + (size_t)po.n * 4);
  L.state_total = pr ? L.s_step + 8 : so;
  return L;
}
}  // namespace vbgs

extern "C" {

vbgs_status vbgs_default_params(vbgs_params* p, int32_t D, int64_t K, int64_t n_max) {
  if (!p) return VBGS_ERR_ARG;
  memset(p, 0, sizeof *p);
  p->abi_version = VBGS_ABI_VERSION;
  p->D = D;
  p->K = K;
  p->n_max = n_max;
  p->kappa0 = 1.0;
  p->nu0 = D + 2.0;
  p->alpha0 = 1.0;
  p->score_prec = D <= 6 ? VBGS_AUTO : VBGS_FP64;
  p->exact = 1;
  p->screen_margin = 0.0;
  p->C = 32;
  p->train_batch = 4096;
  p->cull = 1;
  return VBGS_OK;
}

vbgs_status vbgs_query_sizes(const vbgs_params* p, size_t* state_bytes, size_t* workspace_bytes) {
  const vbgs_status st = check_params(p, nullptr);
  if (st != VBGS_OK) return st;
  if (!state_bytes || !workspace_bytes) return VBGS_ERR_ARG;
  const Layout L = make_layout(*p);
  *state_bytes = L.state_total;
  *workspace_bytes = L.total;
  return VBGS_OK;
}

static bool use_cull(const vbgs_ctx* c) {
  return c->p.score_prec != VBGS_FP64 && c->p.exact == 1 && c->p.cull == 1;
}

// the side streams and their events (culled path only), made with the context so that no stream
// is created while a caller's stream may be capturing; on failure nothing is left behind
static hipError_t make_side(vbgs_ctx* c) {
  if (c->side || !use_cull(c)) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->kl_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->rows_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->feat_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->begin, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (c->begin) hipEventDestroy(c->begin);
    if (c->feat_done) hipEventDestroy(c->feat_done);
    if (c->rows_done) hipEventDestroy(c->rows_done);
    if (c->kl_done) hipEventDestroy(c->kl_done);
    if (c->join) hipEventDestroy(c->join);
    if (c->fork) hipEventDestroy(c->fork);
    if (c->side2) hipStreamDestroy(c->side2);
    if (c->side) hipStreamDestroy(c->side);
    c->side = c->side2 = nullptr;
    c->begin = c->fork = c->join = c->kl_done = c->rows_done = c->feat_done = nullptr;
  }
  return e;
}

// ---- static scratch for callers that cannot allocate ----------------------------------------
// One array per GPU in the library's code object, held until the process ends. In host code its
// name stands for a host-side shadow, not a device address: the address of each GPU's copy is
// looked up once per device with that device current, and only that address is ever used.
static __device__ __align__(256) unsigned char scratch[VBGS_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEV];
}  // namespace

// device address of the current device's scratch (cached per device)
static hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SCRATCH_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// looked up when a context is made (the device current then is the context's); a failure only
// disables vbgs_estep_stats_scratch for this context, and is cleared from HIP's last-error state
static void find_scratch(vbgs_ctx* c) {
  const hipError_t e = scratch_address(&c->scratch);
  if (e != hipSuccess) {
    c->scratch = nullptr;
    c->scratch_err = hipGetErrorString(e);
    (void)hipGetLastError();
  }
}

static vbgs_ctx* new_ctx(const vbgs_params* p, void* state, void* ws) {
  vbgs_ctx* c = new (std::nothrow) vbgs_ctx();
  if (!c) return nullptr;
  c->p = *p;
  c->L = make_layout(*p);
  c->state = state;
  c->ws = ws;
  c->last_N = -1;
  c->post_version = 0;
  c->lse_version = ~(uint64_t)0;
  c->have_stats = false;
  c->order_reset = true;
  c->seg_used = false;
  c->pending_clear = false;
  c->timing = false;
  c->timing_mask = 0;
  c->timers_made = false;
  c->prop_ready = false;
  c->prop_prepared = false;
  const int auto_ns = p->score_prec == VBGS_FP64 ? auto_split_direct(p->K) : auto_split_mfma(c->L.Kpad);
  c->nsplit = p->n_split > 0 ? p->n_split : auto_ns;
  const double T = p->screen_margin > 0 ? p->screen_margin : log((double)p->K) + log(1e12);
  c->T2 = (float)(T * LOG2E);
  return c;
}

vbgs_status vbgs_init(vbgs_ctx** out, const vbgs_params* p, const double* m0, const double* W0, void* state,
                      void* workspace, void* stream) {
  std::string why;
  vbgs_status st = check_params(p, &why);
  if (st != VBGS_OK) return st;
  if (!out || !m0 || !W0 || !state || !workspace) return VBGS_ERR_ARG;
  if (!aligned(state) || !aligned(workspace)) return VBGS_ERR_ARG;
  const int D = p->D;
  // with two blocks the scale matrix is block diagonal: entries across the blocks are ignored
  double W0b[MAXD * MAXD];
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j)
      W0b[i * D + j] = coord_block(i, p->modal_split) == coord_block(j, p->modal_split) ? W0[i * D + j] : 0.0;
  W0 = W0b;
  // W0^{-1} on the host: Cholesky of W0 (rejects non-PD), then invert
  double L[MAXD][MAXD] = {{0}};
  for (int j = 0; j < D; ++j) {
    for (int i = 0; i < D; ++i)
      if (fabs(W0[i * D + j] - W0[j * D + i]) > 1e-12 * (fabs(W0[i * D + j]) + fabs(W0[j * D + i])) + 1e-300)
        return VBGS_ERR_NOT_PD;
    double s = W0[j * D + j];
    for (int t = 0; t < j; ++t) s -= L[j][t] * L[j][t];
    if (!(s > 0) || !isfinite(s)) return VBGS_ERR_NOT_PD;
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < D; ++i) {
      double v = W0[i * D + j];
      for (int t = 0; t < j; ++t) v -= L[i][t] * L[j][t];
      L[i][j] = v / L[j][j];
    }
  }
  double Li[MAXD][MAXD] = {{0}};
  for (int j = 0; j < D; ++j) {
    Li[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < D; ++i) {
      double v = 0.0;
      for (int t = j; t < i; ++t) v += L[i][t] * Li[t][j];
      Li[i][j] = -v / L[i][i];
    }
  }
  Init0 in{};
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double v = 0.0;
      for (int t = 0; t < D; ++t) v += Li[t][a] * Li[t][b];  // W0^{-1} = L^{-T} L^{-1}
      in.W0inv[a * D + b] = v;
    }
  in.alpha0 = p->alpha0;
  in.kappa0 = p->kappa0;
  in.nu0 = p->nu0;
  in.split = p->modal_split;
  vbgs_ctx* c = new_ctx(p, state, workspace);
  if (!c) return VBGS_ERR_ARG;
  find_scratch(c);
  hipError_t e = make_side(c);
  if (e != hipSuccess) {
    delete c;
    return VBGS_ERR_HIP;
  }
  e = launch_init_state(c->dev(), m0, in, S(stream));
  if (e == hipSuccess) e = launch_clear_flags(c->dev(), S(stream));
  if (e != hipSuccess) {
    vbgs_destroy(c);  // releases the side stream too
    return VBGS_ERR_HIP;
  }
  *out = c;
  return VBGS_OK;
}

vbgs_status vbgs_attach(vbgs_ctx** out, const vbgs_params* p, void* state, void* workspace) {
  std::string why;
  vbgs_status st = check_params(p, &why);
  if (st != VBGS_OK) return st;
  if (!out || !state || !workspace || !aligned(state) || !aligned(workspace)) return VBGS_ERR_ARG;
  vbgs_ctx* c = new_ctx(p, state, workspace);
  if (!c) return VBGS_ERR_ARG;
  find_scratch(c);
  if (make_side(c) != hipSuccess) {
    delete c;
    return VBGS_ERR_HIP;
  }
  c->prop_ready = p->proposal == 1;  // a proposal state carries its weights
  c->pending_clear = true;           // done on the stream of the first call that takes one
  *out = c;
  return VBGS_OK;
}

// after vbgs_attach the workspace may hold anything: its sticky flags and counters are cleared on
// the stream of the first call, before that call's own work
static hipError_t settle(vbgs_ctx* c, hipStream_t s) {
  if (!c->pending_clear) return hipSuccess;
  const hipError_t e = launch_clear_flags(c->dev(), s);
  if (e == hipSuccess) c->pending_clear = false;
  return e;
}

#define VBGS_SETTLE(c, stream)                                   \
  do {                                                           \
    const hipError_t e_ = settle((c), S(stream));                \
    if (e_ != hipSuccess) return hipfail((c), e_, "clear flags"); \
  } while (0)


// expectations and coefficient rows, and the KL terms; with culling the MFMA rows are written in
// component order, then gathered into spatial order with the per-row and per-tile bounds
static hipError_t prepare_components(vbgs_ctx* c, hipStream_t s) {
  const DevPtrs d = c->dev();
  hipError_t e;
  if (!use_cull(c)) {
    e = launch_coeffs(d, s);
  } else {
    e = launch_sort_comps(d, s);
    if (e == hipSuccess) e = launch_coeffs(d, s, true, true);
    if (e == hipSuccess) e = launch_tile_info(d, s);
  }
  if (e == hipSuccess) e = launch_kl(d, s);
  return e;
}


static vbgs_status run_pass1(vbgs_ctx* c, const float* X, int64_t N, double* lse_out, void* stream) {
  const DevPtrs d = c->dev();
  EstepCfg cfg{c->p.score_prec, c->p.exact, c->T2, c->nsplit};
  cfg.cull = use_cull(c) ? 1 : 0;
  cfg.seg = cfg.cull;  // (the layout is made below, on the stream that clears the counts)
  c->seg_used = cfg.seg != 0;
  cfg.order_reset = c->order_reset ? 1 : 0;
  const bool cull = use_cull(c);
  const hipStream_t s = S(stream);
  hipError_t e;
  if (cull) {
    // the frame moments first (the components are centred and Hilbert-coded with them; beside them
    // on side2, the kept pairs' segments sized from the last sweep's counts and the sweep's
    // cleared counters), then three streams: the component sort, then the gather of the rows into
    // its order with the tile bounds (side); the alpha sum, the coefficient rows in component
    // order, the point features, and the KL terms (ELBO only) (side2); the point sort and the
    // blocks' dispatch order (the caller's stream, which waits for the gather and the features
    // before the sweep, and for the KL terms after pass 1)
    e = c->side ? hipSuccess : hipErrorInvalidResourceHandle;  // made with the context
    // (the segments and the cleared counters need nothing of this frame: beside the moments)
    if (e == hipSuccess) e = hipEventRecord(c->begin, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side2, c->begin, 0);
    if (e == hipSuccess) e = launch_seg_layout(d, c->side2);
    if (e == hipSuccess) e = launch_pass1(d, cfg, X, N, lse_out, c->side2, 0);
    if (e == hipSuccess) {
      Phase ph(c, 0, s);
      e = launch_frame_prep(d, X, N, s, 0);
    }
    if (e == hipSuccess) e = hipEventRecord(c->fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->fork, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side2, c->fork, 0);
    if (e == hipSuccess) e = launch_coeffs(d, c->side2, true, true);
    if (e == hipSuccess) e = hipEventRecord(c->rows_done, c->side2);
    if (e == hipSuccess) e = launch_frame_prep(d, X, N, c->side2, 1);
    if (e == hipSuccess) e = hipEventRecord(c->feat_done, c->side2);
    if (e == hipSuccess) e = launch_kl(d, c->side2);
    if (e == hipSuccess) e = hipEventRecord(c->kl_done, c->side2);
    if (e == hipSuccess) {
      Phase ph(c, 1, c->side);
      e = launch_sort_comps(d, c->side);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->rows_done, 0);
      if (e == hipSuccess) e = launch_tile_info(d, c->side);
    }
    if (e == hipSuccess) e = hipEventRecord(c->join, c->side);
    if (e == hipSuccess) {
      Phase ph(c, 8, s);
      e = launch_sort_points(d, X, N, s);
      if (e == hipSuccess) e = launch_pass1(d, cfg, X, N, lse_out, s, 4);
    }
    // (the join follows rows_done, which follows the cleared counters)
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->join, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->feat_done, 0);
  } else {
    {
      Phase ph(c, 0, s);
      e = launch_frame_prep(d, X, N, s);
    }
    if (e == hipSuccess) {
      Phase ph(c, 1, s);
      e = prepare_components(c, s);
    }
    if (e == hipSuccess) {
      Phase ph(c, 8, s);
      e = launch_pass1(d, cfg, X, N, lse_out, s, 0);
    }
  }
  if (e == hipSuccess) e = launch_pass1(d, cfg, X, N, lse_out, S(stream), 1);
  if (e == hipSuccess) {
    Phase ph(c, 2, S(stream));  // the screening sweep alone (exact mode), or the whole first pass
    e = launch_pass1(d, cfg, X, N, lse_out, S(stream), 3);
    if (cfg.cull && N > 0) c->order_reset = false;
  }
  if (e == hipSuccess) {
    Phase ph(c, 9, S(stream));
    e = launch_pass1(d, cfg, X, N, lse_out, S(stream), 2);
  }
  if (e == hipSuccess && cull) e = hipStreamWaitEvent(s, c->kl_done, 0);
  return hipfail(c, e, "pass 1");
}

// E-step + statistics into the workspace the context points at (c->ws)
static vbgs_status estep_body(vbgs_ctx* c, const float* X, int64_t N, double* lse_out, double* stats_out,
                              void* stream) {
  vbgs_status st = run_pass1(c, X, N, lse_out, stream);
  if (st != VBGS_OK) return st;
  const DevPtrs d = c->dev();
  EstepCfg cfg{c->p.score_prec, c->p.exact, c->T2, c->nsplit};
  cfg.cull = use_cull(c) ? 1 : 0;
  cfg.seg = cfg.cull;  // (as in run_pass1)
  hipError_t e;
  {
    Phase ph(c, 3, S(stream));
    e = launch_pass2(d, cfg, X, N, S(stream), stats_out);
  }
  if (e == hipSuccess) {
    Phase ph(c, 4, S(stream));
    e = launch_fold(d, cfg, stats_out, S(stream));
  }
  return hipfail(c, e, "pass 2");
}

vbgs_status vbgs_estep_stats(vbgs_ctx* c, const float* X, int64_t N, double* lse_out, double* stats_out,
                             void* stream) {
  if (!c) return VBGS_ERR_ARG;
  if (N < 0 || N > c->p.n_max) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
  if (N > 0 && !X) return fail(c, VBGS_ERR_ARG, "X is NULL");
  VBGS_SETTLE(c, stream);
  const vbgs_status st = estep_body(c, X, N, lse_out, stats_out, stream);
  if (st != VBGS_OK) return st;
  c->last_N = N;
  c->lse_version = c->post_version;
  c->have_stats = true;
  return VBGS_OK;
}

vbgs_status vbgs_estep_stats_scratch(vbgs_ctx* c, const float* X, int64_t N, double* lse_out, double* stats_out,
                                     void* stream) {
  if (!c) return VBGS_ERR_ARG;
  if (N < 0 || N > c->p.n_max) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
  if (N > 0 && !X) return fail(c, VBGS_ERR_ARG, "X is NULL");
  if (c->L.total > VBGS_SCRATCH_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf, "these params need a %zu-byte workspace; the static scratch holds %zu bytes",
             c->L.total, (size_t)VBGS_SCRATCH_BYTES);
    return fail(c, VBGS_ERR_SHAPE, buf);
  }
  if (!c->scratch) return fail(c, VBGS_ERR_HIP, "static scratch unavailable: " + c->scratch_err);
  VBGS_SETTLE(c, stream);
  // the same launches as vbgs_estep_stats with the scratch as the workspace; the context's own
  // workspace and bookkeeping are left as they were
  void* const ws = c->ws;
  const bool order_reset = c->order_reset, seg_used = c->seg_used;
  c->ws = c->scratch;
  c->order_reset = true;  // block costs in the scratch may come from another context
  const DevPtrs sd = c->dev();
  hipError_t e = launch_clear_flags(sd, S(stream));  // flags and counters start at zero
  vbgs_status st = e == hipSuccess ? estep_body(c, X, N, lse_out, stats_out, stream) : hipfail(c, e, "scratch");
  c->ws = ws;
  c->order_reset = order_reset;
  c->seg_used = seg_used;
  if (st != VBGS_OK) return st;
  return hipfail(c, launch_merge_flags(sd.frame(), c->dev().frame(), S(stream)), "scratch flags");
}

vbgs_status vbgs_update(vbgs_ctx* c, int32_t commit, void* stream) {
  if (!c) return VBGS_ERR_ARG;
  if (commit != 0 && commit != 1) return fail(c, VBGS_ERR_ARG, "commit must be 0 or 1");
  if (!c->have_stats) return fail(c, VBGS_ERR_STATE, "vbgs_update needs a preceding vbgs_estep_stats");
  VBGS_SETTLE(c, stream);
  hipError_t e;
  {
    Phase ph(c, 5, S(stream));
    e = launch_update(c->dev(), commit, S(stream));
  }
  if (e != hipSuccess) return hipfail(c, e, "update");
  c->post_version++;
  return VBGS_OK;
}

vbgs_status vbgs_elbo(vbgs_ctx* c, const float* X, int64_t N, double* elbo_dev, void* stream) {
  if (!c || !elbo_dev) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  if (!X) {
    if (c->last_N < 0 || c->lse_version != c->post_version)
      return fail(c, VBGS_ERR_STATE, "no LSE at the current posterior: pass X");
  } else {
    if (N < 0 || N > c->p.n_max) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
    vbgs_status st = run_pass1(c, X, N, nullptr, stream);
    if (st != VBGS_OK) return st;
    c->last_N = N;
    c->lse_version = c->post_version;
  }
  const int64_t np = (c->last_N + 255) / 256;
  Phase ph(c, 6, S(stream));
  return hipfail(c, launch_elbo(c->dev(), np, elbo_dev, S(stream)), "elbo");
}

vbgs_status vbgs_get_params(vbgs_ctx* c, int32_t which, double* alpha, double* kappa, double* m, double* Winv,
                            double* nu, void* stream) {
  if (!c || (which != 0 && which != 1) || !alpha || !kappa || !m || !Winv || !nu) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  return hipfail(c, launch_get_set(c->dev(), which, 0, alpha, kappa, m, Winv, nu, S(stream)), "get_params");
}

vbgs_status vbgs_set_params(vbgs_ctx* c, int32_t which, const double* alpha, const double* kappa,
                            const double* m, const double* Winv, const double* nu, void* stream) {
  if (!c || (which != 0 && which != 1) || !alpha || !kappa || !m || !Winv || !nu) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  hipError_t e = launch_get_set(c->dev(), which, 1, (double*)alpha, (double*)kappa, (double*)m, (double*)Winv,
                                (double*)nu, S(stream));
  if (e != hipSuccess) return hipfail(c, e, "set_params");
  c->post_version++;
  return VBGS_OK;
}

vbgs_status vbgs_reassign(vbgs_ctx* c, const float* X, int64_t N, const double* lse, const double* gumbel,
                          int64_t n, int32_t* out_points, int32_t* out_comps, void* stream) {
  if (!c) return VBGS_ERR_ARG;
  if (N < 0 || N > c->p.n_max) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
  if (n < 0 || n > N || n > c->p.K) return fail(c, VBGS_ERR_SHAPE, "n outside 0..min(N, K)");
  if (N >= (1ll << 25) || c->p.K >= (1ll << 25)) return fail(c, VBGS_ERR_UNSUPPORTED, "N and K must be below 2^25");
  if (n == 0) return VBGS_OK;
  if (!X || !lse || !gumbel) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  hipError_t e = launch_reassign(c->dev(), X, N, lse, gumbel, n, out_points, out_comps, S(stream));
  if (e != hipSuccess) return hipfail(c, e, "reassign");
  c->post_version++;
  return VBGS_OK;
}

vbgs_status vbgs_render(vbgs_ctx* model, vbgs_ctx* sp, const float* Xq, int64_t Nq, double* regress,
                        float* colour_out, double* lse_out, void* stream) {
  if (!model || !sp) return VBGS_ERR_ARG;
  const int D = model->p.D, s = sp->p.D;
  if (s < 1 || s >= D || s > 6) return fail(sp, VBGS_ERR_SHAPE, "the position context needs 1 <= D_s < D, D_s <= 6");
  if (model->p.modal_split > 0 && model->p.modal_split != s)
    return fail(sp, VBGS_ERR_SHAPE, "the position context's D must equal the model's modal_split");
  if (sp->p.K != model->p.K || sp->p.modal_split != 0 || sp->p.proposal != 0)
    return fail(sp, VBGS_ERR_SHAPE, "the position context needs the model's K, modal_split = 0, no proposal");
  if (sp->p.score_prec != VBGS_FP64 && sp->p.exact != 1)
    return fail(sp, VBGS_ERR_UNSUPPORTED, "rendering needs the FP64 path or the exact MFMA mode");
  if (Nq < 0 || Nq > sp->p.n_max) return fail(sp, VBGS_ERR_SHAPE, "Nq outside 0..n_max of the position context");
  if (!regress || (Nq > 0 && (!Xq || !colour_out))) return fail(sp, VBGS_ERR_ARG, "null buffer");
  VBGS_SETTLE(model, stream);
  VBGS_SETTLE(sp, stream);
  hipError_t e = launch_render_marginal(model->dev(), sp->dev(), regress, S(stream));
  if (e != hipSuccess) return hipfail(sp, e, "render marginal");
  sp->post_version++;
  sp->have_stats = false;
  if (Nq == 0) return VBGS_OK;
  vbgs_status st = run_pass1(sp, Xq, Nq, lse_out, stream);
  if (st != VBGS_OK) return st;
  EstepCfg cfg{sp->p.score_prec, sp->p.exact, sp->T2, sp->nsplit};
  cfg.cull = use_cull(sp) ? 1 : 0;
  e = launch_render(sp->dev(), cfg, Xq, Nq, regress, D - s, colour_out, S(stream));
  if (e != hipSuccess) return hipfail(sp, e, "render");
  sp->last_N = Nq;
  sp->lse_version = sp->post_version;
  return VBGS_OK;
}

vbgs_status vbgs_psnr(const float* a, const float* b, int64_t n, double* out, void* stream) {
  if (n < 0 || !out || (n > 0 && (!a || !b))) return VBGS_ERR_ARG;
  return launch_psnr(a, b, n, out, S(stream)) == hipSuccess ? VBGS_OK : VBGS_ERR_HIP;
}

vbgs_status vbgs_sync_status(vbgs_ctx* c, void* stream) {
  if (!c) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  int32_t flags = 0;
  hipError_t e = hipStreamSynchronize(S(stream));
  if (e == hipSuccess)
    e = hipMemcpy(&flags, (char*)c->ws + c->L.frame + offsetof(FrameInfo, flags), sizeof flags,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipfail(c, e, "sync_status");
  if (flags & FLAG_NOT_PD) return fail(c, VBGS_ERR_NOT_PD, "a W^{-1} was not positive definite");
  if (flags & FLAG_NONFINITE) return fail(c, VBGS_ERR_NONFINITE, "non-finite input coordinates");
  return VBGS_OK;
}

vbgs_status vbgs_clear_flags(vbgs_ctx* c, void* stream) {
  if (!c) return VBGS_ERR_ARG;
  const hipError_t e = launch_clear_flags(c->dev(), S(stream));
  if (e == hipSuccess) c->pending_clear = false;
  return hipfail(c, e, "clear_flags");
}

vbgs_status vbgs_counters(vbgs_ctx* c, int64_t out[11], void* stream) {
  if (!c || !out) return VBGS_ERR_ARG;
  VBGS_SETTLE(c, stream);
  FrameInfo f;
  int32_t miss = -1;
  hipError_t e = hipStreamSynchronize(S(stream));
  if (e == hipSuccess) e = hipMemcpy(&f, (char*)c->ws + c->L.frame, sizeof f, hipMemcpyDeviceToHost);
  if (e == hipSuccess && c->seg_used)
    e = hipMemcpy(&miss, (char*)c->ws + c->L.seg_miss, sizeof miss, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipfail(c, e, "counters");
  out[0] = (int64_t)f.refined1;
  out[1] = (int64_t)f.refined2;
  out[2] = c->last_N;
  out[3] = c->p.K;
  out[4] = (int64_t)f.blocks;
  out[5] = c->last_N > 0 ? (c->last_N + P1_PTS - 1) / P1_PTS * (P1_PTS / 64) * (c->L.Kpad / 16) : 0;
  out[6] = (int64_t)f.blocks_cum;
  out[7] = f.n_over;
  out[8] = f.screen_prec;
  out[9] = (int64_t)llround((double)f.screen_slack * 1000.0);
  out[10] = miss;
  return VBGS_OK;
}

// ------------------------------------------------------------------------------------------
// learned proposal
// ------------------------------------------------------------------------------------------
static PArgs make_pargs(vbgs_ctx* c) {
  const Layout& L = c->L;
  char* ws = (char*)c->ws;
  char* st = (char*)c->state;
  const PropOffsets o(c->p.D, c->p.K);
  PArgs a{};
  a.K = c->p.K;
  a.Kpad = L.Kpad;
  a.Bpad = L.Bpad_max;
  a.n_train = o.n;
  a.D = c->p.D;
  a.C = c->p.C > 0 ? c->p.C : 32;
  a.W = reinterpret_cast<float*>(st + L.s_W);
  a.W1 = a.W + o.W1;
  a.b1 = a.W + o.b1;
  a.W2 = a.W + o.W2;
  a.b2 = a.W + o.b2;
  a.E = a.W + o.E;
  a.beta = a.W + o.beta;
  a.mu_in = reinterpret_cast<float*>(st + L.s_mu);
  a.inv_s_in = reinterpret_cast<float*>(st + L.s_is);
  a.m1 = reinterpret_cast<float*>(st + L.s_m1);
  a.m2 = reinterpret_cast<float*>(st + L.s_m2);
  a.step = reinterpret_cast<double*>(st + L.s_step);
  a.Ebf = reinterpret_cast<uint16_t*>(ws + L.p_Ebf);
  a.EbfT = reinterpret_cast<uint16_t*>(ws + L.p_EbfT);
  a.betap = reinterpret_cast<float*>(ws + L.p_betap);
  a.W2T = reinterpret_cast<float*>(ws + L.p_W2T);
  a.h2b = reinterpret_cast<uint16_t*>(ws + L.p_h2b);
  a.tz = reinterpret_cast<float*>(ws + L.p_tz);
  a.tk = reinterpret_cast<int32_t*>(ws + L.p_tk);
  a.tcnt = reinterpret_cast<int32_t*>(ws + L.p_tcnt);
  a.tthr = reinterpret_cast<float*>(ws + L.p_tthr);
  a.f8 = c->p.proposal_prec == VBGS_FP8 ? 1 : 0;
  a.E8 = reinterpret_cast<uint8_t*>(ws + L.p_E8);
  a.sE = reinterpret_cast<float*>(ws + L.p_sE);
  a.h8 = reinterpret_cast<uint8_t*>(ws + L.p_h8);
  a.sh = reinterpret_cast<float*>(ws + L.p_sh);
  a.th1 = reinterpret_cast<float*>(ws + L.p_th1);
  a.th2 = reinterpret_cast<float*>(ws + L.p_th2);
  a.txs = reinterpret_cast<float*>(ws + L.p_txs);
  a.tlse = reinterpret_cast<float*>(ws + L.p_tlse);
  a.tdh2 = reinterpret_cast<float*>(ws + L.p_tdh2);
  a.tdp1 = reinterpret_cast<float*>(ws + L.p_tdp1);
  a.tlpart = reinterpret_cast<float*>(ws + L.p_tlpart);
  a.tdpart = reinterpret_cast<float*>(ws + L.p_tdpart);
  a.twpart = reinterpret_cast<float*>(ws + L.p_twpart);
  a.th2b = reinterpret_cast<uint16_t*>(ws + L.p_th2b);
  a.th2T = reinterpret_cast<uint16_t*>(ws + L.p_th2T);
  a.tloss = reinterpret_cast<double*>(ws + L.p_tloss);
  a.grads = reinterpret_cast<float*>(ws + L.p_grads);
  a.gW1 = a.grads + o.W1;
  a.gb1 = a.grads + o.b1;
  a.gW2 = a.grads + o.W2;
  a.gb2 = a.grads + o.b2;
  a.gE = a.grads + o.E;
  a.gbeta = a.grads + o.beta;
  return a;
}

vbgs_status vbgs_proposal_set(vbgs_ctx* c, const float* W1, const float* b1, const float* W2, const float* b2,
                              const float* E, const float* beta, const float* mu_in, const float* inv_s_in,
                              void* stream) {
  if (!c || !W1 || !b1 || !W2 || !b2 || !E || !beta || !mu_in || !inv_s_in) return VBGS_ERR_ARG;
  if (!c->p.proposal) return fail(c, VBGS_ERR_STATE, "params.proposal is 0");
  VBGS_SETTLE(c, stream);
  PArgs a = make_pargs(c);
  const PropOffsets o(c->p.D, c->p.K);
  const hipStream_t s = S(stream);
  const int64_t H = VBGS_H, D = c->p.D, K = c->p.K;
  hipError_t e = hipMemcpyAsync(a.W + o.W1, W1, H * D * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.W + o.b1, b1, H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.W + o.W2, W2, H * H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.W + o.b2, b2, H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.W + o.E, E, K * H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(a.W + o.beta, beta, K * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_zero_f32((float*)a.mu_in, 2 * MAXD, s);
  if (e == hipSuccess) e = hipMemcpyAsync((float*)a.mu_in, mu_in, D * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync((float*)a.inv_s_in, inv_s_in, D * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_zero_f32(a.m1, o.n, s);
  if (e == hipSuccess) e = launch_zero_f32(a.m2, o.n, s);
  if (e == hipSuccess) e = launch_zero_f32(reinterpret_cast<float*>(a.step), 2, s);
  if (e == hipSuccess) e = launch_prop_prepare(a, s);
  if (e != hipSuccess) return hipfail(c, e, "proposal_set");
  c->prop_ready = true;
  c->prop_prepared = true;
  return VBGS_OK;
}

vbgs_status vbgs_proposal_get(vbgs_ctx* c, float* W1, float* b1, float* W2, float* b2, float* E, float* beta,
                              void* stream) {
  if (!c || !W1 || !b1 || !W2 || !b2 || !E || !beta) return VBGS_ERR_ARG;
  if (!c->p.proposal) return fail(c, VBGS_ERR_STATE, "params.proposal is 0");
  VBGS_SETTLE(c, stream);
  PArgs a = make_pargs(c);
  const PropOffsets o(c->p.D, c->p.K);
  const hipStream_t s = S(stream);
  const int64_t H = VBGS_H, D = c->p.D, K = c->p.K;
  hipError_t e = hipMemcpyAsync(W1, a.W + o.W1, H * D * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b1, a.W + o.b1, H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(W2, a.W + o.W2, H * H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b2, a.W + o.b2, H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(E, a.W + o.E, K * H * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(beta, a.W + o.beta, K * 4, hipMemcpyDeviceToDevice, s);
  return hipfail(c, e, "proposal_get");
}

vbgs_status vbgs_estep_stats_pruned(vbgs_ctx* c, const float* X, int64_t N, const int32_t* audit_idx, int64_t n_audit,
                                    double logmass_bound, double frac_bound, double* lse_out, double* stats_out,
                                    double* report, void* stream) {
  if (!c) return VBGS_ERR_ARG;
  if (!c->p.proposal || !c->prop_ready) return fail(c, VBGS_ERR_STATE, "the proposal has no weights (vbgs_proposal_set)");
  if (N < 0 || N > c->p.n_max) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
  if ((N > 0 && !X) || n_audit < 0 || n_audit > N || (n_audit > 0 && !audit_idx))
    return fail(c, VBGS_ERR_ARG, "bad X / audit arguments");
  if (!isfinite(logmass_bound) || !(frac_bound >= 0.0)) return fail(c, VBGS_ERR_ARG, "bad bounds");
  VBGS_SETTLE(c, stream);
  c->seg_used = false;
  const hipStream_t s = S(stream);
  const DevPtrs d = c->dev();
  EstepCfg cfg{c->p.score_prec, 1, c->T2, 1};
  hipError_t e;
  {
    Phase ph(c, 0, s);
    e = launch_frame_prep(d, X, N, s);
  }
  const bool cull = use_cull(c);
  cfg.cull = cull ? 1 : 0;
  cfg.order_reset = c->order_reset ? 1 : 0;
  if (cull && N > 0) c->order_reset = false;
  if (e == hipSuccess) {
    Phase ph(c, 1, s);
    e = prepare_components(c, s);
  }
  PArgs pa = make_pargs(c);
  if (e == hipSuccess && !c->prop_prepared) {
    e = launch_prop_prepare(pa, s);
    c->prop_prepared = e == hipSuccess;
  }
  EArgs ea = make_eargs(d, cfg, X, N, lse_out);
  int32_t* gate = reinterpret_cast<int32_t*>((char*)c->ws + c->L.p_gate);
  if (e == hipSuccess) {
    Phase ph(c, 7, s);
    MlpOut o{};
    o.npad = N;
    o.h2b = pa.h2b;
    e = launch_mlp_fwd(pa, X, nullptr, N, o, s);
    if (e == hipSuccess) e = launch_topc(pa, ea, N, s);
  }
  if (e == hipSuccess) {
    Phase ph(c, 2, s);
    e = launch_point_lse(ea, c->p.D, N, s);  // exact scores of the candidates, LSE over them
    if (e == hipSuccess)
      e = launch_audit(ea, c->p.D, audit_idx, n_audit, reinterpret_cast<double*>((char*)c->ws + c->L.p_aud),
                       ea.lse2, logmass_bound, frac_bound, gate, report, s);
    if (e == hipSuccess && cull) e = launch_sort_points(d, X, N, s);  // (cheap; only used on fallback)
    if (e == hipSuccess) {  // dense exact E-step, executed only when the audit failed
      EArgs eg = ea;
      eg.gate = gate;
      e = launch_exact_sweep(eg, c->p.score_prec, c->p.D, N, s, cull ? 1 : 0);
    }
  }
  if (e == hipSuccess) {
    Phase ph(c, 3, s);
    ea.stats_out = stats_out;  // final statistics written by the sparse kernels
    e = launch_sparse_stats(ea, c->p.D, N, s);
  }
  if (e == hipSuccess) {
    Phase ph(c, 4, s);
    EstepCfg fc = cfg;
    e = launch_fold(d, fc, stats_out, s);
  }
  if (e != hipSuccess) return hipfail(c, e, "estep_stats_pruned");
  c->last_N = N;
  c->lse_version = c->post_version;
  c->have_stats = true;
  return VBGS_OK;
}

vbgs_status vbgs_proposal_candidates(vbgs_ctx* c, const float* X, int64_t N, int32_t* cand_out, void* stream) {
  if (!c || !cand_out) return VBGS_ERR_ARG;
  if (!c->p.proposal || !c->prop_ready) return fail(c, VBGS_ERR_STATE, "the proposal has no weights");
  if (N < 0 || N > c->p.n_max || (N > 0 && !X)) return fail(c, VBGS_ERR_SHAPE, "N outside 0..n_max");
  VBGS_SETTLE(c, stream);
  const hipStream_t s = S(stream);
  PArgs pa = make_pargs(c);
  hipError_t e = hipSuccess;
  if (!c->prop_prepared) {
    e = launch_prop_prepare(pa, s);
    c->prop_prepared = e == hipSuccess;
  }
  EstepCfg cfg{c->p.score_prec, 1, c->T2, 1};
  const EArgs ea = make_eargs(c->dev(), cfg, X, N, nullptr);
  MlpOut o{};
  o.npad = N;
  o.h2b = pa.h2b;
  if (e == hipSuccess) e = launch_mlp_fwd(pa, X, nullptr, N, o, s);
  if (e == hipSuccess) e = launch_topc(pa, ea, N, s);
  if (e == hipSuccess) e = launch_topc_export(ea, N, pa.C, cand_out, s);
  c->have_stats = false;  // the candidate lists no longer belong to the last E-step
  return hipfail(c, e, "proposal_candidates");
}

vbgs_status vbgs_export_targets(vbgs_ctx* c, const float* X, int64_t N, int32_t* tk, float* tr, void* stream) {
  if (!c || !X || !tk || !tr) return VBGS_ERR_ARG;
  if (c->p.score_prec == VBGS_FP64 || !c->p.exact) return fail(c, VBGS_ERR_UNSUPPORTED, "needs the exact MFMA mode");
  if (!c->have_stats || N != c->last_N) return fail(c, VBGS_ERR_STATE, "N must match the last E-step");
  VBGS_SETTLE(c, stream);
  EstepCfg cfg{c->p.score_prec, 1, c->T2, 1};
  const EArgs ea = make_eargs(c->dev(), cfg, X, N, nullptr);
  return hipfail(c, launch_export_targets(ea, N, tk, tr, S(stream)), "export_targets");
}

vbgs_status vbgs_proposal_train_step(vbgs_ctx* c, const float* X, const int32_t* tk, const float* tr,
                                     const int32_t* batch_idx, int32_t B, float lr, int32_t apply, double* loss_out,
                                     float* grads_out, void* stream) {
  if (!c || !X || !tk || !tr || !batch_idx) return VBGS_ERR_ARG;
  if (!c->p.proposal || !c->prop_ready) return fail(c, VBGS_ERR_STATE, "the proposal has no weights");
  const int64_t Bt = c->p.train_batch > 0 ? c->p.train_batch : 4096;
  if (B < 1 || B > Bt) return fail(c, VBGS_ERR_SHAPE, "B outside 1..train_batch");
  if ((apply != 0 && apply != 1) || !(lr >= 0.0f)) return fail(c, VBGS_ERR_ARG, "bad apply / lr");
  VBGS_SETTLE(c, stream);
  PArgs a = make_pargs(c);
  if (!c->prop_prepared) {
    const hipError_t e = launch_prop_prepare(a, S(stream));
    if (e != hipSuccess) return hipfail(c, e, "proposal_prepare");
    c->prop_prepared = true;
  }
  a.Bpad = ((int64_t)B + 63) / 64 * 64;
  Phase ph(c, 7, S(stream));
  return hipfail(c, launch_train(a, X, tk, tr, batch_idx, B, lr, apply, loss_out, grads_out, S(stream)),
                 "proposal_train_step");
}

vbgs_status vbgs_timing(vbgs_ctx* c, int32_t enable) {
  if (!c || (enable != 0 && enable != 1)) return VBGS_ERR_ARG;
  return vbgs_timing_phases(c, enable ? (1u << VBGS_NPHASE) - 1u : 0u);
}

vbgs_status vbgs_timing_phases(vbgs_ctx* c, uint32_t mask) {
  if (!c || (mask >> VBGS_NPHASE) != 0) return VBGS_ERR_ARG;
  const bool enable = mask != 0;
  if (enable && !c->timers_made) {
    for (int p = 0; p < VBGS_NPHASE; ++p) {
      PhaseTimer& t = c->tm[p];
      for (int i = 0; i < PhaseTimer::RING; ++i) {
        hipError_t e = hipEventCreate(&t.a[i]);
        if (e == hipSuccess) e = hipEventCreate(&t.b[i]);
        if (e != hipSuccess) return hipfail(c, e, "hipEventCreate");
        t.used[i] = false;
      }
      t.head = 0;
      t.ms = 0.0;
      t.count = 0;
    }
    c->timers_made = true;
  }
  c->timing = enable;
  c->timing_mask = mask;
  return VBGS_OK;
}

vbgs_status vbgs_timing_read(vbgs_ctx* c, double ms[VBGS_NPHASE], int64_t counts[VBGS_NPHASE], void* stream) {
  if (!c || !ms || !counts) return VBGS_ERR_ARG;
  hipError_t e = hipStreamSynchronize(S(stream));
  if (e != hipSuccess) return hipfail(c, e, "timing_read");
  for (int p = 0; p < VBGS_NPHASE; ++p) {
    ms[p] = 0.0;
    counts[p] = 0;
    if (!c->timers_made) continue;
    PhaseTimer& t = c->tm[p];
    for (int i = 0; i < PhaseTimer::RING; ++i) harvest(t, i);
    ms[p] = t.ms;
    counts[p] = t.count;
    t.ms = 0.0;
    t.count = 0;
  }
  return VBGS_OK;
}

const char* vbgs_last_error(const vbgs_ctx* c) { return c ? c->err.c_str() : "null context"; }

void vbgs_destroy(vbgs_ctx* c) {
  if (!c) return;
  if (c->side) {  // their work precedes the events that the caller's stream waited on
    hipStreamSynchronize(c->side);
    hipStreamSynchronize(c->side2);
    hipEventDestroy(c->fork);
    hipEventDestroy(c->join);
    hipEventDestroy(c->kl_done);
    hipEventDestroy(c->begin);
    hipEventDestroy(c->rows_done);
    hipEventDestroy(c->feat_done);
    hipStreamDestroy(c->side2);
    hipStreamDestroy(c->side);
  }
  if (c->timers_made)
    for (int p = 0; p < VBGS_NPHASE; ++p)
      for (int i = 0; i < PhaseTimer::RING; ++i) {
        hipEventDestroy(c->tm[p].a[i]);
        hipEventDestroy(c->tm[p].b[i]);
      }
  delete c;
}

}  // extern "C"
