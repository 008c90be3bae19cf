// Internal definitions of the learned candidate proposal.
#pragma once

#include <algorithm>

#include "vbgs_internal.h"

namespace vbgs {

typedef EArgs EArgsLite;

// Offsets of the six trainable arrays inside the flat FP32 parameter block (and its gradient
// and Adam moment copies): W1 (H x D), b1 (H), W2 (H x H), b2 (H), E (K x H), beta (K).
struct PropOffsets {
  int64_t W1, b1, W2, b2, E, beta, n;
  PropOffsets(int D, int64_t K) {
    W1 = 0;
    b1 = (int64_t)VBGS_H * D;
    W2 = b1 + VBGS_H;
    b2 = W2 + (int64_t)VBGS_H * VBGS_H;
    E = b2 + VBGS_H;
    beta = E + K * VBGS_H;
    n = beta + K;
  }
};

struct PArgs {
  int64_t K, Kpad, Bpad, n_train;
  int D, C;
  // weights (state)
  float* W;  // flat trainable block
  const float *W1, *b1, *W2, *b2, *E, *beta, *mu_in, *inv_s_in;
  float *m1, *m2;
  double* step;
  // MFMA operand copies (workspace)
  uint16_t *Ebf, *EbfT;
  float *betap, *W2T;
  // pruned E-step
  uint16_t* h2b;
  float* tz;
  int32_t *tk, *tcnt;
  float* tthr;  // per point: lower bound on its C-th best logit
  // FP8 logits (f8 = 1): e4m3 embedding rows and point rows with the factors undoing their scaling
  int f8;
  uint8_t *E8, *h8;
  float *sE, *sh;
  // training
  float *th1, *th2, *txs, *tlse, *tdh2, *tdp1;
  float *tlpart, *tdpart;  // per component slice: partial (max, sum) of the logits, partial dh2 rows
  float* twpart;           // per batch slice: partial hidden-layer weight gradients
  uint16_t *th2b, *th2T;
  double* tloss;
  float *grads, *gW1, *gb1, *gW2, *gb2, *gE, *gbeta;
};

// component slices of the training passes, so that a minibatch fills the GPU: the logits LSE
// takes enough slices for ~512 workgroups (at most 32), the dh2 product at most 16 with no more than
// 65536 partial rows
inline int train_lse_split(int64_t B) {
  const int64_t wg = (B + 255) / 256, s = (512 + wg - 1) / wg;
  return (int)(s < 1 ? 1 : (s > 32 ? 32 : s));
}
constexpr int TRAIN_W_SPLIT = 16;  // batch slices of the hidden-layer weight gradients
inline int train_dh_split(int64_t B) {
  const int64_t s = 65536 / (B > 0 ? B : 1);
  return (int)(s < 1 ? 1 : (s > 16 ? 16 : s));
}

struct MlpOut {
  int64_t npad;  // rows written (rows >= n are zero)
  float *h1, *h2, *xs;
  uint16_t *h2b, *h2T;
};

hipError_t launch_prop_prepare(const PArgs& a, hipStream_t s);
hipError_t launch_mlp_fwd(const PArgs& a, const float* X, const int32_t* idx, int64_t n, const MlpOut& o,
                          hipStream_t s);
hipError_t launch_topc(const PArgs& a, const EArgsLite& e, int64_t N, hipStream_t s);
hipError_t launch_audit(const EArgsLite& e, int D, const int32_t* idx, int64_t n, double* aud, const double* lse2,
                        double bound, double frac, int32_t* gate, double* report, hipStream_t s);
hipError_t launch_topc_export(const EArgsLite& e, int64_t N, int C, int32_t* out, hipStream_t s);
hipError_t launch_export_targets(const EArgsLite& e, int64_t N, int32_t* tk, float* tr, hipStream_t s);
hipError_t launch_train(const PArgs& a, const float* X, const int32_t* tk, const float* tr, const int32_t* bidx,
                        int64_t B, float lr, int apply, double* loss_out, float* grads_out, hipStream_t s);
hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s);

}  // namespace vbgs
