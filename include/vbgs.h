/*
 * vbgs.h -- C ABI of the MI355X (gfx950) library for the variational-Bayes
 * Gaussian-splatting fit step: per-frame E-step, sufficient statistics,
 * conjugate update and evidence lower bound.
 *
 * Model (Sec. 2.1.2, Fig. 2): each of K components has a Normal-Wishart
 * posterior q(mu_k, Lambda_k) = NW(m_k, kappa_k, W_k, nu_k) and the mixture
 * weights a Dirichlet(alpha). The paper's NIW(m, kappa, V, n) on (mu, Sigma)
 * is the same distribution with W = V^{-1}, nu = n. The fit step of Alg. 1
 * (responsibilities R, statistics Delta S = R^T S_u of Eq. (fused_contr),
 * S <- S + Delta S, closed-form update) becomes:
 *
 *   vbgs_estep_stats : score every point against every component,
 *                      rho_nk = E[ln pi_k] + 1/2 E[ln|Lambda_k|] - D/2 ln(2 pi)
 *                               - 1/2 (D/kappa_k + nu_k (x-m_k)^T W_k (x-m_k)),
 *                      normalise over k (LSE_n), and accumulate
 *                      N_k = sum_n r_nk, S1_k = sum_n r_nk x_n,
 *                      S2_k = sum_n r_nk x_n x_n^T; the N x K responsibility
 *                      matrix is never stored.
 *   vbgs_update      : posterior <- frame prior (+) statistics (conjugate,
 *                      natural parameters); optionally commit it as the
 *                      next frame's prior (replay-free continual update).
 *   vbgs_elbo        : F(q) = sum_n LSE_n - KL(Dir(alpha)||Dir(alpha_p))
 *                      - sum_k KL(NW_k || NW_p,k).
 *
 * Conventions for every entry point:
 *  - Device pointers are caller-owned (e.g. PyTorch tensors), contiguous, on
 *    the device of `stream`. `stream` is a hipStream_t passed as void*
 *    (NULL = the legacy default stream).
 *  - Calls only enqueue work on `stream`: they never synchronise (except
 *    vbgs_sync_status) and never allocate device memory. State and workspace
 *    are caller-provided buffers sized by vbgs_query_sizes. (The culled exact
 *    E-step forks part of its work onto two streams the context made at init,
 *    after an event on `stream`, and `stream` waits on their events before
 *    the call's later work, so `stream` still orders every call.)
 *  - Every call returns a vbgs_status; no C++ exception crosses the ABI.
 *    Argument and shape errors are returned synchronously and leave the
 *    context unchanged. Numeric faults found on the device (a W^{-1} that is
 *    not positive definite, non-finite input points) set sticky device flags
 *    that vbgs_sync_status reports.
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef VBGS_C_ABI_H_
#define VBGS_C_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VBGS_ABI_VERSION 1
#define VBGS_MAX_D 8

typedef struct vbgs_ctx vbgs_ctx;

typedef enum {
  VBGS_OK = 0,
  VBGS_ERR_ARG = -1,         /* null pointer, bad enum, out-of-range scalar */
  VBGS_ERR_SHAPE = -2,       /* D, K or N outside the supported/declared range */
  VBGS_ERR_HIP = -3,         /* a HIP runtime call failed (message in vbgs_last_error) */
  VBGS_ERR_NOT_PD = -4,      /* sticky: some W^{-1} was not positive definite */
  VBGS_ERR_NONFINITE = -5,   /* sticky: non-finite input coordinates */
  VBGS_ERR_STATE = -6,       /* call order: e.g. vbgs_elbo(X=NULL) after an update */
  VBGS_ERR_UNSUPPORTED = -7  /* valid request the library does not implement */
} vbgs_status;

/* Precision of the score GEMM (the dot product of quadratic point features
 * [1, x, upper(x x^T)] with per-component coefficient rows on MFMA).
 * VBGS_FP64 selects the plain direct-form FP64 path (no GEMM). */
typedef enum {
  VBGS_FP64 = 0,    /* direct form (x-m)^T W (x-m) in FP64 on the vector ALUs */
  VBGS_FP32 = 1,    /* v_mfma_f32_16x16x4_f32, FP32 accumulation */
  VBGS_BF16 = 2,    /* v_mfma_f32_16x16x32_bf16, FP32 accumulation */
  VBGS_BF16X3 = 3,  /* split BF16 (hi*hi + hi*lo + lo*hi), FP32 accumulation */
  VBGS_AUTO = 4,    /* exact = 1 only: per E-step, the split-BF16 screen unless its error bound
                       (2^-12 |c| |phi| for the mean coefficient-row and feature norms) exceeds
                       32 log2 units, else the FP32 screen; the choice is made on the device and
                       reported by vbgs_counters (the results are exact either way) */
  VBGS_FP64_CULLED = 6,  /* exact = 1, cull = 1 only: a comparator with the culled sweep's point blocks,
                       seeds and tile / row bounds, every pair within the bounds scored directly in FP64
                       (no MFMA), then the exact mode's LSE and statistics: what the culling alone gives,
                       against the same results. Same params limits as the MFMA precisions (D <= 6). */
  VBGS_FP8 = 5      /* exact = 0 only (a plain tier whose error is reported): every feature and
                       coefficient row scaled by a power of two so that its largest magnitude lies
                       in [224, 448], rounded to OCP e4m3 (nearest even), v_mfma_f32_16x16x32_fp8_fp8
                       with FP32 accumulation, the two scales undone on the FP32 scores. As a screen
                       its error bound (~2^-3 |c| |phi|) would admit nearly every pair, so the exact
                       mode does not take it (VBGS_ERR_UNSUPPORTED) */
} vbgs_prec;

typedef struct {
  int32_t abi_version;     /* must be VBGS_ABI_VERSION */
  int32_t D;               /* feature dimension, 1..8 (MFMA precisions: 1..6) */
  int64_t K;               /* number of components, >= 1 */
  int64_t n_max;           /* largest N any call will pass (workspace sizing); exact MFMA mode: <= 2^23 */
  double kappa0, nu0, alpha0;  /* shared prior scalars: kappa0 > 0, nu0 > D-1, alpha0 > 0 */
  int32_t score_prec;      /* vbgs_prec */
  int32_t exact;           /* MFMA precisions only. 1: the GEMM is a bounded screen and every
                              pair that can carry mass is rescored exactly in FP64 (results
                              match the FP64 path to rounding); 0: the GEMM scores are used
                              as they are (the error is that of the precision) */
  double screen_margin;    /* nats; pairs whose upper bound is more than this below the
                              point's running maximum (pass 1) or its LSE (pass 2) are
                              skipped. <= 0 selects ln(K) + ln(1e12). */
  int32_t n_split;         /* pass-2 point splits; 0 = automatic */
  int32_t proposal;        /* 1: allocate the learned candidate proposal (MFMA precisions, D <= 6) */
  int32_t C;               /* candidates per point proposed by the network, 1..64 (default 32) */
  int32_t train_batch;     /* largest training minibatch, 0..65536 (default 4096) */
  int32_t cull;            /* exact MFMA mode: 1 (default) sorts points and components spatially and
                              skips whole 64-component tiles whose score bound lies below the margin;
                              0 screens every tile */
  int32_t modal_split;     /* 0 (default): one joint Normal-Wishart over all D coordinates.
                              s in 1..D-1: the model of Sec. 2.1.2 with two independent modalities,
                              coordinates [0, s) (spatial) and [s, D) (colour), each with its own
                              Normal-Wishart (kappa, nu, W; both blocks start from kappa0, nu0 and
                              the matching diagonal block of W0, entries of W0 across the blocks are
                              ignored). nu0 must exceed the block sizes minus 1. Needs D <= 7 and
                              proposal = 0 (else VBGS_ERR_UNSUPPORTED). */
  int32_t cull_dims;       /* leading coordinates the culled sweep bounds distances in, 0..3.
                              0 (default): modal_split if it is 1..3, else 2 for D = 5 (pixel
                              u, v, r, g, b) and min(D, 3) otherwise. Any choice gives the same
                              results; coordinates with a much weaker precision than the others
                              only loosen the bounds (slower). */
  int32_t proposal_prec;   /* precision of the proposal's logits h2 . E_k: 0 or VBGS_BF16 (default):
                              v_mfma_f32_16x16x32_bf16, four per 16 x 16 block; VBGS_FP8: every h2 row
                              and embedding row scaled by the power of two that puts its largest
                              magnitude in [224, 448], rounded to OCP e4m3 (nearest even), one
                              v_mfma_scale_f32_16x16x128_f8f6f4 per block (block scales 1), the two
                              row factors undone on the FP32 products. Training stays BF16. */
  int64_t reserved[3];     /* must be zero */
} vbgs_params;

#define VBGS_H 128         /* hidden width of the proposal network (= embedding width) */

/* Fill *p with defaults for (D, K, n_max): kappa0 = 1, nu0 = D + 2, alpha0 = 1,
 * score_prec = VBGS_AUTO (D <= 6; else VBGS_FP64), exact = 1, screen_margin = 0 (automatic). Set
 * an explicit MFMA precision with exact = 0 or with the proposal. */
vbgs_status vbgs_default_params(vbgs_params* p, int32_t D, int64_t K, int64_t n_max);

/* Bytes of caller-owned device memory: `state` persists across calls and frames
 * (frame prior + posterior: a checkpoint of it is a checkpoint of the model);
 * `workspace` is scratch reused by every call (its contents do not need to
 * survive between frames). Both must be 256-byte aligned. */
vbgs_status vbgs_query_sizes(const vbgs_params* p, size_t* state_bytes, size_t* workspace_bytes);

/* Create a context and initialise the state: for every component k the frame
 * prior and the posterior are set to (alpha0, kappa0, m0[k], W0, nu0).
 *   m0      : device, K x D row-major FP64, the prior means.
 *   W0      : HOST, D x D row-major FP64, symmetric positive definite Wishart
 *             scale (the same for every component). Not PD -> VBGS_ERR_NOT_PD.
 *   state, workspace : device buffers of the sizes from vbgs_query_sizes.
 * The state is written by kernels on `stream`; *out is set only on success. */
vbgs_status vbgs_init(vbgs_ctx** out, const vbgs_params* p, const double* m0, const double* W0,
                      void* state, void* workspace, void* stream);

/* Attach a context to an existing state buffer (resume from a checkpoint, e.g. a copy of the
 * state of an earlier context): no kernel runs here; the state must come from a context with the
 * same params. The workspace may hold anything: its sticky flags and counters are cleared on the
 * stream of the first call made with the new context, before that call's own work, so that
 * continuing from the copy gives what the uninterrupted context would have given. */
vbgs_status vbgs_attach(vbgs_ctx** out, const vbgs_params* p, void* state, void* workspace);

/* E-step + sufficient statistics of one frame at the current posterior.
 *   X         : device, N x D row-major FP32 points (N <= n_max; N = 0 allowed).
 *   lse_out   : device, N FP64 or NULL. LSE_n in nats (the per-point ELBO term).
 *   stats_out : device, K x F FP64 or NULL, F = 1 + D + D(D+1)/2, per component
 *               [N_k, S1_k (D), S2_k upper triangle row-major (i <= j)], raw
 *               coordinates. The statistics are also kept in the workspace for
 *               vbgs_update. Reductions are deterministic (fixed order). */
vbgs_status vbgs_estep_stats(vbgs_ctx* ctx, const float* X, int64_t N, double* lse_out,
                             double* stats_out, void* stream);

/* For callers that cannot allocate device memory or must not touch the context's workspace while
 * they run (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * vbgs_estep_stats with, as its workspace, a static device array of VBGS_SCRATCH_BYTES inside the
 * library instead of the context's workspace. Same kernels and launches, same results (bitwise).
 * Allocates nothing: the array is part of the library's code object, one per GPU, held from the
 * library's first use on that GPU until the process ends; its device address is looked up (not
 * allocated) when a context is made.
 *   X, N, lse_out, stats_out: as vbgs_estep_stats (caller-owned inputs and outputs).
 *   The context's workspace and bookkeeping do not change: these statistics are not kept for
 *   vbgs_update, vbgs_elbo(X = NULL) and vbgs_counters do not see this call; the sticky device
 *   flags it raises are added to the context's (vbgs_sync_status reports them).
 * Errors: VBGS_ERR_SHAPE (with the sizes in vbgs_last_error) when the params' workspace
 * (vbgs_query_sizes) exceeds VBGS_SCRATCH_BYTES, e.g. D = 6 exact mode with N = 30000 and
 * K = 4000 fits, c3's N = 307200, K = 100000 does not; VBGS_ERR_HIP if the array's address could
 * not be found. Every call on one GPU, from any context, uses the same array, which keeps the last
 * call's contents (each call clears what must start at zero): calls that overlap in time on one
 * GPU within a process (different streams or threads, any contexts on that device) race and corrupt each
 * other's results; order them on one stream. */
#define VBGS_SCRATCH_BYTES ((size_t)64 << 20)
vbgs_status vbgs_estep_stats_scratch(vbgs_ctx* ctx, const float* X, int64_t N, double* lse_out,
                                     double* stats_out, void* stream);

/* Conjugate update: posterior <- frame prior (+) the last statistics
 * (alpha += N_k, kappa += N_k, nu += N_k, kappa m += S1_k,
 * W^{-1} + kappa m m^T += S2_k). commit = 1 then copies the posterior into the
 * frame prior (end of frame). Needs a preceding vbgs_estep_stats. */
vbgs_status vbgs_update(vbgs_ctx* ctx, int32_t commit, void* stream);

/* Evidence lower bound F(q) at the current posterior against the frame prior,
 * written to elbo_dev (device, 1 FP64). X = NULL reuses sum_n LSE_n of the last
 * vbgs_estep_stats (VBGS_ERR_STATE if the posterior changed since); otherwise
 * the LSE pass runs on X (N points). */
vbgs_status vbgs_elbo(vbgs_ctx* ctx, const float* X, int64_t N, double* elbo_dev, void* stream);

/* Copy the posterior (which = 0) or the frame prior (which = 1) out of / into
 * the state. Device buffers: alpha: K; kappa, nu: K (one block) or K x 2 (modal_split > 0:
 * spatial, colour); m: K x D; Winv: K x D x D (full, symmetric; with two blocks the entries
 * across the blocks read as zero and are ignored when set). Setting does not check positive
 * definiteness (the next E-step flags it). */
vbgs_status vbgs_get_params(vbgs_ctx* ctx, int32_t which, double* alpha, double* kappa, double* m,
                            double* Winv, double* nu, void* stream);
vbgs_status vbgs_set_params(vbgs_ctx* ctx, int32_t which, const double* alpha, const double* kappa,
                            const double* m, const double* Winv, const double* nu, void* stream);

/* Reassignment of under-used components (Alg. 1, `reassign`; Sec. 3.1): sample n points biased
 * towards a low evidence bound and move the means of the n least-used components onto them.
 * X: device N x D FP32 (the frame); lse: device N FP64, the points' log normalisers in nats (the
 * lse_out of a vbgs_estep_stats on X); gumbel: device N FP64 standard Gumbel draws supplied by the
 * caller. Points are taken in decreasing order of gumbel[n] - lse[n] (Gumbel-top-n, i.e. sampling
 * without replacement with probabilities proportional to exp(-lse)), components in increasing
 * order of the posterior alpha; both orders compare the values through their order-preserving
 * 64-bit images with the low 25 bits replaced by the index (ties to the lower index). The i-th
 * point becomes the mean m of the i-th component in the frame prior and in the posterior; no other
 * parameter changes. out_points / out_comps (device int32 n, or NULL) receive the pairs.
 * Requires 0 <= n <= min(N, K) and N, K < 2^25 (VBGS_ERR_SHAPE / VBGS_ERR_UNSUPPORTED);
 * n = 0 does nothing. Invalidates the ELBO of the last E-step, like vbgs_update. */
vbgs_status vbgs_reassign(vbgs_ctx* ctx, const float* X, int64_t N, const double* lse, const double* gumbel,
                          int64_t n, int32_t* out_points, int32_t* out_comps, void* stream);

/* Rendering of the fitted mixture at query positions (the colour that Sec. 5.1's PSNR is taken on).
 * The first s coordinates are the position, the other Dc = D - s the colour. For each query position
 * x the colour is sum_k r_k(x) E[c | x, k]: r_k(x) are the responsibilities of the position marginal
 * of the posterior (the Normal-Wishart (m_s, kappa, ((W^-1)_ss)^-1, nu - Dc); in the two-factor model
 * the position factor itself), scored exactly as vbgs_estep_stats scores points; E[c | x, k] =
 * m_c + (W^-1)_cs ((W^-1)_ss)^-1 (x - m_s) (two-factor model: m_c).
 * model: the fitted context (its posterior is read, nothing in it changes). position: a context the
 * caller created with D = s (= the model's modal_split when that is set), the model's K,
 * modal_split = 0, no proposal, score_prec FP64 or an MFMA precision with exact = 1, n_max >= Nq;
 * its prior and posterior are overwritten with the marginal and its E-step workspace is used (its
 * statistics become invalid for vbgs_update). Xq: device Nq x s FP32 positions. regress: device
 * K x Dc x (1 + s) FP64, caller-owned, receives [m_c, B] per component. colour_out: device Nq x Dc
 * FP32. lse_out: device Nq FP64 (nats, the position marginal's log normaliser) or NULL.
 * A non-positive-definite (W^-1)_ss sets the position context's VBGS_ERR_NOT_PD flag. */
vbgs_status vbgs_render(vbgs_ctx* model, vbgs_ctx* position, const float* Xq, int64_t Nq, double* regress,
                        float* colour_out, double* lse_out, void* stream);

/* PSNR of Sec. 5.1 between two images given as n FP32 values in [0, 1] (values outside are clamped):
 * MSE over all n values of the 0..255-scaled differences, PSNR = 10 log10(255^2 / MSE) (+inf when
 * equal). out: device 2 FP64, [MSE, PSNR]. Deterministic (fixed summation order). */
vbgs_status vbgs_psnr(const float* a, const float* b, int64_t n, double* out, void* stream);

/* Synchronise `stream` and return the sticky device flags (VBGS_ERR_NOT_PD,
 * VBGS_ERR_NONFINITE) or VBGS_OK. Clears nothing; vbgs_clear_flags does. */
vbgs_status vbgs_sync_status(vbgs_ctx* ctx, void* stream);
vbgs_status vbgs_clear_flags(vbgs_ctx* ctx, void* stream);

/* Synchronise `stream` and read counters of the last E-step (exact MFMA mode):
 * out[0] = pairs recorded by the screen sweep, out[1] = pairs kept for the statistics
 * (within the margin of their point's LSE), out[2] = number of points, out[3] = K,
 * out[4] = blocks of 64 points x 16 components the sweep screened on MFMA, out[5] = the
 * number of such blocks without culling (4 per 256-point workgroup and 16 components), out[6] =
 * the blocks screened by all E-steps since vbgs_init or the last vbgs_clear_flags, out[7] = the
 * points whose candidate lists overflowed (their LSE and statistics come from a full rescan),
 * out[8] = the screen precision the sweep used (vbgs_prec), out[9] = the split-BF16 screen's
 * error bound for the mean coefficient-row and feature norms, in 1/1000 log2 units, out[10] =
 * the culled sweep's pair segments: 0 = every kept pair was written into its component's segment
 * (sized from the previous culled E-step's counts), 1 = a pair found no room and the statistics
 * grouped the pairs by a scan of the counts instead (the results are the same either way), -1 =
 * not the culled path. */
vbgs_status vbgs_counters(vbgs_ctx* ctx, int64_t out[11], void* stream);

/* Per-phase timing with HIP events recorded on the stream that runs each phase.
 * Phases: 0 frame moments + features, 1 expectations + coefficient rows, 2 the first pass over
 * all pairs (in exact MFMA mode the screening sweep kernel alone), 3 pass 2 (statistics), 4 fold,
 * 5 update, 6 ELBO reduction, 7 proposal network (forward, logits, top-C, audit), 8 clearing of
 * the transpose counters, 9 exact per-point LSE from the candidates. With culling (exact MFMA
 * mode): 0 the frame moments only, 1 the spatial sort of the components and the gather of their
 * rows with the row and tile bounds (on one of the context's streams), 8 the spatial sort of the
 * points and the sweep's dispatch order; the coefficient rows, the features and the KL terms run
 * on the context's other stream, untimed.
 * vbgs_timing(ctx, 1) creates the events (host-side objects, no device memory) and records
 * every later phase; 0 stops recording. vbgs_timing_read synchronises `stream`, writes the
 * summed duration in ms and the number of recorded launches of each phase, and clears them. */
#define VBGS_NPHASE 10
vbgs_status vbgs_timing(vbgs_ctx* ctx, int32_t enable);
/* As vbgs_timing, recording only the phases p whose bit (1 << p) is set in `mask` (0 stops
 * recording; (1 << VBGS_NPHASE) - 1 is vbgs_timing(ctx, 1)). Each recorded phase adds two events
 * to its stream per launch, and with them some time: a timed loop can record the one phase it
 * needs and leave the others to untimed launches. Errors: VBGS_ERR_ARG for bits >= VBGS_NPHASE. */
vbgs_status vbgs_timing_phases(vbgs_ctx* ctx, uint32_t mask);
vbgs_status vbgs_timing_read(vbgs_ctx* ctx, double ms[VBGS_NPHASE], int64_t counts[VBGS_NPHASE], void* stream);

/* ---------------------------------------------------------------------------------------
 * Learned candidate proposal (needs params.proposal = 1). Not part of the paper's method:
 * a network h2 = relu(W2 relu(W1 x' + b1) + b2), x' = (x - mu_in) * inv_s_in, with logits
 * z_nk = h2_n . E_k + beta_k picks C candidate components per point; only those are scored
 * exactly, and the responsibilities are renormalised over them. Trained on responsibilities
 * of exact E-steps. Weights are FP32 row-major: W1 H x D, b1 H, W2 H x H, b2 H, E K x H,
 * beta K, mu_in D, inv_s_in D (H = VBGS_H), all device pointers.
 * ------------------------------------------------------------------------------------- */

/* Copy weights into the state and reset the Adam moments and step count. */
vbgs_status vbgs_proposal_set(vbgs_ctx* ctx, const float* W1, const float* b1, const float* W2, const float* b2,
                              const float* E, const float* beta, const float* mu_in, const float* inv_s_in,
                              void* stream);
/* Copy the current weights out of the state. */
vbgs_status vbgs_proposal_get(vbgs_ctx* ctx, float* W1, float* b1, float* W2, float* b2, float* E, float* beta,
                              void* stream);

/* E-step + statistics with candidates from the network (top-C of the logits, ties broken on the
 * smaller component index), every candidate scored exactly in FP64, LSE and r over the candidates.
 * Audit: the dense exact LSE of the n_audit points audit_idx (device int32, distinct, < N) gives
 * each one's captured log-mass ln sum_{k in C_n} r_nk = LSE_C(n) - LSE(n) (nats). The frame falls
 * back to the dense exact E-step when ln(mean exp(captured)) < logmass_bound or more than
 * frac_bound of the audited points lie below logmass_bound; the decision is taken on the device
 * and the dense kernels run only then (no host synchronisation). n_audit = 0 disables the audit:
 * the pruned statistics stand unchecked and the report reads [0, NaN, NaN, NaN].
 * report (device, 4 FP64, or NULL): [fallback 0/1, ln mean captured mass, fraction below the
 * bound, minimum captured log-mass]. Outputs as vbgs_estep_stats. */
vbgs_status vbgs_estep_stats_pruned(vbgs_ctx* ctx, const float* X, int64_t N, const int32_t* audit_idx,
                                    int64_t n_audit, double logmass_bound, double frac_bound, double* lse_out,
                                    double* stats_out, double* report, void* stream);

/* Run the network on X (N points) and write each point's C candidates, ascending component
 * index, to cand_out (device, N x C int32; -1 pads when K < C). Logits use BF16 operands with
 * FP32 accumulation; ties at the C-th place are broken by the smaller component index. */
vbgs_status vbgs_proposal_candidates(vbgs_ctx* ctx, const float* X, int64_t N, int32_t* cand_out, void* stream);

/* After a vbgs_estep_stats (exact mode): training targets per point, the kept pairs of the
 * exact E-step (at most 64), tk (device, N x 64 int32, -1 = empty) and their responsibilities
 * tr (device, N x 64 FP32, each pair's FP64 score computed again from X, rounded once).
 * X (device, N x D FP32) must hold the points of that E-step and N its N (the points are not
 * kept by the library; other points give the responsibilities of the kept pairs at those
 * points). VBGS_ERR_ARG for a null pointer; VBGS_ERR_STATE when N differs from that E-step's. */
vbgs_status vbgs_export_targets(vbgs_ctx* ctx, const float* X, int64_t N, int32_t* tk, float* tr, void* stream);

/* One training step of the proposal on a minibatch: rows batch_idx (device int32, B of them) of
 * the points X and of the targets (tk, tr as exported). Loss: mean over the batch of
 * LSE_k(z_nk) - sum_j rbar_nj z_{n,k_j} with rbar the targets renormalised per point; the big
 * products run on BF16 MFMA with FP32 accumulation, master weights FP32.
 * apply = 1: Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8); apply = 0: only gradients.
 * loss_out (device, 1 FP64) or NULL; grads_out (device FP32, the six trainable arrays W1, b1, W2,
 * b2, E, beta concatenated) or NULL. Gradients of E and beta accumulate the sparse target term
 * with FP32 atomics, so they are reproducible to rounding, not bitwise. */
vbgs_status vbgs_proposal_train_step(vbgs_ctx* ctx, const float* X, const int32_t* tk, const float* tr,
                                     const int32_t* batch_idx, int32_t B, float lr, int32_t apply,
                                     double* loss_out, float* grads_out, void* stream);

/* Last error message of this context ("" if none). Never NULL. */
const char* vbgs_last_error(const vbgs_ctx* ctx);

/* Release the host-side context (no device memory is owned). NULL is a no-op. */
void vbgs_destroy(vbgs_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* VBGS_C_ABI_H_ */
