/*
 * cm.h -- C ABI of the MI355X SFFT Carr–Madan pricing library (libcm.so).
 *
 * The library prices European calls with the damped Fourier transform of Carr & Madan
 * (paper Section 2.1) in two ways:
 *   - the SFFT path (paper Section 3): a quantised tensor train (QTT) of the integrand x
 *     (Eq. x), the tensor-train operator of the QFT without its bit reversal (Q_n,
 *     Section 3.2), the zip-up application of that operator, TT rounding, and a readout of
 *     bit-reversed prices (Eq. discretization_dft);
 *   - the dense path: the integrand on all M = 2^n grid points and a Stockham FFT of the
 *     minus-sign unitary DFT (Eq. dft), followed by the same readout.
 *
 * Conventions shared by every call
 *   - Every call is stream-ordered on `stream` (a hipStream_t passed as void*; NULL is the
 *     null stream). No call synchronises the stream, allocates device memory or keeps
 *     global state, except cm_qft_mpo, which synchronises once to report operator ranks.
 *   - All buffers are caller-owned. "device" means device memory of the current HIP
 *     device; "host" means ordinary host memory.
 *   - Complex numbers are interleaved (re, im): float2 for CM_C64, double2 for CM_C128.
 *   - The return value reports call-level errors (bad arguments, undersized workspace,
 *     HIP launch failures), detected before anything is enqueued where possible.
 *     Data-dependent failures of one instance are written to a device status array
 *     (one int32 per instance, cm_status values) and never abort the batch.
 *   - Grid notation: M = 2^n, eta = frequency step, lambda = 2 pi / (M eta) the log-strike
 *     step (grid relation of Section 2.1), k_u = k0 + lambda u, v_j = v0 + j eta.
 */
#ifndef CM_H
#define CM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CM_MAX_N 48          /* largest supported grid exponent n (QTT length)       */
#define CM_RANKS_STRIDE 49   /* int32 entries per instance in cm_tt_batch.ranks      */

typedef enum {
  CM_OK = 0,
  CM_E_INVALID = 1,      /* bad argument, or a workspace smaller than the op needs */
  CM_E_MOMENT = 2,       /* damping moment E[S_T^(alpha+1)] infinite (Eq. damping_moment_condition) */
  CM_E_RANKCAP = 3,      /* a bond hit cap_rank while the truncation error exceeded tol; result still written */
  CM_E_NOCONV = 4,       /* an iteration (Jacobi sweeps, QTT refinement) did not converge */
  CM_E_NONFINITE = 5,    /* NaN or Inf met in the data */
  CM_E_HIP = 6,          /* a HIP runtime call failed */
  CM_E_UNSUPPORTED = 7,  /* valid request outside what this library supports (e.g. n too large for a path) */
} cm_status;

/* CM_VG: Variance Gamma, the log-price a Brownian motion with drift run on an independent
 *        gamma clock (Section 2); cf (1 - i u theta nu + sigma^2 nu u^2/2)^(-T/nu) times the
 *        martingale drift. */
enum { CM_BS = 0, CM_MERTON = 1, CM_HESTON = 2, CM_VG = 3 };
/* CM_QUAD_RECT2: the paper's symmetric rectangle rule (Eq. Ck_from_psi), v0 = -M eta/2,
 *                w_j = eta, price factor 1/(2 pi).
 * CM_QUAD_SIMPSON1: one-sided Simpson rule folded into x (the higher-order option noted at
 *                the end of Section 2.1), v0 = 0, w_j = (eta/3)(3 - (-1)^j - delta_j0),
 *                price factor 1/pi. */
enum { CM_QUAD_RECT2 = 0, CM_QUAD_SIMPSON1 = 1 };
enum { CM_C64 = 0, CM_C128 = 1 };

/* One pricing instance (128 bytes, plain data; arrays of it live in device memory).
 *   p[] : BS {sigma}; Merton {sigma, lambda_J, mu_J, delta_J}; Heston {kappa, theta,
 *         sigma_v, rho, v0}; Variance Gamma {sigma, nu, theta} (nu the variance rate of the
 *         gamma clock; invalid unless 1 - theta nu - sigma^2 nu/2 > 0, which the martingale
 *         drift needs).
 *   k0  : lowest log-strike; NaN selects ln(S0) - pi/eta (at-the-money at u = M/2). */
typedef struct {
  int32_t model, quad, n, flags;
  double S0, r, q, T, alpha, eta;
  double k0;
  double p[5];
  double reserved[2];
} cm_problem;

/* A ragged batch of tensor trains (d_in = 1) or tensor-train operators (d_in = 2).
 * Instance b has n[b] cores; core l (0-based) is a dense array
 *   [r_l][d_out][d_in][r_{l+1}]   (complex, row-major, r_0 = r_n = 1)
 * starting at complex element core_off[b*CM_MAX_N + l] of `cores`. Bond dimensions live in
 * ranks[b*CM_RANKS_STRIDE + l], l = 0..n[b]; calls that produce a TT write them.
 * Core l of a TT of the integrand carries bit j_{l+1} of the frequency index with weight
 * 2^(n-1-l) (most significant first, Eq. discretized_x); core l of an output TT carries
 * the log-strike bit of weight 2^l (bit-reversed order, Section 3.2).
 * Use cm_tt_layout to compute offsets that hold any rank up to cap_rank. */
typedef struct {
  int32_t batch;           /* number of trains                                        */
  int32_t d_out, d_in;     /* physical dimensions per core: TT (2, 1), operator (2, 2) */
  int32_t cap_rank;        /* every bond dimension is at most cap_rank (capacity)      */
  int32_t n_max;           /* host: largest n[b] in the batch                          */
  int32_t dtype;           /* CM_C64 or CM_C128                                        */
  int32_t rank_max;        /* host: largest bond dimension, when known (0 = unknown)   */
  int32_t flags;           /* host: CM_TT_* hints about the cores' canonical form      */
  const int32_t *n;        /* device [batch]                                           */
  int32_t *ranks;          /* device [batch * CM_RANKS_STRIDE]                         */
  const int64_t *core_off; /* device [batch * CM_MAX_N]                                */
  void *cores;             /* device, complex elements of dtype                        */
} cm_tt_batch;

/* cm_tt_batch.flags (host-side hints, set by the calls that produce a train):
 *   CM_TT_LEFT_ORTHO  cores 0..n-2 are left-orthonormal (cm_sfft_apply output); cm_tt_round
 *                     then skips its orthogonalising sweep.
 *   CM_TT_RIGHT_ORTHO cores 1..n-1 are right-orthonormal (cm_build_qtt, cm_tt_round,
 *                     cm_qft_mpo output), the form cm_sfft_apply expects of its inputs.
 * A caller that edits cores must clear the flags. */
#define CM_TT_LEFT_ORTHO 1
#define CM_TT_RIGHT_ORTHO 2

/* Operation identifiers for cm_workspace_bytes. */
enum { CM_OP_QFT_MPO = 0, CM_OP_BUILD_QTT = 1, CM_OP_SFFT_APPLY = 2, CM_OP_TT_ROUND = 3,
       CM_OP_FFT_PRICE = 4, CM_OP_SAMPLE = 5 };

/* Host helper. Writes the capacity layout of one train with n cores into off[0..n-1]
 * (complex-element offsets relative to the train's first core; add a per-train base) and
 * returns the number of complex elements the train needs. Interior bond l is bounded by
 * min(cap_rank, (d_out d_in)^l); bonds 0 and n are 1. Returns -1 on bad arguments. */
int64_t cm_tt_layout(int n, int d_out, int d_in, int cap_rank, int64_t *off);

/* Host helper. Bytes of device workspace the operation needs for `batch` instances of
 * chain length at most n_max and bond dimensions at most cap_rank (0 on bad arguments).
 * For CM_OP_QFT_MPO, batch is the number of operators one call builds (1 for cm_qft_mpo).
 * For CM_OP_FFT_PRICE, n_max is the grid exponent and cap_rank is ignored; for
 * CM_OP_SAMPLE, cap_rank is the train's storage cap y->cap_rank.
 * Sweep ops (CM_OP_BUILD_QTT, CM_OP_SFFT_APPLY, CM_OP_TT_ROUND) run persistent workgroups,
 * one per workspace slab of cm_workspace_bytes(op, 1, n_max, cap_rank, dtype) bytes, each
 * looping over instances b, b + slots, ...: the default size gives min(batch, 2048) slots;
 * any workspace of s >= 1 slabs is accepted and runs min(s, batch) slots, which is how a
 * caller (the autotuner of the Python layer) picks the launch width. */
size_t cm_workspace_bytes(int op, int batch, int n_max, int cap_rank, int dtype);

/* Builds the tensor-train operator of Q_n: the minus-sign unitary DFT of Eq. dft without
 * the final bit reversal (QFT = R_n Q_n, Section 3.2), so that output core l carries
 * log-strike bit 2^l. The operator is assembled exactly from per-bond interpolation of its
 * phase (a construction different from the paper's zip-up of the gate circuit, same
 * operator) and then rounded to relative Frobenius tolerance `tol` with bonds at most
 * cap_rank, leaving cores 1..n-1 right-orthonormal. The result goes to train `slot` of
 * `w` (d_out = d_in = 2); w->n[slot] must already equal n on the device. Sets
 * w->rank_max on the host (this call synchronises `stream` once to read the ranks).
 * Workspace: cm_workspace_bytes(CM_OP_QFT_MPO, 1, n, cap_rank, dtype). */
cm_status cm_qft_mpo(int n, double tol, int cap_rank, cm_tt_batch *w, int slot,
                     void *ws, size_t ws_bytes, void *stream);

/* Operator look-up table (the stored SFFT operators of Sections 3.3 and 4.1: Q_n depends only
 * on n and the tolerance, so it is built once and reused): builds Q_n exactly as cm_qft_mpo
 * does, for every n in [n_lo, n_hi], into train slot n of `w` (w->batch > n_hi, w->n[n] == n
 * on the device), with one workgroup per operator in a single launch. The operators are
 * bit-identical to those of separate cm_qft_mpo calls. Synchronises `stream` once; returns
 * the first non-OK status among the operators.
 * Workspace: cm_workspace_bytes(CM_OP_QFT_MPO, n_hi - n_lo + 1, n_hi, cap_rank, dtype). */
cm_status cm_qft_mpo_table(int n_lo, int n_hi, double tol, int cap_rank, cm_tt_batch *w,
                           void *ws, size_t ws_bytes, void *stream);

/* Builds, for each problem b, the QTT of the integrand
 *   x_j = w_j psi(v_j) exp(-i j eta k0)          (Eq. x; psi from Eq. psi)
 * on j = 0..M-1 with M = 2^prob[b].n (MSB-first cores, Eq. discretized_x), rounded to
 * relative tolerance tol (bond dims <= cap_rank) with cores 1..n-1 right-orthonormal.
 * The exponential factor is the exact rank-1 train of Section 3.3; the smooth remainder
 * is interpolated on an adaptive dyadic partition (piecewise Chebyshev) instead of the
 * paper's TT-cross. prob: device [batch]. x: trains with x->n[b] == prob[b].n and
 * d_out = 2, d_in = 1. status: device [batch] (CM_E_MOMENT for Heston instances whose
 * damping moment explodes before T, CM_E_NONFINITE, CM_E_NOCONV, CM_E_RANKCAP).
 * Workspace: cm_workspace_bytes(CM_OP_BUILD_QTT, batch, x->n_max, cap_rank, dtype). */
cm_status cm_build_qtt(const cm_problem *prob, int batch, double tol, int cap_rank,
                       cm_tt_batch *x, int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* SFFT step (Section 3.2-3.3, Eq. complexity_TTO): y_b = Q_n x_b for every train b,
 * computed by a left-to-right zip-up contraction. At each site the contracted block
 * T[(chi, u)][(w', r')] is factored by Householder QR with column pivoting, stopped at the
 * first rank k whose exact remaining Frobenius tail is at most tol ||x|| / sqrt(n-1); Q_k
 * becomes output core l (left-orthonormal) and R_k P^T the carry into site l+1. Bonds are
 * at most min(cap_rank, 48); a site that would need more sets CM_E_RANKCAP (result still
 * written). The SVD-optimal ranks come from the cm_tt_round that follows. w_by_n holds one
 * operator per chain length: train n of w_by_n is Q_n (so w_by_n->batch > n_max), built by
 * cm_qft_mpo with cores 1..n-1 right-orthonormal and bonds <= 24; x must have cores 1..n-1
 * right-orthonormal (cm_build_qtt and cm_tt_round leave them so). Contractions run in the
 * storage precision (x->dtype == y->dtype == w_by_n->dtype); the pivoted QR runs in FP64.
 * y: trains with y->n[b] == x->n[b], d_out = 2, d_in = 1; on return y->flags =
 * CM_TT_LEFT_ORTHO. status: device [batch].
 * Workspace: cm_workspace_bytes(CM_OP_SFFT_APPLY, batch, x->n_max, cap_rank, dtype). */
cm_status cm_sfft_apply(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank,
                        cm_tt_batch *y, int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cm_sfft_apply without a workspace
 * argument. The zip-up's per-workgroup slabs live in a fixed device array of
 * cm_sfft_apply_noalloc_scratch_bytes() = 256 MiB that the library holds on every device
 * it runs on until the process ends; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine). It runs min(batch, 256 MiB / slab) persistent workgroups,
 * with slab = cm_workspace_bytes(CM_OP_SFFT_APPLY, 1, n_max, cap_rank, dtype) (about
 * 2.5 MB at cap_rank 32, 7.4 MB at 64), so any batch size is accepted; a cap_rank whose
 * single slab exceeds the array returns CM_E_UNSUPPORTED. Arguments, results and status
 * codes are those of cm_sfft_apply, and the output equals its output bit for bit. Every
 * call on a device shares that device's array: calls that overlap on one device (on
 * different streams, or from different host threads) race and must be serialised by the
 * caller. The first call on a device looks up the array's address there (a one-time
 * hipGetSymbolAddress). */
cm_status cm_sfft_apply_noalloc(const cm_tt_batch *w_by_n, const cm_tt_batch *x, double tol, int cap_rank,
                                cm_tt_batch *y, int32_t *status, void *stream);

/* Size in bytes of the fixed device array cm_sfft_apply_noalloc uses. */
size_t cm_sfft_apply_noalloc_scratch_bytes(void);

/* TT rounding (Oseledets 2011; the recompression of Section 3.1) in place: a QR sweep
 * left to right, then truncated SVDs right to left with per-bond threshold
 * tol * ||t|| / sqrt(n-1), bonds <= cap_rank. Afterwards cores 1..n-1 are
 * right-orthonormal. If t->flags has CM_TT_LEFT_ORTHO the first sweep is skipped (the
 * cores are already left-orthonormal). All factorisations in FP64. err_out (device [batch], may be NULL)
 * receives the achieved relative Frobenius error bound. status: device [batch].
 * Workspace: cm_workspace_bytes(CM_OP_TT_ROUND, batch, t->n_max, cap_rank, t->dtype). */
cm_status cm_tt_round(cm_tt_batch *t, double tol, int cap_rank, double *err_out,
                      int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Prices from an SFFT output train (Eq. discretization_dft):
 *   C(k_u) = Re[ exp(-alpha k_u)/(s pi) * exp(-i v0 k_u) * sqrt(M) * y_u ]
 * with s = 2 (rectangle) or 1 (Simpson), where y_u is read from train b at the
 * bit-reversed index of u. strike_idx: device int64 [batch][nk] log-strike indices u in
 * [0, M); prices: device double [batch][nk]. status: device [batch] (may be NULL); an
 * index outside [0, M) yields NaN and CM_E_INVALID for that instance. */
cm_status cm_readout_prices(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx,
                            int nk, double *prices, int32_t *status, void *stream);

/* Observable read-out with exact probabilities (Section 2.2, Eqs. qft_probabilities and
 * qft_observable_price with p_hat = p): the QFT measurement gives p_u = |y_u|^2 / ||x||^2,
 * which loses the phase of y_u, so the price is
 *   C_hat(k_u) = exp(-alpha k_u)/(s pi) * sqrt(M) * |y_u|,
 * equal to |complex price| of cm_readout_prices. Arguments, layout and errors as for
 * cm_readout_prices. */
cm_status cm_readout_observable(const cm_tt_batch *y, const cm_problem *prob, const int64_t *strike_idx,
                                int nk, double *prices, int32_t *status, void *stream);

/* Emulated measurement of the QFT register (Section 2.2, Eq. qft_probabilities): R outcomes
 * per train b drawn from p_u = |y_u|^2 / ||y||^2 without forming the 2^n amplitudes, by
 * exact sequential conditional sampling from bit 0 (weight 1) upward: with the low t bits
 * fixed and q_0, q_1 the masses of the two continuations, bit t is 1 iff U_t (q_0 + q_1) >= q_0.
 * The masses come from right environments (Gram matrices of the partial contractions of
 * cores t+1..n-1) built in FP64; every decision is taken in FP64.
 * uniforms: device double [batch][y->n_max][R] in [0, 1), bit-major (the caller's random
 * numbers: U_t of shot s of train b at [b][t][s]; train b reads levels t < n[b]); out: device int64
 * [batch][R] outcome indices u in [0, 2^n[b]) (bit t of u is bit t of the outcome, the
 * log-strike index of cm_readout_prices); norm2: device double [batch] receives ||y_b||^2.
 * Bonds above 32 give CM_E_UNSUPPORTED for that instance, a zero train CM_E_INVALID, a
 * non-finite one CM_E_NONFINITE; such instances get out = -1. status: device [batch] (may
 * be NULL). R = 0 computes norm2 only.
 * Workspace: cm_workspace_bytes(CM_OP_SAMPLE, batch, y->n_max, y->cap_rank, y->dtype). */
cm_status cm_sample_outcomes(const cm_tt_batch *y, const double *uniforms, int R, int64_t *out,
                             double *norm2, int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Observable prices from R measured outcomes per instance (Eqs. qft_probability_estimator
 * and qft_observable_price): counts[b][i] = number of samples[b][:] equal to strike_idx[b][i],
 * p_hat = counts / R and
 *   C_hat(k_u) = exp(-alpha k_u)/(s pi) * sqrt(M) * sqrt(norm2[b] * p_hat_u).
 * prob: device [batch] (grid of each instance); norm2: device [batch] (||x||^2, e.g. from
 * cm_sample_outcomes); samples: device int64 [batch][R] (entries -1 are skipped, other
 * entries outside [0, M) set CM_E_INVALID); strike_idx: device int64 [batch][nk], strictly
 * increasing per row (a row that is not, or that leaves [0, M), gets NaN prices and
 * CM_E_INVALID); counts: device int32 [batch][nk] (written); prices: device double
 * [batch][nk]. R >= 1. status: device [batch] (may be NULL). */
cm_status cm_shot_prices(const cm_problem *prob, int batch, const double *norm2, const int64_t *samples, int R,
                         const int64_t *strike_idx, int nk, int32_t *counts, double *prices, int32_t *status,
                         void *stream);

/* Dense Carr–Madan baseline (Section 2.1): evaluates x (Eq. x) inside the first FFT pass,
 * applies the minus-sign DFT of Eq. dft with a Stockham FFT in the storage precision, and
 * applies the readout scalars of Eq. discretization_dft in the last pass. x_j is set to
 * exactly zero where |psi| lies below 1e-16 (CM_C64) or 1e-32 (CM_C128) times |psi(0)|, a
 * per-problem cut-off found once by scanning |psi| outward. Every problem must have
 * prob[b].n == n (n <= 30, batch <= 65535). If strike_idx is NULL, prices is [batch][M];
 * otherwise strike_idx is device int64 [batch][nk] and prices is [batch][nk] (gathered).
 * prices holds float for CM_C64 and double for CM_C128. status: device [batch] (may be
 * NULL); a problem that fails its checks gets its code there and NaN prices.
 * Workspace: cm_workspace_bytes(CM_OP_FFT_PRICE, batch, n, 0, dtype). Instances run in launch
 * groups whose pass buffers live in the workspace (one instance per group from n = 22 up,
 * 2^(22-n) below); a larger workspace widens the groups to the largest instance count whose
 * buffers fit (the results are the same). */
cm_status cm_fft_price(const cm_problem *prob, int batch, int n, int dtype, const int64_t *strike_idx,
                       int nk, void *prices, int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------ pricing surrogate
 * A project addition (the paper has no learned component): a multilayer perceptron
 * mapping (kappa, theta, sigma_v, rho, v0, T, k) -- the Heston parameters, the maturity and
 * the log-moneyness k = ln(K/S0) -- to C/S0, trained on SFFT prices by the kernels below
 * and gated so that queries outside its training domain go back to the SFFT path.
 *   xn = (x - shift) * scale;  a1 = silu(W1 xn + b1)  (7 -> 256);
 *   a_l = silu(W_l a_{l-1} + b_l) for l = 2, 3, 4 (256 -> 256);  y = W5 a4 + b5  (256 -> 1);
 *   silu(z) = z / (1 + e^-z).
 * The three 256 x 256 layers run on BF16 MFMA with FP32 accumulation: their weights are the
 * BF16 copies in w_bf16, and each activation operand is split into two BF16 parts
 * (hi + lo) so that its rounding stays near FP32; the 7 -> 256 and 256 -> 1 layers, the
 * loss, and Adam run in FP32.
 * Parameter vector (FP32, CM_MLP_NPARAMS values, row-major, output index first):
 *   W1 [256][7] @0, b1 [256] @1792, W2 [256][256] @2048, b2 @67584, W3 @67840, b3 @133376,
 *   W4 @133632, b4 @199168, W5 [1][256] @199424, b5 @199680. */
#define CM_MLP_NIN 7
#define CM_MLP_WIDTH 256
#define CM_MLP_NPARAMS 199681

typedef struct {
  float *params;       /* device [CM_MLP_NPARAMS] FP32 master parameters */
  uint16_t *w_bf16;    /* device [3][65536] BF16 bit patterns of W2, W3, W4 in MFMA fragment
                        * order: W_l[n][k] at (l - 2) 65536 + 8 (64 (16 (n / 32) + k / 16)
                        * + 32 ((k / 8) mod 2) + n mod 32) + k mod 8 (written by
                        * cm_mlp_sync_bf16 and cm_adam_step; callers only allocate it) */
  float shift[7];      /* host values: input normalisation xn = (x - shift) * scale */
  float scale[7];
} cm_mlp;

/* Bytes of saved pre-activations (Z1..Z4, FP32) that cm_mlp_forward writes for a batch of
 * B rows when asked to, and cm_mlp_backward reads. */
size_t cm_mlp_act_bytes(int B);

/* Refreshes net->w_bf16 from the FP32 master weights (round to nearest even). */
cm_status cm_mlp_sync_bf16(const cm_mlp *net, void *stream);

/* y[b] = network(x[b]) for b < B. x: device float [B][7] raw inputs; y: device float [B].
 * acts: device buffer of acts_bytes bytes. With acts_bytes >= cm_mlp_act_bytes(B) the
 * pre-activations Z1..Z4 are kept there for cm_mlp_backward (training: one launch per
 * layer). Otherwise (inference; acts may be NULL) one fused launch runs all five layers with
 * the activations kept on chip; its outputs equal the training path's to FP32 rounding (the
 * final 256-term sum is added in another order). */
cm_status cm_mlp_forward(const cm_mlp *net, const float *x, int B, float *y, float *acts, size_t acts_bytes,
                         void *stream);

/* grad = sum_b dy[b] * d y[b] / d params, overwriting grad (device float [CM_MLP_NPARAMS]).
 * acts: what cm_mlp_forward saved for the same x. ws: device workspace of
 * cm_mlp_act_bytes(B) / 2 bytes. Column sums over the batch use float atomics, so the
 * summation order (and the last bits) may vary between runs. */
cm_status cm_mlp_backward(const cm_mlp *net, const float *x, const float *acts, const float *dy, int B, float *grad,
                          void *ws, size_t ws_bytes, void *stream);

/* Mean squared error: dy[b] = 2 (y[b] - t[b]) / B and *loss += mean((y - t)^2) (device
 * scalar, accumulated with float atomics; the caller zeroes it). */
cm_status cm_mlp_mse(const float *y, const float *t, int B, float *dy, float *loss, void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected) on every parameter: m, v are device
 * float [CM_MLP_NPARAMS] moment buffers (zero before step 1), step >= 1. Also refreshes
 * w_bf16. */
cm_status cm_adam_step(const cm_mlp *net, const float *grad, float *m, float *v, int step, float lr, float beta1,
                       float beta2, float eps, void *stream);

/* Surrogate decode and gate. The network output z[b] decodes to the price
 * y[b] = C/S0 = e^{z[b]} - out_eps when out_eps > 0 (a network trained on log(C/S0 + out_eps))
 * and y[b] = z[b] when out_eps == 0; y goes to price (device float [B], may be NULL).
 * accept[b] = 1 iff all of:
 *   - every raw input x[b][i] lies in [lo[i], hi[i]] (host arrays of 7: the trusted box);
 *   - y[b] violates the static no-arbitrage bounds max(0, 1 - e^{k - r T}) <= C/S0 <= 1 by at
 *     most res_tol;
 *   - if cell_err is not NULL: the calibrated error of the query's cell is at most err_tol.
 *     cell_err is a device float [nT][nk] table over the box's (T, k) rectangle (cell
 *     iT = floor((T - lo[5]) / (hi[5] - lo[5]) nT), ik likewise from k = x[b][6], clamped to
 *     the grid), holding the largest |network - SFFT| / S0 the caller measured on validation
 *     queries in that cell; NULL skips this check.
 * Otherwise accept[b] = 0 (the caller prices those queries with the SFFT path). */
cm_status cm_surrogate_gate(const float *x, const float *z, int B, const float *lo, const float *hi, float r,
                            float res_tol, float out_eps, const float *cell_err, int nT, int nk, float err_tol,
                            float *price, int32_t *accept, void *stream);

/* Short English text for a status code (static storage). */
const char *cm_status_str(cm_status s);

/* Library version string (static storage). */
const char *cm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CM_H */
