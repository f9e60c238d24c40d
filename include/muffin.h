/*
 * muffin.h - C ABI of the MI355X (gfx950) MUFFIN primal-dual reconstruction library.
 *
 * MUFFIN recovers a sky cube X = [x_1 ... x_L] (L channels of N x N pixels) from dirty images
 * y_l = H_l x_l + n_l, where H_l is convolution by the PSF of channel l (Sec. 2, eq. (model)),
 * by minimising (eq. (reg) with the prior of eq. (RegAll))
 *
 *   sum_l w_l/2 ||y_l - H_l x_l||^2 + 1_{R+}(X) + mu_s sum_l ||W_s x_l||_1 + mu_lambda sum_n ||W_lambda x^n||_1
 *
 * with W_s the isotropic undecimated wavelet transform (IUWT, B3-spline a trous, periodic) and
 * W_lambda the orthonormal cosine transform (DCT-II) of each pixel spectrum, through the
 * primal-dual iteration of Algorithm 1 (Sec. 3).
 *
 * Conventions shared by every entry point:
 *  - Every function returns MUFFIN_OK (0) or a negative MUFFIN_E* code; none aborts or throws.
 *    muffin_last_error() gives a message for the last failure on the calling thread.
 *  - Arrays are FP32, C-contiguous, channel-major:
 *      cube    [L][N][N]           (X, dirty image, PSF, V, gradients)
 *      U       [L][J+1][N][N]      (planes w_1..w_J, then the coarse plane c_J, of each channel;
 *                                   with the union-of-bases prior [L][8][N][N], one plane per basis)
 *    V holds the cosine coefficients of each pixel spectrum, coefficient index first.
 *  - "on_device" arguments: nonzero means the pointer is device memory on the context's device,
 *    zero means host memory.  The library never takes ownership of caller memory: it copies
 *    what it needs into its own buffers.
 *  - A context is bound to one HIP stream given at creation (NULL = the null stream).  Work is
 *    enqueued on a private stream of the library that is ordered after all prior work of the
 *    caller's stream; the caller's stream is made to wait for the library's work before each call
 *    returns, so device outputs are safe to use on the caller's stream.  Calls returning host
 *    values (objective, get_* to host) synchronise.  A context is not thread-safe; distinct
 *    contexts are independent.
 */
#ifndef MUFFIN_H
#define MUFFIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MUFFIN_OK 0
#define MUFFIN_EINVAL (-1)     /* bad argument: size, pointer, parameter out of range */
#define MUFFIN_ENOMEM (-2)     /* device or host allocation failed */
#define MUFFIN_EHIP (-3)       /* a HIP runtime call failed */
#define MUFFIN_ENONFINITE (-4) /* NaN or Inf in an input, or the objective became non-finite */
#define MUFFIN_ESTEP (-5)      /* (tau, sigma, rho) violate the convergence condition */
#define MUFFIN_ESTATE (-6)     /* checkpoint blob does not match the context */

typedef struct muffin_ctx muffin_ctx;

/* Run the IUWT one launch per scale instead of fusing two or three consecutive scales into one
 * launch (the results are the same bit for bit; the fused form moves fewer bytes). */
#define MUFFIN_FLAG_SINGLE_SCALE 1
/* Fused tail (second generation, coarse plane penalised, last scale group a pair): each
 * iteration's analysis ends with one launch that also runs the next iteration's first two adjoint
 * steps over the planes it has just updated.  It moves 12 bytes per voxel fewer, gives the same
 * results bit for bit, and keeps a second copy of three dual planes in memory; but it needs large
 * bands to pay for its longer halo.  By default it is used when the channels alone fill the GPU
 * (L at least the number of compute units) with at least 64 rows per residue class, and
 * muffin_autotune keeps whichever of the fused and the separate launches it measures faster.
 * NO_FUSED_TAIL always runs the two launches separately, FUSED_TAIL always fuses them. */
#define MUFFIN_FLAG_NO_FUSED_TAIL 2
#define MUFFIN_FLAG_FUSED_TAIL 4
/* Union-of-bases prior: on the levels after the first, one workgroup per (tile, channel) runs all
 * eight bases (loading the next basis's input while it filters the current one) when the level has
 * enough tiles and channels to fill the GPU that way, else one workgroup per basis.  UOB_ALL_BASES
 * and UOB_PER_BASIS force either form on every level; the results are the same bit for bit (the
 * objective's FP64 partial sums aside, which are grouped by workgroup). */
#define MUFFIN_FLAG_UOB_ALL_BASES 8
#define MUFFIN_FLAG_UOB_PER_BASIS 16
/* Channel counts L without a radix-2/3 FFT plan (16 < L <= 512): the two cosine transforms of the
 * spectral step (Sec. 2) run either as dense products with a cosine table, or through L-point DFTs
 * in Bluestein's form (a chirp convolution through FFTs of a length M >= 2L - 1 that has a plan).
 * Both agree to FP32 rounding.  By default each L takes the form measured faster (Bluestein for
 * 110 <= L <= 128 and L >= 216); SPECTRAL_DENSE and SPECTRAL_BLUESTEIN force one form. */
#define MUFFIN_FLAG_SPECTRAL_DENSE 32
#define MUFFIN_FLAG_SPECTRAL_BLUESTEIN 64

/* Spatial prior W_s (eq. (RegAll)): the isotropic undecimated wavelet transform MUFFIN uses (Sec. 3,
 * Sec. 4), or the union of the first eight orthonormal Daubechies wavelet bases it is compared with
 * (Sec. 3, Sec. 4 Fig. 3): W_s x = (Psi_1 x, ..., Psi_8 x) / sqrt(8), Psi_n the J-level periodic 2-D
 * DWT with n vanishing moments, each basis's coefficients in the pyramid layout of an N x N plane
 * (after level l the approximation is the top-left (N/2^l)^2 block, the level's horizontal,
 * vertical and diagonal details to its right, below it and diagonally).  With the union of bases,
 * U holds 8 planes per channel, iuwt_gen and penalize_coarse are ignored (every coefficient is
 * penalised), ||W_s||^2 = 1, and N must be divisible by 2^J. */
#define MUFFIN_PRIOR_IUWT 0
#define MUFFIN_PRIOR_UOB 1

/* Problem and algorithm parameters (Sec. 2 eqs. (reg), (RegAll); Sec. 3, Algorithm 1). */
typedef struct {
  int32_t N;                /* image side; N = 2^a or 3 * 2^a with 8 <= N <= 1024 */
  int32_t L;                /* channels, 1 <= L <= 512 */
  int32_t J;                /* wavelet scales, 1 <= J <= 6; the IUWT yields J+1 planes */
  int32_t iuwt_gen;         /* 1 or 2: first or second generation IUWT (the paper uses 2, Sec. 4) */
  int32_t penalize_coarse;  /* 1: the coarse plane is part of W_s's l1 term; 0: it is not */
  int32_t flags;            /* MUFFIN_FLAG_* bits, 0 by default */
  int32_t prior;            /* MUFFIN_PRIOR_IUWT (0, default) or MUFFIN_PRIOR_UOB */
  double mu_s;              /* spatial weight mu_s >= 0 (eq. (RegAll)) */
  double mu_lambda;         /* spectral weight mu_lambda >= 0 (eq. (RegAll)) */
  double tau;               /* primal step; <= 0 selects 0.99 / (beta/2 + sigma ||K||^2) */
  double sigma;             /* dual step > 0 */
  double rho;               /* relaxation, 0 < rho < delta (see muffin_info) */
  const float* chan_weight; /* host [L] weights w_l = 1/sigma_l^2 (eq. (reg)), or NULL for all 1 */
} muffin_params;

/* Create a context: copy the dirty cube y [L][N][N] and the PSF cube [L][N][N] (origin of each PSF
 * at pixel (N/2, N/2)), precompute the transfer functions H_l, b_l = w_l H_l^dagger y_l, the
 * Lipschitz constant beta = max_l w_l ||H_l||^2 and ||K||^2 = mu_s^2 ||W_s||^2 + mu_lambda^2 (FP64),
 * choose tau if needed, and initialise X = U = V = 0 (Algorithm 1, "Initialize").
 * Errors: EINVAL (sizes, NULL pointers, parameters), ENONFINITE (NaN/Inf in dirty or psf),
 * ESTEP (convergence condition violated), ENOMEM, EHIP.  *out is NULL on error. */
int muffin_init(muffin_ctx** out, const muffin_params* p, const float* dirty, const float* psf,
                int inputs_on_device, void* hip_stream);

/* ---------------------------------------------------------------------------------------------
 * Visibility-domain data term (Sec. 2, eq. (viseq)): instead of dirty images and PSFs, the context
 * holds K complex visibilities per channel and minimises
 *
 *   sum_l w_l/2 ||v_l - Phi_l x_l||^2 + 1_{R+}(X) + mu_s sum_l ||W_s x_l||_1 + mu_lambda sum_n ||W_lambda x^n||_1
 *
 * with (Phi_l x)_k = sum over pixels (i, j) of x_ij / n_ij exp(-2 pi i (u_k l_j + v_k m_i + w_k n_ij) / lambda_l):
 * l_j = (j - N/2) cell, m_i = (i - N/2) cell, n_ij = sqrt(1 - l_j^2 - m_i^2); the w n term is the
 * direction-dependent effect that the image-plane model leaves out.  Phi is evaluated exactly (a
 * direct sum over every visibility and pixel, FP64 phases, FP32 products and sums), so a step costs
 * about 2 L K N^2 complex exponentials.  w_l are the channel weights of eq. (reg) (chan_weight, 1 by
 * default).  The gradient of the data term is w_l Re Phi_l^H (Phi_l x_l - v_l); beta is 1.01 times a
 * power-iteration estimate (FP64 norms, power_iters steps from the all-ones cube) of the largest
 * eigenvalue of w_l Re Phi_l^H Phi_l over all channels.  The rest of Algorithm 1 (both priors, the
 * spectral term, relaxation, muffin_step / solve / objective / state calls, the autotuner) is
 * unchanged; out[1] of muffin_objective is sum_l w_l/2 ||v_l - Phi_l x_l||^2.  Not available with
 * visibilities: the warm start, MUFFIN_OP_H / HT, batches.
 * --------------------------------------------------------------------------------------------- */
typedef struct {
  int32_t K;            /* visibilities (baselines) per channel, 1 <= K <= 2^22 */
  double cell;          /* pixel size in direction cosines; every pixel needs l^2 + m^2 < 1 */
  const double* uvw;    /* host [K][3]: baseline (u, v, w) in metres, the same for every channel */
  const double* lambda; /* host [L]: wavelength of each channel in metres (> 0) */
  int32_t power_iters;  /* power iterations for beta, 0 for the default 40 */
} muffin_vis_desc;

/* Create a context with the visibility data term: p as for muffin_init (N a multiple of 8), vis
 * [L][K] complex as interleaved FP32 (re, im) on the host or the device.
 * Initialises X = U = V = 0 (Algorithm 1, "Initialize").  Errors: EINVAL (sizes, NULL pointers,
 * parameters, a pixel outside the unit disc), ENONFINITE (NaN/Inf in uvw or vis, or a power
 * iteration that breaks down), ESTEP, ENOMEM, EHIP.  *out is NULL on error. */
int muffin_init_vis(muffin_ctx** out, const muffin_params* p, const muffin_vis_desc* desc, const float* vis,
                    int vis_on_device, void* hip_stream);
/* Residual Phi_l x_l - v_l of the current X for every channel (not weighted), [L][K] complex as
 * interleaved FP32, into host or device memory (device output is written in place on the
 * context's stream; host output is staged through a device buffer of L K complex values that the
 * context allocates on its first such call and keeps).  EINVAL for an image-plane context. */
int muffin_vis_residual(muffin_ctx* ctx, float* r, int on_device);

/* Run n_iter >= 0 iterations of Algorithm 1 (gradient, primal proximal step, spatial and spectral
 * dual steps, relaxation).  Iterations after the first call replay a captured HIP graph. */
int muffin_step(muffin_ctx* ctx, int32_t n_iter);

/* Stopping rules of muffin_solve (Algorithm 1 ends "until stopping criterion" without naming one). */
#define MUFFIN_STOP_OBJECTIVE 0 /* objective f: gap to f_ref, or relative change between checks */
#define MUFFIN_STOP_CHANGE 1    /* iterates: relative change of X, U and V over one iteration */

/* Iterate until a stopping rule holds (Algorithm 1, "until stopping criterion"), in windows of
 * check_every iterations (the last window may be shorter), at most max_iter iterations.
 *  - MUFFIN_STOP_OBJECTIVE: after each window the objective f (eq. (reg) + eq. (RegAll)) is
 *    evaluated; with f_ref finite the run stops at the first window where (f - f_ref)/|f_ref| <= tol,
 *    otherwise where |f - f_prev| <= tol |f| against the previous window's f.
 *  - MUFFIN_STOP_CHANGE: the last iteration of each window is monitored as by muffin_step_monitored;
 *    the run stops at the first window where max(||dX||/||X||, ||dU||/||U||, ||dV||/||V||) <= tol
 *    (a ratio with a zero change counts as 0); f_ref is ignored and f is evaluated once, at the end.
 * iters_done and f_final (the objective at the end; may be NULL) report where it stopped.
 * Errors: EINVAL (arguments, unknown rule), ENONFINITE if f or the iterates become non-finite
 * (iters_done and f_final still report the state). */
int muffin_solve(muffin_ctx* ctx, int32_t max_iter, int32_t check_every, int32_t rule, double tol, double f_ref,
                 int32_t* iters_done, double* f_final);

/* n_iter >= 1 iterations (Algorithm 1) whose last one is monitored: out receives, in FP64,
 * {||X_k - X_{k-1}||_2, ||X_k||_2, ||U_k - U_{k-1}||_2, ||U_k||_2, ||V_k - V_{k-1}||_2, ||V_k||_2} over the
 * whole cube, the convergence norms of the primal and both dual variables (Sec. 3; a fixed point of
 * the iteration has all three changes zero).  The first call allocates device copies of X, U and V
 * (8 + 4(J+1) bytes per voxel) that the context keeps; the monitored iteration is not part of the
 * captured graph's timing. */
int muffin_step_monitored(muffin_ctx* ctx, int32_t n_iter, double out[6]);

/* Reconstruction SNR of Sec. 4 against a sky truth X* [L][N][N] (host or device):
 * 10 log10(||X*||^2 / ||X - X*||^2) over the cube, sums in FP64 (+inf if X equals X*).  The truth
 * is copied into a scratch buffer of the context; the state is unchanged. */
int muffin_snr(muffin_ctx* ctx, const float* truth, int on_device, double* snr_db);

/* Objective of eq. (reg) + eq. (RegAll) at the current X, reduced in FP64:
 * out[0] total, out[1] data term sum_l w_l/2 ||y_l - H_l x_l||^2, out[2] mu_s-weighted spatial l1,
 * out[3] mu_lambda-weighted spectral l1.  Synchronises. */
int muffin_objective(muffin_ctx* ctx, double out[4]);

/* Scalars of the context (Sec. 3: the step sizes are fixed by the convergence condition of the
 * primal-dual method it cites): out[0] tau, [1] sigma, [2] rho, [3] beta (Lipschitz constant of the
 * data term's gradient), [4] ||K||^2, [5] ||W_s||^2, [6] delta (rho must lie in (0, delta)),
 * [7] iterations done.  Host values, no device work. */
int muffin_info(muffin_ctx* ctx, double out[8]);

/* Initial point (Algorithm 1, "Initialize"; Sec. 4, calibration step 2 starts the full method from
 * step 1's X): X = max(x0, 0), which keeps X inside the positivity constraint, and U = V = 0.
 * x0 is [L][N][N] on the host or the device; the caller keeps it. */
int muffin_set_x(muffin_ctx* ctx, const float* x0, int on_device);
/* Copy out the primal variable X [L][N][N] and the dual variables U (one decomposition per channel,
 * eq. (anaylsespat): [L][J+1][N][N] for the IUWT, [L][8][N][N] for the union of bases) and V [L][N][N]
 * (cosine coefficients of each pixel spectrum) of Algorithm 1, into caller memory (host or device). */
int muffin_get_x(muffin_ctx* ctx, float* x, int on_device);
int muffin_get_u(muffin_ctx* ctx, float* u, int on_device);
int muffin_get_v(muffin_ctx* ctx, float* v, int on_device);

/* Checkpoint of the state (X, U, V) of Algorithm 1, so that a run (e.g. a calibration of Sec. 4
 * spread over several jobs) can stop and resume: a host blob holding a header (sizes, parameters,
 * iteration count) and X, U, V.  muffin_state_size gives its size in bytes; get_state needs a
 * caller buffer of at least that size (EINVAL otherwise).  muffin_set_state rejects a blob written
 * by a context of other sizes or parameters with ESTATE.  Restoring and continuing reproduces an
 * uninterrupted run bit for bit. */
int muffin_state_size(muffin_ctx* ctx, size_t* bytes);
int muffin_get_state(muffin_ctx* ctx, void* blob, size_t bytes);
int muffin_set_state(muffin_ctx* ctx, const void* blob, size_t bytes);

/* Single operators on device arrays, for per-operator parity checks.  in/out are device
 * pointers on the context's device with the sizes given per operator:
 *   MUFFIN_OP_H        cube -> cube       H_l x_l (Sec. 2, eq. (model))
 *   MUFFIN_OP_HT       cube -> cube       H_l^dagger y_l
 *   MUFFIN_OP_GRAD     cube -> cube       w_l H_l^dagger (H_l x_l - y_l) (Algorithm 1, eq. (grad))
 *   MUFFIN_OP_IUWT     cube -> U          W_s x_l per channel
 *   MUFFIN_OP_IUWT_ADJ U -> cube          W_s^dagger u_l per channel (eq. (adjointspat) without mu_s)
 *   MUFFIN_OP_DCT      cube -> cube       X W_lambda (cosine coefficients of each pixel spectrum)
 *   MUFFIN_OP_IDCT     cube -> cube       V W_lambda^dagger
 *   MUFFIN_OP_IUWT_SCHED cube -> U        W_s x_l per channel through the iteration's own analysis
 *                                         launches (the scale groups of the spatial dual step, the
 *                                         fused tail when the context uses it) applied to zero dual
 *                                         planes with sigma mu_s = rho = 1 (eq. (anaylsespat)): valid
 *                                         where every |W_s x| <= 1, since the dual step saturates;
 *                                         the coarse plane only when it is penalised (else 0)
 *   MUFFIN_OP_PHI      cube -> [L][K] complex (interleaved FP32)   Phi_l x_l (Sec. 2, eq. (viseq))
 *   MUFFIN_OP_PHI_ADJ  [L][K] complex -> cube                     Re Phi_l^H r_l
 * With visibilities, MUFFIN_OP_GRAD is w_l Re Phi_l^H (Phi_l x_l - v_l); the PHI operators need a
 * visibility context and H / HT an image-plane one (EINVAL otherwise).
 * The context's state is not changed.  EINVAL for an unknown op. */
#define MUFFIN_OP_H 1
#define MUFFIN_OP_HT 2
#define MUFFIN_OP_GRAD 3
#define MUFFIN_OP_IUWT 4
#define MUFFIN_OP_IUWT_ADJ 5
#define MUFFIN_OP_DCT 6
#define MUFFIN_OP_IDCT 7
#define MUFFIN_OP_IUWT_SCHED 8
#define MUFFIN_OP_PHI 9
#define MUFFIN_OP_PHI_ADJ 10
int muffin_apply_op(muffin_ctx* ctx, int op, const float* in, float* out);

/* Measurement, not part of the paper's method: time n_iter iterations of Algorithm 1 with HIP
 * events on the library's stream, without graph replay, and report average device milliseconds:
 *   ms[0] whole iteration, [1] spatial adjoint (IUWT^dagger), [2] gradient (FFT passes, or the
 *   visibility kernels),
 *   [3] fused spectral kernel, [4] spatial analysis and dual update; [5..7] are 0;
 *   ms[8 + 2k] mean duration of one launch of kind k and ms[9 + 2k] launches of kind k per
 *   iteration, for the second-generation band kernels: k = 0 one analysis scale with its dual
 *   step, 1 one adjoint Horner step, 2 the last analysis scale with the coarse plane's dual step,
 *   3 two analysis scales in one launch, 4 two adjoint steps in one launch, 5 the last two
 *   analysis scales with the coarse plane's dual step, 6 three analysis scales in one launch,
 *   7 three adjoint steps in one launch, 8 the last three analysis scales with the coarse plane's
 *   dual step, 9 the last two analysis scales with the coarse plane's dual step fused with the
 *   next iteration's first two adjoint steps (which then leave the adjoint phase); k = 10, 11
 *   are 0, and so is every kind of a first-generation context.
 * Each kernel family (adjoint, analysis) is bracketed in every other iteration, so n_iter >= 2.
 * The iterations advance the state like muffin_step. */
int muffin_profile(muffin_ctx* ctx, int32_t n_iter, double ms[32]);

/* Measurement, not part of the paper's method: time n_iter iterations of Algorithm 1 (graph
 * replay) with HIP events on the library's stream: *ms is the total device time.  Advances the
 * state like muffin_step. */
int muffin_step_timed(muffin_ctx* ctx, int32_t n_iter, double* ms);

/* ---------------------------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method): a CNN that maps a dirty channel image,
 * normalised by its PSF's main-lobe gain, to an estimate of the reconstructed image; the primal-dual
 * iteration refines from max(estimate, 0).  Four 3x3 convolutions 1 -> 32 -> 32 -> 32 -> 1 with
 * circular padding, bias, ReLU after the first three; BF16 weights and activations (rounded to
 * nearest even), FP32 accumulation; MSE loss and Adam (beta 0.9 / 0.999, eps 1e-8) on FP32 master
 * weights.  Parameters are one FP32 vector in the order w1[32][1][3][3], b1[32], w2[32][32][3][3],
 * b2[32], w3[32][32][3][3], b3[32], w4[1][32][3][3], b4[1] (19105 values); tap [a][e] reads the
 * input at offset (a - 1, e - 1).  Image batches are device FP32 arrays [B][N][N] with N a multiple
 * of 32.  A network object is bound to a HIP stream like a context and is not thread-safe.
 * --------------------------------------------------------------------------------------------- */
typedef struct muffin_cnn muffin_cnn;
/* Create with He-normal weights drawn from a counter-based generator seeded by seed; features
 * must be 32. */
int muffin_cnn_create(muffin_cnn** out, int32_t features, uint64_t seed, void* hip_stream);
/* Number of FP32 parameters of the network (19105). */
int muffin_cnn_param_count(muffin_cnn* net, int32_t* n);
/* Copy the FP32 parameter vector to or from host memory (n must equal the count); set_params
 * also resets the Adam moments. */
int muffin_cnn_get_params(muffin_cnn* net, float* params, int32_t n);
int muffin_cnn_set_params(muffin_cnn* net, const float* params, int32_t n);
/* out = network output (before the positive-part projection) for B images. */
int muffin_cnn_predict(muffin_cnn* net, const float* in, float* out, int32_t B, int32_t N);
/* Mean squared error against target and its gradient (host [count], may be NULL), no update. */
int muffin_cnn_loss_grad(muffin_cnn* net, const float* in, const float* target, int32_t B, int32_t N,
                         double* loss, float* grad);
/* One Adam step of learning rate lr on the mean squared error; *loss (may be NULL) is the loss
 * before the step. */
int muffin_cnn_train_step(muffin_cnn* net, const float* in, const float* target, int32_t B, int32_t N,
                          float lr, double* loss);
/* Single layer (1..4), for parity checks.  x: device FP32 [B][Cin][N][N], rounded to BF16 inside.
 * op 0: out = pre-activation z [B][Cout][N][N] (bias added).  op 1: given dz [B][Cout][N][N]
 * (rounded to BF16 inside), out = input gradient [B][Cin][N][N] without activation mask (zeros
 * for layer 1) and dparams (host) = weight then bias gradients of the layer. */
int muffin_cnn_layer(muffin_cnn* net, int32_t layer, int32_t op, const float* x, const float* dz,
                     float* out, float* dparams, int32_t B, int32_t N);
/* Allocation-free inference, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same network output
 * as muffin_cnn_predict, bit for bit, computed with a workspace the library holds in a static
 * device array (two BF16 activation planes of 2^20 pixels x 32 features, 128 MiB per GPU, kept
 * until the process ends) instead of workspaces allocated on first use.  in and out are device
 * arrays [B][N][N]; planes are processed in chunks of floor(2^20 / N^2), so N^2 <= 2^20 (N <= 1024,
 * N a multiple of 32), else EINVAL.  The call allocates nothing and launches no memset.  Every call
 * on one GPU shares that GPU's workspace: calls that overlap in time on one GPU (two networks, two
 * streams, two threads) race and must be ordered by the caller. */
int muffin_cnn_predict_noalloc(muffin_cnn* net, const float* in, float* out, int32_t B, int32_t N);
/* Release a network and its device buffers (NULL is accepted). */
void muffin_cnn_free(muffin_cnn* net);
/* Warm start: X = max(CNN(y_l / g_l), 0) channel by channel, U = V = 0, where g_l is the sum of
 * psf_l over the 9 x 9 window centred on its origin.  N must be a multiple of 32.  The network's
 * stream is ordered after the context's and the context's after the network's, without host
 * synchronisation. */
int muffin_warm_start(muffin_ctx* ctx, muffin_cnn* net);
/* The network input the warm start builds, y_l / g_l as above, written to out [L][N][N] (host or
 * device), so that a caller can train on or check exactly what muffin_warm_start feeds the network. */
int muffin_warm_input(muffin_ctx* ctx, float* out, int on_device);

/* Release a context and every device buffer it owns (NULL is accepted); waits for its stream. */
void muffin_free(muffin_ctx* ctx);

/* Launch tuning, not part of the paper's method.  Autotuner: times every band height (rows per
 * workgroup) of the IUWT band kernels with every split of a band's residue classes mod 2^j over
 * 1, 2, 4 or 8 workgroups ("class groups", up to 2^j), for each scale of this context's sizes,
 * keeps the fastest (process-wide, per image side, scale and kernel family) and recaptures the
 * iteration.  Only scratch planes are written: the state is unchanged.  report (may be NULL)
 * receives a JSON description of the candidates ("rows x groups") and choices (each with its
 * kernel family, rows and class groups), truncated to report_len.  None of these choices changes
 * a result bit. */
int muffin_autotune(muffin_ctx* ctx, int32_t reps, char* report, size_t report_len);

/* Kernel families of the IUWT launches, as the autotuner's report names them. */
#define MUFFIN_FAMILY_ANALYSIS 0          /* one scale, second generation: analysis + dual step */
#define MUFFIN_FAMILY_ADJOINT 1           /* one scale, second generation: adjoint Horner step */
#define MUFFIN_FAMILY_ANALYSIS_G1 2       /* one scale, first generation: analysis + dual step */
#define MUFFIN_FAMILY_ADJOINT_G1 3        /* one scale, first generation: adjoint step */
#define MUFFIN_FAMILY_PAIR_ANALYSIS 5     /* two scales: analysis + dual steps */
#define MUFFIN_FAMILY_PAIR_ADJOINT 6      /* two adjoint Horner steps */
#define MUFFIN_FAMILY_TRIPLE_ANALYSIS 7   /* three scales: analysis + dual steps */
#define MUFFIN_FAMILY_TRIPLE_ADJOINT 8    /* three adjoint Horner steps */
#define MUFFIN_FAMILY_FUSED_PAIR 9        /* last analysis pair + next iteration's first adjoint pair */
#define MUFFIN_FAMILY_PAIR_ANALYSIS_G1 10 /* first generation: two scales of analysis */
#define MUFFIN_FAMILY_PAIR_ADJOINT_G1 11  /* first generation: two adjoint steps */

/* Launch tuning: record band rows (0: back to the default) and class groups (0 or 1: one
 * workgroup per band) for the launches of image side N at scale j of one family, as the autotuner
 * would, e.g. to restore an earlier report's choices without timing again.  rows must divide N;
 * class_groups must be a power of two up to min(2^j, 8).  Process-wide; applies to iterations
 * captured afterwards (a context captures its iteration on its first step after creation or after
 * muffin_autotune).  EINVAL for a value out of range. */
int muffin_set_band_tiles(int32_t N, int32_t j, int32_t family, int32_t rows, int32_t class_groups);

/* ---------------------------------------------------------------------------------------------
 * Batches of independent cubes of uneven sizes (not part of the paper's method).  Cubes that share
 * N, J, generation, coarse weighting, mu_s, sigma and rho form one group: the per-channel phases
 * run once over the packed channels of all cubes of a group, the per-pixel spectral step and the
 * objective per cube (with the cube's own L, mu_lambda and tau).  Each group replays a captured
 * graph on its own stream; groups run concurrently.  p, dirty and psf are arrays of n_cubes entries;
 * every cube must pass muffin_init's checks.  Cube indices follow the input order.
 * --------------------------------------------------------------------------------------------- */
typedef struct muffin_batch muffin_batch;
int muffin_batch_init(muffin_batch** out, int32_t n_cubes, const muffin_params* p, const float* const* dirty,
                      const float* const* psf, int inputs_on_device, void* hip_stream);
/* n_iter iterations of Algorithm 1 for every cube of the batch (graph replay, groups concurrent). */
int muffin_batch_step(muffin_batch* batch, int32_t n_iter);
/* n_iter iterations of every cube; *ms is the device time between two events of the caller's stream. */
int muffin_batch_step_timed(muffin_batch* batch, int32_t n_iter, double* ms);
/* Per cube, as muffin_objective (eq. (reg) + eq. (RegAll)) and muffin_get_x. */
int muffin_batch_objective(muffin_batch* batch, int32_t cube, double out[4]);
int muffin_batch_get_x(muffin_batch* batch, int32_t cube, float* x, int on_device);
/* Initial point of one cube of the batch (Algorithm 1, "Initialize"), as muffin_set_x: its X becomes
 * max(x0, 0) and its U and V zero; the other cubes are unchanged. */
int muffin_batch_set_x(muffin_batch* batch, int32_t cube, const float* x0, int on_device);
/* The warm start's network input of one cube of the batch [L][N][N], as muffin_warm_input. */
int muffin_batch_warm_input(muffin_batch* batch, int32_t cube, float* out, int on_device);
/* SNR of one cube of the batch against its truth [L][N][N], as muffin_snr. */
int muffin_batch_snr(muffin_batch* batch, int32_t cube, const float* truth, int on_device, double* snr_db);
/* Per cube, as muffin_info; the autotuner over every group, as muffin_autotune; release. */
int muffin_batch_info(muffin_batch* batch, int32_t cube, double out[8]);
int muffin_batch_autotune(muffin_batch* batch, int32_t reps, char* report, size_t report_len);
void muffin_batch_free(muffin_batch* batch);

/* The scaling filter of Daubechies' orthonormal wavelet with n vanishing moments (1 <= n <= 8; 2n
 * taps into h[0..2n), len >= 2n) as the library builds it for the union-of-bases prior, in FP64
 * (host only: Daubechies' spectral factorisation, minimum phase, largest taps first).  EINVAL for
 * other n or a short buffer. */
int muffin_uob_filter(int32_t n, double* h, int32_t len);

/* Checked builds (test infrastructure, not part of the paper's method): in a library built with
 * MF_CHECKED every instrumented kernel index outside its bound is counted, and replaced by an index
 * in bounds so that the kernel completes.  *count = the number caught since the last call, then
 * zero.  The normal build returns EINVAL (count 0). */
int muffin_debug_oob(uint64_t* count);

/* Error reporting: a fixed text for each MUFFIN_E* code, and the message of the last failure on the
 * calling thread (valid until the next failing call on that thread). */
const char* muffin_strerror(int code);
const char* muffin_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MUFFIN_H */
