/*
 * adjwave.h - C ABI of the MI355X (gfx950) library for the deblurring operator
 * A = R W, its adjoint A^* = W^* R^*, one FISTA iteration on eq. (1), and the
 * blind-channel convolution adjoint pair.
 *
 * Paper: J. Folberth and S. Becker, "Efficient Adjoint Computation for Wavelet
 * and Convolution Operators", IEEE Signal Processing Magazine, Lecture Notes,
 * 2016.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory   Every data pointer is a DEVICE pointer owned by the caller. The
 *          library never allocates device memory in these calls: buffers for
 *          intermediates come from the caller as a workspace whose size
 *          aw_workspace_size() reports. Descriptor structs are host memory,
 *          read during the call only.
 * Streams  Work is enqueued on `stream` (a hipStream_t passed as void*; NULL
 *          means the default stream). No call synchronises the device; the
 *          caller orders reads of outputs after the stream.
 * Layout   Images are row-major [batch][rows][cols]. Coefficient vectors are
 *          [batch][ncoef] with subbands a_J, H_J, V_J, D_J, H_{J-1}, ...,
 *          D_1, each row-major (K^r_j x K^c_j). H = high-pass along rows and
 *          low-pass along columns, V = low-pass along rows and high-pass along
 *          columns, D = high-pass along both.
 * dtype    AW_F32 or AW_F64, for every floating-point buffer of a call.
 * Errors   A negative aw_status. Arguments are validated on the host before
 *          anything is enqueued; on error nothing is launched and
 *          aw_last_error() returns a message (thread-local). AW_EHIP reports a
 *          HIP launch error; its message carries the HIP error string.
 * Threads  Entry points are thread-safe; calls that share a workspace or an
 *          output buffer must be ordered by the caller.
 */
#ifndef ADJWAVE_H
#define ADJWAVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AW_OK = 0,
  AW_EINVAL = -1,        /* invalid argument (NULL, size, filter, radius ...) */
  AW_EUNSUPPORTED = -2,  /* valid request that this build does not implement */
  AW_EHIP = -3           /* HIP runtime / launch failure                     */
} aw_status;

typedef enum { AW_F32 = 0, AW_F64 = 1 } aw_dtype;

/* Boundary handling of the wavelet transform (Sec. "A few signal extensions").
 *  AW_BC_ZPD     zero boundary: the zero-boundary core alone (no explicit
 *                extension); K = floor((N + L - 1)/2) per band.
 *  AW_BC_SYM     half-point symmetric extension by L' = L - 1 on each side,
 *                fold weights 1/mult (the paper's (E_sym^dagger)^*);
 *                K = floor((N + 3L - 3)/2).
 *  AW_BC_PER     critically sampled circular transform (square, orthogonal):
 *                c[k] = sum_q f[q] y[(2k+q) mod N], K = N/2; every level's
 *                length must be even.
 *  AW_BC_PER_EXT periodic extension by L' with fold weights 1/mult (the
 *                paper's E_per and (E_per^dagger)^*); K as for AW_BC_SYM. */
typedef enum { AW_BC_ZPD = 0, AW_BC_SYM = 1, AW_BC_PER = 2, AW_BC_PER_EXT = 3 } aw_bc;

#define AW_MAX_TAPS 16
#define AW_MAX_LEVELS 8
#define AW_MAX_RADIUS 12

/* Multi-level 2-D wavelet transform of a rows x cols image.
 * Orthogonal (biorthogonal = 0): lo[0..filter_len) is the reconstruction
 * low-pass filter h (orthonormal even shifts, sum sqrt(2)); the high-pass is
 * g[k] = (-1)^k h[L-1-k]; every operator uses (h, g).
 * Biorthogonal (biorthogonal = 1, Sec. "The adjoint for biorthogonal
 * wavelets"): lo is the synthesis low-pass h_s and lo_analysis the analysis
 * low-pass h_a (sum_k h_s[k] h_a[k+2m] = delta_m); W and its true adjoint W^*
 * use (h_s, g_s) with g_s[k] = (-1)^k h_a[L-1-k], so W^* = W~^dagger_zpd
 * (E^dagger)^* (eq. 4) analyses with the dual filters; W^dagger and
 * (W^dagger)^* use (h_a, g_a) with g_a[k] = (-1)^k h_s[L-1-k].
 * filter_len must be 2, 8, 10 or 16 (Haar, Daubechies-4, CDF 9/7 or
 * Daubechies-5, Daubechies-8); 1 <= levels <= AW_MAX_LEVELS. */
typedef struct {
  int32_t rows, cols;
  int32_t levels;
  int32_t filter_len;
  int32_t bc; /* aw_bc */
  double lo[AW_MAX_TAPS];
  int32_t biorthogonal;
  double lo_analysis[AW_MAX_TAPS];
} aw_wavelet;

/* Separable blur R with half-point reflexive boundaries (Sec. "Example 1"):
 * (R x)[i] = sum_{u=-r}^{r} g[u] x[refl(i-u)] along rows, then columns;
 * taps[u + radius] = g[u]; 0 <= radius <= AW_MAX_RADIUS. The taps need not be
 * symmetric: blur_adjoint applies the structural adjoint in every case. */
typedef struct {
  int32_t rows, cols, radius;
  double taps[2 * AW_MAX_RADIUS + 1];
} aw_blur;

/* ------------------------------------------------------------ utilities */

/* Message of the last failing call on this thread ("" if none). */
const char* aw_last_error(void);

/* Orthonormal minimum-phase Daubechies scaling filter of length `taps`
 * (2, 4, ..., 16), by spectral factorisation (host computation; writes taps
 * doubles to lo_out, sum sqrt(2)). Sec. "The adjoint for orthogonal wavelets"
 * names Haar and Daubechies wavelets. */
aw_status aw_daubechies(int32_t taps, double* lo_out);

/* Biorthogonal CDF 9/7 low-pass pair as length-10 filters (host
 * computation): the p = 4 product filter 2 cos^8(w/2) P(sin^2(w/2)) split
 * into the 7-tap synthesis filter (the real root of P) and the 9-tap analysis
 * filter (the complex pair), both symmetric about index 4 (synthesis taps at
 * 1..7, analysis taps at 0..8), each summing to sqrt(2). Sec. "The adjoint for
 * biorthogonal wavelets" runs its second experiment with this pair. */
aw_status aw_cdf97(double* lo_syn_out, double* lo_ana_out);

/* Normalised Gaussian PSF taps g[u] ~ exp(-u^2/(2 sigma^2)), |u| <= radius
 * (host computation; writes 2*radius+1 doubles; 0 <= radius <= 16384: the
 * direct blur takes radius <= AW_MAX_RADIUS, the DCT route any of these). */
aw_status aw_gaussian_psf(double sigma, int32_t radius, double* taps_out);

/* Coefficient layout: ncoef per image and the per-level sizes along rows and
 * columns, sub_rows[0] = rows, sub_rows[j] = K^r_j (arrays of levels+1
 * entries; either may be NULL). */
aw_status aw_wavelet_layout(const aw_wavelet* w, int64_t* ncoef, int32_t* sub_rows,
                            int32_t* sub_cols);

/* Workspace bytes that every entry point below needs for this problem and
 * batch (w or b may be NULL when the call does not use it). */
aw_status aw_workspace_size(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype,
                            int32_t batch, size_t* bytes);

/* ------------------------------------------------------ wavelet operators */

/* img = W coef: multi-level synthesis (reconstruction), per level
 * W = E^dagger Phi^* (Sec. "A few signal extensions"). */
aw_status wavelet_synth(const aw_wavelet* w, aw_dtype dtype, int32_t batch, const void* coef,
                        void* img, void* workspace, size_t workspace_bytes, void* stream);

/* coef = W^* img: the true adjoint of wavelet_synth, per level
 * W^* = W^*_zpd (E^dagger)^* (eq. 2; for orthogonal filters W^*_zpd is the
 * zero-boundary analysis). */
aw_status wavelet_synth_adjoint(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                                const void* img, void* coef, void* workspace,
                                size_t workspace_bytes, void* stream);

/* coef = W^dagger img: wavelet analysis, per level W^dagger = W^dagger_zpd E
 * (Sec. "A few signal extensions"); the "pseudoinverse approximation" of W^*. */
aw_status aw_wavelet_analysis(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                              const void* img, void* coef, void* workspace,
                              size_t workspace_bytes, void* stream);

/* img = (W^dagger)^* coef = per level E^* Phi^* (synthesis with a summing
 * fold); the adjoint of aw_wavelet_analysis. */
aw_status aw_wavelet_analysis_adjoint(const aw_wavelet* w, aw_dtype dtype, int32_t batch,
                                      const void* coef, void* img, void* workspace,
                                      size_t workspace_bytes, void* stream);

/* --------------------------------------------------------- blur operators */

/* y = R x (Sec. "Example 1": Gaussian PSF, reflexive boundaries). x != y. */
aw_status blur(const aw_blur* b, aw_dtype dtype, int32_t batch, const void* x, void* y,
               void* stream);

/* x = R^* y: correlation with the PSF on the extended domain, halo folded back
 * by summation onto its reflexive preimages. x != y. */
aw_status blur_adjoint(const aw_blur* b, aw_dtype dtype, int32_t batch, const void* y,
                       void* x, void* stream);

/* y = R x by DCT-II diagonalisation (Sec. "Example 1": for reflexive
 * boundaries R can be applied in O(N log N); pays off over the direct
 * kernels for wide PSFs). With half-point reflexive boundaries (repeating with
 * period 2N) and a symmetric PSF g of any radius, each axis of R is
 * C^{-1} diag(lambda) C with C the DCT-II and lambda_k = g_0 + 2 sum_{u>=1}
 * g_u cos(pi k u / N); then R^* = R. The plan holds the eigenvalues and the
 * FFT / DCT twiddle tables of both axes, computed on the host in FP64 and
 * stored in the plan's dtype (device memory, freed by destroy). rows and cols: powers of two in
 * [2, 4096]; taps: host array of 2*radius+1 doubles, symmetric to 1e-14
 * relative (else AW_EUNSUPPORTED), 0 <= radius <= 16384. */
typedef struct aw_blur_dct aw_blur_dct;
aw_status aw_blur_dct_create(int32_t rows, int32_t cols, int32_t radius, const double* taps,
                             aw_dtype dtype, aw_blur_dct** plan);
aw_status aw_blur_dct_destroy(aw_blur_dct* plan);
/* Workspace of aw_blur_dct_apply: two images per batch entry. */
aw_status aw_blur_dct_workspace(const aw_blur_dct* plan, int32_t batch, size_t* bytes);
/* y = R x for batch images [batch][rows][cols] in the plan's dtype (x may
 * alias y): five passes (row transform, transpose, column transform with the
 * eigenvalue scaling and inverse, transpose, row inverse). */
aw_status aw_blur_dct_apply(const aw_blur_dct* plan, int32_t batch, const void* x, void* y,
                            void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------- composed operators */

/* img = A coef = R W coef (eq. 1). w and b must describe the same image size. */
aw_status aw_apply_A(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                     const void* coef, void* img, void* workspace, size_t workspace_bytes,
                     void* stream);

/* img = A coef - b_obs (b_obs NULL: img = A coef), the residual of eq. (1),
 * with the finest synthesis level and the blur in one tile pass: each tile
 * synthesises the part of W coef its blur window reaches straight into LDS, so
 * the full-resolution W coef never reaches memory (coarser levels run as in
 * aw_apply_A). Bitwise equal to aw_apply_A (minus b_obs). Float32 only;
 * boundaries zpd, sym or per; filter length 2, 8 or 16; rows and cols at least
 * radius + 1 (and at least L - 1 for sym). Other requests return
 * AW_EUNSUPPORTED. Same workspace as aw_apply_A. aw_apply_A is the faster of
 * the two on gfx950 (the window's halo is synthesised by every tile that
 * reads it and the larger LDS footprint lowers occupancy); this entry point
 * offers the pass that writes no intermediate image. */
aw_status aw_apply_A_fused(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                           const void* coef, const void* b_obs, void* img, void* workspace,
                           size_t workspace_bytes, void* stream);

/* coef = A^* img = W^* R^* img (the gradient map of Sec. "Example 1"). */
aw_status aw_apply_A_adjoint(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype,
                             int32_t batch, const void* img, void* coef, void* workspace,
                             size_t workspace_bytes, void* stream);

/* coef = A^* img = W^* R^* img with the blur adjoint and the finest analysis
 * level in one tile pass: each tile computes R^* img over the image samples its
 * window reads and analyses them from LDS, so R^* img never reaches memory
 * (coarser levels run as in aw_apply_A_adjoint). Bitwise equal to
 * aw_apply_A_adjoint. Float32 only; boundaries zpd or sym (images of at least
 * L - 1 samples per axis for sym); filter length 2, 8 or 16. Other requests
 * return AW_EUNSUPPORTED. Same workspace as aw_apply_A_adjoint, which is the
 * faster of the two on gfx950 (this entry point trades the intermediate
 * image for recomputed blur halos and a larger LDS footprint). */
aw_status aw_apply_A_adjoint_fused(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype,
                                   int32_t batch, const void* img, void* coef, void* workspace,
                                   size_t workspace_bytes, void* stream);

/* ------------------------------- multi-channel blind channel estimation */

/* Sec. "Example 2", eq. 6: C channels h_c (length K) observe one source s
 * (length N); x_c = h_c * s (full linear convolution, length M = K+N-1).
 * For all channels at once:
 *   resid[c]        = h_c * s - x_obs[c]   (x_obs NULL: no subtraction)
 *   grad_h[c]       = S^* resid[c]:  grad_h[c][n] = sum_{k<N} s[k] resid[c][k+n]
 *   grad_s_parts[c] = H_c^* resid[c]: sum_{k<K} h_c[k] resid[c][k+n]
 *   grad_s          = sum_c grad_s_parts[c] (channels in order; needs grad_s_parts)
 *   rnorm[c]        = ||resid[c]||^2 (device doubles)
 * h [C][K], x_obs and resid [C][M], grad_s_parts [C][N], s and grad_s [N];
 * grad_h, grad_s_parts, grad_s and rnorm may be NULL. These are the gradients
 * of 1/2 ||h_c * s - x_c||^2 (the data term of eq. 6 carries no 1/2: its
 * gradients are twice these). resid must not alias the inputs. */
aw_status aw_conv_multichannel(aw_dtype dtype, int32_t channels, int32_t K, int32_t N,
                               const void* h, const void* s, const void* x_obs, void* resid,
                               void* grad_h, void* grad_s_parts, void* grad_s, double* rnorm,
                               void* stream);

/* The softened TV term of eq. 6 per row b of h [batch][K]:
 *   value[b] = sum_{j<K-1} L_delta((D h_b)_j),  (D h)_j = h_{j+1} - h_j,
 *   L_delta(z) = z^2/2 (|z| <= delta), delta (|z| - delta/2) otherwise,
 *   grad[b][j] += gscale * (D^* clip(D h_b, -delta, delta))_j,
 * with (D^* v)_j = v_{j-1} - v_j and v_{-1} = v_{K-1} = 0 (the gradient of
 * gscale * value). value (device doubles) and grad may be NULL; delta > 0. */
aw_status aw_huber_tv(aw_dtype dtype, int32_t batch, int32_t K, const void* h, double delta,
                      double gscale, void* grad, double* value, void* stream);

/* Proximal gradient step for an l1 term: out = soft(x - step g, thresh),
 * soft(v, t) = sign(v) max(|v| - t, 0), over n entries; stats (device doubles
 * [3], or NULL) = [sum g (out - x), sum (out - x)^2, sum |out|], the terms of
 * a backtracking test. out must not alias x or g; step, thresh >= 0. One
 * workgroup: meant for channel and source vectors, not images. */
aw_status aw_prox_l1(aw_dtype dtype, int64_t n, const void* x, const void* g, double step,
                     double thresh, void* out, double* stats, void* stream);

/* ------------------------------------------------------------------ FISTA */

/* State of FISTA (Beck & Teboulle) on eq. (1) for `batch` independent images
 * sharing one size, filter and PSF.
 *   x      [batch][ncoef]  x_{k-1} on entry, x_k on return (in place)
 *   y      [batch][ncoef]  y_k on entry, y_{k+1} on return (in place)
 *   resid  [batch][rows][cols]  written: A y_k - b
 *   obj    device doubles [batch][2] or NULL: written when want_objective:
 *          obj[2i] = 1/2 ||A y_k - b||^2, obj[2i+1] = ||x_k||_1
 *   k      iteration index (>= 1), incremented by fista_step
 *   t      t_k (t_1 = 1), replaced by t_{k+1} by fista_step
 *   gradient  AW_GRAD_ADJOINT (0, the zero-initialised default): the
 *          gradient W^* R^* (A y - b) with the true adjoint; AW_GRAD_PINV: W^dagger in
 *          the place of W^*, the approximation that Sec. "The adjoint for
 *          orthogonal wavelets" compares with the true adjoint (the two coincide
 *          for zpd and per). Other values: AW_EINVAL.                       */
typedef enum { AW_GRAD_ADJOINT = 0, AW_GRAD_PINV = 1 } aw_gradient_map;

typedef struct {
  void* x;
  void* y;
  void* resid;
  double* obj;
  int64_t k;
  double t;
  int32_t gradient;
} aw_fista_state;

/* One FISTA iteration with constant step 1/L:
 *   x_k = soft(y_k - A^*(A y_k - b)/L, lambda/L),
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,
 *   y_{k+1} = x_k + ((t_k - 1)/t_{k+1}) (x_k - x_{k-1}).
 * b is [batch][rows][cols]. L > 0, lambda >= 0. */
aw_status fista_step(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                     const void* b_obs, double L, double lambda, aw_fista_state* state,
                     int32_t want_objective, void* workspace, size_t workspace_bytes,
                     void* stream);

/* fista_step for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same iteration, arguments and results as fista_step, with the
 * workspace taken from a static device array of the library (64 MiB,
 * 67108864 bytes, held on every GPU the library runs on until the process
 * ends) instead of a caller's buffer. Nothing is allocated or freed; the
 * caller still passes b, the state's x, y, resid and obj. Problems whose
 * aw_workspace_size(w, b, dtype, batch) exceeds 64 MiB fail with AW_EINVAL
 * before any device work (2048 x 2048 FP32 at db4, J = 4 needs 38 MiB).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (none of it is read before it is written within a call): calls
 * that overlap on one GPU, on different streams or threads, race. */
aw_status fista_step_noalloc(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                             const void* b_obs, double L, double lambda, aw_fista_state* state,
                             int32_t want_objective, void* stream);

/* The second half of fista_step, from an image-space gradient: with
 * grad = R^*(A y_k - b) (or the gradient of any other smooth term in image
 * space), the coefficient gradient W^* grad (W^dagger grad with
 * AW_GRAD_PINV) is consumed level by level by the update
 *   x_k = soft(y_k - W^* grad / L, lambda/L),  y_{k+1} = x_k + beta_k (x_k - x_{k-1}),
 * with t_k, beta_k and the state's k, t advanced as in fista_step (Beck &
 * Teboulle's step as used in Sec. "Example 1: An Image Deblurring Problem").
 * grad is a device image [batch][rows][cols] (read only); state->resid and
 * the blur are not used. With want_l1 and state->obj, obj[2i+1] = ||x_k||_1
 * (obj[2i] untouched). The workspace is sized by aw_workspace_size(w, NULL,
 * ...). Fails with AW_EINVAL on NULL pointers, batch < 1, L <= 0, lambda < 0,
 * k < 1, t < 1 or an unknown gradient map. */
aw_status aw_fista_update(const aw_wavelet* w, aw_dtype dtype, int32_t batch, const void* grad,
                          double L, double lambda, aw_fista_state* state, int32_t want_l1,
                          void* workspace, size_t workspace_bytes, void* stream);

/* Objective of eq. (1) at x: obj[3i] = 1/2 ||A x_i - b_i||^2,
 * obj[3i+1] = ||x_i||_1, obj[3i+2] = obj[3i] + lambda obj[3i+1]
 * (obj: device doubles [batch][3]; fixed-order reductions, reproducible). */
aw_status aw_objective(const aw_wavelet* w, const aw_blur* b, aw_dtype dtype, int32_t batch,
                       const void* b_obs, double lambda, const void* x, double* obj,
                       void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------ batched FISTA (uneven) */

/* Opaque plan for FISTA on n independent FP32 problems of uneven image size,
 * wavelet depth, filter length and PSF (each with its own aw_wavelet /
 * aw_blur; boundary modes zero, symmetric or circular, every level at least
 * as long as the extension width). Creation validates and sizes; binding
 * uploads per-stage tile queues (the plan's own device memory, freed by
 * aw_batch_destroy). aw_batch_step then only enqueues kernels whose varying
 * inputs live in device memory, so one iteration can be captured into a
 * hipGraph once and replayed. */
typedef struct aw_batch aw_batch;

aw_status aw_batch_create(int32_t n, const aw_wavelet* w, const aw_blur* b, aw_batch** plan);
/* Releases the plan and everything it owns; the plan is gone even when a
 * runtime error is reported (AW_EHIP, the first error met). */
aw_status aw_batch_destroy(aw_batch* plan);

/* coef_off / img_off: n+1 element offsets of problem i in the concatenated
 * coefficient / image buffers (either may be NULL); workspace bytes. */
aw_status aw_batch_layout(const aw_batch* plan, int64_t* coef_off, int64_t* img_off,
                          size_t* workspace_bytes);

/* Tunables: cfg[0..2] tile-shape variant (0 full-height, 1 half-height
 * tiles) of the synthesis, analysis and blur kernels, the analysis also 2
 * (full height for the finest level, half height for the coarser ones) and
 * 3 (half height for 16-tap filters, full height for the others), the
 * blur also 2 (full-height tiles, and one launch per blur stage: every PSF
 * zero-padded to the batch's largest radius, the same values as per-radius
 * launches);
 * cfg[3] streams (1..4) over which the kernel classes of one stage run
 * concurrently (each class to the stream with the least estimated work).
 * Rebuilds the tile queues of a bound plan. */
aw_status aw_batch_set_config(aw_batch* plan, const int32_t* cfg);

/* Bind device buffers: b_obs (concatenated images), x, y (concatenated
 * coefficients, in/out) and the workspace; FISTA step 1/L and lambda. Blocking
 * (uploads descriptor tables and the beta_k table). */
aw_status aw_batch_bind(aw_batch* plan, const void* b_obs, void* x, void* y, void* workspace,
                        size_t workspace_bytes, double lambda, double L);

/* Device addresses inside the bound workspace: the iteration counter k
 * (int32), per-problem active flags (int32[n]; 0 skips every tile of that
 * problem) and per-problem partials obj[n][3] of the last step
 * (1/2 ||A y_k - b||^2, ||x_k||_1, ||x_k - x_{k-1}||^2). */
aw_status aw_batch_control(const aw_batch* plan, int32_t** counter, int32_t** active,
                           double** obj);

/* k = 1, all problems active, x = y = 0 (kernels on stream). */
aw_status aw_batch_reset(aw_batch* plan, void* stream);

/* One FISTA iteration for every active problem (kernels only). */
aw_status aw_batch_step(aw_batch* plan, void* stream);

/* Message of the last failing aw_batch_* call on this thread. */
const char* aw_batch_last_error(void);

/* ------------------------------------------------- convolution adjoints */

/* Blind-channel pair (Sec. "Example 2"), `batch` independent (h, s) pairs:
 *   resid[t]  = (h * s)[t] - x_obs[t],  t < K+N-1  (full linear convolution)
 *   grad_h[n] = sum_{k<N} s[k] resid[k+n], n < K  (S^* r, cross-correlation)
 *   grad_s[n] = sum_{k<K} h[k] resid[k+n], n < N  (H^* r)
 * h: [batch][K], s: [batch][N], x_obs/resid: [batch][K+N-1]. x_obs may be
 * NULL (treated as zero). grad_h / grad_s may be NULL (not computed).
 * resid must not alias the inputs. */
aw_status conv_adjoint_pair(aw_dtype dtype, int32_t batch, int32_t K, int32_t N, const void* h,
                            const void* s, const void* x_obs, void* resid, void* grad_h,
                            void* grad_s, void* stream);

/* ----------------------------------------------- learned warm start (CNN) */
/* The paper solves eq. (1) by FISTA from x = 0 (Sec. "The adjoint for
 * orthogonal wavelets"); these calls add a learned start x_0 for it, with the
 * zero start kept as fallback. Network: six 3x3 convolution layers
 * 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, zero 'same' padding, a bias per output
 * channel, ReLU after the first five; a layer computes
 *   out[o][y][x] = bias[o] + sum_{i,ky,kx} w[o][i][ky][kx] in[i][y+ky-1][x+kx-1].
 * The image u = b + CNN(b) is mapped to coefficients by the wavelet analysis
 * W^dagger (aw_wavelet_analysis) and x_0 = soft(W^dagger u, lambda / L)
 * (aw_soft_threshold). Training minimises ||W^dagger u - x*||^2 (aw_sq_error),
 * backpropagated through (W^dagger)^* (aw_wavelet_analysis_adjoint),
 * aw_cnn_backward and aw_adam_step.
 *
 * Parameters  FP32 master vector of AW_CNN_PARAMS values, layer by layer, each
 *             as weight [out][in][3][3] then bias [out].
 * Precision   Weights and activations are rounded to BF16 (nearest even);
 *             products accumulate in FP32 (v_mfma_f32_32x32x16_bf16 for the
 *             32-channel layers). The input image enters the first layer in
 *             FP32; the incoming gradient du is rounded to BF16 where it
 *             enters a convolution; biases stay FP32.
 * Activations [5][batch][rows][cols][32] BF16 (uint16 bit patterns), the
 *             outputs y_1..y_5 of layers 1..5 after ReLU (AW_CNN_ACT_BYTES per
 *             pixel). Gradients at the pre-activations of layers 1..5 use the
 *             same layout. */
#define AW_CNN_CHANNELS 32
#define AW_CNN_PARAMS 37601
#define AW_CNN_ACT_BYTES 320 /* 5 layers x 32 channels x 2 bytes per pixel */

/* Sizes: packed parameter buffer (bytes), activation buffer (bytes, also the
 * size of the activation-gradient buffer) and the backward workspace (bytes)
 * for `batch` images of rows x cols. Any output pointer may be NULL. */
aw_status aw_cnn_sizes(int32_t batch, int32_t rows, int32_t cols, size_t* packed_bytes,
                       size_t* act_bytes, size_t* workspace_bytes);

/* Device-side conversion of the FP32 master parameters (AW_CNN_PARAMS) into
 * the packed BF16 layouts the kernels read (forward and mirrored-transposed
 * copies). Call after every parameter update. */
aw_status aw_cnn_pack(const float* params, void* packed, void* stream);

/* u = b + CNN(b) for b: [batch][rows][cols] FP32; acts receives y_1..y_5
 * (needed by aw_cnn_backward). u must not alias b. */
aw_status aw_cnn_forward(const void* packed, int32_t batch, int32_t rows, int32_t cols,
                         const float* b, void* acts, float* u, void* stream);

/* Gradient of <du, CNN(b)> in the parameters: grad (FP32, AW_CNN_PARAMS,
 * overwritten, master layout) from the activations of aw_cnn_forward and du
 * ([batch][rows][cols] FP32). dacts receives the gradients at the
 * pre-activations of layers 1..5. Workspace size from aw_cnn_sizes.
 * Deterministic (fixed-order reductions). */
aw_status aw_cnn_backward(const void* packed, int32_t batch, int32_t rows, int32_t cols,
                          const float* b, const void* acts, const float* du, void* dacts,
                          float* grad, void* workspace, size_t workspace_bytes, void* stream);

/* Adam (Kingma & Ba 2015, Algorithm 1) on n FP32 values, step t >= 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
aw_status aw_adam_step(float* params, float* m, float* v, const float* grad, int64_t n,
                       int32_t step, double lr, double beta1, double beta2, double eps,
                       void* stream);

/* r = c - target over n FP32 values: grad = scale * 2 r (grad may be NULL)
 * and *loss = sum r^2 (one FP64 device value, fixed-order sum). The
 * workspace holds aw_sq_error_workspace(n) bytes. */
aw_status aw_sq_error(int64_t n, const float* c, const float* target, double scale, float* grad,
                      double* loss, void* workspace, size_t workspace_bytes, void* stream);
aw_status aw_sq_error_workspace(int64_t n, size_t* bytes);

/* out = sign(in) max(|in| - tau, 0) over n FP32 values (out may equal in). */
aw_status aw_soft_threshold(int64_t n, const float* in, double tau, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ADJWAVE_H */
