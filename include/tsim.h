/*
 * tsim.h -- C ABI of the MI355X dense-field phase-to-space (DF-P2S)
 * turbulence renderer (Chimitt, Zhang, Mao, Chan, "Real-Time Dense Field
 * Phase-to-Space Simulation of Imaging through Atmospheric Turbulence").
 *
 * The per-frame hot path is
 *   (a) tsim_sample_zernike : per-pixel Zernike coefficient fields drawn by
 *       FFT colouring of independent unit-variance fields followed by
 *       per-pixel mixing with the Noll matrix factor (Sec. III-C, Eq. (9));
 *   (b) tsim_p2s            : Zernike vector -> weights on K PSF basis
 *       functions (Sec. II-C, Eq. (7)), either by exact pupil-FFT PSFs
 *       (Eq. (2)) and projection, or by a small learned network;
 *   (c) tsim_render         : the basis-weighted blur of Eq. (8);
 *   (d) tsim_warp           : the tilt modes (Noll 2, 3) as a bilinear warp.
 *
 * Conventions for every call
 *   - Return codes: TSIM_OK (0) or a negative TSIM_E* code.  No exception
 *     crosses the ABI.  Arguments are validated before any launch.
 *   - Device pointers are caller-owned device memory (hipMalloc or torch),
 *     256-byte aligned, row-major, frame-major.  The plan owns only its own
 *     tables.  Host pointers are read during the call only.
 *   - Launches are asynchronous on the given stream (NULL = default stream);
 *     kernel faults surface at the caller's next synchronisation.
 *   - A plan is immutable after creation: concurrent calls on different
 *     streams are safe if each uses its own workspace.
 *   - Buffer extents cannot be checked through bare pointers: the caller
 *     guarantees that every buffer has the shape and element type stated
 *     for it (the Python binding checks them before each call).
 *   - A failing call also records its status and name for tsim_last_error
 *     on the calling thread.
 */
#ifndef TSIM_H
#define TSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsim_plan tsim_plan;
typedef void *tsim_stream; /* a hipStream_t */

enum {
  TSIM_OK = 0,
  TSIM_EINVAL = -1,      /* bad argument (pointer, size, parameter)        */
  TSIM_ENOMEM = -2,      /* device or host allocation failed               */
  TSIM_EDEVICE = -3,     /* no usable gfx950 device or a HIP runtime error */
  TSIM_EARTEFACT = -4,   /* basis or network weights missing or malformed  */
  TSIM_EUNSUPPORTED = -5 /* valid request this build does not implement    */
};

enum { TSIM_P2S_EXACT = 0, TSIM_P2S_LEARNED = 1 };
enum { TSIM_FP32 = 0, TSIM_BF16 = 1 };

#define TSIM_N_MODES 35  /* Noll j = 2..36 (Sec. II-B keeps N = 36 modes; piston dropped) */
#define TSIM_MAX_MODES 65 /* Noll j = 2..66: complete radial orders up to 10 */

/*
 * Problem statement (Sec. II and its footnote on s = (x - x')/D).
 *
 *   H, W, C        image rows, columns, channels (1 <= H, W <= 4096, 1 <= C <= 4)
 *   Gh, Gw         zero-padded periodic FFT grid for the sampler; powers of
 *                  two, 64 <= G <= 4096, Gh >= H, Gw >= W
 *   n_modes        number of Zernike modes sampled, Noll j = 2..n_modes + 1:
 *                  35 (Noll 2..36, radial orders up to 7, the paper's
 *                  N = 36 with piston dropped), or 44, 54, 65 (complete
 *                  radial orders up to 8, 9, 10: Sec. II-B notes that N
 *                  can be raised at some cost in speed).  Coefficient
 *                  planes are [frames][n_modes][H][W] throughout.  The
 *                  learned P2S form and tsim_structure_function take
 *                  n_modes = 35 only (TSIM_EUNSUPPORTED otherwise).
 *   pixel_pitch_over_d
 *                  one image pixel in units of the aperture diameter D
 *                  (the displacement unit of the Zernike space).  If <= 0 it
 *                  is derived from the optics as L*lambda/(2 D^2): the image
 *                  pixel is the Nyquist angle lambda/(2D) seen over path L.
 *   aperture_d_m, wavelength_m, path_length_m
 *                  D, lambda, L in metres (used only when the pitch is <= 0)
 *   alias_fold     spectral aliases folded per axis (0..4; 2 recommended)
 *   pupil_n        P, pupil samples per side for exact PSFs (64 or 128); the
 *                  circular aperture spans P/2 samples, so one PSF sample is
 *                  one image pixel
 *   psf_t          T, odd PSF support: 9, 15, 21, 31 or 33 with P = 64, 33 or
 *                  65 with P = 128 (the exact-PSF kernels' sizes); in BF16
 *                  plans also one of 15, 21, 33, 65, excluding K > 112 with
 *                  C = 4 and T = 65 (the BF16 blur's image tile and basis
 *                  staging exceed the LDS there).  Other values:
 *                  TSIM_EUNSUPPORTED at plan creation.
 *   basis_k        K, number of PSF basis functions (1 <= K <= 128)
 *   basis          host [K][T*T] float64, orthonormal rows (Eq. (7)); copied.
 *                  May be NULL for a plan that only samples and warps.
 *   p2s_mode       TSIM_P2S_EXACT or TSIM_P2S_LEARNED
 *   precision      TSIM_FP32 (plain form) or TSIM_BF16 (learned form: BF16
 *                  network and basis contraction, FP32 accumulation)
 *   subharmonic_levels
 *                  0..4 (0: off).  Subharmonic compensation of the tilt
 *                  fields (Noll 2, 3), the low-frequency remedy named in
 *                  Sec. IV-B: level p adds the 8 cells of size (1/(Gw ds),
 *                  1/(Gh ds))/3^p around the DC bin (ds = pixel pitch over
 *                  D) as 4 random cosine waves per mode, and the two tilt
 *                  spectra are normalised over grid bins and cells together,
 *                  so each field keeps unit variance.  See tsim_plan_table
 *                  what = 4 and tsim_sample_zernike.
 */
typedef struct tsim_params {
  int32_t H, W, C;
  int32_t Gh, Gw;
  int32_t n_modes;
  double pixel_pitch_over_d;
  double aperture_d_m, wavelength_m, path_length_m;
  int32_t alias_fold;
  int32_t pupil_n;
  int32_t psf_t;
  int32_t basis_k;
  const double *basis;
  int32_t p2s_mode;
  int32_t precision;
  int32_t subharmonic_levels;
} tsim_params;

/* Build the FP64 plan tables on the host and upload them: the Noll matrix
 * A_0 and its lower Cholesky factor L (Sec. III-C: L L^T = A_0), the folded
 * unit-mean per-mode spectra of the autocovariances A_ii (Sec. III-B/III-C),
 * the Zernike pupil table for exact PSFs (Eq. (2), (5)) and the basis.  Uses
 * the current HIP device.  On error *out is NULL. */
int tsim_plan_create(const tsim_params *p, tsim_plan **out);

/* The host half of plan creation without any device: validates `p`, builds
 * the FP64 tables and copies table `what` (numbering of tsim_plan_table) to
 * host_out.  For inspection and CPU-side tests of the plan builder. */
int tsim_host_tables(const tsim_params *p, int what, double *host_out, size_t count);

/* Free the plan's device tables.  NULL is accepted. */
int tsim_plan_destroy(tsim_plan *plan);

/* Bytes of caller-provided device workspace needed by calls on `frames`
 * frames: the larger of the sampler's pass-1 intermediate (frames x 18 x
 * H x Gw complex samples, chunked to about 2 GB) and the exact-P2S PSF
 * buffer (up to 2^20 pixels x T*T floats).  The same workspace may be reused by consecutive calls on one
 * stream. */
int tsim_workspace_bytes(const tsim_plan *plan, int frames, size_t *bytes);

/* Copy a plan table to host memory as float64, for inspection and tests.
 *   what = 0: A_0 at D/r0 = 1, [N][N] (N = n_modes)
 *   what = 1: L, [N][N] lower triangular
 *   what = 2: sqrt of the quarter spectra, [N][Gw/2+1][Gh/2+1] (ky fastest)
 *   what = 3: pixel pitch over D, [1]
 *   what = 4: subharmonic wave amplitudes, [2 modes][4 levels][4 cells]
 *             (Noll 2, 3; level p = 1..4; cells (m, n) = (1,0), (1,1),
 *             (0,1), (-1,1)), zero beyond subharmonic_levels
 * `count` is the number of doubles `host_out` can hold. */
int tsim_plan_table(const tsim_plan *plan, int what, double *host_out, size_t count);

/* (a) Zernike fields for `frames` frames (Sec. III-C):
 *   step 1: for field q = 0..17 (modes 2+2q and 3+2q in its real and
 *           imaginary parts), Hermitian white noise from Philox4x32-10 with
 *           key (seed lo, seed hi) and counter (canonical bin, q, frame0+f,
 *           0) is coloured by the square-root spectra and inverse-FFT'd on
 *           the Gh x Gw grid (unitary scaling), then cropped to H x W;
 *           with subharmonic levels, the tilt fields ybar_2, ybar_3 gain
 *           sum over levels p and cells (m, n) of A cos t + B sin t,
 *           t = 2 pi (m x / (Gw 3^p) + n y / (Gh 3^p)) at pixel (x, y),
 *           where (A2, B2, A3, B3) are the amplitudes of table 4 times the
 *           four Gaussians of the Philox call with counter (cell, p,
 *           frame0+f, 5);
 *   step 2: a_x = (D/r0)^{5/6} L ybar_x at every pixel.
 *   d_over_r0 : host [frames], each > 0 and finite
 *   zern      : device [frames][N][H][W] float32, output
 *   ws        : device workspace of tsim_workspace_bytes(plan, frames) */
int tsim_sample_zernike(const tsim_plan *plan, int frames, const float *d_over_r0,
                        uint64_t seed, uint64_t frame0, float *zern, void *ws,
                        tsim_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fields as tsim_sample_zernike, bit for bit, with no workspace argument and
 * no allocation of any kind.  The pass-1 intermediate lives in a fixed
 * device array of the library, TSIM_NOALLOC_SCRATCH_BYTES (256 MiB) on each
 * GPU the library runs on, held until the process ends; its address is
 * looked up at plan creation.  Frames are processed in chunks that fit it.
 *   Limit: one frame's intermediate, ceil(N / 2) * H * Gw * 8 bytes (18
 *   fields for N = 35), must fit the array (e.g. 768 x 1024 on a 2048-wide
 *   grid fits, 2160 x 3840 on 4096 does not): larger plans return
 *   TSIM_EUNSUPPORTED before any launch.
 *   Every call on one GPU shares that GPU's array, so calls that overlap in
 *   time on one GPU (other threads, other streams without ordering) race;
 *   calls on one stream are ordered and safe.  The array's contents from
 *   the previous call are never read.  Launches are not traced.
 *   d_over_r0 : host [frames], each > 0 and finite
 *   zern      : device [frames][N][H][W] float32, output, 256-byte aligned */
#define TSIM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int tsim_sample_zernike_noalloc(const tsim_plan *plan, int frames, const float *d_over_r0,
                                uint64_t seed, uint64_t frame0, float *zern,
                                tsim_stream stream);

/* Launch forms of the field sampler (the two passes of tsim_sample_zernike,
 * Sec. III-A / III-C), chosen per plan.  Every form computes the same
 * transforms and sums, so the fields do not depend on it; only the time does.
 *   pass-1 columns: columns of the grid one block transforms (NC columns of
 *     Gh points in LDS; (NC / 2) Gh must be 1024, 2048 or 4096 draws);
 *   pass-2 form: 1 = two rows per 256-thread block (W <= 1024), 2 = the same
 *     with twice the outputs per thread (W <= 512), 3 = one row per
 *     1024-thread block.
 * tsim_plan_autotune times each candidate of each pass on the caller's
 * buffers (a warm-up, then the best of three timed runs, HIP events on the
 * stream) and keeps the fastest in the plan; a candidate replaces the
 * built-in form only when at least 3% faster.  It synchronises the stream,
 * overwrites zern and ws, and changes the plan: call it before the plan is
 * used on other threads.
 *   frames : frames of the workload to time (at most one pass-1 chunk is used)
 *   zern   : device [frames][N][H][W] float32 scratch, 256-byte aligned
 *   ws     : device workspace of tsim_workspace_bytes(plan, frames) bytes
 * tsim_plan_set_tuning forces a form (0 = the built-in choice; TSIM_EINVAL
 * for a form the plan's shape does not allow); tsim_plan_tuning returns the
 * forms in effect. */
int tsim_plan_autotune(tsim_plan *plan, int frames, float *zern, void *ws, tsim_stream stream);
int tsim_plan_set_tuning(tsim_plan *plan, int columns, int rows_form);
int tsim_plan_tuning(const tsim_plan *plan, int *columns, int *rows_form);

/* Spatial tilt statistics of coefficient planes (the spatial validation of
 * Sec. IV-B): for Noll 2 and 3, the tilt correlation (mean product) and the
 * differential tilt variance (mean squared difference) of all pixel pairs at
 * lags d = 0..max_lag along x and along y, over `frames` frames.  Pairs stay
 * inside the frame: H (W - d) per frame for an x lag, (H - d) W for a y lag.
 * Row sums are FP32, their total FP64 in a fixed order (deterministic).
 *   zern     : device [frames][N][H][W] float32, 256-byte aligned (e.g. the
 *              output of tsim_sample_zernike)
 *   max_lag  : 0 <= max_lag <= 256, below H and W
 *   host_out : host [2 modes][2 axes (x, y)][2 (correlation, DTV)][max_lag+1]
 *              float64, written on success
 *   ws       : device workspace of tsim_tilt_stats_ws_bytes(plan, frames,
 *              max_lag) bytes, 256-byte aligned
 * Synchronises `stream` before returning.  TSIM_EINVAL on a bad argument. */
int tsim_tilt_stats_ws_bytes(const tsim_plan *plan, int frames, int max_lag, size_t *bytes);
int tsim_tilt_stats(const tsim_plan *plan, int frames, const float *zern, int max_lag,
                    double *host_out, void *ws, tsim_stream stream);

/* Phase structure function over the aperture (the aperture statistics of
 * Sec. IV-B; Eq. (4) gives its Kolmogorov form 6.88 (r/r0)^{5/3}): with
 * phi = sum_{j=2}^{36} a_j Z_j on a 64 x 64 pupil grid (aperture 32 samples
 * across, points strictly inside), D(r) is the mean of
 * (phi(p) - phi(p + r x))^2 over the pairs inside the aperture and over all
 * pixels and frames, for r = 0..30 samples (r/D = r/32).  The device part
 * is the coefficients' second moments C_jk = mean a_j a_k (FP32 tile sums,
 * FP64 total in a fixed order); D(r) = sum_jk C_jk mean(dZ_j dZ_k) follows on
 * the host.
 *   zern         : device [frames][N][H][W] float32, 256-byte aligned
 *   host_out     : host [31] float64, D(r)
 *   host_moments : host [35][35] float64 (C), or NULL
 *   ws           : device workspace of tsim_structure_function_ws_bytes
 * Synchronises `stream` before returning. */
int tsim_structure_function_ws_bytes(const tsim_plan *plan, int frames, size_t *bytes);
int tsim_structure_function(const tsim_plan *plan, int frames, const float *zern, double *host_out,
                            double *host_moments, void *ws, tsim_stream stream);

/* Long- and short-exposure optical transfer functions (the aperture
 * statistics of Sec. IV-B): one realisation's OTF is the autocorrelation of
 * the generalised pupil, H(xi) = sum_x G(x) conj(G(x - xi)) with
 * G = P exp(-j phi) and phi = sum_j a_j Z_j over the plan's modes, Noll 2..N+1; the long-
 * exposure OTF is its mean over realisations, the short-exposure OTF the
 * same with the tilt-corrected phase (the plane of best fit over the
 * aperture, i.e. the Zernike tilts Noll 2 and 3, removed).  Every pixel of
 * every frame is one realisation.  The pupil grid is the plan's P x P
 * (P = 64 only: aperture 32 samples across, points strictly inside), and H
 * is normalised so that H(0) = 1.  The device sums |DFT(G)|^2 over the
 * realisations (FP32 per block, FP64 across blocks, fixed order); the host
 * takes the inverse DFT of the mean in FP64.  Synchronises the stream.
 *   zern           : device [frames][N][H][W] float32, 256-byte aligned
 *   short_exposure : 0 for the long-exposure OTF, 1 for the short-exposure
 *   host_out       : host [2][64][64] float64, real then imaginary part,
 *                    lag (dy, dx) at index (32 + dy, 32 + dx), dy, dx in
 *                    [-32, 32); written on success
 *   ws             : device workspace of tsim_otf_ws_bytes(plan, frames)
 *                    bytes, 256-byte aligned
 * TSIM_EUNSUPPORTED for plans with P != 64. */
int tsim_otf_ws_bytes(const tsim_plan *plan, int frames, size_t *bytes);
int tsim_otf(const tsim_plan *plan, int frames, const float *zern, int short_exposure,
             double *host_out, void *ws, tsim_stream stream);

/* (a') Temporally correlated Zernike fields by an auto-regressive process,
 * the low-order workaround the paper gives for spatio-temporal correlation
 * (Sec. III-E): the unit-variance fields of frame t follow
 *   ybar_t = alpha ybar_{t-1} + sqrt(1 - alpha^2) w_t,
 * with w_t the independent fields tsim_sample_zernike draws for frame
 * frame0 + t, and frame t is mixed with its own (D/r0_t)^{5/6} L.  Each
 * field keeps its spatial statistics; frames t and t + k correlate by
 * alpha^k.  Computed on the mixed fields as
 *   a_t = alpha (s_t / s_{t-1}) a_{t-1} + sqrt(1 - alpha^2) a_t^new,
 * s = (D/r0)^{5/6}, which is the same recursion.
 *   alpha          : in [0, 1]
 *   zern_prev      : device [N][H][W] float32, the coefficients of the frame
 *                    before frame0, or NULL to start the sequence from
 *                    frame0's own (already stationary) draw; must not
 *                    overlap zern
 *   d_over_r0_prev : that frame's D/r0 (> 0; ignored when zern_prev is NULL)
 *   other arguments as tsim_sample_zernike (same workspace size). */
int tsim_sample_zernike_ar(const tsim_plan *plan, int frames, const float *d_over_r0,
                           uint64_t seed, uint64_t frame0, float alpha, const float *zern_prev,
                           float d_over_r0_prev, float *zern, void *ws, tsim_stream stream);

/* (b) Basis weights beta[f][y][x][k] from Zernike fields (Sec. II-C).
 *   Exact form: the per-pixel PSF of Eq. (2) from modes 4..36 on the P x P
 *   pupil, cropped to T x T around the zero frequency and normalised to unit
 *   sum, projected on the basis (beta = Psi h).
 *   Learned form: the network set by tsim_plan_set_mlp.  A learned plan with
 *   no network yet runs the exact form (the fallback; tsim_p2s_form tells
 *   which form runs).
 *   Output float32 in FP32 plans and bfloat16 in BF16 plans, either form.
 *   zern : device [frames][N][H][W] float32
 *   beta : device [frames][H][W][K] float32, or in BF16 plans
 *          [frames][H][W][KP] bfloat16 with KP = K rounded up to 32, 64, 112
 *          or 128 (entries K..KP-1 written as 0) */
int tsim_p2s(const tsim_plan *plan, int frames, const float *zern, void *beta, void *ws,
             tsim_stream stream);

/* The form tsim_p2s runs on this plan now: *form = TSIM_P2S_LEARNED for a
 * learned plan holding a network, else TSIM_P2S_EXACT (exact plans, and
 * learned plans without one, which fall back to the exact path). */
int tsim_p2s_form(const tsim_plan *plan, int *form);

/* (c) Eq. (8): out_c(x) = sum_k beta_k(x) sum_u psi_k(u) img_c(clamp(x - u)),
 * u in [-(T-1)/2, (T-1)/2]^2, a true convolution with replicated borders.
 *   img, out : device [frames][C][H][W] float32, img != out
 *   beta     : device [frames][H][W][K] float32, or in BF16 plans
 *              [frames][H][W][KP] bfloat16 as written by tsim_p2s (entries
 *              K..KP-1 must be finite; they meet zero basis rows)
 * The BF16 form evaluates Eq. (8) in the order sum_u (sum_k beta_k psi_k(u))
 * img(x - u) with BF16 operands and FP32 accumulation; it returns
 * TSIM_EUNSUPPORTED for the one shape whose image tile and basis staging do
 * not fit the LDS (K > 112 with C = 4 and T = 65), and both forms for frames
 * of 4 GiB or more (C * H * W * 4 bytes). */
int tsim_render(const tsim_plan *plan, int frames, const float *img, const void *beta,
                float *out, void *ws, tsim_stream stream);

/* (d) Tilt warp: out_c(x) = bilinear(img_c, x - t_x) with the four taps
 * clamped to the image and t_x = -(4/pi) (a_{x,2}, a_{x,3}) pixels, read
 * from planes 0 and 1 of zern (a pure tilt a_2 moves the Eq. (2) PSF by
 * -4 a_2/pi samples).
 *   img, out : device [frames][C][H][W] float32, img != out
 *   zern     : device [frames][N][H][W] float32 */
int tsim_warp(const tsim_plan *plan, int frames, const float *img, const float *zern,
              float *out, tsim_stream stream);

/* Batches of frames of mixed sizes (many frames and uneven image sizes per
 * launch): each item is one plan's frames through the whole path of
 * Sec. III-C and Eq. (8) -- tsim_sample_zernike, tsim_p2s, tsim_render
 * into `blur`, tsim_warp into `out` -- and tsim_batch_create records the
 * calls of all items, in item order, into one HIP graph that the library
 * captures on a private stream and instantiates; tsim_batch_launch replays
 * it on the caller's stream.  Every replay recomputes the same frames
 * (same seed, frame counters and D/r0) from the buffers' current contents:
 * refill `img` between launches to render new images.
 *   Each item: plan, frames >= 1, d_over_r0 host [frames] (read at create),
 *   frame0 (the frame counter of its first frame), and device buffers as
 *   for the individual calls, all 256-byte aligned, owned by the caller and
 *   kept alive and unmoved until tsim_batch_destroy: img, blur, out
 *   [frames][C][H][W] float32 (three distinct buffers), zern
 *   [frames][N][H][W] float32, beta per the plan's precision, ws of at
 *   least tsim_workspace_bytes(plan, frames) bytes (items may share one ws:
 *   the graph runs them in order).  The plans must outlive the batch.
 *   Every item is checked before anything is recorded (TSIM_EINVAL,
 *   TSIM_EARTEFACT without a basis); tsim_batch_launch returns
 *   TSIM_EDEVICE if the replay cannot be queued. */
typedef struct tsim_batch tsim_batch;
typedef struct tsim_batch_item {
  const tsim_plan *plan;
  int frames;
  const float *d_over_r0;
  uint64_t frame0;
  const float *img;
  float *zern;
  void *beta;
  float *blur;
  float *out;
  void *ws;
} tsim_batch_item;
int tsim_batch_create(const tsim_batch_item *items, int n_items, uint64_t seed,
                      tsim_batch **out);
int tsim_batch_launch(const tsim_batch *batch, tsim_stream stream);
int tsim_batch_destroy(tsim_batch *batch);

/* The whole per-frame path of Sec. III-C and Eq. (8) in one call: Zernike
 * fields (as tsim_sample_zernike), basis weights (as tsim_p2s, in the plan's
 * form), the blur of Eq. (8) (as tsim_render) and the tilt warp (as
 * tsim_warp), so that out[f] = warp(blur(img[f])).  Frames go through the
 * four steps in groups of `group` frames (the last group may be smaller);
 * a group's fields, weights and blurred frames live in `ws`, so the
 * workspace is set by the group, not by `frames`, and the weights of the
 * whole call never exist at once.  The result equals the four individual
 * calls on the same frames bit for bit, for any group size (frame f's
 * fields depend only on seed, frame0 + f and d_over_r0[f]).
 *   group     : frames per group, 1..65535; tsim_frame_group gives the
 *               largest group whose fields, weights and blurred frames fit
 *               about 1 GiB (e.g. 10 frames of 512 x 512 x 3 in a BF16
 *               plan with K = 100, 7 in an FP32 plan, one 3840 x 2160
 *               frame)
 *   d_over_r0 : host [frames], each > 0 and finite
 *   img, out  : device [frames][C][H][W] float32, distinct, 256-byte aligned
 *   zern_out  : device [frames][N][H][W] float32 to keep the fields, or NULL
 *               (then they live in ws only)
 *   ws        : device workspace of tsim_frame_workspace_bytes(plan, group)
 *               bytes, 256-byte aligned, owned by the caller (once a
 *               network is set on the plan, the size leaves out the exact
 *               form's PSF buffer; query it after tsim_plan_set_mlp)
 * Asynchronous on `stream`.  TSIM_EINVAL on a bad argument, TSIM_EARTEFACT
 * without a basis, TSIM_EUNSUPPORTED for a shape the blur does not build;
 * all checked before the first launch. */
int tsim_frame_group(const tsim_plan *plan, int *group);
int tsim_frame_workspace_bytes(const tsim_plan *plan, int group, size_t *bytes);
int tsim_frame(const tsim_plan *plan, int frames, int group, const float *d_over_r0,
               uint64_t seed, uint64_t frame0, const float *img, float *zern_out,
               float *out, void *ws, tsim_stream stream);

/* Exact PSFs of Eq. (2) for n Zernike vectors:
 *   zvec : device [n][N] float32 (N the plan's n_modes; modes 4..N+1 enter
 *          the phase);  psf : device [n][T*T] float32, unit sum. */
int tsim_psf_exact(const tsim_plan *plan, int n, const float *zvec, float *psf,
                   tsim_stream stream);

/* PSF basis of Eq. (7) by PCA over a database of exact PSFs (Sec. II-C).
 * Draws n_psf Zernike vectors a = (D/r0)^{5/6} L g (g ~ N(0, I) from Philox
 * counters (i, w, 0, 1), D/r0 uniform in [dr_lo, dr_hi] from word 0 of
 * (i, 9, 0, 1)), computes their exact T x T PSFs (modes 4..36) on the device,
 * forms the FP64 Gram matrix of the PSF matrix, and returns its top-K
 * eigenvectors (the uncentred principal components), each signed so its sum
 * is non-negative (ties: largest-magnitude entry positive).  K, T and P come
 * from the plan, which need not hold a basis.  Synchronous; allocates and
 * frees its own device buffers.
 *   basis_out : host [K][T*T] float64, output (orthonormal rows)
 *   eig_out   : host [K] float64 eigenvalues, descending (may be NULL)
 * Returns TSIM_EARTEFACT if the eigen-solver does not converge. */
int tsim_basis_build(const tsim_plan *plan, int n_psf, uint64_t seed, double dr_lo, double dr_hi,
                     double *basis_out, double *eig_out);

/* ---- The learned P2S map (Sec. II-C: a small neural network maps each
 * pixel's Zernike vector to its PSF-basis weights) ----
 *
 * Network: 35 -> 256 -> 256 -> 256 -> K, exact (erf) GELU after the hidden
 * layers.  Input x_j = a_j * inv_s_j (the tilt slots Noll 2, 3 carry
 * inv_s = 0: tilt is applied by tsim_warp); output beta = s_out * y + mu.
 * Products run on BF16 matrix cores with FP32 accumulation; master weights,
 * biases, Adam moments and the loss are FP32.  Parameters are one flat FP32
 * array: for layer l = 0..3, W_l [out][in] at off_w[l] and b_l [out] at
 * off_b[l] (tsim_mlp_layout).  A tsim_mlp is not thread-safe. */
typedef struct tsim_mlp tsim_mlp;

/* Allocate a network for the plan's K with training batch `batch`;
 * weights ~ N(0, 1/fan_in) from Philox counters (i, 0, layer, 3) under key
 * `seed`, biases 0; inv_s_j = 1/sqrt(A_0[j][j] 2.75^{5/3}), mu = 0, s_out = 1. */
int tsim_mlp_create(const tsim_plan *plan, int batch, uint64_t seed, tsim_mlp **out);
int tsim_mlp_destroy(tsim_mlp *net);
int tsim_mlp_param_count(const tsim_mlp *net, size_t *count);
int tsim_mlp_layout(const tsim_mlp *net, size_t *off_w /*[4]*/, size_t *off_b /*[4]*/);

/* Copy out / in (host float32): what = 0 parameters [param_count],
 * 1 gradients of the last tsim_mlp_grad/train step [param_count] (get only),
 * 2 inv_s [35], 3 mu [K], 4 s_out [1], 5 AdamW first moments [param_count],
 * 6 AdamW second moments [param_count], 7 training counters [2] = {optimiser
 * steps taken, cosine schedule length (0: each tsim_mlp_train call spans its
 * own steps)}, whole numbers below 2^24.  Parameters, moments and counters
 * together are a training checkpoint: a network restored from them continues
 * bit-identically.  Setting what = 0 also refreshes the BF16 weight copies.
 * Synchronises the device. */
int tsim_mlp_get(const tsim_mlp *net, int what, float *host, size_t count);
int tsim_mlp_set(tsim_mlp *net, int what, const float *host, size_t count);

/* Training pairs from the exact path: n_pairs Zernike vectors a = (D/r0)^{5/6}
 * L g (Philox counters (i, w, 0, 2), D/r0 uniform in [dr_lo, dr_hi] from word
 * 0 of (i, 9, 0, 2)) and their exact projected weights (Eq. (2) + Eq. (7)).
 *   zvec : device [n_pairs][35] f32;  beta : device [n_pairs][K] f32
 *   ws   : device, tsim_mlp_data_ws_bytes(plan, n_pairs) bytes (PSFs of one
 *          chunk: at most 2^20 pairs and about 5 GB) */
int tsim_mlp_data_ws_bytes(const tsim_plan *plan, int n_pairs, size_t *bytes);
int tsim_mlp_make_data(const tsim_plan *plan, int n_pairs, uint64_t seed, float dr_lo, float dr_hi,
                       float *zvec, float *beta, void *ws, tsim_stream stream);

/* Loss (mean over batch and outputs of (y - (target - mu)/s_out)^2) and its
 * gradients for one batch, without updating.  zvec [batch][35], target
 * [batch][K] device f32; loss_host may be NULL. */
int tsim_mlp_grad(tsim_mlp *net, int batch, const float *zvec, const float *target,
                  float *loss_host, tsim_stream stream);

/* Set the output normalisation from training targets [n_pairs][K] (device):
 * mu = per-output mean, s_out = RMS deviation from mu over all outputs. */
int tsim_mlp_fit_output(tsim_mlp *net, const float *target, int n_pairs, tsim_stream stream);

/* The plan's network on n_vec Zernike vectors: zvec [n_vec][35] device f32
 * -> beta [n_vec][K] device f32 (BF16 products, FP32 accumulation). */
int tsim_mlp_predict(const tsim_plan *plan, int n_vec, const float *zvec, float *beta,
                     tsim_stream stream);

/* `steps` AdamW steps (beta1 0.9, beta2 0.999, eps 1e-8, no weight decay,
 * cosine learning rate lr_max -> lr_min) on consecutive batches of the
 * pairs (wrapping around).  Step t of the network's life (t = 0, 1, ...,
 * counted across calls) trains on pairs [t B, (t + 1) B) modulo n_pairs,
 * uses bias correction 1 - beta^(t + 1), and, with a schedule length S set
 * through tsim_mlp_set(what = 7), the rate lr_min + (lr_max - lr_min)(1 +
 * cos(pi min(t, S - 1) / (S - 1))) / 2; with S = 0 the cosine spans this
 * call's steps.  Weight-gradient partial sums are added in a fixed order, so
 * the parameters are bit-reproducible.  loss_host [steps] may be NULL. */
int tsim_mlp_train(tsim_mlp *net, const float *zvec, const float *target, int n_pairs, int steps,
                   float lr_max, float lr_min, float *loss_host, tsim_stream stream);

/* Copy the network into the plan for tsim_p2s in TSIM_P2S_LEARNED mode
 * (BF16 weights padded to the inference layout).  Must not run
 * concurrently with tsim_p2s on the plan.  In learned mode tsim_p2s writes
 * beta as float32 [F][H][W][K] in TSIM_FP32 plans and as bfloat16
 * [F][H][W][KP] (KP = K rounded up to 32, 64, 112 or 128, zero padded) in
 * TSIM_BF16 plans, the layout tsim_render then reads. */
int tsim_plan_set_mlp(tsim_plan *plan, const tsim_mlp *net);

/* Kernel tracing.  tsim_trace_enable(1) clears the counters and brackets
 * every later kernel launch of the library with two HIP events recorded on
 * the launch's stream; tsim_trace_enable(0) stops.  tsim_trace_count and
 * tsim_trace_get wait for the recorded events, then report per kernel name
 * the number of launches and their summed duration in milliseconds.  Not
 * for use while a stream is being captured into a graph. */
int tsim_trace_enable(int on);
int tsim_trace_count(int *n_kernels);
int tsim_trace_get(int index, char *name, size_t name_len, double *total_ms, int *launches);

/* Human-readable text for a status code. */
const char *tsim_status_string(int status);

/* The status of the most recent failing call on the calling thread
 * (TSIM_OK if none since the last query) and, if msg is not NULL, a
 * NUL-terminated text naming the call (at most msg_len bytes).  Reading it
 * clears it. */
int tsim_last_error(char *msg, size_t msg_len);

/* Wait for all work queued on `stream`; a device fault of an earlier
 * asynchronous launch is returned as TSIM_EDEVICE (and recorded for
 * tsim_last_error with the runtime's text). */
int tsim_sync(tsim_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* TSIM_H */
