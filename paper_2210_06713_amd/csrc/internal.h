// Internal declarations shared by the host plan builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/tsim.h"

#define TSIM_FIELDS 18        // complex fields carrying the 35 real modes (the default plan)
constexpr int kMaxModes = TSIM_MAX_MODES;   // Noll 2..66
// mode counts a plan takes: complete radial orders up to 7, 8, 9, 10
constexpr bool modes_supported(int n) { return n == 35 || n == 44 || n == 54 || n == 65; }
// Chebyshev terms per axis of the pupil phase series: the modes' highest
// radial order plus one (8 for Noll 2..36, 11 otherwise)
constexpr int cheb_terms(int n) { return n == 35 ? 8 : 11; }
#define TSIM_PSF_MODE0 2      // first mode index (0-based, Noll 4) inside the PSF

constexpr int kProjectTile = 128;  // pixels per projection block (P2S chunks are multiples)

struct tsim_plan {
  tsim_params p;
  double ds;                   // pixel pitch over D
  int Gh, Gw, H, W, C, P, T, K;
  int N, NF, NCH;              // modes (Noll 2..N+1), complex sampler fields, Chebyshev terms
  int KP;                      // K padded to 32, 64, 112 or 128
  // host FP64 copies (for tsim_plan_table)
  std::vector<double> A0;      // [N][N] at D/r0 = 1
  std::vector<double> L;       // [N][N] lower
  std::vector<double> sqrtS;   // [N][Gw/2+1][Gh/2+1]
  std::vector<double> subh;    // [2][4][4] subharmonic wave amplitudes (tilt modes)
  std::vector<double> basis;   // [K][T*T]
  // device tables
  float *d_sqrtS = nullptr;    // [N][Gw/2+1][Gh/2+1] float32
  float2 *d_tw_h = nullptr;    // twiddles exp(+2 pi i k / Gh), k < Gh/2
  float2 *d_tw_w = nullptr;    // twiddles exp(+2 pi i k / Gw), k < Gw/2
  float *d_L = nullptr;        // [N][N] float32 lower
  float *d_zcheb = nullptr;    // [N-2][NCH][NCH] 2D Chebyshev coefficients of modes 4..N+1 over the aperture
  float *d_basis = nullptr;    // [K][T*T] float32
  float *d_basis_t = nullptr;  // [T*T][KP] float32 (tap-major, zero padded)
  uint16_t *d_basis_bf = nullptr;  // [groups of 32 tap pairs][2][32][KP + 8] bfloat16, zero padded
  uint16_t *d_basis_h3 = nullptr;  // basis x 2^10 as FP16 (hi, lo) pairs in matrix-core fragment order:
                                   // [ceil(T*T/32)][2][ceil(KP/32)][64][2][8] (projection)
  uint16_t *d_basis_h3r = nullptr;  // basis x 2^10 as FP16 (hi, lo) in fragment order for the plain blur:
                                    // [ceil(T*T/32)][KP/16][2][64][8]
  // sampler launch forms (0 = the built-in choice): pass-1 columns per
  // block, pass-2 form (1 = two rows per 256-thread block, 2 = the same
  // with twice the columns per thread, 3 = one row per 1024-thread block);
  // set by tsim_plan_autotune / tsim_plan_set_tuning
  int tune_nc = 0, tune_rows = 0;
  uint16_t *d_mlp_w = nullptr;     // packed BF16 network weights (inference layout)
  float *d_mlp_f = nullptr;        // biases, input scales, output means (FP32)
  float mlp_s_out = 1.f;
};

struct tsim_mlp;

// Brackets one kernel launch with timing events when tracing is enabled.
class TraceScope {
 public:
  TraceScope(const char *name, hipStream_t s);
  ~TraceScope();
  TraceScope(const TraceScope &) = delete;
  TraceScope &operator=(const TraceScope &) = delete;

 private:
  hipStream_t s_;
  int slot_;
};

// Launches on the calling thread are not traced while one is alive (for
// calls that must create no events).
class TraceQuiet {
 public:
  TraceQuiet();
  ~TraceQuiet();
  TraceQuiet(const TraceQuiet &) = delete;
  TraceQuiet &operator=(const TraceQuiet &) = delete;
};

// ---- launchers (sampler.hip) ----
int launch_sampler(const tsim_plan *pl, int frames, const float *scale_host, uint64_t seed,
                   uint64_t frame0, float *zern, void *ws, hipStream_t s);
size_t sampler_ws_bytes(const tsim_plan *pl, int frames);
// the sampler's candidate launch forms for the plan's shape (built-in
// choice first); out arrays of at least 4 entries, returns the count
int sampler_pass1_forms(const tsim_plan *pl, int *nc);
int sampler_pass2_forms(const tsim_plan *pl, int *form);
// one pass of the sampler alone with a given form, for timing (frames <=
// one chunk, ws as for tsim_sample_zernike, zern of frames frames)
int launch_sampler_pass(const tsim_plan *pl, int pass, int frames, float *zern, void *ws, hipStream_t s);
bool sampler_form_valid(const tsim_plan *pl, int nc, int rows);
int pass1_nc(const tsim_plan *pl);    // effective pass-1 columns per block
int pass2_form(const tsim_plan *pl);  // effective pass-2 form (1, 2, 3)
int sampler_chunk_frames(const tsim_plan *pl, int frames);  // frames per pass-1 launch
int launch_sampler_ar(const tsim_plan *pl, int frames, const float *scale_host, float alpha,
                      const float *zern_prev, float scale_prev, uint64_t seed, uint64_t frame0,
                      float *zern, void *ws, hipStream_t s);

// ---- allocation-free sampling (noalloc.hip): looks up the device address
// of the library's fixed scratch array for the current device, once ----
int noalloc_scratch_init();

// ---- launchers (stats.hip) ----
size_t tilt_stats_ws_bytes(const tsim_plan *pl, int frames, int max_lag);
int launch_tilt_stats(const tsim_plan *pl, int frames, const float *zern, int max_lag, double *host_out,
                      void *ws, hipStream_t s);
size_t moments_ws_bytes(const tsim_plan *pl, int frames);
// mean a_j a_k over all pixels and frames, host [35][35] float64
int launch_moments(const tsim_plan *pl, int frames, const float *zern, double *host_out, void *ws,
                   hipStream_t s);

// sum over rows of part[rows][n_out] in FP64, in a fixed order, into the
// device array out[n_out]
int launch_partial_sum(const float *part, size_t rows, int n_out, double *out, hipStream_t s);

// ---- optical transfer functions (psf.hip): the sums over all pixels of
// all frames of |DFT(P exp(-i phi))|^2 on the 64 x 64 pupil grid, into the
// device array dev_sums[64][64] (DFT order, kx fastest); workspace of
// otf_ws_bytes (the sums' array may be its tail) ----
size_t otf_ws_bytes(const tsim_plan *pl, int frames);
int launch_otf_sums(const tsim_plan *pl, int frames, const float *zern, int short_exposure, void *ws,
                    double *dev_sums, hipStream_t s);

// ---- structure function (plan.cpp, host) ----
constexpr int kSfPupil = 64;            // pupil grid: aperture 32 samples across
constexpr int kSfLags = kSfPupil / 2 - 1;  // separations r = 0..30 samples
void structure_function_from_moments(const double *C, double *out);

// ---- launchers (psf.hip) ----
int launch_psf_exact(const tsim_plan *pl, int n, const float *zvec, float *psf, hipStream_t s);
// beta: float32 [pixels][K], or with out_bf16 bfloat16 [pixels][KP] (zero padded)
int launch_p2s_exact(const tsim_plan *pl, int frames, const float *zern, void *beta, int out_bf16, void *ws,
                     hipStream_t s);
size_t p2s_ws_bytes(const tsim_plan *pl, int frames);
size_t p2s_chunk_pixels(const tsim_plan *pl, size_t total);

// ---- launchers (project.hip) ----
int launch_project(const tsim_plan *pl, const float *h, int n, void *beta, int out_bf16, hipStream_t s);

// ---- launchers (mlp.hip) ----
int plan_set_mlp_impl(tsim_plan *pl, const tsim_mlp *n);
int launch_mlp_infer(const tsim_plan *pl, const float *zern, int hw, size_t n_pix, void *beta,
                     int out_bf16, int kb, hipStream_t s);

// ---- launchers (render.hip) ----
int launch_render_fp32(const tsim_plan *pl, int frames, const float *img, const float *beta,
                       float *out, hipStream_t s);
int launch_render_bf16(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta,
                       float *out, hipStream_t s);
int launch_render_f32_mfma(const tsim_plan *pl, int frames, const float *img, const float *beta,
                           float *out, hipStream_t s);
// shapes the BF16 blur is built for: T in {15, 21, 33, 65} and an image
// tile plus basis staging that fit the LDS (all but KP = 128, C = 4, T = 65)
bool render_bf16_supported(int KP, int T, int C);
// PSF supports the exact-PSF kernels are built for: P = 64 with T in {9, 15,
// 21, 31, 33} and P = 128 with T in {33, 65} for 35 modes; T = 33 (P = 64)
// and T in {33, 65} (P = 128) for more
bool psf_size_supported(int P, int T, int n_modes);
int launch_warp(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out,
                hipStream_t s);

// ---- status of the C ABI (status.cpp): records a failing call's status
// and name for tsim_last_error, returns st unchanged ----
int note_status(const char *fn, int st);
// a reason for the status the next note_status records (a string literal)
void note_detail(const char *why);

#define TSIM_HIP_CHECK(expr)                 \
  do {                                       \
    if ((expr) != hipSuccess) return TSIM_EDEVICE; \
  } while (0)
