// Per-frame entry points of the C ABI: argument validation, then launches.
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace {

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

bool frames_ok(const tsim_plan *pl, int frames) {
  return pl && frames >= 1 && frames <= 65535;  // frames index grid z
}

}  // namespace

extern "C" {

int tsim_workspace_bytes(const tsim_plan *pl, int frames, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return TSIM_EINVAL;
  size_t a = sampler_ws_bytes(pl, frames);
  size_t b = p2s_ws_bytes(pl, frames);
  *bytes = a > b ? a : b;
  return TSIM_OK;
}

int tsim_sample_zernike(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed,
                        uint64_t frame0, float *zern, void *ws, tsim_stream stream) {
  if (!frames_ok(pl, frames) || !d_over_r0 || !zern || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;  // 32-bit frame counter
  std::vector<float> scale(static_cast<size_t>(frames));
  for (int f = 0; f < frames; ++f) {
    double v = d_over_r0[f];
    if (!(v > 0.0) || !std::isfinite(v)) return TSIM_EINVAL;
    scale[f] = float(std::pow(v, 5.0 / 6.0));
  }
  return launch_sampler(pl, frames, scale.data(), seed, frame0, zern, ws,
                        static_cast<hipStream_t>(stream));
}

int tsim_tilt_stats_ws_bytes(const tsim_plan *pl, int frames, int max_lag, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return TSIM_EINVAL;
  if (max_lag < 0 || max_lag > 256 || max_lag >= pl->H || max_lag >= pl->W) return TSIM_EINVAL;
  *bytes = tilt_stats_ws_bytes(pl, frames, max_lag);
  return TSIM_OK;
}

int tsim_tilt_stats(const tsim_plan *pl, int frames, const float *zern, int max_lag, double *host_out,
                    void *ws, tsim_stream stream) {
  if (!frames_ok(pl, frames) || !zern || !host_out || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (max_lag < 0 || max_lag > 256 || max_lag >= pl->H || max_lag >= pl->W) return TSIM_EINVAL;
  return launch_tilt_stats(pl, frames, zern, max_lag, host_out, ws, static_cast<hipStream_t>(stream));
}

int tsim_structure_function_ws_bytes(const tsim_plan *pl, int frames, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return TSIM_EINVAL;
  *bytes = moments_ws_bytes(pl, frames);
  return TSIM_OK;
}

int tsim_structure_function(const tsim_plan *pl, int frames, const float *zern, double *host_out,
                            double *host_moments, void *ws, tsim_stream stream) {
  if (!frames_ok(pl, frames) || !zern || !host_out || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  std::vector<double> C(size_t(TSIM_N_MODES) * TSIM_N_MODES);
  int st = launch_moments(pl, frames, zern, C.data(), ws, static_cast<hipStream_t>(stream));
  if (st != TSIM_OK) return st;
  structure_function_from_moments(C.data(), host_out);
  if (host_moments)
    for (size_t i = 0; i < C.size(); ++i) host_moments[i] = C[i];
  return TSIM_OK;
}

int tsim_sample_zernike_ar(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed,
                           uint64_t frame0, float alpha, const float *zern_prev, float d_over_r0_prev,
                           float *zern, void *ws, tsim_stream stream) {
  if (!frames_ok(pl, frames) || !d_over_r0 || !zern || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (!(alpha >= 0.f && alpha <= 1.f)) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;
  float sprev = 1.f;
  if (zern_prev) {
    if (!aligned(zern_prev)) return TSIM_EINVAL;
    if (!(d_over_r0_prev > 0.f) || !std::isfinite(d_over_r0_prev)) return TSIM_EINVAL;
    const size_t plane = size_t(TSIM_N_MODES) * pl->H * pl->W * sizeof(float);
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(zern), a1 = a0 + plane * size_t(frames);
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(zern_prev), b1 = b0 + plane;
    if (b0 < a1 && a0 < b1) return TSIM_EINVAL;  // overlap
    sprev = float(std::pow(double(d_over_r0_prev), 5.0 / 6.0));
  }
  std::vector<float> scale(static_cast<size_t>(frames));
  for (int f = 0; f < frames; ++f) {
    double v = d_over_r0[f];
    if (!(v > 0.0) || !std::isfinite(v)) return TSIM_EINVAL;
    scale[f] = float(std::pow(v, 5.0 / 6.0));
  }
  return launch_sampler_ar(pl, frames, scale.data(), alpha, zern_prev, sprev, seed, frame0, zern, ws,
                           static_cast<hipStream_t>(stream));
}

int tsim_p2s(const tsim_plan *pl, int frames, const float *zern, void *beta, void *ws,
             tsim_stream stream) {
  if (!frames_ok(pl, frames) || !zern || !beta || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(beta) || !aligned(ws)) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->p.p2s_mode == TSIM_P2S_LEARNED) {
    if (!pl->d_mlp_w) return TSIM_EARTEFACT;
    const bool bf = pl->p.precision == TSIM_BF16;
    return launch_mlp_infer(pl, zern, pl->H * pl->W, size_t(frames) * pl->H * pl->W, beta, bf ? 1 : 0,
                            bf ? pl->KP : pl->K, s);
  }
  if (pl->p.precision != TSIM_FP32) return TSIM_EUNSUPPORTED;
  return launch_p2s_exact(pl, frames, zern, static_cast<float *>(beta), ws, s);
}

int tsim_render(const tsim_plan *pl, int frames, const float *img, const void *beta, float *out,
                void *ws, tsim_stream stream) {
  (void)ws;
  if (!frames_ok(pl, frames) || !img || !beta || !out) return TSIM_EINVAL;
  if (img == out) return TSIM_EINVAL;
  if (!aligned(img) || !aligned(beta) || !aligned(out)) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  if (pl->p.precision == TSIM_BF16)
    return launch_render_bf16(pl, frames, img, static_cast<const uint16_t *>(beta), out,
                              static_cast<hipStream_t>(stream));
  // FP32 matrix cores for the instantiated shape (K = 100, T = 33), else the vector-ALU kernel
  const int st = launch_render_f32_mfma(pl, frames, img, static_cast<const float *>(beta), out,
                                        static_cast<hipStream_t>(stream));
  if (st != TSIM_EUNSUPPORTED) return st;
  return launch_render_fp32(pl, frames, img, static_cast<const float *>(beta), out,
                            static_cast<hipStream_t>(stream));
}

int tsim_warp(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out,
              tsim_stream stream) {
  if (!frames_ok(pl, frames) || !img || !zern || !out) return TSIM_EINVAL;
  if (img == out) return TSIM_EINVAL;
  if (!aligned(img) || !aligned(zern) || !aligned(out)) return TSIM_EINVAL;
  return launch_warp(pl, frames, img, zern, out, static_cast<hipStream_t>(stream));
}

int tsim_plan_set_mlp(tsim_plan *pl, const tsim_mlp *net) {
  if (!pl || !net) return TSIM_EINVAL;
  return plan_set_mlp_impl(pl, net);
}

int tsim_psf_exact(const tsim_plan *pl, int n, const float *zvec, float *psf, tsim_stream stream) {
  if (!pl || n < 1 || !zvec || !psf) return TSIM_EINVAL;
  if (!aligned(zvec) || !aligned(psf)) return TSIM_EINVAL;
  return launch_psf_exact(pl, n, zvec, psf, static_cast<hipStream_t>(stream));
}

}  // extern "C"
