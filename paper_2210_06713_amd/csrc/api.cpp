// Per-frame entry points of the C ABI: argument validation, then launches.
// Every entry point records a failing status for tsim_last_error.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "internal.h"

// A captured, instantiated graph of a batch's calls (tsim_batch_create).
struct tsim_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_items = 0;
};

namespace {

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

bool frames_ok(const tsim_plan *pl, int frames) {
  return pl && frames >= 1 && frames <= 65535;  // frames index grid z
}

// (D/r0)^{5/6} per frame, the mixing scale of Eq. (9); false on a bad value
bool frame_scales(const float *d_over_r0, int frames, std::vector<float> &scale) {
  scale.resize(static_cast<size_t>(frames));
  for (int f = 0; f < frames; ++f) {
    const double v = d_over_r0[f];
    if (!(v > 0.0) || !std::isfinite(v)) return false;
    scale[f] = float(std::pow(v, 5.0 / 6.0));
  }
  return true;
}

int sample_impl(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed, uint64_t frame0,
                float *zern, void *ws, hipStream_t s) {
  if (!frames_ok(pl, frames) || !d_over_r0 || !zern || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;  // 32-bit frame counter
  std::vector<float> scale;
  if (!frame_scales(d_over_r0, frames, scale)) return TSIM_EINVAL;
  return launch_sampler(pl, frames, scale.data(), seed, frame0, zern, ws, s);
}

int stats_impl(const tsim_plan *pl, int frames, const float *zern, int max_lag, double *host_out, void *ws,
               hipStream_t s) {
  if (!frames_ok(pl, frames) || !zern || !host_out || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (max_lag < 0 || max_lag > 256 || max_lag >= pl->H || max_lag >= pl->W) return TSIM_EINVAL;
  return launch_tilt_stats(pl, frames, zern, max_lag, host_out, ws, s);
}

int sf_impl(const tsim_plan *pl, int frames, const float *zern, double *host_out, double *host_moments, void *ws,
            hipStream_t s) {
  if (!frames_ok(pl, frames) || !zern || !host_out || !ws) return TSIM_EINVAL;
  if (pl->N != TSIM_N_MODES) return TSIM_EUNSUPPORTED;   // moments and pair table of 35 modes
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  std::vector<double> C(size_t(TSIM_N_MODES) * TSIM_N_MODES);
  int st = launch_moments(pl, frames, zern, C.data(), ws, s);
  if (st != TSIM_OK) return st;
  structure_function_from_moments(C.data(), host_out);
  if (host_moments)
    for (size_t i = 0; i < C.size(); ++i) host_moments[i] = C[i];
  return TSIM_OK;
}

int sample_ar_impl(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed, uint64_t frame0,
                   float alpha, const float *zern_prev, float d_over_r0_prev, float *zern, void *ws,
                   hipStream_t s) {
  if (!frames_ok(pl, frames) || !d_over_r0 || !zern || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (!(alpha >= 0.f && alpha <= 1.f)) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;
  float sprev = 1.f;
  if (zern_prev) {
    if (!aligned(zern_prev)) return TSIM_EINVAL;
    if (!(d_over_r0_prev > 0.f) || !std::isfinite(d_over_r0_prev)) return TSIM_EINVAL;
    const size_t plane = size_t(pl->N) * pl->H * pl->W * sizeof(float);
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(zern), a1 = a0 + plane * size_t(frames);
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(zern_prev), b1 = b0 + plane;
    if (b0 < a1 && a0 < b1) return TSIM_EINVAL;  // overlap
    sprev = float(std::pow(double(d_over_r0_prev), 5.0 / 6.0));
  }
  std::vector<float> scale;
  if (!frame_scales(d_over_r0, frames, scale)) return TSIM_EINVAL;
  return launch_sampler_ar(pl, frames, scale.data(), alpha, zern_prev, sprev, seed, frame0, zern, ws, s);
}

// Mean OTF over all pixels of all frames (Sec. IV-B): the device sums
// |DFT(G)|^2 over the vectors; the host takes the inverse 64 x 64 DFT of the
// mean in FP64, moves lag 0 to index 32 and divides by the number of
// aperture samples (H(0) = 1).
int otf_impl(const tsim_plan *pl, int frames, const float *zern, int short_exposure, double *host_out, void *ws,
             hipStream_t s) {
  if (!frames_ok(pl, frames) || !zern || !host_out || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  if (short_exposure != 0 && short_exposure != 1) return TSIM_EINVAL;
  if (pl->P != 64) return TSIM_EUNSUPPORTED;
  constexpr int P = 64;
  const size_t n = size_t(frames) * pl->H * pl->W;
  double *dev_sums = reinterpret_cast<double *>(static_cast<char *>(ws) + otf_ws_bytes(pl, frames) -
                                                size_t(P) * P * sizeof(double));
  int st = launch_otf_sums(pl, frames, zern, short_exposure, ws, dev_sums, s);
  if (st != TSIM_OK) return st;
  std::vector<double> S(size_t(P) * P);
  if (hipMemcpyAsync(S.data(), dev_sums, S.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return TSIM_EDEVICE;
  int n_ap = 0;
  for (int r = -16; r < 16; ++r)
    for (int c = -16; c < 16; ++c) n_ap += (r * r + c * c < 256);
  // H[ly][lx] = (1 / P^2) sum_k mean S[ky][kx] exp(+2 pi i (ky ly + kx lx) / P), separably
  std::vector<double> cw(P), sw(P);
  for (int j = 0; j < P; ++j) {
    cw[j] = std::cos(2.0 * 3.14159265358979323846 * j / P);
    sw[j] = std::sin(2.0 * 3.14159265358979323846 * j / P);
  }
  std::vector<double> Tr(size_t(P) * P), Ti(size_t(P) * P);   // [ky][lx]
  for (int ky = 0; ky < P; ++ky)
    for (int lx = 0; lx < P; ++lx) {
      double re = 0.0, im = 0.0;
      for (int kx = 0; kx < P; ++kx) {
        const double v = S[size_t(ky) * P + kx];
        const int j = (kx * lx) % P;
        re += v * cw[j];
        im += v * sw[j];
      }
      Tr[size_t(ky) * P + lx] = re;
      Ti[size_t(ky) * P + lx] = im;
    }
  const double scale = 1.0 / (double(n) * P * P * n_ap);
  for (int ly = 0; ly < P; ++ly)
    for (int lx = 0; lx < P; ++lx) {
      double re = 0.0, im = 0.0;
      for (int ky = 0; ky < P; ++ky) {
        const int j = (ky * ly) % P;
        const double a = Tr[size_t(ky) * P + lx], b = Ti[size_t(ky) * P + lx];
        re += a * cw[j] - b * sw[j];
        im += a * sw[j] + b * cw[j];
      }
      const size_t o = size_t((ly + P / 2) % P) * P + (lx + P / 2) % P;
      host_out[o] = re * scale;
      host_out[size_t(P) * P + o] = im * scale;
    }
  return TSIM_OK;
}

// The form tsim_p2s runs: the network once one is set on a learned plan,
// else the exact pupil-FFT path (also the learned form's fallback).
int p2s_form(const tsim_plan *pl) {
  return (pl->p.p2s_mode == TSIM_P2S_LEARNED && pl->d_mlp_w && pl->d_mlp_f) ? TSIM_P2S_LEARNED : TSIM_P2S_EXACT;
}

int p2s_impl(const tsim_plan *pl, int frames, const float *zern, void *beta, void *ws, hipStream_t s) {
  if (!frames_ok(pl, frames) || !zern || !beta || !ws) return TSIM_EINVAL;
  if (!aligned(zern) || !aligned(beta) || !aligned(ws)) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  const bool bf = pl->p.precision == TSIM_BF16;
  if (p2s_form(pl) == TSIM_P2S_LEARNED)
    return launch_mlp_infer(pl, zern, pl->H * pl->W, size_t(frames) * pl->H * pl->W, beta, bf ? 1 : 0,
                            bf ? pl->KP : pl->K, s);
  return launch_p2s_exact(pl, frames, zern, beta, bf ? 1 : 0, ws, s);
}

int render_impl(const tsim_plan *pl, int frames, const float *img, const void *beta, float *out, hipStream_t s) {
  if (!frames_ok(pl, frames) || !img || !beta || !out) return TSIM_EINVAL;
  if (img == out) return TSIM_EINVAL;
  if (!aligned(img) || !aligned(beta) || !aligned(out)) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  if (pl->p.precision == TSIM_BF16)
    return launch_render_bf16(pl, frames, img, static_cast<const uint16_t *>(beta), out, s);
  // FP32 matrix cores for the instantiated shape (K = 100, T = 33 or 65), else the vector-ALU kernel
  const int st = launch_render_f32_mfma(pl, frames, img, static_cast<const float *>(beta), out, s);
  if (st != TSIM_EUNSUPPORTED) return st;
  return launch_render_fp32(pl, frames, img, static_cast<const float *>(beta), out, s);
}

int warp_impl(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out, hipStream_t s) {
  if (!frames_ok(pl, frames) || !img || !zern || !out) return TSIM_EINVAL;
  if (img == out) return TSIM_EINVAL;
  if (!aligned(img) || !aligned(zern) || !aligned(out)) return TSIM_EINVAL;
  return launch_warp(pl, frames, img, zern, out, s);
}

hipStream_t hs(tsim_stream s) { return static_cast<hipStream_t>(s); }

// One item's four calls on stream s, in the order of the path (sample, P2S,
// blur, warp), with the same checks as the individual entry points.
int batch_item_calls(const tsim_batch_item &it, uint64_t seed, hipStream_t s) {
  int st = sample_impl(it.plan, it.frames, it.d_over_r0, seed, it.frame0, it.zern, it.ws, s);
  if (st == TSIM_OK) st = p2s_impl(it.plan, it.frames, it.zern, it.beta, it.ws, s);
  if (st == TSIM_OK) st = render_impl(it.plan, it.frames, it.img, it.beta, it.blur, s);
  if (st == TSIM_OK) st = warp_impl(it.plan, it.frames, it.blur, it.zern, it.out, s);
  return st;
}

// ---- the whole path in one call, group by group of frames ----
// A group's fields, weights and blurred frames live in the workspace, so its
// size is set by the group, not by the number of frames of the call.
constexpr size_t kFrameGroupBudget = size_t(1) << 30;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t beta_px_bytes(const tsim_plan *pl) {
  return pl->p.precision == TSIM_BF16 ? size_t(pl->KP) * 2 : size_t(pl->K) * 4;
}

int frame_group_default(const tsim_plan *pl) {
  const size_t per = size_t(pl->H) * pl->W * (size_t(pl->N) * 4 + beta_px_bytes(pl) + size_t(pl->C) * 4);
  const size_t g = kFrameGroupBudget / per;
  return int(std::max<size_t>(1, std::min<size_t>(g, 65535)));
}

// workspace layout of one group: fields | weights | blurred frames | step workspace
struct FrameWs {
  float *zern;
  void *beta;
  float *blur;
  void *step;
};

size_t frame_ws_bytes(const tsim_plan *pl, int group, FrameWs *lay, void *base) {
  const size_t hw = size_t(pl->H) * pl->W;
  const size_t zb = align256(size_t(group) * pl->N * hw * 4);
  const size_t bb = align256(size_t(group) * hw * beta_px_bytes(pl));
  const size_t ib = align256(size_t(group) * pl->C * hw * 4);
  // the exact form's PSF buffer only where P2S may take the exact form (a
  // plan's network, once set, stays set)
  const size_t pb = p2s_form(pl) == TSIM_P2S_LEARNED ? 0 : p2s_ws_bytes(pl, group);
  const size_t sb = std::max(sampler_ws_bytes(pl, group), pb);
  if (lay) {
    char *c = static_cast<char *>(base);
    lay->zern = reinterpret_cast<float *>(c);
    lay->beta = c + zb;
    lay->blur = reinterpret_cast<float *>(c + zb + bb);
    lay->step = c + zb + bb + ib;
  }
  return zb + bb + ib + std::max<size_t>(sb, 256);
}

int frame_impl(const tsim_plan *pl, int frames, int group, const float *d_over_r0, uint64_t seed,
               uint64_t frame0, const float *img, float *zern_out, float *out, void *ws, hipStream_t s) {
  if (!frames_ok(pl, frames) || !frames_ok(pl, group) || !d_over_r0 || !img || !out || !ws)
    return TSIM_EINVAL;
  if (!aligned(img) || !aligned(out) || !aligned(ws) || (zern_out && !aligned(zern_out))) return TSIM_EINVAL;
  if (img == out) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;
  std::vector<float> scale;
  if (!frame_scales(d_over_r0, frames, scale)) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  if (pl->p.precision == TSIM_BF16 && !render_bf16_supported(pl->KP, pl->T, pl->C)) return TSIM_EUNSUPPORTED;
  FrameWs w{};
  frame_ws_bytes(pl, group, &w, ws);
  const size_t hw = size_t(pl->H) * pl->W;
  const size_t img_frame = size_t(pl->C) * hw, zern_frame = size_t(pl->N) * hw;
  for (int g0 = 0; g0 < frames; g0 += group) {
    const int n = std::min(group, frames - g0);
    float *zern = zern_out ? zern_out + size_t(g0) * zern_frame : w.zern;
    int st = sample_impl(pl, n, d_over_r0 + g0, seed, frame0 + uint64_t(g0), zern, w.step, s);
    if (st == TSIM_OK) st = p2s_impl(pl, n, zern, w.beta, w.step, s);
    if (st == TSIM_OK) st = render_impl(pl, n, img + size_t(g0) * img_frame, w.beta, w.blur, s);
    if (st == TSIM_OK) st = warp_impl(pl, n, w.blur, zern, out + size_t(g0) * img_frame, s);
    if (st != TSIM_OK) return st;
  }
  return TSIM_OK;
}

int batch_check(const tsim_batch_item &it) {
  const tsim_plan *pl = it.plan;
  if (!frames_ok(pl, it.frames) || !it.d_over_r0 || !it.img || !it.zern || !it.beta || !it.blur || !it.out ||
      !it.ws)
    return TSIM_EINVAL;
  if (!aligned(it.img) || !aligned(it.zern) || !aligned(it.beta) || !aligned(it.blur) || !aligned(it.out) ||
      !aligned(it.ws))
    return TSIM_EINVAL;
  if (it.img == it.blur || it.blur == it.out || it.img == it.out) return TSIM_EINVAL;
  if (it.frame0 + uint64_t(it.frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;
  for (int f = 0; f < it.frames; ++f)
    if (!(it.d_over_r0[f] > 0.f) || !std::isfinite(it.d_over_r0[f])) return TSIM_EINVAL;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  if (pl->p.precision == TSIM_BF16 && !render_bf16_supported(pl->KP, pl->T, pl->C)) return TSIM_EUNSUPPORTED;
  return TSIM_OK;
}

int batch_create_impl(const tsim_batch_item *items, int n_items, uint64_t seed, tsim_batch **out) {
  if (!out) return TSIM_EINVAL;
  *out = nullptr;
  if (!items || n_items < 1 || n_items > 4096) return TSIM_EINVAL;
  for (int i = 0; i < n_items; ++i) {
    const int st = batch_check(items[i]);
    if (st != TSIM_OK) return st;
  }
  tsim_batch *b = new (std::nothrow) tsim_batch();
  if (!b) return TSIM_ENOMEM;
  b->n_items = n_items;
  // capture on a private stream (default priority); the launchers' one-time
  // set-up (LDS limits) is not a stream operation, hence relaxed mode, and
  // launches are not traced (no event nodes in the graph)
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return TSIM_EDEVICE;
  }
  int st = TSIM_OK;
  {
    TraceQuiet quiet;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
      st = TSIM_EDEVICE;
    } else {
      for (int i = 0; i < n_items && st == TSIM_OK; ++i) st = batch_item_calls(items[i], seed, cs);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (st == TSIM_OK && (e != hipSuccess || !g)) st = TSIM_EDEVICE;
      if (g && st != TSIM_OK) (void)hipGraphDestroy(g);
      if (st == TSIM_OK) b->graph = g;
    }
  }
  (void)hipStreamDestroy(cs);
  if (st == TSIM_OK && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
    st = TSIM_EDEVICE;
  if (st != TSIM_OK) {
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return st;
  }
  *out = b;
  return TSIM_OK;
}

}  // namespace

extern "C" {

int tsim_batch_create(const tsim_batch_item *items, int n_items, uint64_t seed, tsim_batch **out) {
  return note_status("tsim_batch_create", batch_create_impl(items, n_items, seed, out));
}

int tsim_batch_launch(const tsim_batch *batch, tsim_stream stream) {
  if (!batch || !batch->exec) return note_status("tsim_batch_launch", TSIM_EINVAL);
  if (hipGraphLaunch(batch->exec, hs(stream)) != hipSuccess) return note_status("tsim_batch_launch", TSIM_EDEVICE);
  return TSIM_OK;
}

int tsim_batch_destroy(tsim_batch *batch) {
  if (!batch) return TSIM_OK;
  if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
  if (batch->graph) (void)hipGraphDestroy(batch->graph);
  delete batch;
  return TSIM_OK;
}

}  // extern "C"

namespace {

// Times each candidate launch form of the sampler's two passes on the
// caller's buffers (one warm-up, best of three, HIP events on the stream)
// and keeps the fastest in the plan; a candidate replaces the built-in form
// only if it is at least 3% faster.
int autotune_impl(tsim_plan *pl, int frames, float *zern, void *ws, hipStream_t s) {
  if (!frames_ok(pl, frames) || !zern || !ws || !aligned(zern) || !aligned(ws)) return TSIM_EINVAL;
  const int nf = sampler_chunk_frames(pl, frames);
  TraceQuiet quiet;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return TSIM_EDEVICE;
  }
  int st = TSIM_OK;
  auto time_pass = [&](int pass, float *ms) {
    st = launch_sampler_pass(pl, pass, nf, zern, ws, s);
    float best = 1e30f;
    for (int r = 0; r < 3 && st == TSIM_OK; ++r) {
      float t = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess) st = TSIM_EDEVICE;
      if (st == TSIM_OK) st = launch_sampler_pass(pl, pass, nf, zern, ws, s);
      if (st == TSIM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        st = TSIM_EDEVICE;
      best = std::min(best, t);
    }
    *ms = best;
  };
  const int nc0 = pl->tune_nc, rows0 = pl->tune_rows;
  int cand[4], n = sampler_pass1_forms(pl, cand);
  int best_nc = cand[0];
  float best_t = 0.f;
  for (int i = 0; i < n && st == TSIM_OK; ++i) {
    pl->tune_nc = cand[i];
    float t = 0.f;
    time_pass(1, &t);
    if (i == 0 || t < 0.97f * best_t) {
      best_t = t;
      best_nc = cand[i];
    }
  }
  pl->tune_nc = best_nc;
  n = sampler_pass2_forms(pl, cand);
  int best_rows = cand[0];
  for (int i = 0; i < n && st == TSIM_OK; ++i) {
    pl->tune_rows = cand[i];
    float t = 0.f;
    time_pass(2, &t);
    if (i == 0 || t < 0.97f * best_t) {
      best_t = t;
      best_rows = cand[i];
    }
  }
  pl->tune_rows = best_rows;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TSIM_OK) {
    pl->tune_nc = nc0;
    pl->tune_rows = rows0;
  }
  return st;
}

}  // namespace

extern "C" {

int tsim_plan_autotune(tsim_plan *plan, int frames, float *zern, void *ws, tsim_stream stream) {
  return note_status("tsim_plan_autotune", autotune_impl(plan, frames, zern, ws, hs(stream)));
}

int tsim_plan_set_tuning(tsim_plan *plan, int columns, int rows_form) {
  if (!plan || columns < 0 || rows_form < 0 || rows_form > 3 || !sampler_form_valid(plan, columns, rows_form))
    return note_status("tsim_plan_set_tuning", TSIM_EINVAL);
  plan->tune_nc = columns;
  plan->tune_rows = rows_form;
  return TSIM_OK;
}

int tsim_plan_tuning(const tsim_plan *plan, int *columns, int *rows_form) {
  if (!plan || !columns || !rows_form) return note_status("tsim_plan_tuning", TSIM_EINVAL);
  *columns = pass1_nc(plan);
  *rows_form = pass2_form(plan);
  return TSIM_OK;
}

int tsim_workspace_bytes(const tsim_plan *pl, int frames, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return note_status("tsim_workspace_bytes", TSIM_EINVAL);
  size_t a = sampler_ws_bytes(pl, frames);
  size_t b = p2s_ws_bytes(pl, frames);
  *bytes = a > b ? a : b;
  return TSIM_OK;
}

int tsim_sample_zernike(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed,
                        uint64_t frame0, float *zern, void *ws, tsim_stream stream) {
  return note_status("tsim_sample_zernike", sample_impl(pl, frames, d_over_r0, seed, frame0, zern, ws, hs(stream)));
}

int tsim_tilt_stats_ws_bytes(const tsim_plan *pl, int frames, int max_lag, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return note_status("tsim_tilt_stats_ws_bytes", TSIM_EINVAL);
  if (max_lag < 0 || max_lag > 256 || max_lag >= pl->H || max_lag >= pl->W)
    return note_status("tsim_tilt_stats_ws_bytes", TSIM_EINVAL);
  *bytes = tilt_stats_ws_bytes(pl, frames, max_lag);
  return TSIM_OK;
}

int tsim_tilt_stats(const tsim_plan *pl, int frames, const float *zern, int max_lag, double *host_out,
                    void *ws, tsim_stream stream) {
  return note_status("tsim_tilt_stats", stats_impl(pl, frames, zern, max_lag, host_out, ws, hs(stream)));
}

int tsim_structure_function_ws_bytes(const tsim_plan *pl, int frames, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return note_status("tsim_structure_function_ws_bytes", TSIM_EINVAL);
  *bytes = moments_ws_bytes(pl, frames);
  return TSIM_OK;
}

int tsim_structure_function(const tsim_plan *pl, int frames, const float *zern, double *host_out,
                            double *host_moments, void *ws, tsim_stream stream) {
  return note_status("tsim_structure_function",
                     sf_impl(pl, frames, zern, host_out, host_moments, ws, hs(stream)));
}

int tsim_otf_ws_bytes(const tsim_plan *pl, int frames, size_t *bytes) {
  if (!bytes || !frames_ok(pl, frames)) return note_status("tsim_otf_ws_bytes", TSIM_EINVAL);
  if (pl->P != 64) return note_status("tsim_otf_ws_bytes", TSIM_EUNSUPPORTED);
  *bytes = otf_ws_bytes(pl, frames);
  return TSIM_OK;
}

int tsim_otf(const tsim_plan *pl, int frames, const float *zern, int short_exposure, double *host_out, void *ws,
             tsim_stream stream) {
  return note_status("tsim_otf", otf_impl(pl, frames, zern, short_exposure, host_out, ws, hs(stream)));
}

int tsim_sample_zernike_ar(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed,
                           uint64_t frame0, float alpha, const float *zern_prev, float d_over_r0_prev,
                           float *zern, void *ws, tsim_stream stream) {
  return note_status("tsim_sample_zernike_ar", sample_ar_impl(pl, frames, d_over_r0, seed, frame0, alpha,
                                                              zern_prev, d_over_r0_prev, zern, ws, hs(stream)));
}

int tsim_p2s(const tsim_plan *pl, int frames, const float *zern, void *beta, void *ws, tsim_stream stream) {
  return note_status("tsim_p2s", p2s_impl(pl, frames, zern, beta, ws, hs(stream)));
}

int tsim_p2s_form(const tsim_plan *pl, int *form) {
  if (!pl || !form) return note_status("tsim_p2s_form", TSIM_EINVAL);
  *form = p2s_form(pl);
  return TSIM_OK;
}

int tsim_render(const tsim_plan *pl, int frames, const float *img, const void *beta, float *out,
                void *ws, tsim_stream stream) {
  (void)ws;
  return note_status("tsim_render", render_impl(pl, frames, img, beta, out, hs(stream)));
}

int tsim_warp(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out,
              tsim_stream stream) {
  return note_status("tsim_warp", warp_impl(pl, frames, img, zern, out, hs(stream)));
}

int tsim_plan_set_mlp(tsim_plan *pl, const tsim_mlp *net) {
  if (!pl || !net) return note_status("tsim_plan_set_mlp", TSIM_EINVAL);
  return note_status("tsim_plan_set_mlp", plan_set_mlp_impl(pl, net));
}

int tsim_frame_group(const tsim_plan *pl, int *group) {
  if (!pl || !group) return note_status("tsim_frame_group", TSIM_EINVAL);
  *group = frame_group_default(pl);
  return TSIM_OK;
}

int tsim_frame_workspace_bytes(const tsim_plan *pl, int group, size_t *bytes) {
  if (!bytes || !frames_ok(pl, group)) return note_status("tsim_frame_workspace_bytes", TSIM_EINVAL);
  *bytes = frame_ws_bytes(pl, group, nullptr, nullptr);
  return TSIM_OK;
}

int tsim_frame(const tsim_plan *pl, int frames, int group, const float *d_over_r0, uint64_t seed,
               uint64_t frame0, const float *img, float *zern_out, float *out, void *ws, tsim_stream stream) {
  return note_status("tsim_frame", frame_impl(pl, frames, group, d_over_r0, seed, frame0, img, zern_out, out, ws,
                                              hs(stream)));
}

int tsim_psf_exact(const tsim_plan *pl, int n, const float *zvec, float *psf, tsim_stream stream) {
  if (!pl || n < 1 || !zvec || !psf) return note_status("tsim_psf_exact", TSIM_EINVAL);
  if (!aligned(zvec) || !aligned(psf)) return note_status("tsim_psf_exact", TSIM_EINVAL);
  return note_status("tsim_psf_exact", launch_psf_exact(pl, n, zvec, psf, hs(stream)));
}

}  // extern "C"
