// Field sampling without any allocation: tsim_sample_zernike_noalloc runs
// the same two sampler passes as tsim_sample_zernike (Sec. III-A circulant
// sampling, Sec. III-C two-step generation, Eq. (9)), with the pass-1
// intermediate in a fixed device array of this library instead of a caller
// workspace.  For callers that cannot allocate device memory (code under
// graph capture, serving loops).
//
// The array's device address is looked up once per device, with that device
// current, at plan creation (noalloc_scratch_init); host code uses only that
// address.  Frames are processed in chunks whose intermediate fits the
// array, so any frame count works as long as one frame's intermediate
// (fields * H * Gw * 8 bytes, fields = ceil(n_modes / 2)) fits in kScratchBytes.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace {

// TSIM_NOALLOC_SCRATCH_BYTES = 256 MiB: one 768 x 1024 frame on a
// 2048-wide grid (226 MB), three 512 x 512 frames on a 1024-wide grid, 14
// frames of 256 x 256 on a 512-wide grid per chunk.
constexpr size_t kScratchBytes = TSIM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr int kMaxChunkFrames = 64;  // the sampler's per-launch frame table

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

int scratch_for_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TSIM_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return TSIM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TSIM_EDEVICE;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TSIM_OK;
}

int sample_noalloc_impl(const tsim_plan *pl, int frames, const float *d_over_r0, uint64_t seed,
                        uint64_t frame0, float *zern, hipStream_t s) {
  if (!pl || frames < 1 || frames > 65535 || !d_over_r0 || !zern) return TSIM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(zern) & 255u) != 0) return TSIM_EINVAL;
  if (frame0 + uint64_t(frames) > (uint64_t(1) << 32)) return TSIM_EINVAL;
  const size_t per_frame = size_t(pl->NF) * pl->H * size_t(pl->Gw) * 2 * sizeof(float);
  if (per_frame > kScratchBytes) {
    note_detail("one frame's intermediate exceeds the fixed scratch array (TSIM_NOALLOC_SCRATCH_BYTES)");
    return TSIM_EUNSUPPORTED;
  }
  // every frame's scale is checked before the first launch
  for (int f = 0; f < frames; ++f) {
    const double v = d_over_r0[f];
    if (!(v > 0.0) || !std::isfinite(v)) return TSIM_EINVAL;
  }
  void *ws = nullptr;
  int st = scratch_for_current_device(&ws);
  if (st != TSIM_OK) return st;
  TraceQuiet quiet;  // tracing would create timing events
  int chunk = int(std::min<size_t>(kScratchBytes / per_frame, size_t(kMaxChunkFrames)));
  const size_t plane = size_t(pl->N) * pl->H * pl->W;
  float scale[kMaxChunkFrames];
  for (int f0 = 0; f0 < frames; f0 += chunk) {
    const int nf = std::min(chunk, frames - f0);
    for (int i = 0; i < nf; ++i) scale[i] = float(std::pow(double(d_over_r0[f0 + i]), 5.0 / 6.0));
    // pass 1 writes every row y < H of every slot of the intermediate before
    // pass 2 reads it, so the array's previous contents never matter
    st = launch_sampler(pl, nf, scale, seed, frame0 + uint64_t(f0), zern + size_t(f0) * plane, ws, s);
    if (st != TSIM_OK) return st;
  }
  return TSIM_OK;
}

}  // namespace

int noalloc_scratch_init() {
  void *p = nullptr;
  return scratch_for_current_device(&p);
}

extern "C" {

int tsim_sample_zernike_noalloc(const tsim_plan *plan, int frames, const float *d_over_r0, uint64_t seed,
                                uint64_t frame0, float *zern, tsim_stream stream) {
  return note_status("tsim_sample_zernike_noalloc",
                     sample_noalloc_impl(plan, frames, d_over_r0, seed, frame0, zern,
                                         static_cast<hipStream_t>(stream)));
}

}  // extern "C"
