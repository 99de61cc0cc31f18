// Image formation: the basis-weighted blur of Eq. (8) and the tilt warp.
//
// k_render_fp32: one thread per output pixel of a 16 x 16 tile.  The image
// tile with its (T-1)/2 halo (borders replicated) sits in LDS for every
// channel; the pixel's K weights sit in registers.  For each tap u the
// reconstructed PSF value h(u) = sum_k beta_k psi_k(u) is formed once and
// applied to all channels, so the sum of Eq. (8) is evaluated in the
// reconstruct-first order, sum_u (sum_k beta_k psi_k(u)) I(x - u), which is
// the same quantity with about C times fewer multiply-adds.
//
// k_warp: out(x) = bilinear(img, x - t_x), t_x = -(4/pi)(a_2, a_3).
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

constexpr int kTile = 16;

template <int KP>
__global__ void __launch_bounds__(256)
k_render_fp32(const float *__restrict__ img, const float *__restrict__ beta,
              const float *__restrict__ psi_t /*[T*T][KP]*/, float *__restrict__ out, int H, int W,
              int C, int T, int K) {
  extern __shared__ float tile[];  // [C][S][S], S = kTile + T - 1
  const int r = (T - 1) / 2;
  const int S = kTile + T - 1;
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * kTile, tx0 = blockIdx.x * kTile;
  const float *imf = img + size_t(f) * C * H * W;
  for (int e = threadIdx.x; e < C * S * S; e += blockDim.x) {
    int c = e / (S * S);
    int rem = e - c * S * S;
    int sy = rem / S, sx = rem - sy * S;
    int gy = min(max(ty0 + sy - r, 0), H - 1);
    int gx = min(max(tx0 + sx - r, 0), W - 1);
    tile[e] = imf[(size_t(c) * H + gy) * W + gx];
  }
  const int ly = threadIdx.x / kTile, lx = threadIdx.x % kTile;
  const int y = ty0 + ly, x = tx0 + lx;
  const bool valid = (y < H) && (x < W);
  float b[KP];
  const float *bp = beta + ((size_t(f) * H + (valid ? y : 0)) * W + (valid ? x : 0)) * K;
#pragma unroll
  for (int k = 0; k < KP; ++k) b[k] = (k < K) ? bp[k] : 0.f;
  __syncthreads();
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int uy = -r; uy <= r; ++uy) {
    // offset u = (ux, uy) reads img(x - u): tile index (ly + r - uy, lx + r - ux)
    const int rowb = (ly + r - uy) * S + lx + r;
    const float *pt = psi_t + size_t((uy + r) * T) * KP;
    for (int ux = -r; ux <= r; ++ux, pt += KP) {
      float h = 0.f;
#pragma unroll
      for (int k = 0; k < KP; ++k) h = fmaf(b[k], pt[k], h);
      const int idx = rowb - ux;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < C) acc[c] = fmaf(h, tile[c * S * S + idx], acc[c]);
    }
  }
  if (valid) {
    float *o = out + size_t(f) * C * H * W;
    for (int c = 0; c < C; ++c) o[(size_t(c) * H + y) * W + x] = acc[c];
  }
}

__global__ void __launch_bounds__(256)
k_warp(const float *__restrict__ img, const float *__restrict__ zern, float *__restrict__ out,
       int H, int W, int C, int nmodes, int tiles_x, int tiles_y, int n_tiles) {
  // Tiles of 64 x 4 pixels, so the source rows a tile reads (its own rows
  // shifted by the local tilt) are shared within the block; workgroups go to
  // the 8 XCDs in turn, so XCD k is given the contiguous band of tiles
  // [k n / 8, (k + 1) n / 8) (rows of tiles, frame by frame) and neighbouring
  // tiles read their common source rows through one L2.
  const int band = (n_tiles + 7) / 8;
  const int t = int(blockIdx.x % 8u) * band + int(blockIdx.x / 8u);
  if (t >= n_tiles) return;
  const int per_frame = tiles_x * tiles_y;
  const int f = t / per_frame, tr = t - f * per_frame;
  const int y = (tr / tiles_x) * 4 + int(threadIdx.x >> 6);
  const int x = (tr % tiles_x) * 64 + int(threadIdx.x & 63);
  if (x >= W || y >= H) return;
  const size_t plane = size_t(H) * W;
  const float *zf = zern + size_t(f) * nmodes * plane;
  const float k = -1.27323954473516268f;  // -4/pi pixels per radian of tilt
  const float tx = k * zf[size_t(y) * W + x];
  const float ty = k * zf[plane + size_t(y) * W + x];
  // sample point x - t = (x - floor(t) - 1) + (1 - frac(t)): the integer part
  // is exact and the fraction keeps the precision of t itself, which
  // float(x) - t would lose at large x (ulp 2^-12 at x ~ 4000)
  const float tix = floorf(tx), tiy = floorf(ty);
  float fx = 1.f - (tx - tix), fy = 1.f - (ty - tiy);  // in (0, 1]
  // clamp in float first so huge displacements cannot overflow the int cast;
  // beyond +-(size + 2) both taps sit on the border whatever the fraction
  int x0 = x - int(fminf(fmaxf(tix, -float(W) - 2.f), float(W) + 2.f)) - 1;
  int y0 = y - int(fminf(fmaxf(tiy, -float(H) - 2.f), float(H) + 2.f)) - 1;
  if (fx >= 1.f) {
    fx -= 1.f;
    x0 += 1;
  }
  if (fy >= 1.f) {
    fy -= 1.f;
    y0 += 1;
  }
  const int x0c = min(max(x0, 0), W - 1), x1c = min(max(x0 + 1, 0), W - 1);
  const int y0c = min(max(y0, 0), H - 1), y1c = min(max(y0 + 1, 0), H - 1);
  const float *imf = img + size_t(f) * C * plane;
  float *of = out + size_t(f) * C * plane;
  for (int c = 0; c < C; ++c) {
    const float *p = imf + size_t(c) * plane;
    float v00 = p[size_t(y0c) * W + x0c], v01 = p[size_t(y0c) * W + x1c];
    float v10 = p[size_t(y1c) * W + x0c], v11 = p[size_t(y1c) * W + x1c];
    float top = fmaf(fx, v01 - v00, v00);
    float bot = fmaf(fx, v11 - v10, v10);
    of[size_t(c) * plane + size_t(y) * W + x] = fmaf(fy, bot - top, top);
  }
}

}  // namespace

// The image tile takes C (16 + T - 1)^2 floats of LDS: up to 100 KB (T = 65,
// C = 4), beyond the default 64 KB of dynamic LDS, so the kernel's limit is
// raised to the tile's size (gfx950 allows 160 KB per block).
template <int KP>
int launch_fp32_kp(const tsim_plan *pl, int frames, const float *img, const float *beta, float *out,
                   size_t lds, hipStream_t s) {
  const int H = pl->H, W = pl->W, C = pl->C, T = pl->T, K = pl->K;
  if (lds > 64 * 1024) {
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return TSIM_EDEVICE;
    if (lds > size_t(max_lds)) return TSIM_EUNSUPPORTED;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_render_fp32<KP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
      return TSIM_EDEVICE;
  }
  dim3 grid((W + kTile - 1) / kTile, (H + kTile - 1) / kTile, frames);
  hipLaunchKernelGGL(k_render_fp32<KP>, grid, dim3(256), lds, s, img, beta, pl->d_basis_t, out, H, W, C, T, K);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

int launch_render_fp32(const tsim_plan *pl, int frames, const float *img, const float *beta,
                       float *out, hipStream_t s) {
  const int S = kTile + pl->T - 1;
  const size_t lds = size_t(pl->C) * S * S * sizeof(float);
  TraceScope tr("k_render_fp32", s);
  switch (pl->KP) {
    case 32: return launch_fp32_kp<32>(pl, frames, img, beta, out, lds, s);
    case 64: return launch_fp32_kp<64>(pl, frames, img, beta, out, lds, s);
    case 112: return launch_fp32_kp<112>(pl, frames, img, beta, out, lds, s);
    default: return launch_fp32_kp<128>(pl, frames, img, beta, out, lds, s);
  }
}

int launch_warp(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out,
                hipStream_t s) {
  const int tiles_x = (pl->W + 63) / 64, tiles_y = (pl->H + 3) / 4;
  const size_t n_tiles = size_t(tiles_x) * tiles_y * size_t(frames);
  if (n_tiles > size_t(1) << 30) return TSIM_EUNSUPPORTED;
  const unsigned blocks = unsigned((n_tiles + 7) / 8 * 8);
  TraceScope tr("k_warp", s);
  hipLaunchKernelGGL(k_warp, dim3(blocks), dim3(256), 0, s, img, zern, out, pl->H, pl->W, pl->C, pl->N, tiles_x,
                     tiles_y, int(n_tiles));
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
