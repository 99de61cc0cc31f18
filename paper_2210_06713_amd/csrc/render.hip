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
       int H, int W, int C) {
  const int f = blockIdx.z;
  const int y = blockIdx.y;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= W) return;
  const size_t plane = size_t(H) * W;
  const float *zf = zern + size_t(f) * TSIM_N_MODES * plane;
  const float k = -1.27323954473516268f;  // -4/pi pixels per radian of tilt
  const float tx = k * zf[size_t(y) * W + x];
  const float ty = k * zf[plane + size_t(y) * W + x];
  const float px = float(x) - tx, py = float(y) - ty;
  const float fx0 = floorf(px), fy0 = floorf(py);
  const float fx = px - fx0, fy = py - fy0;
  // clamp in float first so huge displacements cannot overflow the int cast
  const int x0 = int(fminf(fmaxf(fx0, -1.f), float(W)));
  const int y0 = int(fminf(fmaxf(fy0, -1.f), float(H)));
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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 ld_bf8(const uint16_t *p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

// k_render_bf16: the learned form's blur.  Block = 8 x 16 output pixels,
// wave w owns rows 2w and 2w+1 (32 pixels = one MFMA row block).  For each
// block of 32 taps the matrix cores form htilde[32 px][32 taps] = beta (BF16)
// x psi (BF16) with FP32 accumulation; each lane then multiplies its 16
// (pixel, tap) values by the image samples I(x - u) from LDS and keeps
// per-pixel partial sums; a 32-lane reduction finishes the tap sum.  The psi
// tap tiles are staged through double-buffered LDS shared by the 4 waves.
template <int KS>
__global__ void __launch_bounds__(256)
k_render_bf16(const float *__restrict__ img, const uint16_t *__restrict__ beta,
              const uint16_t *__restrict__ psi /*[ntiles*32][KS*16]*/, float *__restrict__ out,
              int H, int W, int C, int T, int ntiles) {
  constexpr int TH = 8, TW = 16, KB = KS * 16, PLD = KB + 8;  // padded psi rows (bank spread)
  __shared__ __attribute__((aligned(16))) uint16_t ps[2][32 * PLD];
  extern __shared__ float tile[];
  const int R = (T - 1) / 2;
  const int SH = TH + T - 1, SW = TW + T - 1;
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const float *imf = img + size_t(f) * C * H * W;
  for (int e = threadIdx.x; e < C * SH * SW; e += blockDim.x) {
    const int c = e / (SH * SW);
    const int rem = e - c * SH * SW;
    const int sy = rem / SW, sx = rem - sy * SW;
    const int gy = min(max(ty0 + sy - R, 0), H - 1);
    const int gx = min(max(tx0 + sx - R, 0), W - 1);
    tile[e] = imf[(size_t(c) * H + gy) * W + gx];
  }
  // stage psi tile 0: 32 rows x KB bf16 = 32 * KS * 2 chunks of 16 B
  auto stage = [&](int t, int buf) {
    for (int e = threadIdx.x; e < 32 * KS * 2; e += 256) {
      const int row = e / (KS * 2), ch = e - row * (KS * 2);
      *reinterpret_cast<uint4 *>(&ps[buf][row * PLD + ch * 8]) =
          *reinterpret_cast<const uint4 *>(psi + size_t(32 * t + row) * KB + ch * 8);
    }
  };
  stage(0, 0);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bf16x8 a[KS];
  {
    const int m = lane & 31;
    const int y = ty0 + 2 * w + (m >> 4), x = tx0 + (m & 15);
    const bool ok = (y < H) && (x < W);
    const uint16_t *bp = beta + ((size_t(f) * H + (ok ? y : 0)) * W + (ok ? x : 0)) * KB + 8 * (lane >> 5);
#pragma unroll
    for (int s = 0; s < KS; ++s) a[s] = ok ? ld_bf8(bp + 16 * s) : bf16x8{};
  }
  int base[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    base[r] = (2 * w + (m >> 4) + R) * SW + (m & 15) + R;
  }
  float sum[16][4];
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) sum[r][c] = 0.f;
  __syncthreads();
  const int plane = SH * SW;
  for (int t = 0; t < ntiles; ++t) {
    const int cur = t & 1;
    if (t + 1 < ntiles) stage(t + 1, cur ^ 1);
    f32x16 acc = {};
    const uint16_t *pp = &ps[cur][(lane & 31) * PLD + 8 * (lane >> 5)];
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[s], ld_bf8(pp + 16 * s), acc, 0, 0, 0);
    const int n = 32 * t + (lane & 31);
    const int nn = n < T * T ? n : 0;  // padded taps carry psi = 0
    const int uy = nn / T - R, ux = nn - (nn / T) * T - R;
    const int off = uy * SW + ux;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int idx = base[r] - off;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < C) sum[r][c] = fmaf(acc[r], tile[c * plane + idx], sum[r][c]);
    }
    __syncthreads();  // tile t+1 staged; everyone done with tile t's buffer
  }
  // reduce over the 32 lanes that hold the same pixel rows
#pragma unroll
  for (int r = 0; r < 16; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c >= C) continue;
      float v = sum[r][c];
#pragma unroll
      for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o);
      sum[r][c] = v;
    }
  if ((lane & 31) == 0) {
    float *of = out + size_t(f) * C * H * W;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int y = ty0 + 2 * w + (m >> 4), x = tx0 + (m & 15);
      if (y < H && x < W)
        for (int c = 0; c < C; ++c) of[(size_t(c) * H + y) * W + x] = sum[r][c];
    }
  }
}

}  // namespace

int launch_render_fp32(const tsim_plan *pl, int frames, const float *img, const float *beta,
                       float *out, hipStream_t s) {
  const int H = pl->H, W = pl->W, C = pl->C, T = pl->T, K = pl->K;
  const int S = kTile + T - 1;
  size_t lds = size_t(C) * S * S * sizeof(float);
  if (lds > 64 * 1024) return TSIM_EUNSUPPORTED;
  dim3 grid((W + kTile - 1) / kTile, (H + kTile - 1) / kTile, frames);
  const int KP = pl->KP;
  TraceScope tr("k_render_fp32", s);
  if (KP == 32)
    hipLaunchKernelGGL(k_render_fp32<32>, grid, dim3(256), lds, s, img, beta, pl->d_basis_t, out, H, W, C, T, K);
  else if (KP == 64)
    hipLaunchKernelGGL(k_render_fp32<64>, grid, dim3(256), lds, s, img, beta, pl->d_basis_t, out, H, W, C, T, K);
  else if (KP == 112)
    hipLaunchKernelGGL(k_render_fp32<112>, grid, dim3(256), lds, s, img, beta, pl->d_basis_t, out, H, W, C, T, K);
  else
    hipLaunchKernelGGL(k_render_fp32<128>, grid, dim3(256), lds, s, img, beta, pl->d_basis_t, out, H, W, C, T, K);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

int launch_warp(const tsim_plan *pl, int frames, const float *img, const float *zern, float *out,
                hipStream_t s) {
  dim3 grid((pl->W + 255) / 256, pl->H, frames);
  TraceScope tr("k_warp", s);
  hipLaunchKernelGGL(k_warp, grid, dim3(256), 0, s, img, zern, out, pl->H, pl->W, pl->C);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

int launch_render_bf16(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta,
                       float *out, hipStream_t s) {
  const int H = pl->H, W = pl->W, C = pl->C, T = pl->T;
  const int SH = 8 + T - 1, SW = 16 + T - 1;
  size_t lds = size_t(C) * SH * SW * sizeof(float);
  if (lds > 64 * 1024 || !pl->d_basis_bf) return TSIM_EUNSUPPORTED;
  dim3 grid((W + 15) / 16, (H + 7) / 8, frames);
  const int ntiles = (T * T + 31) / 32;
  TraceScope tr("k_render_bf16", s);
  switch (pl->KP) {
    case 32: hipLaunchKernelGGL(k_render_bf16<2>, grid, dim3(256), lds, s, img, beta, pl->d_basis_bf, out, H, W, C, T, ntiles); break;
    case 64: hipLaunchKernelGGL(k_render_bf16<4>, grid, dim3(256), lds, s, img, beta, pl->d_basis_bf, out, H, W, C, T, ntiles); break;
    case 112: hipLaunchKernelGGL(k_render_bf16<7>, grid, dim3(256), lds, s, img, beta, pl->d_basis_bf, out, H, W, C, T, ntiles); break;
    case 128: hipLaunchKernelGGL(k_render_bf16<8>, grid, dim3(256), lds, s, img, beta, pl->d_basis_bf, out, H, W, C, T, ntiles); break;
    default: return TSIM_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
