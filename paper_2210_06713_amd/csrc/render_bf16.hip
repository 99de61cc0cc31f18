// The learned form's blur on the BF16 matrix cores (Eq. (8), evaluated in
// the reconstruct-first order sum_u (sum_k beta_k psi_k(u)) I(x - u)).
//
// Block = 8 x 16 output pixels, 4 waves; wave w owns the 32 pixels of rows
// 2w, 2w+1.  For each block of 32 taps the matrix cores form
// htilde[32 px][32 taps] = beta (BF16, rows = pixels) x psi^T (BF16), FP32
// accumulation, so every lane owns ONE tap (column) for 16 of the 32 pixels:
// it multiplies them by the image samples I(x - u) read from the LDS tile at
// compile-time offsets from a per-lane base and keeps C x 16 running sums,
// summed over the lanes once at the end.  Tap blocks are software-
// pipelined: the psi fragments of block t+2 are in flight and the products
// of block t+1 are issued while the epilogue of block t runs.
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Fragments are kept as four 32-bit words and reinterpreted only at the
// matrix-core call: copies of 8 x bf16 vectors between pipeline stages
// otherwise get split into 16-bit lanes and re-packed with byte permutes.
__device__ __forceinline__ uint4 ld_frag(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }

__device__ __forceinline__ f32x16 mfma_bf16(const uint4 &a, const uint4 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}

template <int KS, int T, int C>
__global__ void __launch_bounds__(256)
k_render_bf16(const float *__restrict__ img, const uint16_t *__restrict__ beta,
              const uint16_t *__restrict__ psi /*[ntiles*32][KS*16]*/, float *__restrict__ out,
              int H, int W) {
  constexpr int TH = 8, TW = 16, KB = KS * 16;
  constexpr int R = (T - 1) / 2;
  constexpr int SH = TH + T - 1, SW = TW + T - 1, PLANE = SH * SW;
  constexpr int NT = (T * T + 31) / 32;
  extern __shared__ float tile[];             // [C][SH][SW]
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const float *imf = img + size_t(f) * C * H * W;
  for (int e = threadIdx.x; e < C * PLANE; e += 256) {
    const int c = e / PLANE;
    const int rem = e - c * PLANE;
    const int sy = rem / SW, sx = rem - sy * SW;
    const int gy = min(max(ty0 + sy - R, 0), H - 1);
    const int gx = min(max(tx0 + sx - R, 0), W - 1);
    tile[e] = imf[(size_t(c) * H + gy) * W + gx];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pn = lane & 31, g = lane >> 5;
  // A operand: beta of pixel pn of the wave (rows 2w, 2w+1 of the block)
  uint4 b[KS];
  {
    const int py = 2 * w + (pn >> 4), px = pn & 15;
    const int y = ty0 + py, x = tx0 + px;
    const bool ok = (y < H) && (x < W);
    const uint16_t *bp = beta + ((size_t(f) * H + (ok ? y : 0)) * W + (ok ? x : 0)) * KB + 8 * g;
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = ok ? ld_frag(bp + 16 * s) : make_uint4(0u, 0u, 0u, 0u);
  }
  // B operand: psi^T column = tap pn of the 32-tap block, k-slice 8g..8g+7
  const uint16_t *prow = psi + size_t(pn) * KB + 8 * g;  // + t*32*KB
  // the lane's accumulator rows are pixels m_r + 4g, m_r = 8(r/4) + r%4: all in
  // one tile row, so pixel position = wave base + 4g + (compile-time part)
  const int pbase = (2 * w + R) * SW + R + 4 * g;
  __syncthreads();

  float sum[C][16];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[c][r] = 0.f;
  auto epilogue = [&](const f32x16 &acc, int t) {
    // this lane's tap u = 32t + pn, offset (uy - R) SW + (ux - R); padded taps carry 0
    const int u = 32 * t + pn;
    const int uy = u / T, ux = u - uy * T;
    const int lb = pbase - ((u < T * T) ? (uy - R) * SW + (ux - R) : 0);
    const float *tl = tile + lb;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = 8 * (r >> 2) + (r & 3);
      const int o = (m >> 4) * SW + (m & 15);
      const float v = acc[r];
#pragma unroll
      for (int c = 0; c < C; ++c) sum[c][r] = fmaf(v, tl[c * PLANE + o], sum[c][r]);
    }
  };
  uint4 pa[KS], pq[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) pa[s] = ld_frag(prow + 16 * s);
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll
  for (int s = 0; s < KS; ++s) acc0 = mfma_bf16(b[s], pa[s], acc0);
  if (NT > 1) {
#pragma unroll
    for (int s = 0; s < KS; ++s) pq[s] = ld_frag(prow + size_t(32) * KB + 16 * s);
  }
  for (int t = 0; t < NT; t += 2) {
    // block t+1: products (its psi was loaded an iteration earlier); block t+2: loads
    if (t + 1 < NT) {
      acc1 = f32x16{};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc1 = mfma_bf16(b[s], pq[s], acc1);
    }
    if (t + 2 < NT) {
#pragma unroll
      for (int s = 0; s < KS; ++s) pa[s] = ld_frag(prow + size_t(32 * (t + 2)) * KB + 16 * s);
    }
    epilogue(acc0, t);
    if (t + 1 < NT) {
      if (t + 2 < NT) {
        acc0 = f32x16{};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc0 = mfma_bf16(b[s], pa[s], acc0);
      }
      if (t + 3 < NT) {
#pragma unroll
        for (int s = 0; s < KS; ++s) pq[s] = ld_frag(prow + size_t(32 * (t + 3)) * KB + 16 * s);
      }
      epilogue(acc1, t + 1);
    }
  }
  // the 32 lanes of a half hold the 32 taps-columns of the same 16 pixels: sum them
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float v = sum[c][r];
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      sum[c][r] = v;
    }
  }
  // lane pn < 16 of each half writes pixel m_pn + 4g
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (pn != r) continue;
    const int m = 8 * (r >> 2) + (r & 3) + 4 * g;
    const int y = ty0 + 2 * w + (m >> 4), x = tx0 + (m & 15);
    if (y < H && x < W) {
      float *of = out + size_t(f) * C * H * W + size_t(y) * W + x;
      const size_t pl = size_t(H) * W;
#pragma unroll
      for (int c = 0; c < C; ++c) of[c * pl] = sum[c][r];
    }
  }
}

// The plain form's blur on the FP32 matrix cores (v_mfma_f32_32x32x2f32),
// same block/wave/lane layout as the BF16 kernel: htilde^T[32 taps][32 px] =
// psi x beta^T over K2 = K/2 k-steps of two.  psi2 holds, for tap n and lane
// half g, the values psi[2s + g][n] for s = 0..K2P-1 contiguously, so a lane
// streams its k-values with 16-byte loads; beta is FP32 [px][K].
template <int K2, int T>
__global__ void __launch_bounds__(256)
k_render_f32m(const float *__restrict__ img, const float *__restrict__ beta,
              const float *__restrict__ psi2 /*[ntaps][2][K2P]*/, float *__restrict__ out, int H,
              int W, int C, int K) {
  constexpr int TH = 8, TW = 16;
  constexpr int K2P = (K2 + 3) / 4 * 4;
  constexpr int R = (T - 1) / 2;
  constexpr int SH = TH + T - 1, SW = TW + T - 1, PLANE = SH * SW;
  constexpr int NT = (T * T + 31) / 32;
  extern __shared__ float tile[];
  __shared__ short offtab[NT * 32];
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const float *imf = img + size_t(f) * C * H * W;
  for (int e = threadIdx.x; e < C * PLANE; e += 256) {
    const int c = e / PLANE;
    const int rem = e - c * PLANE;
    const int sy = rem / SW, sx = rem - sy * SW;
    const int gy = min(max(ty0 + sy - R, 0), H - 1);
    const int gx = min(max(tx0 + sx - R, 0), W - 1);
    tile[e] = imf[(size_t(c) * H + gy) * W + gx];
  }
  for (int e = threadIdx.x; e < NT * 32; e += 256) {
    const int uy = e / T - R, ux = e % T - R;
    offtab[e] = (e < T * T) ? uy * SW + ux : 0;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 5, pn = lane & 31;
  const int py = 2 * w + (pn >> 4), px = pn & 15;
  const int y = ty0 + py, x = tx0 + px;
  const bool ok = (y < H) && (x < W);
  float b[K2];
  {
    const float *bp = beta + ((size_t(f) * H + (ok ? y : 0)) * W + (ok ? x : 0)) * K;
#pragma unroll
    for (int s = 0; s < K2; ++s) b[s] = (ok && 2 * s + g < K) ? bp[2 * s + g] : 0.f;
  }
  const int pbase = (py + R) * SW + px + R;
  const float *prow = psi2 + (size_t(pn) * 2 + g) * K2P;
  const size_t tstride = size_t(32) * 2 * K2P;
  const int mrow = 4 * g;
  __syncthreads();
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  f32x16 acc0 = {};
  // psi of tap block t + 1 is loaded while block t goes through the matrix cores
  float4 cur[K2P / 4], nxt[K2P / 4];
  {
    const float4 *pp = reinterpret_cast<const float4 *>(prow);
#pragma unroll
    for (int q = 0; q < K2P / 4; ++q) cur[q] = pp[q];
  }
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) {
      const float4 *pp = reinterpret_cast<const float4 *>(prow + size_t(t + 1) * tstride);
#pragma unroll
      for (int q = 0; q < K2P / 4; ++q) nxt[q] = pp[q];
    }
    acc0 = f32x16{};
#pragma unroll
    for (int q = 0; q < K2P / 4; ++q) {
      const float4 a = cur[q];
      if (4 * q + 0 < K2) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b[4 * q + 0], acc0, 0, 0, 0);
      if (4 * q + 1 < K2) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b[4 * q + 1], acc0, 0, 0, 0);
      if (4 * q + 2 < K2) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b[4 * q + 2], acc0, 0, 0, 0);
      if (4 * q + 3 < K2) acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b[4 * q + 3], acc0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < K2P / 4; ++q) cur[q] = nxt[q];
    const short *ot = offtab + 32 * t + mrow;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int idx = pbase - ot[8 * (r >> 2) + (r & 3)];
      const float v = acc0[r];
      s0 = fmaf(v, tile[idx], s0);
      if (C > 1) s1 = fmaf(v, tile[PLANE + idx], s1);
      if (C > 2) s2 = fmaf(v, tile[2 * PLANE + idx], s2);
      if (C > 3) s3 = fmaf(v, tile[3 * PLANE + idx], s3);
    }
  }
  s0 += __shfl_xor(s0, 32);
  s1 += __shfl_xor(s1, 32);
  s2 += __shfl_xor(s2, 32);
  s3 += __shfl_xor(s3, 32);
  if (lane < 32 && ok) {
    float *of = out + size_t(f) * C * H * W + size_t(y) * W + x;
    const size_t pl = size_t(H) * W;
    of[0] = s0;
    if (C > 1) of[pl] = s1;
    if (C > 2) of[2 * pl] = s2;
    if (C > 3) of[3 * pl] = s3;
  }
}

// Dynamic LDS of the image tile; tiles above 64 KB (T = 65) need the
// device's larger workgroup limit, checked here and raised on the kernel.
template <typename Kern>
int prepare_lds(Kern kern, size_t lds, int T) {
  const size_t stat = sizeof(short) * size_t((T * T + 31) / 32 * 32);
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return TSIM_EDEVICE;
  if (lds + stat > size_t(max_lds)) return TSIM_EUNSUPPORTED;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(lds)) != hipSuccess)
    return TSIM_EDEVICE;
  return TSIM_OK;
}

template <int KS, int T, int C>
int launch_ks_tc(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta, float *out,
                 hipStream_t s) {
  const int H = pl->H, W = pl->W;
  dim3 grid((W + 15) / 16, (H + 7) / 8, frames);
  const size_t lds = size_t(C) * (8 + T - 1) * (16 + T - 1) * sizeof(float);
  const int st = prepare_lds(k_render_bf16<KS, T, C>, lds, T);
  if (st != TSIM_OK) return st;
  hipLaunchKernelGGL((k_render_bf16<KS, T, C>), grid, dim3(256), lds, s, img, beta, pl->d_basis_bf, out, H, W);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

template <int KS, int T>
int launch_ks_t(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta, float *out,
                hipStream_t s) {
  switch (pl->C) {
    case 1: return launch_ks_tc<KS, T, 1>(pl, frames, img, beta, out, s);
    case 2: return launch_ks_tc<KS, T, 2>(pl, frames, img, beta, out, s);
    case 3: return launch_ks_tc<KS, T, 3>(pl, frames, img, beta, out, s);
    case 4: return launch_ks_tc<KS, T, 4>(pl, frames, img, beta, out, s);
    default: return TSIM_EUNSUPPORTED;
  }
}

template <int KS>
int launch_ks(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta, float *out,
              hipStream_t s) {
  switch (pl->T) {
    case 65: return launch_ks_t<KS, 65>(pl, frames, img, beta, out, s);
    case 33: return launch_ks_t<KS, 33>(pl, frames, img, beta, out, s);
    case 21: return launch_ks_t<KS, 21>(pl, frames, img, beta, out, s);
    case 15: return launch_ks_t<KS, 15>(pl, frames, img, beta, out, s);
    default: return TSIM_EUNSUPPORTED;
  }
}

}  // namespace

int launch_render_f32_mfma(const tsim_plan *pl, int frames, const float *img, const float *beta,
                           float *out, hipStream_t s) {
  const int H = pl->H, W = pl->W, C = pl->C, T = pl->T;
  if (!pl->d_basis_k2 || pl->K != 100 || (T != 33 && T != 65)) return TSIM_EUNSUPPORTED;
  dim3 grid((W + 15) / 16, (H + 7) / 8, frames);
  const size_t lds = size_t(C) * (8 + T - 1) * (16 + T - 1) * sizeof(float);
  const int st = T == 33 ? prepare_lds(k_render_f32m<50, 33>, lds, T) : prepare_lds(k_render_f32m<50, 65>, lds, T);
  if (st != TSIM_OK) return st;
  TraceScope tr("k_render_fp32", s);
  if (T == 33)
    hipLaunchKernelGGL((k_render_f32m<50, 33>), grid, dim3(256), lds, s, img, beta, pl->d_basis_k2, out,
                       H, W, C, pl->K);
  else
    hipLaunchKernelGGL((k_render_f32m<50, 65>), grid, dim3(256), lds, s, img, beta, pl->d_basis_k2, out,
                       H, W, C, pl->K);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

int launch_render_bf16(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta,
                       float *out, hipStream_t s) {
  if (!pl->d_basis_bf) return TSIM_EUNSUPPORTED;
  TraceScope tr("k_render_bf16", s);
  switch (pl->KP) {
    case 32: return launch_ks<2>(pl, frames, img, beta, out, s);
    case 64: return launch_ks<4>(pl, frames, img, beta, out, s);
    case 112: return launch_ks<7>(pl, frames, img, beta, out, s);
    case 128: return launch_ks<8>(pl, frames, img, beta, out, s);
    default: return TSIM_EUNSUPPORTED;
  }
}
