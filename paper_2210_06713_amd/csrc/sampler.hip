// DF-P2S Zernike-field sampler (Sec. III-A circulant sampling, Sec. III-C
// two-step generation, Eq. (9)).
//
// Pass 1 (k_sampler_cols): for field q (Noll modes 2+2q, 3+2q in its real
// and imaginary parts) and a strip of NC adjacent frequency columns kx, the
// Hermitian white noise of every bin is drawn in registers from Philox,
// coloured by the square-root spectra, and inverse-transformed along ky in
// LDS; rows y < H of the result are written to the workspace V[f][q][y][kx].
// Pass 2 (k_sampler_rows_mix): one block per output row y inverse-transforms
// V[f][q][y][:] along kx for every field, keeps columns x < W, and mixes the
// 35 unit-variance fields at each pixel with (D/r0)^{5/6} L before writing
// the 35 coefficient planes.  Only rows y < H survive pass 1 and only columns
// x < W pass 2 (crop of the top-left corner of the periodic grid).
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

using namespace tsim;

constexpr int kLdsFloat2 = 8192;  // 64 KB of complex samples per pass-1 block
constexpr int kMaxFramesPerLaunch = 64;

struct FrameScales {
  float s[kMaxFramesPerLaunch];
};

__global__ void __launch_bounds__(256)
k_sampler_cols(const float *__restrict__ sqrtS, const float2 *__restrict__ tw, float2 *__restrict__ V,
               int Gh, int Gw, int log2h, int H, int NC, uint32_t key0, uint32_t key1,
               uint32_t frame_base) {
  extern __shared__ float2 lds[];
  const int q = blockIdx.y;
  const int fl = blockIdx.z;  // frame within this launch
  const uint32_t frame = frame_base + uint32_t(fl);
  const int c0 = blockIdx.x * NC;
  const int qh = Gh / 2 + 1, qw = Gw / 2 + 1;
  const int ma = 2 * q, mb = 2 * q + 1;  // 0-based mode indices (Noll 2+2q, 3+2q)
  const bool has_b = mb < TSIM_N_MODES;
  const float rs2 = 0.70710678118654752f;

  for (int e = threadIdx.x; e < NC * Gh; e += blockDim.x) {
    const int col = e >> log2h;
    const int ky = e & (Gh - 1);
    const int kx = c0 + col;
    const int mky = (Gh - ky) & (Gh - 1);
    const int mkx = (Gw - kx) & (Gw - 1);
    const uint32_t lin = uint32_t(ky) * Gw + kx;
    const uint32_t lin_m = uint32_t(mky) * Gw + mkx;
    const uint32_t canon = lin < lin_m ? lin : lin_m;
    u32x4 r = philox4x32_10(u32x4{canon, uint32_t(q), frame, 0u}, key0, key1);
    float2 g01 = box_muller(r.x, r.y);
    float2 g23 = box_muller(r.z, r.w);
    float2 wa, wb;
    if (lin == lin_m) {
      wa = make_float2(g01.x, 0.f);
      wb = make_float2(g23.x, 0.f);
    } else {
      wa = make_float2(g01.x * rs2, g01.y * rs2);
      wb = make_float2(g23.x * rs2, g23.y * rs2);
      if (lin > lin_m) {
        wa.y = -wa.y;
        wb.y = -wb.y;
      }
    }
    const int kxq = kx < qw ? kx : Gw - kx;
    const int kyq = ky < qh ? ky : Gh - ky;
    const float sa = sqrtS[(size_t(ma) * qw + kxq) * qh + kyq];
    const float sb = has_b ? sqrtS[(size_t(mb) * qw + kxq) * qh + kyq] : 0.f;
    // U = sa Wa + i sb Wb
    float2 u = make_float2(sa * wa.x - sb * wb.y, sa * wa.y + sb * wb.x);
    lds[col * Gh + bitrev(uint32_t(ky), log2h)] = u;
  }
  __syncthreads();
  lds_fft_dit(lds, Gh, log2h, NC, Gh, tw);
  const float norm = rsqrtf(float(Gh) * float(Gw));
  float2 *Vout = V + (size_t(fl) * TSIM_FIELDS + q) * size_t(H) * Gw;
  for (int e = threadIdx.x; e < H * NC; e += blockDim.x) {
    const int y = e / NC;
    const int col = e - y * NC;
    float2 v = lds[col * Gh + y];
    Vout[size_t(y) * Gw + c0 + col] = make_float2(v.x * norm, v.y * norm);
  }
}

template <int PX, int NT>
__global__ void __launch_bounds__(NT)
k_sampler_rows_mix(const float2 *__restrict__ V, const float2 *__restrict__ tw,
                   const float *__restrict__ Lmat, float *__restrict__ zern, int Gw, int log2w,
                   int H, int W, FrameScales scales, int frame_out0) {
  extern __shared__ float2 lds[];
  const int y = blockIdx.x;
  const int fl = blockIdx.y;
  const int nthr = NT;
  float acc[TSIM_N_MODES][PX];
#pragma unroll
  for (int j = 0; j < TSIM_N_MODES; ++j)
#pragma unroll
    for (int k = 0; k < PX; ++k) acc[j][k] = 0.f;

  for (int q = 0; q < TSIM_FIELDS; ++q) {
    const float2 *row = V + ((size_t(fl) * TSIM_FIELDS + q) * H + y) * size_t(Gw);
    for (int kx = threadIdx.x; kx < Gw; kx += nthr) lds[bitrev(uint32_t(kx), log2w)] = row[kx];
    __syncthreads();
    lds_fft_dit(lds, Gw, log2w, 1, Gw, tw);
    float ya[PX], yb[PX];
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      int x = threadIdx.x + k * nthr;
      float2 z = (x < W) ? lds[x] : make_float2(0.f, 0.f);
      ya[k] = z.x;
      yb[k] = z.y;
    }
    __syncthreads();  // lds is overwritten by the next field
    // a_j += L[j][2q] ybar_{2q} + L[j][2q+1] ybar_{2q+1} (L lower triangular)
    const int ta = 2 * q, tb = 2 * q + 1;
#pragma unroll
    for (int j = 0; j < TSIM_N_MODES; ++j) {
      const float la = Lmat[j * TSIM_N_MODES + ta];
      const float lb = (tb < TSIM_N_MODES) ? Lmat[j * TSIM_N_MODES + tb] : 0.f;
#pragma unroll
      for (int k = 0; k < PX; ++k) acc[j][k] = fmaf(la, ya[k], fmaf(lb, yb[k], acc[j][k]));
    }
  }
  const float sc = scales.s[fl];
  float *out = zern + size_t(frame_out0 + fl) * TSIM_N_MODES * size_t(H) * W + size_t(y) * W;
#pragma unroll
  for (int j = 0; j < TSIM_N_MODES; ++j)
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      int x = threadIdx.x + k * nthr;
      if (x < W) out[size_t(j) * H * W + x] = acc[j][k] * sc;
    }
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

int frames_per_chunk(const tsim_plan *pl, int frames) {
  // bound the pass-1 intermediate to ~2 GB and the launch's scale table
  size_t per = size_t(TSIM_FIELDS) * pl->H * size_t(pl->Gw) * sizeof(float2);
  size_t cap = size_t(2) << 30;
  int n = int(std::max<size_t>(1, cap / per));
  n = std::min(n, kMaxFramesPerLaunch);
  return std::min(n, frames);
}

}  // namespace

size_t sampler_ws_bytes(const tsim_plan *pl, int frames) {
  if (frames < 1) return 0;
  int n = frames_per_chunk(pl, frames);
  return size_t(n) * TSIM_FIELDS * pl->H * size_t(pl->Gw) * sizeof(float2);
}

int launch_sampler(const tsim_plan *pl, int frames, const float *scale_host, uint64_t seed,
                   uint64_t frame0, float *zern, void *ws, hipStream_t s) {
  const int Gh = pl->Gh, Gw = pl->Gw, H = pl->H, W = pl->W;
  const int log2h = ilog2(Gh), log2w = ilog2(Gw);
  int NC = std::min(kLdsFloat2 / Gh, 32);
  NC = std::min(NC, Gw);
  const uint32_t key0 = uint32_t(seed & 0xffffffffu), key1 = uint32_t(seed >> 32);
  float2 *V = static_cast<float2 *>(ws);
  const int chunk = frames_per_chunk(pl, frames);
  for (int f0 = 0; f0 < frames; f0 += chunk) {
    const int nf = std::min(chunk, frames - f0);
    dim3 g1(Gw / NC, TSIM_FIELDS, nf);
    {
      TraceScope tr("k_sampler_cols", s);
      hipLaunchKernelGGL(k_sampler_cols, g1, dim3(256), size_t(NC) * Gh * sizeof(float2), s, pl->d_sqrtS,
                       pl->d_tw_h, V, Gh, Gw, log2h, H, NC, key0, key1,
                       uint32_t(frame0 + uint64_t(f0)));
    }
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
    FrameScales sc;
    for (int i = 0; i < kMaxFramesPerLaunch; ++i) sc.s[i] = 0.f;
    for (int i = 0; i < nf; ++i) sc.s[i] = scale_host[f0 + i];
    dim3 g2(H, nf);
    size_t lds = size_t(Gw) * sizeof(float2);
    TraceScope tr("k_sampler_rows_mix", s);
    if (W <= 256)
      hipLaunchKernelGGL((k_sampler_rows_mix<1, 256>), g2, dim3(256), lds, s, V, pl->d_tw_w, pl->d_L,
                         zern, Gw, log2w, H, W, sc, f0);
    else if (W <= 512)
      hipLaunchKernelGGL((k_sampler_rows_mix<2, 256>), g2, dim3(256), lds, s, V, pl->d_tw_w, pl->d_L,
                         zern, Gw, log2w, H, W, sc, f0);
    else if (W <= 1024)
      hipLaunchKernelGGL((k_sampler_rows_mix<4, 256>), g2, dim3(256), lds, s, V, pl->d_tw_w, pl->d_L,
                         zern, Gw, log2w, H, W, sc, f0);
    else
      hipLaunchKernelGGL((k_sampler_rows_mix<4, 1024>), g2, dim3(1024), lds, s, V, pl->d_tw_w, pl->d_L,
                         zern, Gw, log2w, H, W, sc, f0);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  return TSIM_OK;
}
