// Exact per-pixel PSFs (Eq. (2)) and their projection on the PSF basis
// (Eq. (7)): the plain form of the phase-to-space step.
//
// k_psf64 (pupil P = 64, aperture diameter 32 samples, crop T <= 33):
// 32 lanes (half a wavefront) own one pixel.  The pupil function
// P(xi) exp(-i phi(xi)) is non-zero only on the 31 x 31 window around the
// pupil centre, and only the 33 x 33 lowest frequencies of the 64 x 64 DFT are
// kept, so the DFT is pruned on both sides: a 64-point DFT of 32 samples at
// 33 frequencies splits into the 32-point DFTs of x[c] (even frequencies)
// and x[c] exp(-2 pi i c/64) (odd frequencies).  Stage 1: lane = pupil row,
// two register FFT-32s along x.  Stage 2 (after an LDS transpose): lane =
// frequency column, two FFT-32s along y; the 33rd column is a direct
// 32-term DFT shared by the lanes.  |.|^2, unit-sum normalisation, write.
//
// k_psf128 (pupil P = 128, crop T <= 65): the same pruned DFT with one
// wavefront per pixel and register FFT-64s; see the kernel.
//
// The projection of these PSFs on the basis (Eq. (7)) is in project.hip.
#include <algorithm>

#include "common.cuh"
#include "internal.h"
#include "cheb32.h"
#include "cheb64.h"
#include "twiddle128.h"
#include "twiddle64.h"

namespace {

using tsim::cmul;

constexpr int kZPad = 36;  // modes 4..36 padded to 36 floats per pupil sample

template <int LOG>
constexpr int brev(int v) {
  int r = 0;
  for (int b = 0; b < LOG; ++b) r |= ((v >> b) & 1) << (LOG - 1 - b);
  return r;
}

__device__ __forceinline__ float2 f2add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 f2sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Forward N-point DFT in registers (N = 32 or 64), natural order in and out:
// radix-2 decimation in time; the stage twiddle exp(-2 pi i j / (2 hs)) is
// W64[j * 32 / hs], with the factor -i applied as a swap.
template <int N>
__device__ __forceinline__ void fft_fwd(float2 (&x)[N]) {
  constexpr int LOG = N == 32 ? 5 : 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = brev<LOG>(i);
    if (j > i) {
      float2 t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
#pragma unroll
  for (int hs = 1; hs < N; hs <<= 1) {
#pragma unroll
    for (int g = 0; g < N; g += 2 * hs) {
#pragma unroll
      for (int j = 0; j < hs; ++j) {
        float2 a = x[g + j], b = x[g + j + hs];
        const int k = j * (32 / hs);
        float2 t;
        if (k == 0) {
          t = b;
        } else if (k == 16) {
          t = make_float2(b.y, -b.x);
        } else {
          t = cmul(make_float2(kW64re[k], kW64im[k]), b);
        }
        x[g + j] = f2add(a, t);
        x[g + j + hs] = f2sub(a, t);
      }
    }
  }
}

// value of the 64-point DFT at signed frequency k in [-16, 16] from the two
// 32-point DFTs: even k from E, odd k from O
__device__ __forceinline__ float2 pick(const float2 (&E)[32], const float2 (&O)[32], int k) {
  return (k & 1) ? O[((k - 1) >> 1) & 31] : E[(k >> 1) & 31];
}

// This lane's row coefficients d_p = sum_q C[p][q] T_q(y) of the pixel's 2D
// Chebyshev phase series C (NCH x NCH, from LDS), y the row's normalised
// coordinate.
template <int NCH>
__device__ __forceinline__ void row_series(const float *cb, float y, float (&d)[NCH]) {
  float ty[NCH];
  ty[0] = 1.f;
  ty[1] = y;
#pragma unroll
  for (int q = 2; q < NCH; ++q) ty[q] = fmaf(2.f * y, ty[q - 1], -ty[q - 2]);
#pragma unroll
  for (int p = 0; p < NCH; ++p) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NCH; ++q) s = fmaf(cb[NCH * p + q], ty[q], s);
    d[p] = s;
  }
}

// Modes in a pixel's phase (Noll 4..N+1) for a series of NCH terms: at
// most 33 for NCH = 8 (Noll 4..36), 63 for NCH = 11 (Noll 4..66).
template <int NCH>
constexpr int kMaxPhaseModes = NCH == 8 ? 33 : 63;

// The pixel's phase as a 2D Chebyshev series, entry e of C (row-major p, q):
// sum over the modes of a_j E[j][e], E the plan's table, zero padded to
// kMaxPhaseModes<NCH> modes of NCH^2 entries (a_j = 0 beyond the plan's).
template <int NCH>
__device__ __forceinline__ float cheb_entry(const float (&a)[kMaxPhaseModes<NCH>], const float *zc, int e) {
  float c = 0.f;
#pragma unroll
  for (int j = 0; j < kMaxPhaseModes<NCH>; ++j) c = fmaf(a[j], zc[j * NCH * NCH + e], c);
  return c;
}

// This pixel's coefficients of the phase modes 4..N+1 (nm = N - 2 of them;
// 33 for NCH = 8), zero beyond: the loads are unconditional (a clamped mode
// index), so they all go out together.
template <int NCH>
__device__ __forceinline__ void phase_coeffs(const float *zp, size_t hw, int nm, float (&a)[kMaxPhaseModes<NCH>]) {
#pragma unroll
  for (int t = 0; t < kMaxPhaseModes<NCH>; ++t) {
    const int tt = NCH == 8 ? t : min(t, nm - 1);
    const float v = zp[size_t(tt + TSIM_PSF_MODE0) * hw];
    a[t] = (NCH == 8 || t < nm) ? v : 0.f;
  }
}

template <int T, int NCH>
__global__ void __launch_bounds__(256)
k_psf64(const float *__restrict__ zern, int hw, int nmodes, size_t p_base, int n_pix,
        const float *__restrict__ zc, float *__restrict__ psf) {
  constexpr int NCC = NCH * NCH, NMAX = kMaxPhaseModes<NCH>;
  const int nm = nmodes - 2;
  constexpr int R = (T - 1) / 2;  // crop radius, <= 16
  constexpr int LS = 33;          // LDS row stride (complex)
  __shared__ float2 s1[8][32 * LS];
  __shared__ float cbuf[8][NCC];  // per pixel: 2D Chebyshev coefficients of the phase
  const int lane = threadIdx.x & 31;
  const int slot = threadIdx.x >> 5;  // half-wave within the block
  float2 *buf = s1[slot];
  const int p = blockIdx.x * 8 + slot;
  const bool active = p < n_pix;
  const int pc = active ? p : 0;

  // Zernike coefficients of modes 4..N+1 of this pixel
  float a[NMAX];
  {
    const size_t pg = p_base + size_t(pc);  // pixel index into zern
    const size_t fr = pg / size_t(hw), yx = pg - fr * size_t(hw);
    const float *zp = zern + fr * nmodes * size_t(hw) + yx;
    phase_coeffs<NCH>(zp, size_t(hw), nm, a);
  }

  // the pixel's phase as a 2D Chebyshev series C[p][q] = sum_j a_j E[j][p][q]
  // (lane: entries 2 lane, 2 lane + 1 for 8 terms; lane, lane + 32, ... for
  // 11), shared through LDS
  if constexpr (NCH == 8) {
    float c0 = 0.f, c1 = 0.f;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
      c0 = fmaf(a[j], zc[j * NCC + 2 * lane], c0);
      c1 = fmaf(a[j], zc[j * NCC + 2 * lane + 1], c1);
    }
    cbuf[slot][2 * lane] = c0;
    cbuf[slot][2 * lane + 1] = c1;
  } else {
#pragma unroll
    for (int e = lane; e < NCC; e += 32) cbuf[slot][e] = cheb_entry<NCH>(a, zc, e);
  }
  __syncthreads();

  // ---- stage 1: lane = window row wr, pupil row offset r' = wr - 16 ----
  float2 E[32], O[32];
  {
    const int wr = lane;
    const int rp = wr - 16;
    // this row's phase as a Chebyshev series in x: phi(x) = sum_p d_p T_p(x)
    float d[NCH];
    row_series<NCH>(cbuf[slot], float(rp) * 0.0625f, d);
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      const int cp = (n < 16) ? n : n - 32;  // signed column offset
      float2 v = make_float2(0.f, 0.f);
      if (rp * rp + cp * cp < 256) {
        float phi = 0.f;
#pragma unroll
        for (int p = 0; p < NCH; ++p) phi = fmaf(d[p], kChebCol[n][p], phi);
        // exp(-i phi) with the hardware sine/cosine (input in revolutions)
        const float rev = phi * 0.15915494309189535f;
        v = make_float2(__builtin_amdgcn_cosf(rev), -__builtin_amdgcn_sinf(rev));
      }
      E[n] = v;
      const int k = (cp + 64) & 63;  // exp(-2 pi i c'/64)
      O[n] = cmul(make_float2(kW64re[k], kW64im[k]), v);
    }
    fft_fwd<32>(E);
    fft_fwd<32>(O);
    // X1[r'][kx] for kx in [-16, 16] -> buf[wr][kx + 16]
#pragma unroll
    for (int kx = -16; kx <= 16; ++kx) buf[wr * LS + kx + 16] = pick(E, O, kx);
  }
  __syncthreads();

  // ---- stage 2: lane = frequency column kx = lane - 16 ----
  float h[T];
  float hx[2] = {0.f, 0.f};  // column kx = +16: rows ky = lane - 16 and (lane 0) ky = +16
  float total = 0.f;
  {
    const int col = lane;
#pragma unroll
    for (int n = 0; n < 32; ++n) {
      const int rp = (n < 16) ? n : n - 32;
      float2 v = buf[(rp + 16) * LS + col];
      E[n] = v;
      const int k = (rp + 64) & 63;
      O[n] = cmul(make_float2(kW64re[k], kW64im[k]), v);
    }
    fft_fwd<32>(E);
    fft_fwd<32>(O);
    const int kx = lane - 16;
#pragma unroll
    for (int ky = -R; ky <= R; ++ky) {
      float2 v = pick(E, O, ky);
      float m = v.x * v.x + v.y * v.y;
      h[ky + R] = m;
      if (kx >= -R && kx <= R) total += m;
    }
    if (R == 16) {
      // direct DFT of the column kx = +16 over rows r' in [-16, 15]
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int ky = (s == 0) ? lane - 16 : 16;
        if (s == 1 && lane != 0) break;
        float2 acc = make_float2(0.f, 0.f);
        // twiddle exp(-2 pi i ky r'/64) for r' = -16, -15, ... by recurrence
        const int k0 = (-16 * ky + 64 * 64) & 63, k1 = (ky + 64) & 63;
        float2 tw = make_float2(kW64re[k0], kW64im[k0]);
        const float2 step = make_float2(kW64re[k1], kW64im[k1]);
        for (int wr = 0; wr < 32; ++wr) {
          acc = f2add(acc, cmul(tw, buf[wr * LS + 32]));
          tw = cmul(tw, step);
        }
        float m = acc.x * acc.x + acc.y * acc.y;
        hx[s] = m;
        total += m;
      }
    }
  }
  // unit-sum normalisation over the T x T crop (32-lane reduction)
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) total += __shfl_xor(total, off, 32);
  const float inv = 1.0f / total;
  if (active) {
    float *out = psf + size_t(p) * T * T;
    const int kx = lane - 16;
    if (kx >= -R && kx <= R) {
#pragma unroll
      for (int ky = -R; ky <= R; ++ky) out[(ky + R) * T + (kx + R)] = h[ky + R] * inv;
    }
    if (R == 16) {
      out[(lane - 16 + R) * T + (16 + R)] = hx[0] * inv;
      if (lane == 0) out[(16 + R) * T + (16 + R)] = hx[1] * inv;
    }
  }
}

// k_psf128 (pupil P = 128, aperture diameter 64 samples, crop T <= 65):
// two wavefronts own one pixel.  The aperture fits the 64 x 64 window of
// offsets [-32, 32) and the 65 x 65 lowest frequencies of the 128 x 128 DFT
// are kept; a 128-point DFT of 64 samples at frequencies [-32, 32] splits
// into the 64-point DFTs of x[c] (even frequencies) and
// x[c] exp(-2 pi i c/128) (odd frequencies).  Wave 0 takes the even and
// wave 1 the odd frequencies of both passes, so a lane holds one 64-point
// transform at a time.
// Stage 1: lane = pupil row; wave 1 forms its samples as
// exp(-i (phi + 2 pi c/128)) from the phase directly.  The outputs go to an
// LDS buffer of the 64 rows x 65 frequencies.
// Stage 2: lane = frequency column kx in [-32, 32); the column kx = +32 is a
// direct 64-term DFT (row ky = +32 of it: twiddles (-i)^r', a wave sum),
// taken by wave 0.  The unit-sum normalisation adds the two waves' sums.
template <int T, int NCH>
__global__ void __launch_bounds__(128)
k_psf128(const float *__restrict__ zern, int hw, int nmodes, size_t p_base, const float *__restrict__ zc,
         float *__restrict__ psf) {
  constexpr int NCC = NCH * NCH, NMAX = kMaxPhaseModes<NCH>;
  const int nm = nmodes - 2;
  constexpr int R = (T - 1) / 2;  // crop radius, <= 32
  constexpr int LS = 65;          // LDS row stride (complex)
  constexpr int MR = R / 2;       // even ky = 2m, m in [-MR, MR]; odd ky = 2m + 1, m in [-MR, MR - 1]
  static_assert(R % 2 == 0, "the crop radius splits into even and odd rows");
  __shared__ float2 buf[64 * LS];
  __shared__ float cbuf[NCC];     // 2D Chebyshev coefficients of the phase
  __shared__ float part[2];       // the two waves' sums over the crop
  const int lane = threadIdx.x & 63;
  const int odd = threadIdx.x >> 6;  // 0: even frequencies, 1: odd
  const size_t p = blockIdx.x;

  {
    float a[NMAX];
    const size_t pg = p_base + p;
    const size_t fr = pg / size_t(hw), yx = pg - fr * size_t(hw);
    const float *zp = zern + fr * nmodes * size_t(hw) + yx;
    phase_coeffs<NCH>(zp, size_t(hw), nm, a);
#pragma unroll
    for (int e = threadIdx.x; e < NCC; e += 128) cbuf[e] = cheb_entry<NCH>(a, zc, e);
  }
  __syncthreads();

  float2 X[64];
  // ---- stage 1: lane = window row wr, pupil row offset r' = wr - 32 ----
  {
    const int rp = lane - 32;
    float d[NCH];
    row_series<NCH>(cbuf, float(rp) * 0.03125f, d);
#pragma unroll
    for (int n = 0; n < 64; ++n) {
      const int cp = (n < 32) ? n : n - 64;
      float2 v = make_float2(0.f, 0.f);
      if (rp * rp + cp * cp < 1024) {
        float phi = 0.f;
#pragma unroll
        for (int q = 0; q < NCH; ++q) phi = fmaf(d[q], kChebCol64[n][q], phi);
        const float rev = fmaf(phi, 0.15915494309189535f, odd ? float(cp) * 0.0078125f : 0.f);
        v = make_float2(__builtin_amdgcn_cosf(rev), -__builtin_amdgcn_sinf(rev));
      }
      X[n] = v;
    }
    fft_fwd<64>(X);
    // X1[r'][kx] for kx in [-32, 32] -> buf[wr][kx + 32]: kx = 2m + odd at X[m]
    float2 *row = buf + lane * LS;
    if (odd) {
#pragma unroll
      for (int m = -16; m <= 15; ++m) row[2 * m + 1 + 32] = X[m & 63];
    } else {
#pragma unroll
      for (int m = -16; m <= 16; ++m) row[2 * m + 32] = X[m & 63];
    }
  }
  __syncthreads();

  // ---- stage 2: lane = frequency column kx = lane - 32 ----
  const int kx = lane - 32;
  float hx = 0.f, hx32 = 0.f;  // column kx = +32: row ky = lane - 32, and row ky = +32
  if (R == 32 && !odd) {
    float2 acc = make_float2(0.f, 0.f);
    const int ky = lane - 32;
    for (int wr = 0; wr < 64; ++wr) {
      const float rev = float((ky * (wr - 32)) & 127) * (1.0f / 128.0f);
      const float2 w = make_float2(__builtin_amdgcn_cosf(rev), -__builtin_amdgcn_sinf(rev));
      acc = f2add(acc, cmul(w, buf[wr * LS + 64]));
    }
    hx = acc.x * acc.x + acc.y * acc.y;
    // ky = +32: exp(-2 pi i 32 r'/128) = (-i)^r'; lane = row
    const float2 v = buf[lane * LS + 64];
    const int q = (lane - 32) & 3;
    float2 t = q == 0 ? v : q == 1 ? make_float2(v.y, -v.x) : q == 2 ? make_float2(-v.x, -v.y)
                                                                      : make_float2(-v.y, v.x);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      t.x += __shfl_xor(t.x, off, 64);
      t.y += __shfl_xor(t.y, off, 64);
    }
    hx32 = t.x * t.x + t.y * t.y;
  }
#pragma unroll
  for (int n = 0; n < 64; ++n) {
    const int r = (n < 32) ? n : n - 64;
    const float2 v = buf[(r + 32) * LS + lane];
    X[n] = odd ? cmul(make_float2(kW128re[r & 127], kW128im[r & 127]), v) : v;
  }
  fft_fwd<64>(X);
  // |X|^2 at ky = 2m + odd, m in [-MR, MR] (the last only for even ky)
  float h[2 * MR + 1];
#pragma unroll
  for (int m = -MR; m <= MR; ++m) {
    const float2 v = X[m & 63];
    h[m + MR] = v.x * v.x + v.y * v.y;
  }
  float total = (R == 32 && !odd) ? hx + (lane == 0 ? hx32 : 0.f) : 0.f;
  if (kx >= -R && kx <= R) {
#pragma unroll
    for (int m = -MR; m <= MR; ++m)
      if (!odd || m < MR) total += h[m + MR];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) total += __shfl_xor(total, off, 64);
  if (lane == 0) part[odd] = total;
  __syncthreads();
  const float inv = 1.0f / (part[0] + part[1]);
  float *out = psf + p * T * T;
  if (kx >= -R && kx <= R) {
#pragma unroll
    for (int m = -MR; m <= MR; ++m)
      if (!odd || m < MR) out[(2 * m + odd + R) * T + (kx + R)] = h[m + MR] * inv;
  }
  if (R == 32 && !odd) {
    out[(lane - 32 + R) * T + (32 + R)] = hx * inv;
    if (lane == 0) out[(32 + R) * T + (32 + R)] = hx32 * inv;
  }
}

int launch_psf_impl(const tsim_plan *pl, const float *zern, int hw, size_t p_base, int n, float *psf,
                    hipStream_t s) {
  const float *zt = pl->d_zcheb;
  const int N = pl->N;
  const bool wide = pl->NCH == 11;   // more than 35 modes
  if (pl->P == 128) {
    TraceScope tr("k_psf128", s);
    if (pl->T == 65 && !wide)
      hipLaunchKernelGGL((k_psf128<65, 8>), dim3(n), dim3(128), 0, s, zern, hw, N, p_base, zt, psf);
    else if (pl->T == 33 && !wide)
      hipLaunchKernelGGL((k_psf128<33, 8>), dim3(n), dim3(128), 0, s, zern, hw, N, p_base, zt, psf);
    else if (pl->T == 65)
      hipLaunchKernelGGL((k_psf128<65, 11>), dim3(n), dim3(128), 0, s, zern, hw, N, p_base, zt, psf);
    else if (pl->T == 33)
      hipLaunchKernelGGL((k_psf128<33, 11>), dim3(n), dim3(128), 0, s, zern, hw, N, p_base, zt, psf);
    else
      return TSIM_EUNSUPPORTED;
    return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
  }
  if (pl->P != 64) return TSIM_EUNSUPPORTED;
  dim3 grid((n + 7) / 8);
  TraceScope tr("k_psf64", s);
  if (wide) {
    if (pl->T != 33) return TSIM_EUNSUPPORTED;
    hipLaunchKernelGGL((k_psf64<33, 11>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf);
    return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
  }
  switch (pl->T) {
    case 33: hipLaunchKernelGGL((k_psf64<33, 8>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf); break;
    case 31: hipLaunchKernelGGL((k_psf64<31, 8>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf); break;
    case 21: hipLaunchKernelGGL((k_psf64<21, 8>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf); break;
    case 15: hipLaunchKernelGGL((k_psf64<15, 8>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf); break;
    case 9: hipLaunchKernelGGL((k_psf64<9, 8>), grid, dim3(256), 0, s, zern, hw, N, p_base, n, zt, psf); break;
    default: return TSIM_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

// The optical transfer functions of Sec. IV-B need the whole 64 x 64
// spectrum of each generalised pupil G = P exp(-i phi): the OTF is the
// autocorrelation of G, i.e. the inverse DFT of |DFT(G)|^2, and its sample
// mean over coefficient vectors is the inverse DFT of the mean |DFT(G)|^2.
// k_otf64 (P = 64): one wavefront per block takes the vectors s = block,
// block + grid, ... in turn.  Stage 1: lanes 0-31 take window row wr = lane
// and its 32-point DFT at even frequencies (E), lanes 32-63 the same row's
// odd frequencies (O, input times exp(-2 pi i c'/64)); the 32 x 64 row
// spectra go to LDS.  Stage 2: lane = frequency column kx = 2 (lane % 32) +
// lane / 32, the even and odd row frequencies of the column by two more
// 32-point DFTs; |.|^2 of all 64 is added to the lane's running sums.  At
// the end the block writes its 64 x 64 sums (kx fastest, frequencies in
// DFT order).  With TILT = false the tilt modes (Noll 2, 3: 2x and 2y on the
// unit disc) enter the phase's Chebyshev series; TILT = true leaves them out
// (the short-exposure OTF's tilt-corrected phase).
template <bool TILT, int NCH>
__global__ void __launch_bounds__(64)
k_otf64(const float *__restrict__ zern, int hw, int nmodes, size_t n, const float *__restrict__ zc,
        float *__restrict__ part) {
  constexpr int LS = 33, NCC = NCH * NCH, NMAX = kMaxPhaseModes<NCH>;
  const int nm = nmodes - 2;
  __shared__ float2 buf[2][32 * LS];
  __shared__ float cbuf[NCC];
  const int lane = threadIdx.x;
  const int par = lane >> 5, m = lane & 31;
  float acc[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) acc[k] = 0.f;
  for (size_t smp = blockIdx.x; smp < n; smp += gridDim.x) {
    const size_t fr = smp / size_t(hw), yx = smp - fr * size_t(hw);
    const float *zp = zern + fr * nmodes * size_t(hw) + yx;
    {
      // Chebyshev coefficients of the phase: modes 4..N+1 from the plan's
      // table; the tilts 2 a2 x (entry p = 1, q = 0) and 2 a3 y (p = 0,
      // q = 1) unless removed
#pragma unroll
      for (int e = lane; e < NCC; e += 64) {
        float c = 0.f;
#pragma unroll
        for (int j = 0; j < NMAX; ++j) {
          const int jj = NCH == 8 ? j : min(j, nm - 1);
          const float v = zp[size_t(jj + TSIM_PSF_MODE0) * hw];
          c = fmaf((NCH == 8 || j < nm) ? v : 0.f, zc[j * NCC + e], c);
        }
        if (!TILT) {
          if (e == NCH) c = fmaf(2.f, zp[0], c);
          if (e == 1) c = fmaf(2.f, zp[size_t(hw)], c);
        }
        cbuf[e] = c;
      }
    }
    __syncthreads();
    {
      // ---- stage 1: row wr = m, parity par ----
      const int rp = m - 16;
      float d[NCH];
      row_series<NCH>(cbuf, float(rp) * 0.0625f, d);
      float2 X[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const int cp = (k < 16) ? k : k - 32;  // signed column offset
        float2 v = make_float2(0.f, 0.f);
        if (rp * rp + cp * cp < 256) {
          float phi = 0.f;
#pragma unroll
          for (int q = 0; q < NCH; ++q) phi = fmaf(d[q], kChebCol[k][q], phi);
          const float rev = phi * 0.15915494309189535f;
          v = make_float2(__builtin_amdgcn_cosf(rev), -__builtin_amdgcn_sinf(rev));
        }
        if (par) {
          const int w = (cp + 64) & 63;
          v = cmul(make_float2(kW64re[w], kW64im[w]), v);
        }
        X[k] = v;
      }
      fft_fwd<32>(X);
#pragma unroll
      for (int k = 0; k < 32; ++k) buf[par][m * LS + k] = X[k];
    }
    __syncthreads();
    {
      // ---- stage 2: column kx = 2 m + par (row spectra of parity par, entry m) ----
      // even row frequencies, then odd ones (the column re-read from LDS,
      // so one 32-point array is live at a time)
#pragma unroll
      for (int odd = 0; odd < 2; ++odd) {
        float2 X[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
          const int rp = (k < 16) ? k : k - 32;
          const float2 v = buf[par][(rp + 16) * LS + m];
          const int w = (rp + 64) & 63;
          X[k] = odd ? cmul(make_float2(kW64re[w], kW64im[w]), v) : v;
        }
        fft_fwd<32>(X);
#pragma unroll
        for (int k = 0; k < 32; ++k) acc[2 * k + odd] += X[k].x * X[k].x + X[k].y * X[k].y;
      }
    }
    __syncthreads();  // cbuf and buf are rewritten by the next vector
  }
  float *out = part + size_t(blockIdx.x) * 4096 + 2 * m + par;
#pragma unroll
  for (int ky = 0; ky < 64; ++ky) out[ky * 64] = acc[ky];
}

}  // namespace

bool psf_size_supported(int P, int T, int n_modes) {
  if (n_modes != 35) return (P == 64 && T == 33) || (P == 128 && (T == 65 || T == 33));
  if (P == 128) return T == 65 || T == 33;
  if (P == 64) return T == 33 || T == 31 || T == 21 || T == 15 || T == 9;
  return false;
}

// pixels per P2S chunk: at most 2^20 pixels and about 5 GB of PSFs, in whole
// projection tiles (bounds the PSF workspace)
size_t p2s_chunk_pixels(const tsim_plan *pl, size_t total) {
  const size_t per = size_t(pl->T) * pl->T * sizeof(float);
  size_t cap = std::min(size_t(1) << 20, (size_t(5) << 30) / per / kProjectTile * kProjectTile);
  return std::min(total, std::max(cap, size_t(kProjectTile)));
}


size_t p2s_ws_bytes(const tsim_plan *pl, int frames) {
  size_t total = size_t(frames) * pl->H * pl->W;
  return p2s_chunk_pixels(pl, total) * size_t(pl->T) * pl->T * sizeof(float);
}

int launch_psf_exact(const tsim_plan *pl, int n, const float *zvec, float *psf, hipStream_t s) {
  return launch_psf_impl(pl, zvec, 1, 0, n, psf, s);
}

int launch_p2s_exact(const tsim_plan *pl, int frames, const float *zern, void *beta, int out_bf16, void *ws,
                     hipStream_t s) {
  const int hw = pl->H * pl->W;
  const size_t total = size_t(frames) * hw;
  const size_t chunk = p2s_chunk_pixels(pl, total);
  // bytes of one pixel's weights in the output layout
  const size_t row = out_bf16 ? size_t(pl->KP) * 2 : size_t(pl->K) * 4;
  float *h = static_cast<float *>(ws);
  for (size_t p0 = 0; p0 < total; p0 += chunk) {
    const int n = int(std::min(chunk, total - p0));
    int st = launch_psf_impl(pl, zern, hw, p0, n, h, s);
    if (st != TSIM_OK) return st;
    st = launch_project(pl, h, n, static_cast<char *>(beta) + p0 * row, out_bf16, s);
    if (st != TSIM_OK) return st;
  }
  return TSIM_OK;
}

// ---- optical transfer functions (Sec. IV-B) ----
constexpr int kOtfMaxBlocks = 2048;

size_t otf_blocks(size_t n) { return std::max<size_t>(1, std::min<size_t>(kOtfMaxBlocks, (n + 63) / 64)); }

size_t otf_ws_bytes(const tsim_plan *pl, int frames) {
  const size_t n = size_t(frames) * pl->H * pl->W;
  return otf_blocks(n) * 4096 * sizeof(float) + 4096 * sizeof(double);
}

int launch_otf_sums(const tsim_plan *pl, int frames, const float *zern, int short_exposure, void *ws,
                    double *dev_sums, hipStream_t s) {
  if (pl->P != 64) return TSIM_EUNSUPPORTED;
  const int hw = pl->H * pl->W;
  const size_t n = size_t(frames) * hw;
  const size_t blocks = otf_blocks(n);
  float *part = static_cast<float *>(ws);
  {
    TraceScope tr("k_otf64", s);
    const int N = pl->N;
    if (pl->NCH == 8) {
      if (short_exposure)
        hipLaunchKernelGGL((k_otf64<true, 8>), dim3(unsigned(blocks)), dim3(64), 0, s, zern, hw, N, n, pl->d_zcheb,
                           part);
      else
        hipLaunchKernelGGL((k_otf64<false, 8>), dim3(unsigned(blocks)), dim3(64), 0, s, zern, hw, N, n, pl->d_zcheb,
                           part);
    } else {
      if (short_exposure)
        hipLaunchKernelGGL((k_otf64<true, 11>), dim3(unsigned(blocks)), dim3(64), 0, s, zern, hw, N, n,
                           pl->d_zcheb, part);
      else
        hipLaunchKernelGGL((k_otf64<false, 11>), dim3(unsigned(blocks)), dim3(64), 0, s, zern, hw, N, n,
                           pl->d_zcheb, part);
    }
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  return launch_partial_sum(part, blocks, 4096, dev_sums, s);
}
