// Exact projection of PSFs on the PCA basis (Eq. (7)): beta = Psi h per
// pixel, a dense [pixels x T^2] x [T^2 x K] contraction.
//
// The FP32 matrix instructions of this chip run at the rate of its FP32
// vector ALU, on which the PSF kernels already spend their time, so the
// contraction runs on the 16-bit matrix cores instead, at FP32 accuracy:
// every operand is split into two FP16 numbers, x = x_hi + x_lo with
// x_hi = fp16(x) and x_lo = fp16(x - x_hi), and the product is
// Psi_hi h_hi + Psi_hi h_lo + Psi_lo h_hi with FP32 accumulation.  The
// dropped term Psi_lo h_lo and the rounding of the two parts are each below
// 2^-22 of |Psi h|, about 1e-6 of every product; the products of FP16
// numbers and their sums are exact FP32 operations.  Operands are scaled
// into FP16's normal range first (h by 2^12, PSFs summing to 1; Psi by
// 2^10, rows of unit norm) and the sums scaled back by 2^-22.
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kHScale = 4096.f;                    // 2^12
constexpr float kOutScale = 1.f / (4096.f * 1024.f);  // 2^-22

__device__ __forceinline__ f32x16 mfma_f16(const uint4 &a, const uint4 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                0, 0);
}

// beta[p][k] = sum_t psi[k][t] h[p][t] on v_mfma_f32_32x32x16_f16, A = the
// basis (rows = outputs), B = the PSFs (columns = pixels).  Block: 128 pixels,
// 4 waves; wave w owns pixels [32 w, 32 w + 32) and NT 32-row output tiles.
// Taps go in chunks of 64 (four 16-tap matrix-core steps).  Per chunk the
// block stages its 128 pixels' 64 taps in LDS by coalesced row loads
// (thread: 32 taps of pixel rows, consecutive threads consecutive taps) and
// the chunk's basis fragments (hi and lo, in fragment order in the plan
// table); the global loads of chunk c + 1 are in flight in registers while
// the matrix cores work on chunk c.  A lane's B fragment is its pixel's taps
// 8 (l / 32) + 0..7 of the step, split into FP16 hi and lo on the fly.
constexpr int CT = 64;       // taps per chunk
constexpr int HS = CT + 4;   // LDS row stride of the staged PSF taps (floats; 16-byte aligned groups of 8)

template <int NT, bool OUT_BF16>
__global__ void __launch_bounds__(256)
k_project_h3(const float *__restrict__ h, const uint4 *__restrict__ psi /*[chunks][4][NT][64][2] x 8 f16*/,
             void *__restrict__ beta, int n, int T2, int K, int KB) {
  constexpr int SPC = CT / 16;          // matrix-core steps per chunk
  constexpr int CH = SPC * NT * 64 * 2;  // uint4 per chunk
  constexpr int PER = CH / 256;          // of them per thread
  constexpr int HPT = kProjectTile * CT / 256;  // staged PSF values per thread
  __shared__ uint4 ps[CH];
  __shared__ __attribute__((aligned(16))) float hs[kProjectTile * HS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p0 = blockIdx.x * kProjectTile;
  const int nchunk = (T2 + CT - 1) / CT;

  // staging loads: element e = threadIdx.x + 256 i is pixel e / 64, tap
  // e % 64 of the chunk; pixels past n read pixel n - 1 and taps past T^2
  // the row's last tap, so every load is unconditional (the basis table is
  // zero past T^2, and such pixels are not stored).  Rows of a full block
  // are 4 pixels apart; only the last block clamps.
  // (element offsets fit 32 bits: a P2S chunk holds at most about 5 GB of PSFs)
  const int tt = threadIdx.x & (CT - 1), prow = threadIdx.x / CT;
  const bool full = p0 + kProjectTile <= n;
  const uint32_t rbase = uint32_t(p0 + prow) * uint32_t(T2), rstep = 4u * uint32_t(T2);
  float hv[HPT];
  auto hload = [&](int t0) {
    const uint32_t t = uint32_t(min(t0 + tt, T2 - 1));
    if (full) {
#pragma unroll
      for (int i = 0; i < HPT; ++i) hv[i] = h[rbase + rstep * uint32_t(i) + t];
    } else {
#pragma unroll
      for (int i = 0; i < HPT; ++i) hv[i] = h[uint32_t(min(p0 + prow + 4 * i, n - 1)) * uint32_t(T2) + t];
    }
  };
  // the chunk's basis fragments, PER (= 2 NT) per thread, as named values
  // (an array of them ends up in scratch memory)
  const uint4 *pp = psi + threadIdx.x;
  uint4 pv0, pv1, pv2, pv3, pv4, pv5, pv6, pv7;
  auto pload = [&]() {
    pv0 = pp[0];
    pv1 = pp[256];
    if constexpr (PER > 2) { pv2 = pp[512]; pv3 = pp[768]; }
    if constexpr (PER > 4) { pv4 = pp[1024]; pv5 = pp[1280]; }
    if constexpr (PER > 6) { pv6 = pp[1536]; pv7 = pp[1792]; }
  };
  auto pstore = [&]() {
    ps[threadIdx.x] = pv0;
    ps[threadIdx.x + 256] = pv1;
    if constexpr (PER > 2) { ps[threadIdx.x + 512] = pv2; ps[threadIdx.x + 768] = pv3; }
    if constexpr (PER > 4) { ps[threadIdx.x + 1024] = pv4; ps[threadIdx.x + 1280] = pv5; }
    if constexpr (PER > 6) { ps[threadIdx.x + 1536] = pv6; ps[threadIdx.x + 1792] = pv7; }
  };
  static_assert(PER == 2 * NT && PER <= 8, "two basis fragments per thread and output tile");
  pload();

  f32x16 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = f32x16{};
  hload(0);
  const float *hb = hs + (32 * w + (lane & 31)) * HS + 8 * (lane >> 5);
  for (int c = 0; c < nchunk; ++c) {
    pstore();
#pragma unroll
    for (int i = 0; i < HPT; ++i) hs[(prow + 4 * i) * HS + tt] = hv[i];
    __syncthreads();
    if (c + 1 < nchunk) {
      hload(CT * (c + 1));
      pp += CH;
      pload();
    }
#pragma unroll
    for (int s = 0; s < SPC; ++s) {
      // this step's PSF values as FP16 pairs
      const float4 u0 = *reinterpret_cast<const float4 *>(hb + 16 * s);
      const float4 u1 = *reinterpret_cast<const float4 *>(hb + 16 * s + 4);
      const f32x8 v = f32x8{u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w} * kHScale;
      const f16x8 hi = __builtin_convertvector(v, f16x8);
      const f16x8 lo = __builtin_convertvector(v - __builtin_convertvector(hi, f32x8), f16x8);
      const uint4 bhi = __builtin_bit_cast(uint4, hi), blo = __builtin_bit_cast(uint4, lo);
      uint4 ahi[NT], alo[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        ahi[j] = ps[((s * NT + j) * 64 + lane) * 2];
        alo[j] = ps[((s * NT + j) * 64 + lane) * 2 + 1];
      }
      // the three products of each tile, tiles interleaved so consecutive
      // matrix-core instructions are independent
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = mfma_f16(ahi[j], bhi, acc[j]);
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = mfma_f16(ahi[j], blo, acc[j]);
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = mfma_f16(alo[j], bhi, acc[j]);
    }
    __syncthreads();
  }
  const int pix = p0 + 32 * w + (lane & 31);
  if (pix >= n) return;
  // D layout: lane holds column (pixel) lane % 32, rows 8 i + 4 (lane / 32) + r
#pragma unroll
  for (int j = 0; j < NT; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 32 * j + 8 * i + 4 * (lane >> 5) + r;
        const float v = acc[j][4 * i + r] * kOutScale;
        if constexpr (OUT_BF16) {
          if (k < KB) static_cast<__bf16 *>(beta)[size_t(pix) * KB + k] = __bf16(k < K ? v : 0.f);
        } else {
          if (k < K) static_cast<float *>(beta)[size_t(pix) * K + k] = v;
        }
      }
}

}  // namespace

int launch_project(const tsim_plan *pl, const float *h, int n, void *beta, int out_bf16, hipStream_t s) {
  const int T2 = pl->T * pl->T, KB = out_bf16 ? pl->KP : pl->K;
  const int nt = (pl->KP + 31) / 32;  // the plan table's output tiles (KP >= KB)
  dim3 grid((n + kProjectTile - 1) / kProjectTile);
  TraceScope tr("k_project", s);
  const uint4 *psi = reinterpret_cast<const uint4 *>(pl->d_basis_h3);
#define TSIM_PJ(NT, BF) \
  hipLaunchKernelGGL((k_project_h3<NT, BF>), grid, dim3(256), 0, s, h, psi, beta, n, T2, pl->K, KB)
  switch (nt) {
    case 1: if (out_bf16) TSIM_PJ(1, true); else TSIM_PJ(1, false); break;
    case 2: if (out_bf16) TSIM_PJ(2, true); else TSIM_PJ(2, false); break;
    case 3: if (out_bf16) TSIM_PJ(3, true); else TSIM_PJ(3, false); break;
    case 4: if (out_bf16) TSIM_PJ(4, true); else TSIM_PJ(4, false); break;
    default: return TSIM_EUNSUPPORTED;
  }
#undef TSIM_PJ
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
