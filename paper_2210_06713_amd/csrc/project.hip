// Exact projection of PSFs on the PCA basis (Eq. (7)): beta = Psi h per
// pixel, a dense [pixels x T^2] x [T^2 x K] contraction on the FP32 matrix
// cores.
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

// beta[p][k] = sum_t h[p][t] psi[k][t] on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32).  Block: 128 pixels x 16 NT outputs, 4 waves;
// wave w owns pixels [32w, 32w + 32) as two 16-row tiles and all NT 16-wide
// output tiles, so padding K = 100 costs 12 columns (NT = 7) rather than 28.
// 32-tap chunks of h and psi^T are staged through LDS (h rows padded against
// bank conflicts), and the global loads of chunk c + 1 are in flight in
// registers while the matrix cores work on chunk c.
constexpr int PJ_PX = kProjectTile, PJ_TK = 32, PJ_N = 128;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// OUT_BF16: beta rows of KB bfloat16 (K weights, zeros up to KB <= 16 PJ_NT),
// the layout BF16 plans use; else rows of K floats.
template <int PJ_NT, bool OUT_BF16>  // 16-wide output tiles: 7 for KB <= 112, 8 up to 128
__global__ void __launch_bounds__(256)
k_project_mfma(const float *__restrict__ h, const float *__restrict__ psi_t128 /*[T2][128]*/,
               void *__restrict__ beta, int n, int T2, int K, int KB) {
  __shared__ float As[PJ_PX][PJ_TK + 1];
  __shared__ __attribute__((aligned(16))) float Bs[PJ_TK][PJ_N];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;   // MFMA row/column in the tile, k within the step
  const int p0 = blockIdx.x * PJ_PX;
  constexpr int NA = PJ_PX * PJ_TK / 256, NB = PJ_TK * PJ_N / 4 / 256;
  float ra[NA];
  float4 rb[NB];
  auto gload = [&](int t0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = threadIdx.x + i * 256;
      const int px = e >> 5, tt = e & 31;
      const int gp = p0 + px, gt = t0 + tt;
      ra[i] = (gp < n && gt < T2) ? h[size_t(gp) * T2 + gt] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = threadIdx.x + i * 256;
      const int tt = e >> 5, c4 = e & 31;
      const int gt = t0 + tt;
      rb[i] = (gt < T2) ? *reinterpret_cast<const float4 *>(psi_t128 + size_t(gt) * PJ_N + 4 * c4)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  f32x4 acc[2][PJ_NT];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < PJ_NT; ++j) acc[i][j] = f32x4{};
  gload(0);
  for (int t0 = 0; t0 < T2; t0 += PJ_TK) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = threadIdx.x + i * 256;
      As[e >> 5][e & 31] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = threadIdx.x + i * 256;
      *reinterpret_cast<float4 *>(&Bs[e >> 5][4 * (e & 31)]) = rb[i];
    }
    __syncthreads();
    if (t0 + PJ_TK < T2) gload(t0 + PJ_TK);
#pragma unroll
    for (int s = 0; s < PJ_TK / 4; ++s) {
      const int k = 4 * s + lk;
      const float a0 = As[w * 32 + li][k], a1 = As[w * 32 + 16 + li][k];
#pragma unroll
      for (int j = 0; j < PJ_NT; ++j) {
        const float b = Bs[k][16 * j + li];
        acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b, acc[0][j], 0, 0, 0);
        acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b, acc[1][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // C layout: lane holds column li of the tile, rows 4 lk + r
#pragma unroll
  for (int j = 0; j < PJ_NT; ++j) {
    const int k = 16 * j + li;
    if (k >= (OUT_BF16 ? KB : K)) continue;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gp = p0 + w * 32 + 16 * i + 4 * lk + r;
        if (gp >= n) continue;
        if constexpr (OUT_BF16)
          static_cast<__bf16 *>(beta)[size_t(gp) * KB + k] = __bf16(k < K ? acc[i][j][r] : 0.f);
        else
          static_cast<float *>(beta)[size_t(gp) * K + k] = acc[i][j][r];
      }
  }
}

}  // namespace

int launch_project(const tsim_plan *pl, const float *h, int n, void *beta, int out_bf16, hipStream_t s) {
  const int T2 = pl->T * pl->T, KB = out_bf16 ? pl->KP : pl->K;
  dim3 grid((n + PJ_PX - 1) / PJ_PX);
  TraceScope tr("k_project", s);
  if (KB <= 112) {
    if (out_bf16)
      hipLaunchKernelGGL((k_project_mfma<7, true>), grid, dim3(256), 0, s, h, pl->d_basis_t128, beta, n, T2, pl->K, KB);
    else
      hipLaunchKernelGGL((k_project_mfma<7, false>), grid, dim3(256), 0, s, h, pl->d_basis_t128, beta, n, T2, pl->K, KB);
  } else {
    if (out_bf16)
      hipLaunchKernelGGL((k_project_mfma<8, true>), grid, dim3(256), 0, s, h, pl->d_basis_t128, beta, n, T2, pl->K, KB);
    else
      hipLaunchKernelGGL((k_project_mfma<8, false>), grid, dim3(256), 0, s, h, pl->d_basis_t128, beta, n, T2, pl->K, KB);
  }
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
