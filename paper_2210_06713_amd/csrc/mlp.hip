// The learned phase-to-space map (Sec. II-C: a small network turns each
// pixel's Zernike vector into its PSF-basis weights): a 35 -> 256 -> 256 ->
// 256 -> K perceptron with exact (erf) GELU, trained and evaluated with BF16
// matrix-core (MFMA) products and FP32 accumulation, FP32 master weights and
// AdamW.
//
// Kernels
//   k_gemm_bf16<EPI>   C = A B over an LDS-staged 64 x 64 tile (4 waves, one
//                      32x32x16 BF16 MFMA tile each), any operand strides, so
//                      the forward (X W^T), input-gradient (dZ W) and weight-
//                      gradient (dZ^T X) products share it; fused epilogues
//                      add the bias and apply GELU or its derivative.
//   k_mlp_infer        fused per-pixel inference for the P2S step: a block
//                      of 8 waves carries 128 pixels through all four
//                      layers in two pipelined halves (one half's GELU on
//                      the vector ALU while the matrix cores take the other
//                      half's products), activations staying in LDS, weights
//                      in fragment order streamed from L2 three k-steps
//                      ahead of their products.
//   k_prep, k_mse_grad, k_colsum_*, k_adamw, k_init_normal, k_draws: data
//                      preparation, loss, bias gradients, optimiser, seeded
//                      initialisation and training-pair draws.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.cuh"
#include "internal.h"

namespace {

using namespace tsim;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16, nearest with ties to even (the hardware conversion)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, __bf16(f)); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
// two floats -> two bfloat16 in one word (lo = first), nearest-even, one
// packed conversion
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{lo, hi}), bf16x2));
}

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Fragments stay four 32-bit words until the matrix-core call: copies of
// 8 x bf16 vectors otherwise get split into 16-bit lanes and re-packed.
__device__ __forceinline__ uint4 load8(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }

__device__ __forceinline__ f32x16 mfma_bf16(const uint4 &a, const uint4 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_BIAS_F32 = 2, EPI_GELU_GRAD = 3 };

constexpr int GT = 64, GK = 32, GKP = GK + 8;

// C[m][n] = sum_k A(m,k) B(k,n); A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
template <int EPI>
__global__ void __launch_bounds__(256)
k_gemm_bf16(const uint16_t *__restrict__ A, long sam, long sak, const uint16_t *__restrict__ B,
            long sbk, long sbn, int M, int N, int Kd, const float *__restrict__ bias,
            float *__restrict__ Z, float *__restrict__ outf, uint16_t *__restrict__ outb, int ldc) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GT][GKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GKP];
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wm = w >> 1, wn = w & 1;
  f32x16 acc = {};
  // split-K: block z reduces over k in [z * kchunk, (z + 1) * kchunk)
  const int kchunk = ((Kd + int(gridDim.z) - 1) / int(gridDim.z) + GK - 1) / GK * GK;
  const int kbeg = blockIdx.z * kchunk, kend = min(Kd, kbeg + kchunk);
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    for (int e = threadIdx.x; e < GT * GK; e += 256) {
      int m, k;
      if (sak == 1) { m = e / GK; k = e % GK; } else { m = e % GT; k = e / GT; }
      const int gm = m0 + m, gk = k0 + k;
      As[m][k] = (gm < M && gk < Kd) ? A[gm * sam + gk * sak] : uint16_t(0);
      int n, kb;
      if (sbk == 1) { n = e / GK; kb = e % GK; } else { n = e % GT; kb = e / GT; }
      const int gn = n0 + n, gkb = k0 + kb;
      Bs[n][kb] = (gn < N && gkb < Kd) ? B[gkb * sbk + gn * sbn] : uint16_t(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 16) {
      const uint4 a = load8(&As[wm * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
      const uint4 b = load8(&Bs[wn * 32 + (lane & 31)][kk + 8 * (lane >> 5)]);
      acc = mfma_bf16(a, b, acc);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int n = n0 + wn * 32 + (lane & 31);
    if (m >= M || n >= N) continue;
    const size_t o = size_t(m) * ldc + n;
    const float v = acc[r];
    if (EPI == EPI_F32) {
      // split-K block z writes its partial product to slice z (z = 0 unsplit)
      outf[size_t(blockIdx.z) * size_t(M) * ldc + o] = v;
    } else if (EPI == EPI_BIAS_F32) {
      outf[o] = v + bias[n];
    } else if (EPI == EPI_BIAS_GELU) {
      const float z = v + bias[n];
      Z[o] = z;
      outb[o] = f2bf(gelu(z));
    } else {
      const float dz = v * gelu_grad(Z[o]);
      outf[o] = dz;
      outb[o] = f2bf(dz);
    }
  }
}

// dst[i] = sum over z of part[z][i], z in increasing order: the split-K
// partial products added in a fixed order, so training is bit-reproducible
__global__ void k_sum_parts(const float *__restrict__ part, int splits, size_t count, float *__restrict__ dst) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[size_t(z) * count + i];
    dst[i] = s;
  }
}

// network input: x = a * inv_s (tilt slots carry inv_s = 0), bf16; targets
// standardised (beta - mu) / s_out
__global__ void k_prep(const float *__restrict__ a, const float *__restrict__ beta, int n_total,
                       int start, int B, const float *__restrict__ inv_s, const float *__restrict__ mu,
                       float inv_sout, int K, uint16_t *__restrict__ x, float *__restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int src = (start + i) % n_total;
  for (int j = 0; j < TSIM_N_MODES; ++j)
    x[size_t(i) * TSIM_N_MODES + j] = f2bf(a[size_t(src) * TSIM_N_MODES + j] * inv_s[j]);
  if (beta)
    for (int k = 0; k < K; ++k) t[size_t(i) * K + k] = (beta[size_t(src) * K + k] - mu[k]) * inv_sout;
}

// dY = 2 (Y - T) / (B K); loss += mean square
__global__ void k_mse_grad(const float *__restrict__ Y, const float *__restrict__ T, int n,
                           float scale, float *__restrict__ dzf, uint16_t *__restrict__ dzb,
                           float *__restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    const float g = 2.f * d * scale;
    dzf[i] = g;
    dzb[i] = f2bf(g);
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] * scale);
}

// db[n] = sum_m dZ[m][n]
// Column sums db[n] = sum_m dz[m][n] (M x N, N <= 256) in two passes with a
// fixed order: blocks of 64 columns x one chunk of rows write partial sums,
// then the partials are added in chunk order.
constexpr int CS_CHUNKS = 256;
__global__ void k_colsum_part(const float *__restrict__ dz, int M, int N, int rows, float *__restrict__ part) {
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int m0 = blockIdx.y * rows, m1 = min(M, m0 + rows);
  __shared__ float red[4][64];
  float s = 0.f;
  if (n < N)
    for (int m = m0 + g; m < m1; m += 4) s += dz[size_t(m) * N + n];
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && n < N)
    part[size_t(blockIdx.y) * N + n] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                       red[3][threadIdx.x];
}

__global__ void k_colsum_fin(const float *__restrict__ part, int chunks, int N, float *__restrict__ db) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += part[size_t(c) * N + n];
  db[n] = s;
}

// part holds CS_CHUNKS * N floats
void colsum(hipStream_t s, const float *dz, int M, int N, float *db, float *part) {
  const int chunks = std::max(1, std::min(CS_CHUNKS, (M + 255) / 256));
  const int rows = (M + chunks - 1) / chunks;
  hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, chunks), dim3(256), 0, s, dz, M, N, rows, part);
  hipLaunchKernelGGL(k_colsum_fin, dim3((N + 255) / 256), dim3(256), 0, s, part, chunks, N, db);
}

// sum of squared deviations from mu over [n][K] (output scale of the network)
__global__ void k_sqdev(const float *__restrict__ beta, const float *__restrict__ mu, size_t nel, int K,
                        float *__restrict__ acc) {
  __shared__ float red[256];
  float s = 0.f;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nel; i += size_t(gridDim.x) * blockDim.x) {
    const float d = beta[i] - mu[i % K];
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, red[0]);
}

__global__ void k_scale(float *__restrict__ v, int n, float s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] *= s;
}

__global__ void k_adamw(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, uint16_t *__restrict__ wb, int n, float lr, float b1,
                        float omb1, float b2, float omb2, float c1, float c2, float eps, float wd) {
  // omb1 = 1 - beta1 and omb2 = 1 - beta2 come rounded once from double:
  // 1.f - float(0.999) would be 1.3e-5 away from 0.001
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
  w[i] = wi;
  wb[i] = f2bf(wi);
}

__global__ void k_init_normal(float *__restrict__ w, uint16_t *__restrict__ wb, int n, float std,
                              uint32_t key0, uint32_t key1, uint32_t stream) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u32x4 r = philox4x32_10(u32x4{uint32_t(i), 0u, stream, 3u}, key0, key1);
  const float v = box_muller(r.x, r.y).x * std;
  w[i] = v;
  wb[i] = f2bf(v);
}

// training pairs: a = (D/r0)^{5/6} L g, g from Philox (i, w, 0, 2), D/r0 from (i, 9, 0, 2)
__global__ void k_draws(const float *__restrict__ Lmat, float *__restrict__ zvec, int n,
                        uint32_t key0, uint32_t key1, float lo, float hi, uint32_t tag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float g[36];
#pragma unroll
  for (int w = 0; w < 9; ++w) {
    u32x4 r = philox4x32_10(u32x4{uint32_t(i), uint32_t(w), 0u, tag}, key0, key1);
    float2 a = box_muller(r.x, r.y), b = box_muller(r.z, r.w);
    g[4 * w] = a.x; g[4 * w + 1] = a.y; g[4 * w + 2] = b.x; g[4 * w + 3] = b.y;
  }
  u32x4 r = philox4x32_10(u32x4{uint32_t(i), 9u, 0u, tag}, key0, key1);
  const float sc = powf(lo + (hi - lo) * u01(r.x), 5.0f / 6.0f);
  for (int j = 0; j < TSIM_N_MODES; ++j) {
    float s = 0.f;
    for (int k = 0; k <= j; ++k) s = fmaf(Lmat[j * TSIM_N_MODES + k], g[k], s);
    zvec[size_t(i) * TSIM_N_MODES + j] = s * sc;
  }
}

// ----------------------------------------------------------- inference ----
constexpr int HID = 256;
constexpr int IN_PAD = 48;   // 35 inputs padded to three 16-wide k-steps
constexpr int ACT_LD = HID + 8;
constexpr int IPX = 128;     // pixels per inference block (four 32-row tiles)

// The inference GELU, z Phi(z) = max(z, 0) - |z| erfc(|z| / sqrt 2) / 2 (one
// expression for both signs), with erfc by Abramowitz & Stegun 7.1.28:
// erfc(x) = (1 + a1 x + ... + a6 x^6)^-16, |error| <= 3e-7; the coefficients
// below are a_i 2^(-i/2) (argument |z| / sqrt 2) times 2^(1/16) (the factor
// 1/2), so one reciprocal and four squarings give erfc(|z| / sqrt 2) / 2.
__device__ __forceinline__ float gelu_fast(float z) {
  const float a = fabsf(z);
  const float p = fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(5.6212996640e-06f, a, 5.1055209009e-05f), a, 3.9686137011e-05f), a,
                                      3.4227392389e-03f), a, 2.2076998457e-02f), a, 5.2075163037e-02f), a,
                       1.0442737824e+00f);
  float r = __builtin_amdgcn_rcpf(p);
  r *= r;
  r *= r;
  r *= r;
  r *= r;
  return fmaf(-a, r, fmaxf(z, 0.f));
}

// Weight fragments of one layer for this wave, WD k-steps in flight: the
// loads for k-step s + WD are issued as soon as k-step s has been consumed,
// and the first WD k-steps of a layer while the previous layer's activations
// are formed.
constexpr int WD = 3;
template <int NT>
struct WRing {
  uint4 f[WD][NT];
};

// The weights are stored in matrix-core fragment order: for a layer of R
// rows (neurons) and KS = ldw / 16 k-steps, fragment (row tile nt, k-step s)
// is 1 KB at byte ((nt KS + s) 64 + lane) 16, lane l holding row
// 32 nt + l % 32, columns 16 s + 8 (l / 32) + 0..7; a wave's fragment load is
// one contiguous kilobyte.  Uniform base, 32-bit per-lane byte offset.
__device__ __forceinline__ uint4 wfrag(const uint16_t *__restrict__ W, uint32_t lane_off, uint32_t off) {
  return *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(W) + (lane_off + off));
}

struct InferParams {
  const uint16_t *W1, *W2, *W3, *W4;  // 256 x 48, 256 x 256, 256 x 256, 128 x 256 bf16, fragment order
  const float *b1, *b2, *b3, *b4;     // [256] x3, [128]
  const float *inv_s;                 // [35]
  const float *mu;                    // [128] output means (0 beyond K)
  float s_out;
  int K, KB;                          // outputs, row stride of beta
  int out_bf16;
};

// GELU(acc + bias) of quads [Q0, Q1) of a pixel half's products (quad =
// four adjacent neurons of one pixel, one 8-byte LDS write): quad idx is
// tile i = idx / (4 NT) of the half, neuron tile t = (idx / 4) % NT, group
// q = idx % 4 of the accumulator registers.
template <int NT, int Q0, int Q1>
__device__ __forceinline__ void gelu_quads(uint16_t *act, const f32x16 (&acc)[2][NT], const float *bias, int n0,
                                           int half, int lane) {
#pragma unroll
  for (int idx = Q0; idx < Q1; ++idx) {
    const int i = idx / (4 * NT), t = (idx / 4) % NT, q = idx % 4;
    const int n = n0 + 32 * t + 8 * q + 4 * (lane >> 5);
    const int m = 32 * (2 * half + i) + (lane & 31);
    const float4 bn = *reinterpret_cast<const float4 *>(bias + n);
    const f32x16 &a = acc[i][t];
    uint2 w;
    w.x = pack_bf16(gelu_fast(a[4 * q] + bn.x), gelu_fast(a[4 * q + 1] + bn.y));
    w.y = pack_bf16(gelu_fast(a[4 * q + 2] + bn.z), gelu_fast(a[4 * q + 3] + bn.w));
    *reinterpret_cast<uint2 *>(act + m * ACT_LD + n) = w;
  }
}

// Inference is pipelined over the two 64-pixel halves of a block: each
// wave owns one 32-neuron tile of every hidden layer, so its accumulators
// fit 128 registers and four waves share a SIMD.

// Steps S.. of a phase: acc[i] = W[32 nt0 + .][k] x
// act[tile tile0 + i][k]^T for RT pixel tiles, with the GELU of the other
// half's two tiles of the step before (gacc, 8 quads) spread over the
// k-steps.
template <int RT, int KS, bool GELU, int S = 0>
struct Phase8 {
  __device__ __forceinline__ static void step(uint16_t *act, const uint16_t *__restrict__ W, uint32_t lo,
                                              f32x16 (&acc)[RT][1], WRing<1> &ring, uint4 (&an)[RT],
                                              const uint16_t *arow, const f32x16 (&gacc)[2][1],
                                              const float *gbias, int gn0, int ghalf, int lane) {
    if constexpr (S < KS) {
      uint4 a[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = an[i];
      if constexpr (S + 1 < KS) {
#pragma unroll
        for (int i = 0; i < RT; ++i) an[i] = load8(arow + 32 * i * ACT_LD + (S + 1) * 16);
      }
#pragma unroll
      for (int i = 0; i < RT; ++i) acc[i][0] = mfma_bf16(ring.f[S % WD][0], a[i], acc[i][0]);
      if constexpr (S + WD < KS) ring.f[S % WD][0] = wfrag(W, lo, uint32_t((S + WD) * 1024));
      if constexpr (GELU) gelu_quads<1, S * 8 / KS, (S + 1) * 8 / KS>(act, gacc, gbias, gn0, ghalf, lane);
      Phase8<RT, KS, GELU, S + 1>::step(act, W, lo, acc, ring, an, arow, gacc, gbias, gn0, ghalf, lane);
    }
  }
};

template <int RT, int KS, bool GELU>
__device__ __forceinline__ void phase8(uint16_t *act, int tile0, const uint16_t *__restrict__ W, int nt0,
                                       f32x16 (&acc)[RT][1], WRing<1> &ring, const f32x16 (&gacc)[2][1],
                                       const float *gbias, int gn0, int ghalf, int lane) {
#pragma unroll
  for (int i = 0; i < RT; ++i) acc[i][0] = f32x16{};
  const uint32_t lo = uint32_t(lane * 16 + nt0 * KS * 1024);
  const uint16_t *arow = act + (32 * tile0 + (lane & 31)) * ACT_LD + 8 * (lane >> 5);
  uint4 an[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) an[i] = load8(arow + 32 * i * ACT_LD);
  Phase8<RT, KS, GELU>::step(act, W, lo, acc, ring, an, arow, gacc, gbias, gn0, ghalf, lane);
}

template <int KS>
__device__ __forceinline__ void w_prefetch1(WRing<1> &ring, const uint16_t *__restrict__ W, int nt0, int lane) {
  const uint32_t lo = uint32_t(lane * 16 + nt0 * KS * 1024);
#pragma unroll
  for (int d = 0; d < WD && d < KS; ++d) ring.f[d][0] = wfrag(W, lo, uint32_t(d * 1024));
}

// Output epilogue of one 32-pixel tile and one 32-output tile (n0w):
// beta = (acc + b4) s_out + mu, four adjacent basis weights of a pixel per store.
__device__ __forceinline__ void mlp_out_tile(const f32x16 &acc, const InferParams &ip, const float *b4,
                                             const float *mu, size_t p, int n0w, int lane, size_t n_pix,
                                             void *__restrict__ beta) {
  if (p >= n_pix) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = n0w + 8 * q + 4 * (lane >> 5);
    if (n >= ip.KB) continue;
    const float4 bn = *reinterpret_cast<const float4 *>(b4 + n);
    const float4 mn = *reinterpret_cast<const float4 *>(mu + n);
    const float bv[4] = {bn.x, bn.y, bn.z, bn.w}, mv[4] = {mn.x, mn.y, mn.z, mn.w};
    float y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = (n + j < ip.K) ? (acc[4 * q + j] + bv[j]) * ip.s_out + mv[j] : 0.f;
    if ((ip.KB & 3) == 0) {   // whole, aligned quads
      if (ip.out_bf16) {
        uint2 wv;
        wv.x = pack_bf16(y[0], y[1]);
        wv.y = pack_bf16(y[2], y[3]);
        *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(beta) + p * ip.KB + n) = wv;
      } else {
        *reinterpret_cast<float4 *>(static_cast<float *>(beta) + p * ip.KB + n) = make_float4(y[0], y[1], y[2], y[3]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (n + j >= ip.KB) break;
        if (ip.out_bf16)
          static_cast<uint16_t *>(beta)[p * ip.KB + n + j] = f2bf(y[j]);
        else
          static_cast<float *>(beta)[p * ip.KB + n + j] = y[j];
      }
    }
  }
}

// Block: 128 pixels in two halves of 64 (two 32-row tiles each), 8 waves.
// Wave w computes the neurons [32 w, +32) of each hidden layer for all 128
// pixels, one half at a time (a weight fragment feeds two products); in the
// output layer it takes output tile w % 4 of pixel tile w / 4 of the half.
// The halves are pipelined: while the matrix cores take layer l for one
// half, the vector ALU forms the other half's GELU activations of the layer
// before, in place in LDS.  One barrier per phase (every wave has read the
// rows a phase overwrites, and written the rows the next phase reads).
// Biases and output means are staged in LDS.
__global__ void __launch_bounds__(512, 4)
k_mlp_infer(const float *__restrict__ zern, int hw, size_t n_pix, InferParams ip, void *__restrict__ beta) {
  __shared__ __attribute__((aligned(16))) uint16_t act[IPX * ACT_LD];
  __shared__ __attribute__((aligned(16))) float sb[3 * HID + 128 + 128];   // b1 b2 b3 b4 mu
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t pb = size_t(blockIdx.x) * IPX;
  const int n0 = w * 32;
  constexpr int K1 = IN_PAD / 16, KH = HID / 16;
  WRing<1> ring;
  w_prefetch1<K1>(ring, ip.W1, w, lane);
  for (int e = threadIdx.x; e < 3 * HID + 256; e += 512) {
    float v;
    if (e < HID) v = ip.b1[e];
    else if (e < 2 * HID) v = ip.b2[e - HID];
    else if (e < 3 * HID) v = ip.b3[e - 2 * HID];
    else if (e < 3 * HID + 128) v = ip.b4[e - 3 * HID];
    else v = ip.mu[e - 3 * HID - 128];
    sb[e] = v;
  }
  {
    // inputs: thread -> pixel (tid % 128), modes [12 (tid / 128), +12)
    const int px = threadIdx.x & 127, j0 = (threadIdx.x >> 7) * 12;
    const size_t p = pb + px;
    const bool ok = p < n_pix;
    const size_t pc = ok ? p : 0;
    const size_t fr = pc / size_t(hw), yx = pc - fr * size_t(hw);
    const float *zp = zern + fr * TSIM_N_MODES * size_t(hw) + yx;
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const int j = j0 + q;
      const float v = (ok && j < TSIM_N_MODES) ? zp[size_t(j) * hw] * ip.inv_s[j] : 0.f;
      act[px * ACT_LD + j] = f2bf(v);
    }
  }
  __syncthreads();
  const float *b1 = sb, *b2 = sb + HID, *b3 = sb + 2 * HID, *b4 = sb + 3 * HID, *mu = sb + 3 * HID + 128;
  f32x16 A[2][1], B[2][1];
  phase8<2, K1, false>(act, 0, ip.W1, w, A, ring, B, nullptr, 0, 0, lane);     // layer 1, half 0
  w_prefetch1<K1>(ring, ip.W1, w, lane);
  __syncthreads();
  phase8<2, K1, true>(act, 2, ip.W1, w, B, ring, A, b1, n0, 0, lane);          // layer 1 half 1 + GELU1 half 0
  w_prefetch1<KH>(ring, ip.W2, w, lane);
  __syncthreads();
  phase8<2, KH, true>(act, 0, ip.W2, w, A, ring, B, b1, n0, 1, lane);          // layer 2 half 0 + GELU1 half 1
  w_prefetch1<KH>(ring, ip.W2, w, lane);
  __syncthreads();
  phase8<2, KH, true>(act, 2, ip.W2, w, B, ring, A, b2, n0, 0, lane);          // layer 2 half 1 + GELU2 half 0
  w_prefetch1<KH>(ring, ip.W3, w, lane);
  __syncthreads();
  phase8<2, KH, true>(act, 0, ip.W3, w, A, ring, B, b2, n0, 1, lane);          // layer 3 half 0 + GELU2 half 1
  w_prefetch1<KH>(ring, ip.W3, w, lane);
  __syncthreads();
  phase8<2, KH, true>(act, 2, ip.W3, w, B, ring, A, b3, n0, 0, lane);          // layer 3 half 1 + GELU3 half 0
  const int ot = w & 3, pt = w >> 2;   // output tile and pixel tile (within a half) of this wave
  w_prefetch1<KH>(ring, ip.W4, ot, lane);
  __syncthreads();
  f32x16 A1[1][1], B1[1][1];
  phase8<1, KH, true>(act, pt, ip.W4, ot, A1, ring, B, b3, n0, 1, lane);       // layer 4 half 0 + GELU3 half 1
  w_prefetch1<KH>(ring, ip.W4, ot, lane);
  __syncthreads();
  phase8<1, KH, false>(act, 2 + pt, ip.W4, ot, B1, ring, B, nullptr, 0, 0, lane);   // layer 4 half 1
  mlp_out_tile(A1[0][0], ip, b4, mu, pb + 32 * pt + (lane & 31), 32 * ot, lane, n_pix, beta);
  mlp_out_tile(B1[0][0], ip, b4, mu, pb + 32 * (2 + pt) + (lane & 31), 32 * ot, lane, n_pix, beta);
}


template <int EPI>
int gemm(hipStream_t s, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn,
         int M, int N, int Kd, const float *bias, float *Z, float *outf, uint16_t *outb, int ldc,
         int splits = 1) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
  hipLaunchKernelGGL(k_gemm_bf16<EPI>, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, M, N, Kd,
                     bias, Z, outf, outb, ldc);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

}  // namespace

// ------------------------------------------------------------------ host --
struct tsim_mlp {
  int K = 0, B = 0;
  size_t n_par = 0;
  size_t off_w[4], off_b[4];
  int din[4], dout[4];
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // flat FP32
  uint16_t *wb = nullptr;                                         // flat BF16 copy
  float *inv_s = nullptr, *mu = nullptr;                          // [35], [K]
  float s_out = 1.f;
  uint16_t *x = nullptr, *act[3] = {nullptr, nullptr, nullptr}, *dzb = nullptr;
  float *z[3] = {nullptr, nullptr, nullptr}, *y = nullptr, *t = nullptr, *dzf = nullptr;
  float *loss = nullptr;
  float *colpart = nullptr;                                      // [CS_CHUNKS][256] column-sum partials
  float *gpart = nullptr;                                        // [splits][dout * din] split-K partials
  int step = 0;                                                  // step within the current call (loss slot)
  long long t_done = 0;                                          // optimiser steps taken so far
  long long sched = 0;                                           // cosine schedule length (0: per call)
  std::vector<double> A0diag;
};

namespace {

void mlp_free(tsim_mlp *n) {
  if (!n) return;
  void *ptrs[] = {n->w, n->g, n->m, n->v, n->wb, n->inv_s, n->mu, n->x, n->act[0], n->act[1],
                  n->act[2], n->dzb, n->z[0], n->z[1], n->z[2], n->y, n->t, n->dzf, n->loss, n->colpart,
                  n->gpart};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete n;
}

template <class T>
bool dalloc(T **p, size_t n) {
  return hipMalloc(p, std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess;
}

// split-K of the weight gradients: at most this many blocks per product, so
// the partials (splits x dout x din <= kMaxSplitBlocks x GT x GT floats) fit
// one buffer
constexpr int kMaxSplitBlocks = 512;

// forward + backward for the current batch (x, t already prepared)
int mlp_fwd_bwd(tsim_mlp *n, int Bsz, hipStream_t s) {
  const int H = HID, K = n->K;
  int st;
  const uint16_t *Wb[4];
  for (int l = 0; l < 4; ++l) Wb[l] = n->wb + n->off_w[l];
  const float *bf[4];
  for (int l = 0; l < 4; ++l) bf[l] = n->w + n->off_b[l];
  // forward
  if ((st = gemm<EPI_BIAS_GELU>(s, n->x, TSIM_N_MODES, 1, Wb[0], 1, TSIM_N_MODES, Bsz, H, TSIM_N_MODES,
                                 bf[0], n->z[0], nullptr, n->act[0], H)) != TSIM_OK) return st;
  for (int l = 1; l < 3; ++l)
    if ((st = gemm<EPI_BIAS_GELU>(s, n->act[l - 1], H, 1, Wb[l], 1, H, Bsz, H, H, bf[l], n->z[l],
                                   nullptr, n->act[l], H)) != TSIM_OK) return st;
  if ((st = gemm<EPI_BIAS_F32>(s, n->act[2], H, 1, Wb[3], 1, H, Bsz, K, H, bf[3], nullptr, n->y,
                                nullptr, K)) != TSIM_OK) return st;
  // loss gradient
  const int nel = Bsz * K;
  hipLaunchKernelGGL(k_mse_grad, dim3(std::min(1024, (nel + 255) / 256)), dim3(256), 0, s, n->y, n->t,
                     nel, 1.0f / float(nel), n->dzf, n->dzb, n->loss + n->step);
  // backward: layer l has input act[l-1] (x for l = 0), output gradient dZ (dzf/dzb, width dout)
  for (int l = 3; l >= 0; --l) {
    const int dout = n->dout[l], din = n->din[l];
    const uint16_t *in = (l == 0) ? n->x : n->act[l - 1];
    // dW = dZ^T X: M = dout, N = din, reduction over the batch, split over
    // the batch so that ~512 blocks run; the partial products are added in
    // split order by a second kernel (no atomics: bit-reproducible)
    const int tiles = ((dout + GT - 1) / GT) * ((din + GT - 1) / GT);
    const int splits = std::max(1, std::min(Bsz / 256, kMaxSplitBlocks / tiles));
    float *gw = n->g + n->off_w[l];
    if ((st = gemm<EPI_F32>(s, n->dzb, 1, dout, in, din, 1, dout, din, Bsz, nullptr, nullptr,
                            splits > 1 ? n->gpart : gw, nullptr, din, splits)) != TSIM_OK) return st;
    if (splits > 1) {
      const size_t cnt = size_t(dout) * din;
      hipLaunchKernelGGL(k_sum_parts, dim3(unsigned(std::min<size_t>((cnt + 255) / 256, 1024))), dim3(256), 0, s,
                         n->gpart, splits, cnt, gw);
    }
    colsum(s, n->dzf, Bsz, dout, n->g + n->off_b[l], n->colpart);
    if (l > 0) {
      // dA = dZ W (M = batch, N = din, reduction over dout), then dZ_prev = dA * GELU'(Z_prev).
      // dZ of width din is written after the product has consumed dZ of width dout,
      // so the two share buffers only across separate launches (stream order).
      if ((st = gemm<EPI_GELU_GRAD>(s, n->dzb, dout, 1, Wb[l], din, 1, Bsz, din, dout, nullptr,
                                    n->z[l - 1], n->dzf + size_t(Bsz) * 256, n->dzb + size_t(Bsz) * 256,
                                    din)) != TSIM_OK) return st;
      // move the new dZ to the front of the buffers
      if (hipMemcpyAsync(n->dzf, n->dzf + size_t(Bsz) * 256, size_t(Bsz) * din * sizeof(float),
                         hipMemcpyDeviceToDevice, s) != hipSuccess) return TSIM_EDEVICE;
      if (hipMemcpyAsync(n->dzb, n->dzb + size_t(Bsz) * 256, size_t(Bsz) * din * sizeof(uint16_t),
                         hipMemcpyDeviceToDevice, s) != hipSuccess) return TSIM_EDEVICE;
    }
  }
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

}  // namespace

namespace {

int mlp_create_impl(const tsim_plan *pl, int batch, uint64_t seed, tsim_mlp **out) {
  if (!pl || !out || batch < 1 || batch > (1 << 20)) return TSIM_EINVAL;
  *out = nullptr;
  if (pl->K > 128 || pl->N != TSIM_N_MODES) return TSIM_EUNSUPPORTED;   // 35 network inputs
  tsim_mlp *n = new (std::nothrow) tsim_mlp();
  if (!n) return TSIM_ENOMEM;
  n->K = pl->K;
  n->B = batch;
  const int dims[5] = {TSIM_N_MODES, HID, HID, HID, pl->K};
  size_t off = 0;
  for (int l = 0; l < 4; ++l) {
    n->din[l] = dims[l];
    n->dout[l] = dims[l + 1];
    n->off_w[l] = off;
    off += size_t(dims[l]) * dims[l + 1];
    off = (off + 63) & ~size_t(63);
    n->off_b[l] = off;
    off += dims[l + 1];
    off = (off + 63) & ~size_t(63);
  }
  n->n_par = off;
  const size_t B = batch;
  bool ok = dalloc(&n->w, off) && dalloc(&n->g, off) && dalloc(&n->m, off) && dalloc(&n->v, off) &&
            dalloc(&n->wb, off) && dalloc(&n->inv_s, TSIM_N_MODES) && dalloc(&n->mu, 128) &&
            dalloc(&n->x, B * TSIM_N_MODES) && dalloc(&n->y, B * pl->K) && dalloc(&n->t, B * pl->K) &&
            dalloc(&n->dzf, 2 * B * 256) && dalloc(&n->dzb, 2 * B * 256) && dalloc(&n->loss, 1 << 20) &&
            dalloc(&n->colpart, size_t(CS_CHUNKS) * 256) && dalloc(&n->gpart, size_t(kMaxSplitBlocks) * GT * GT);
  for (int l = 0; l < 3 && ok; ++l) ok = dalloc(&n->act[l], B * HID) && dalloc(&n->z[l], B * HID);
  if (!ok) {
    mlp_free(n);
    return TSIM_ENOMEM;
  }
  if (hipMemset(n->w, 0, off * 4) != hipSuccess || hipMemset(n->g, 0, off * 4) != hipSuccess ||
      hipMemset(n->m, 0, off * 4) != hipSuccess ||
      hipMemset(n->v, 0, off * 4) != hipSuccess || hipMemset(n->wb, 0, off * 2) != hipSuccess ||
      hipMemset(n->mu, 0, 128 * 4) != hipSuccess || hipMemset(n->loss, 0, (1 << 20) * 4) != hipSuccess) {
    mlp_free(n);
    return TSIM_EDEVICE;
  }
  // seeded initialisation: W ~ N(0, 1/fan_in), biases 0 (Philox counters (i, 0, layer, 3))
  for (int l = 0; l < 4; ++l) {
    const int cnt = n->din[l] * n->dout[l];
    const float sd = 1.0f / std::sqrt(float(n->din[l]));
    hipLaunchKernelGGL(k_init_normal, dim3((cnt + 255) / 256), dim3(256), 0, 0, n->w + n->off_w[l],
                       n->wb + n->off_w[l], cnt, sd, uint32_t(seed), uint32_t(seed >> 32), uint32_t(l));
  }
  // input scales: 1 / sqrt(A0[j][j] (D/r0)^{5/3}) at D/r0 = 2.75, tilt slots 0
  std::vector<float> inv(TSIM_N_MODES, 0.f);
  for (int j = 2; j < TSIM_N_MODES; ++j)
    inv[j] = float(1.0 / std::sqrt(pl->A0[size_t(j) * TSIM_N_MODES + j] * std::pow(2.75, 5.0 / 3.0)));
  if (hipMemcpy(n->inv_s, inv.data(), inv.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    mlp_free(n);
    return TSIM_EDEVICE;
  }
  *out = n;
  return TSIM_OK;
}

int mlp_destroy_impl(tsim_mlp *n) {
  mlp_free(n);
  return TSIM_OK;
}

int mlp_param_count_impl(const tsim_mlp *n, size_t *count) {
  if (!n || !count) return TSIM_EINVAL;
  *count = n->n_par;
  return TSIM_OK;
}

int mlp_layout_impl(const tsim_mlp *n, size_t *off_w, size_t *off_b) {
  if (!n || !off_w || !off_b) return TSIM_EINVAL;
  for (int l = 0; l < 4; ++l) {
    off_w[l] = n->off_w[l];
    off_b[l] = n->off_b[l];
  }
  return TSIM_OK;
}

int mlp_get_impl(const tsim_mlp *n, int what, float *host, size_t count) {
  if (!n || !host) return TSIM_EINVAL;
  const float *src = nullptr;
  size_t cnt = n->n_par;
  switch (what) {
    case 0: src = n->w; break;
    case 1: src = n->g; break;
    case 2: src = n->inv_s; cnt = TSIM_N_MODES; break;
    case 3: src = n->mu; cnt = size_t(n->K); break;
    case 4:
      if (count < 1) return TSIM_EINVAL;
      host[0] = n->s_out;
      return TSIM_OK;
    case 5: src = n->m; break;
    case 6: src = n->v; break;
    case 7:
      if (count < 2) return TSIM_EINVAL;
      host[0] = float(n->t_done);
      host[1] = float(n->sched);
      return TSIM_OK;
    default: return TSIM_EINVAL;
  }
  if (count < cnt) return TSIM_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return TSIM_EDEVICE;
  return hipMemcpy(host, src, cnt * 4, hipMemcpyDeviceToHost) == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

int mlp_set_impl(tsim_mlp *n, int what, const float *host, size_t count) {
  if (!n || !host) return TSIM_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return TSIM_EDEVICE;
  switch (what) {
    case 0: {
      if (count != n->n_par) return TSIM_EINVAL;
      std::vector<uint16_t> b(n->n_par);
      for (size_t i = 0; i < n->n_par; ++i) {
        uint32_t u;
        std::memcpy(&u, &host[i], 4);
        b[i] = uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
      }
      if (hipMemcpy(n->w, host, n->n_par * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(n->wb, b.data(), n->n_par * 2, hipMemcpyHostToDevice) != hipSuccess)
        return TSIM_EDEVICE;
      return TSIM_OK;
    }
    case 2:
      if (count != TSIM_N_MODES) return TSIM_EINVAL;
      return hipMemcpy(n->inv_s, host, count * 4, hipMemcpyHostToDevice) == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
    case 3:
      if (count != size_t(n->K)) return TSIM_EINVAL;
      return hipMemcpy(n->mu, host, count * 4, hipMemcpyHostToDevice) == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
    case 4:
      if (count != 1 || !(host[0] > 0.f)) return TSIM_EINVAL;
      n->s_out = host[0];
      return TSIM_OK;
    case 5:
    case 6:
      if (count != n->n_par) return TSIM_EINVAL;
      return hipMemcpy(what == 5 ? n->m : n->v, host, count * 4, hipMemcpyHostToDevice) == hipSuccess
                 ? TSIM_OK
                 : TSIM_EDEVICE;
    case 7: {
      // whole numbers in [0, 2^24), where float holds every integer exactly
      if (count != 2) return TSIM_EINVAL;
      for (int i = 0; i < 2; ++i)
        if (!(host[i] >= 0.f && host[i] < 16777216.f) || host[i] != std::floor(host[i])) return TSIM_EINVAL;
      n->t_done = static_cast<long long>(host[0]);
      n->sched = static_cast<long long>(host[1]);
      return TSIM_OK;
    }
    default: return TSIM_EINVAL;
  }
}

int mlp_data_ws_bytes_impl(const tsim_plan *pl, int n_pairs, size_t *bytes) {
  if (!pl || n_pairs < 1 || !bytes) return TSIM_EINVAL;
  *bytes = p2s_chunk_pixels(pl, size_t(n_pairs)) * size_t(pl->T) * pl->T * sizeof(float);
  return TSIM_OK;
}

int mlp_make_data_impl(const tsim_plan *pl, int n_pairs, uint64_t seed, float dr_lo, float dr_hi,
                       float *zvec, float *beta, void *ws, tsim_stream stream) {
  if (!pl || n_pairs < 1 || !zvec || !beta || !ws) return TSIM_EINVAL;
  if (pl->N != TSIM_N_MODES) return TSIM_EUNSUPPORTED;
  if (!pl->d_basis) return TSIM_EARTEFACT;
  if (!(dr_lo > 0.f) || !(dr_hi >= dr_lo)) return TSIM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_draws, dim3((n_pairs + 255) / 256), dim3(256), 0, s, pl->d_L, zvec, n_pairs,
                     uint32_t(seed), uint32_t(seed >> 32), dr_lo, dr_hi, 2u);
  if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  const size_t chunk = p2s_chunk_pixels(pl, size_t(n_pairs));
  for (size_t p0 = 0; p0 < size_t(n_pairs); p0 += chunk) {
    const int cnt = int(std::min(chunk, size_t(n_pairs) - p0));
    int st = launch_psf_exact(pl, cnt, zvec + p0 * TSIM_N_MODES, static_cast<float *>(ws), s);
    if (st != TSIM_OK) return st;
    st = launch_project(pl, static_cast<float *>(ws), cnt, beta + p0 * pl->K, 0, s);
    if (st != TSIM_OK) return st;
  }
  return TSIM_OK;
}

int mlp_grad_impl(tsim_mlp *n, int batch, const float *zvec, const float *target, float *loss_host,
                  tsim_stream stream) {
  if (!n || batch < 1 || batch > n->B || !zvec || !target) return TSIM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_prep, dim3((batch + 255) / 256), dim3(256), 0, s, zvec, target, batch, 0, batch,
                     n->inv_s, n->mu, 1.0f / n->s_out, n->K, n->x, n->t);
  if (hipMemsetAsync(n->loss + n->step, 0, 4, s) != hipSuccess) return TSIM_EDEVICE;
  int st = mlp_fwd_bwd(n, batch, s);
  if (st != TSIM_OK) return st;
  if (loss_host) {
    if (hipStreamSynchronize(s) != hipSuccess) return TSIM_EDEVICE;
    if (hipMemcpy(loss_host, n->loss + n->step, 4, hipMemcpyDeviceToHost) != hipSuccess) return TSIM_EDEVICE;
  }
  return TSIM_OK;
}

int mlp_fit_output_impl(tsim_mlp *n, const float *target, int n_pairs, tsim_stream stream) {
  if (!n || !target || n_pairs < 1) return TSIM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  colsum(s, target, n_pairs, n->K, n->mu, n->colpart);
  hipLaunchKernelGGL(k_scale, dim3(1), dim3(128), 0, s, n->mu, n->K, 1.0f / float(n_pairs));
  if (hipMemsetAsync(n->loss, 0, 4, s) != hipSuccess) return TSIM_EDEVICE;
  const size_t nel = size_t(n_pairs) * n->K;
  hipLaunchKernelGGL(k_sqdev, dim3(1024), dim3(256), 0, s, target, n->mu, nel, n->K, n->loss);
  float sq = 0.f;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(&sq, n->loss, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return TSIM_EDEVICE;
  const float rms = std::sqrt(sq / float(nel));
  if (!(rms > 0.f) || !std::isfinite(rms)) return TSIM_EINVAL;
  n->s_out = rms;
  return TSIM_OK;
}

int mlp_predict_impl(const tsim_plan *pl, int n_vec, const float *zvec, float *beta, tsim_stream stream) {
  if (!pl || n_vec < 1 || !zvec || !beta) return TSIM_EINVAL;
  if (!pl->d_mlp_w) return TSIM_EARTEFACT;
  return launch_mlp_infer(pl, zvec, 1, size_t(n_vec), beta, 0, pl->K, static_cast<hipStream_t>(stream));
}

int mlp_train_impl(tsim_mlp *n, const float *zvec, const float *target, int n_pairs, int steps,
                   float lr_max, float lr_min, float *loss_host, tsim_stream stream) {
  if (!n || !zvec || !target || n_pairs < n->B || steps < 1 || steps > (1 << 20)) return TSIM_EINVAL;
  if (!(lr_max > 0.f) || !(lr_min >= 0.f)) return TSIM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipMemsetAsync(n->loss, 0, size_t(steps) * 4, s) != hipSuccess) return TSIM_EDEVICE;
  const int B = n->B;
  const double b1 = 0.9, b2 = 0.999;
  for (int it = 0; it < steps; ++it) {
    n->step = it;
    const long long tg = n->t_done;  // global step: batch position, schedule, bias correction
    const int start = int((static_cast<unsigned long long>(tg) * unsigned(B)) % size_t(n_pairs));
    hipLaunchKernelGGL(k_prep, dim3((B + 255) / 256), dim3(256), 0, s, zvec, target, n_pairs, start, B,
                       n->inv_s, n->mu, 1.0f / n->s_out, n->K, n->x, n->t);
    int st = mlp_fwd_bwd(n, B, s);
    if (st != TSIM_OK) return st;
    double prog;
    if (n->sched > 0)
      prog = n->sched > 1 ? double(std::min(tg, n->sched - 1)) / double(n->sched - 1) : 1.0;
    else
      prog = steps > 1 ? double(it) / double(steps - 1) : 1.0;
    const float lr = float(lr_min + 0.5 * (lr_max - lr_min) * (1.0 + std::cos(3.14159265358979 * prog)));
    const double t = double(tg + 1);
    hipLaunchKernelGGL(k_adamw, dim3(int((n->n_par + 255) / 256)), dim3(256), 0, s, n->w, n->g, n->m,
                       n->v, n->wb, int(n->n_par), lr, float(b1), float(1.0 - b1), float(b2),
                       float(1.0 - b2), float(1.0 - std::pow(b1, t)), float(1.0 - std::pow(b2, t)), 1e-8f,
                       0.0f);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
    ++n->t_done;
  }
  n->step = 0;
  if (loss_host) {
    if (hipStreamSynchronize(s) != hipSuccess) return TSIM_EDEVICE;
    if (hipMemcpy(loss_host, n->loss, size_t(steps) * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return TSIM_EDEVICE;
  }
  return TSIM_OK;
}

}  // namespace

extern "C" {
int tsim_mlp_create(const tsim_plan *pl, int batch, uint64_t seed, tsim_mlp **out) {
  return note_status("tsim_mlp_create", mlp_create_impl(pl, batch, seed, out));
}

int tsim_mlp_destroy(tsim_mlp *n) {
  return note_status("tsim_mlp_destroy", mlp_destroy_impl(n));
}

int tsim_mlp_param_count(const tsim_mlp *n, size_t *count) {
  return note_status("tsim_mlp_param_count", mlp_param_count_impl(n, count));
}

int tsim_mlp_layout(const tsim_mlp *n, size_t *off_w, size_t *off_b) {
  return note_status("tsim_mlp_layout", mlp_layout_impl(n, off_w, off_b));
}

int tsim_mlp_get(const tsim_mlp *n, int what, float *host, size_t count) {
  return note_status("tsim_mlp_get", mlp_get_impl(n, what, host, count));
}

int tsim_mlp_set(tsim_mlp *n, int what, const float *host, size_t count) {
  return note_status("tsim_mlp_set", mlp_set_impl(n, what, host, count));
}

int tsim_mlp_data_ws_bytes(const tsim_plan *pl, int n_pairs, size_t *bytes) {
  return note_status("tsim_mlp_data_ws_bytes", mlp_data_ws_bytes_impl(pl, n_pairs, bytes));
}

int tsim_mlp_make_data(const tsim_plan *pl, int n_pairs, uint64_t seed, float dr_lo, float dr_hi, float *zvec,
                       float *beta, void *ws, tsim_stream stream) {
  return note_status("tsim_mlp_make_data",
                     mlp_make_data_impl(pl, n_pairs, seed, dr_lo, dr_hi, zvec, beta, ws, stream));
}

int tsim_mlp_grad(tsim_mlp *n, int batch, const float *zvec, const float *target, float *loss_host,
                  tsim_stream stream) {
  return note_status("tsim_mlp_grad", mlp_grad_impl(n, batch, zvec, target, loss_host, stream));
}

int tsim_mlp_fit_output(tsim_mlp *n, const float *target, int n_pairs, tsim_stream stream) {
  return note_status("tsim_mlp_fit_output", mlp_fit_output_impl(n, target, n_pairs, stream));
}

int tsim_mlp_predict(const tsim_plan *pl, int n_vec, const float *zvec, float *beta, tsim_stream stream) {
  return note_status("tsim_mlp_predict", mlp_predict_impl(pl, n_vec, zvec, beta, stream));
}

int tsim_mlp_train(tsim_mlp *n, const float *zvec, const float *target, int n_pairs, int steps, float lr_max,
                   float lr_min, float *loss_host, tsim_stream stream) {
  return note_status("tsim_mlp_train",
                     mlp_train_impl(n, zvec, target, n_pairs, steps, lr_max, lr_min, loss_host, stream));
}

}  // extern "C"

// Pack the network into the plan's inference layout (padded BF16 weights).
int plan_set_mlp_impl(tsim_plan *pl, const tsim_mlp *n) {
  if (!pl || !n || n->K != pl->K) return TSIM_EINVAL;
  if (pl->N != TSIM_N_MODES) return TSIM_EUNSUPPORTED;
  if (hipDeviceSynchronize() != hipSuccess) return TSIM_EDEVICE;
  std::vector<float> w(n->n_par), inv(TSIM_N_MODES), mu(n->K);
  if (hipMemcpy(w.data(), n->w, w.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(inv.data(), n->inv_s, inv.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(mu.data(), n->mu, mu.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return TSIM_EDEVICE;
  auto bf = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
  };
  // row-major, zero padded: W1 [256][48] | W2 [256][256] | W3 [256][256] | W4 [128][256]
  const size_t s1 = size_t(HID) * IN_PAD, s2 = size_t(HID) * HID, s4 = size_t(128) * HID;
  std::vector<uint16_t> rm(s1 + 2 * s2 + s4, 0);
  for (int o = 0; o < HID; ++o)
    for (int i = 0; i < TSIM_N_MODES; ++i) rm[size_t(o) * IN_PAD + i] = bf(w[n->off_w[0] + size_t(o) * TSIM_N_MODES + i]);
  for (int l = 1; l < 3; ++l)
    for (size_t e = 0; e < s2; ++e) rm[s1 + (l - 1) * s2 + e] = bf(w[n->off_w[l] + e]);
  for (int o = 0; o < n->K; ++o)
    for (int i = 0; i < HID; ++i) rm[s1 + 2 * s2 + size_t(o) * HID + i] = bf(w[n->off_w[3] + size_t(o) * HID + i]);
  // the same matrices in matrix-core fragment order (the kernel's wfrag):
  // element (row r, column k) of an R x 16 KS layer goes to
  // ((r / 32 * KS + k / 16) * 64 + r % 32 + 32 (k % 16 / 8)) * 8 + k % 8
  std::vector<uint16_t> pk(rm.size(), 0);
  const size_t base[4] = {0, s1, s1 + s2, s1 + 2 * s2};
  const int rows[4] = {HID, HID, HID, 128}, cols[4] = {IN_PAD, HID, HID, HID};
  for (int l = 0; l < 4; ++l) {
    const int ks = cols[l] / 16;
    for (int r = 0; r < rows[l]; ++r)
      for (int k = 0; k < cols[l]; ++k) {
        const size_t dst = (size_t((r / 32) * ks + k / 16) * 64 + r % 32 + 32 * ((k % 16) / 8)) * 8 + k % 8;
        pk[base[l] + dst] = rm[base[l] + size_t(r) * cols[l] + k];
      }
  }
  // FP32: b1 | b2 | b3 | b4[128] | inv_s[35] (pad 64) | mu[128]
  std::vector<float> fb(3 * HID + 128 + 64 + 128, 0.f);
  for (int l = 0; l < 3; ++l)
    for (int o = 0; o < HID; ++o) fb[l * HID + o] = w[n->off_b[l] + o];
  for (int o = 0; o < n->K; ++o) fb[3 * HID + o] = w[n->off_b[3] + o];
  for (int j = 0; j < TSIM_N_MODES; ++j) fb[3 * HID + 128 + j] = inv[j];
  for (int o = 0; o < n->K; ++o) fb[3 * HID + 128 + 64 + o] = mu[o];
  if (!pl->d_mlp_w && hipMalloc(&pl->d_mlp_w, pk.size() * 2) != hipSuccess) return TSIM_ENOMEM;
  if (!pl->d_mlp_f && hipMalloc(&pl->d_mlp_f, fb.size() * 4) != hipSuccess) return TSIM_ENOMEM;
  if (hipMemcpy(pl->d_mlp_w, pk.data(), pk.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pl->d_mlp_f, fb.data(), fb.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return TSIM_EDEVICE;
  pl->mlp_s_out = n->s_out;
  return TSIM_OK;
}

int launch_mlp_infer(const tsim_plan *pl, const float *zern, int hw, size_t n_pix, void *beta,
                     int out_bf16, int kb, hipStream_t s) {
  if (!pl->d_mlp_w) return TSIM_EARTEFACT;
  InferParams ip;
  const size_t s1 = size_t(HID) * IN_PAD, s2 = size_t(HID) * HID;
  ip.W1 = pl->d_mlp_w;
  ip.W2 = pl->d_mlp_w + s1;
  ip.W3 = pl->d_mlp_w + s1 + s2;
  ip.W4 = pl->d_mlp_w + s1 + 2 * s2;
  ip.b1 = pl->d_mlp_f;
  ip.b2 = pl->d_mlp_f + HID;
  ip.b3 = pl->d_mlp_f + 2 * HID;
  ip.b4 = pl->d_mlp_f + 3 * HID;
  ip.inv_s = pl->d_mlp_f + 3 * HID + 128;
  ip.mu = pl->d_mlp_f + 3 * HID + 128 + 64;
  ip.s_out = pl->mlp_s_out;
  ip.K = pl->K;
  ip.KB = kb;
  ip.out_bf16 = out_bf16;
  const size_t blocks = (n_pix + IPX - 1) / IPX;
  TraceScope tr("k_mlp_infer", s);
  hipLaunchKernelGGL(k_mlp_infer, dim3(unsigned(blocks)), dim3(512), 0, s, zern, hw, n_pix, ip, beta);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
