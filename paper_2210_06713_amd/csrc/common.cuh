// Device helpers shared by the HIP kernels: Philox4x32-10, Box-Muller, and
// an in-place radix-2^2 decimation-in-time FFT on LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tsim {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit multiplies with the Weyl key schedule.
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = uint64_t(0xD2511F53u) * c.x;
    uint64_t p1 = uint64_t(0xCD9E8D57u) * c.z;
    uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// u = ((x >> 9) + 0.5) 2^-23: in (0, 1) and exact in binary32.
__device__ __forceinline__ float u01(uint32_t x) {
  return (float(x >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// Box-Muller pair from two 32-bit words.
__device__ __forceinline__ float2 box_muller(uint32_t a, uint32_t b) {
  float u0 = u01(a), u1 = u01(b);
  float r = sqrtf(-2.0f * logf(u0));
  float s, c;
  sincospif(2.0f * u1, &s, &c);
  return make_float2(r * c, r * s);
}

// Box-Muller on the hardware transcendental units: r = sqrt(-2 ln 2 log2 u0)
// and the cosine/sine of 2 pi u1 (v_sin/v_cos take revolutions), each a few
// ulp from the correctly rounded value; u0 >= 2^-24 is a normal number.
__device__ __forceinline__ float2 box_muller_hw(uint32_t a, uint32_t b) {
  const float u0 = u01(a), u1 = u01(b);
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u0));
  return make_float2(r * __builtin_amdgcn_cosf(u1), r * __builtin_amdgcn_sinf(u1));
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t v, int log2n) {
  return __builtin_bitreverse32(v) >> (32 - log2n);
}

// LDS element index with one padding slot per 32 complex samples: strided
// and bit-reversed access patterns then spread over all banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// Twiddle exp(sign 2 pi i k / n) for k < n/2 from the quarter table
// twq[k] (k < n/4): the second quarter is the first times exp(sign i pi/2).
__device__ __forceinline__ float2 twiddle(const float2 *twq, int k, int quarter, float sign) {
  const bool hi = k >= quarter;
  const float2 t = twq[hi ? k - quarter : k];
  return hi ? make_float2(-sign * t.y, sign * t.x) : t;
}

// Copy the quarter twiddle table (n/4 entries of `tw`, which holds
// exp(sign 2 pi i k / n) for k < n/2) into LDS; the caller synchronises.
__device__ __forceinline__ void load_twiddles(float2 *twq, const float2 *__restrict__ tw, int n) {
  for (int k = threadIdx.x; k < (n >> 2); k += blockDim.x) twq[k] = tw[k];
}

// In-place decimation-in-time FFT over `ncol` independent lines of length n
// (power of two, >= 4) stored line-major in LDS (`buf[line * stride +
// lpad(i)]`), input in bit-reversed order, output natural.  The twiddles
// come from the LDS quarter table `twq` of exp(sign 2 pi i k / n), which
// also sets the direction.  Two radix-2 stages are fused per pass (radix
// 2^2), so a length-1024 transform takes five barriers.  All threads of the
// block take part; the caller synchronises before and after.
__device__ inline void lds_fft_dit(float2 *buf, int n, int log2n, int ncol, int stride, const float2 *twq,
                                   float sign) {
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int quarter = n >> 2;
  int h = 1;
  int lh = 0;
  while (h < n) {
    if (2 * h < n) {
      // stages of span h and 2h on quadruples (i, i+h, i+2h, i+3h)
      const int groups = ncol << (log2n - 2);
      const int tstep1 = n / (2 * h);   // omega_{2h}^j = w[j * n/(2h)]
      const int tstep2 = n / (4 * h);   // omega_{4h}^j = w[j * n/(4h)], index < n/4
      for (int g = tid; g < groups; g += nthr) {
        int line = g >> (log2n - 2);
        int gg = g & ((n >> 2) - 1);
        int j = gg & (h - 1);
        int i = ((gg >> lh) << (lh + 2)) + j;
        float2 *b = buf + line * stride;
        float2 x0 = b[lpad(i)], x1 = b[lpad(i + h)], x2 = b[lpad(i + 2 * h)], x3 = b[lpad(i + 3 * h)];
        float2 w1 = twiddle(twq, j * tstep1, quarter, sign);
        float2 w2 = twq[j * tstep2];
        float2 t1 = cmul(w1, x1), t3 = cmul(w1, x3);
        float2 a0 = make_float2(x0.x + t1.x, x0.y + t1.y);
        float2 a1 = make_float2(x0.x - t1.x, x0.y - t1.y);
        float2 a2 = make_float2(x2.x + t3.x, x2.y + t3.y);
        float2 a3 = make_float2(x2.x - t3.x, x2.y - t3.y);
        float2 u2 = cmul(w2, a2);
        // omega_{4h}^{j+h} = omega_{4h}^j * omega_4, omega_4 = (0, sign)
        float2 w3 = make_float2(-sign * w2.y, sign * w2.x);
        float2 u3 = cmul(w3, a3);
        b[lpad(i)] = make_float2(a0.x + u2.x, a0.y + u2.y);
        b[lpad(i + 2 * h)] = make_float2(a0.x - u2.x, a0.y - u2.y);
        b[lpad(i + h)] = make_float2(a1.x + u3.x, a1.y + u3.y);
        b[lpad(i + 3 * h)] = make_float2(a1.x - u3.x, a1.y - u3.y);
      }
      h <<= 2;
      lh += 2;
    } else {
      const int groups = ncol << (log2n - 1);
      const int tstep1 = n / (2 * h);
      for (int g = tid; g < groups; g += nthr) {
        int line = g >> (log2n - 1);
        int gg = g & ((n >> 1) - 1);
        int j = gg & (h - 1);
        int i = ((gg >> lh) << (lh + 1)) + j;
        float2 *b = buf + line * stride;
        float2 x0 = b[lpad(i)], x1 = b[lpad(i + h)];
        float2 t1 = cmul(twiddle(twq, j * tstep1, quarter, sign), x1);
        b[lpad(i)] = make_float2(x0.x + t1.x, x0.y + t1.y);
        b[lpad(i + h)] = make_float2(x0.x - t1.x, x0.y - t1.y);
      }
      h <<= 1;
      lh += 1;
    }
    __syncthreads();
  }
}

}  // namespace tsim
