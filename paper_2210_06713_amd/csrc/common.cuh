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

// LDS layout of the transform lines: line l of length n (power of two,
// >= 64) occupies buf[l * n, (l + 1) * n), and its element i sits at
// i ^ x, where x (5 bits) folds the index bits 5-9 and 10-14 and the line
// term `lt` (the line number shifted so that the lines read out together
// land on different banks) into bits 0-4.  Bits >= 5 are untouched, so the
// map is a bijection of [0, n) for every line.  With 64 banks of 4 bytes
// (8-byte accesses served 32 lanes at a time), the 32 lanes of a half-wave
// then touch 32 different bank pairs in a bit-reversed scatter of
// consecutive indices (the top five index bits vary), in the radix-4
// butterflies at spans 1, 64, 256 and 1024 (index bits 2-6 or 0-4 vary), in
// natural-order rows and in reads across lines; spans 4 and 16 keep two-way
// conflicts.
__device__ __forceinline__ int lds_swz(int i, int lt) { return i ^ (((i >> 5) ^ (i >> 10) ^ lt) & 31); }

// Number of LDS twiddles lds_fft_dit reads for length n: the radix-4 passes
// at spans h = 1, 4, 16, ... (while 2h < n) take h entries each, and an odd
// log2 n adds the final radix-2 pass's quarter table of n/4 entries.
__host__ __device__ constexpr int fft_twiddle_count(int log2n) {
  return ((1 << (2 * (log2n / 2))) - 1) / 3 + ((log2n & 1) ? (1 << log2n) / 4 : 0);
}

// Fill the LDS twiddle table from `tw`, which holds exp(sign 2 pi i k / n)
// for k < n/2: the radix-4 pass at span h reads omega_{4h}^j (j < h) at
// offset (h - 1)/3, so consecutive lanes read consecutive entries; for odd
// log2 n, omega_n^k (k < n/4) follows.  The caller synchronises.
__device__ __forceinline__ void load_twiddles(float2 *tws, const float2 *__restrict__ tw, int n, int log2n) {
  const int r4 = ((1 << (2 * (log2n / 2))) - 1) / 3;
  const int total = fft_twiddle_count(log2n);
  for (int k = threadIdx.x; k < total; k += blockDim.x) {
    if (k < r4) {
      int h = 1;
      while ((4 * h - 1) / 3 <= k) h *= 4;
      const int j = k - (h - 1) / 3;
      tws[k] = tw[j * (n / (4 * h))];
    } else {
      tws[k] = tw[k - r4];
    }
  }
}

// In-place decimation-in-time FFT over `nlines` independent lines of length
// n (power of two, 64 <= n <= 32768) in the LDS layout of lds_swz, line l
// with line term l << lsh; input in bit-reversed order, output natural.
// The twiddles come from the table of load_twiddles, whose source table
// also sets the direction `sign`.  Two radix-2 stages are fused per pass
// (radix 2^2: spans h and 2h on quadruples i, i+h, i+2h, i+3h), so a
// length-1024 transform takes five barriers.  All threads of the block
// take part; the caller synchronises before and after.
__device__ inline void lds_fft_dit(float2 *buf, int n, int log2n, int nlines, int lsh, const float2 *tws,
                                   float sign) {
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  int h = 1;
  int lh = 0;
  int toff = 0;  // offset of the pass's twiddles
  // The swizzle is linear over XOR and the offsets k h (k < 4) occupy index
  // bits lh, lh + 1, which are clear in a quadruple's base i, so element
  // i + k h sits at lds_swz(i, lt) ^ lds_swz(k h, 0): one swizzle per
  // butterfly and three pass-uniform offsets.
  while (h < n) {
    if (2 * h < n) {
      const int groups = nlines << (log2n - 2);
      const int d1 = lds_swz(h, 0), d2 = lds_swz(2 * h, 0), d3 = lds_swz(3 * h, 0);
      for (int g = tid; g < groups; g += nthr) {
        const int line = g >> (log2n - 2);
        const int gg = g & ((n >> 2) - 1);
        const int j = gg & (h - 1);
        const int i = ((gg >> lh) << (lh + 2)) + j;
        float2 *b = buf + line * n;
        const int lt = line << lsh;
        const int p0 = lds_swz(i, lt), p1 = p0 ^ d1, p2 = p0 ^ d2, p3 = p0 ^ d3;
        const float2 x0 = b[p0], x1 = b[p1], x2 = b[p2], x3 = b[p3];
        // omega_{4h}^j from the table; omega_{2h}^j is its square and
        // omega_{4h}^{j+h} = omega_{4h}^j * omega_4, omega_4 = (0, sign)
        const float2 w2 = tws[toff + j];
        const float2 w1 = make_float2(w2.x * w2.x - w2.y * w2.y, 2.f * w2.x * w2.y);
        const float2 t1 = cmul(w1, x1), t3 = cmul(w1, x3);
        const float2 a0 = make_float2(x0.x + t1.x, x0.y + t1.y);
        const float2 a1 = make_float2(x0.x - t1.x, x0.y - t1.y);
        const float2 a2 = make_float2(x2.x + t3.x, x2.y + t3.y);
        const float2 a3 = make_float2(x2.x - t3.x, x2.y - t3.y);
        const float2 u2 = cmul(w2, a2);
        const float2 w3 = make_float2(-sign * w2.y, sign * w2.x);
        const float2 u3 = cmul(w3, a3);
        b[p0] = make_float2(a0.x + u2.x, a0.y + u2.y);
        b[p2] = make_float2(a0.x - u2.x, a0.y - u2.y);
        b[p1] = make_float2(a1.x + u3.x, a1.y + u3.y);
        b[p3] = make_float2(a1.x - u3.x, a1.y - u3.y);
      }
      toff += h;
      h <<= 2;
      lh += 2;
    } else {
      // final radix-2 pass (odd log2 n): span h = n/2, omega_n^j, j < n/2,
      // from the quarter table after the radix-4 twiddles
      const int groups = nlines << (log2n - 1);
      const int quarter = n >> 2;
      const int d1 = lds_swz(h, 0);
      for (int g = tid; g < groups; g += nthr) {
        const int line = g >> (log2n - 1);
        const int j = g & ((n >> 1) - 1);
        float2 *b = buf + line * n;
        const int lt = line << lsh;
        const int p0 = lds_swz(j, lt), p1 = p0 ^ d1;
        const float2 x0 = b[p0], x1 = b[p1];
        const bool hi = j >= quarter;
        const float2 tq = tws[toff + (hi ? j - quarter : j)];
        const float2 w = hi ? make_float2(-sign * tq.y, sign * tq.x) : tq;
        const float2 t1 = cmul(w, x1);
        b[p0] = make_float2(x0.x + t1.x, x0.y + t1.y);
        b[p1] = make_float2(x0.x - t1.x, x0.y - t1.y);
      }
      h <<= 1;
      lh += 1;
    }
    __syncthreads();
  }
}

}  // namespace tsim
