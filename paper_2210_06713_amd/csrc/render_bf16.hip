// The learned form's blur on the BF16 matrix cores (Eq. (8), evaluated in
// the reconstruct-first order sum_u (sum_k beta_k psi_k(u)) I(x - u)).
//
// Taps are taken in pairs (ux, ux + 1) of horizontally adjacent kernel
// columns.  A block covers TH x 16 output pixels with TH / 2 waves; wave w
// owns the 32 pixels of rows 2w, 2w + 1.  For each group of 32 tap pairs the
// matrix cores form two 32 x 32 products htilde = beta (BF16, rows = pixels)
// x psi^T (BF16) with FP32 accumulation, one for the left and one for the
// right taps of the pairs, so every lane owns the two taps of one pair for 16
// pixels, in runs of 4 horizontally adjacent pixels.  A run meets 5 distinct
// image samples for its 8 products, read from an FP32 LDS tile whose rows
// are split by the parity of the column (pairs step the column by two) and
// padded to a stride congruent to the pair count per kernel row modulo 32,
// so the 32 lanes of a half-wave, which walk consecutive tap pairs, hit 32
// distinct banks.  The products are FP32 vector FMAs, which co-issue with
// the matrix-core instructions; each matrix-core instruction is followed in
// the schedule by a slice of the previous group's FMAs.  The per-lane sums
// over taps are reduced across the 32 lanes that share pixels once at the
// end.
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// Fragments are kept as four 32-bit words and reinterpreted only at the
// matrix-core call: copies of 8 x bf16 vectors between pipeline stages
// otherwise get split into 16-bit lanes and re-packed with byte permutes.
__device__ __forceinline__ uint4 ld_frag(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }

__device__ __forceinline__ f32x16 mfma_bf16(const uint4 &a, const uint4 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}

// Geometry of the paired-tap blur for kernel size T, TH output rows per block
// and KP basis coefficients per tap.  Tile word (c, sy, parity, k) =
// I(column 2k + parity) sits at c CH + sy RSR + parity SWH + k, k < SWH;
// the row stride RSR >= 2 SWH is congruent to the pair count per kernel row
// modulo 32, and a lane's words of one channel lie within 255 words of its
// base.  The basis is staged in groups of 32 tap pairs, rows of KPP = KP + 8
// coefficients (the 16-byte pad keeps the lanes' 16-byte reads on distinct
// banks), in a ring of three stages: while group tp is multiplied, group
// tp + 1 is resident and group tp + 2 is being copied into the stage that
// group tp - 1 has just left.
template <int T, int TH, int KP, int C>
struct PairGeom {
  static_assert(T % 2 == 1, "odd kernel size");
  static constexpr int R = (T - 1) / 2;
  static constexpr int NPX = (T + 1) / 2;          // tap pairs per kernel row (last one half padding)
  static constexpr int NP = T * NPX;               // tap pairs
  static constexpr int NTP = (NP + 31) / 32;       // groups of 32 pairs
  static constexpr int SH = TH + T - 1;            // tile rows
  static constexpr int SW = 16 + T - 1;            // tile columns (even)
  static constexpr int SWH = SW / 2;               // columns of one parity
  static constexpr int RSR = 2 * SWH + ((NPX - 2 * SWH) % 32 + 32) % 32;
  static constexpr int CH = SH * RSR;              // one channel
  static constexpr int KPP = KP + 8;
  static constexpr int GB = 64 * KPP * 2;          // bytes of one group: [2 sides][32 pairs][KPP]
  static constexpr int NCH = GB / 1024;            // 1 KB wave copies per group
  static constexpr size_t BASE = size_t(C) * CH * 4 + size_t(NTP) * 32 * 4;   // tile + lane bases
  static constexpr int NS = 3;
  static constexpr size_t LDS = BASE + size_t(NS) * GB;
  static constexpr bool kFits = LDS <= 160 * 1024;
  static_assert(GB % 1024 == 0, "whole wave copies");
  static_assert(RSR + SWH + 5 < 256, "read offsets");
};

// Two waves per SIMD (at most 256 registers); four channels' sums or a
// 128-wide basis need more.
template <int KS, int T, int C>
constexpr bool kWide = C > 3 || KS > 7;

// Copies one 1 KB piece of a basis group from global memory straight into
// LDS: lane l moves bytes 16 l .. 16 l + 15 of the piece.  The LDS address
// of the piece must be the same for the whole wave (it goes through M0).
__device__ __forceinline__ void copy_to_lds(const char *src_piece, uint32_t lds_piece, int lane) {
  asm volatile(
      "s_mov_b32 m0, %0\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %1, %2"
      :
      : "s"(lds_piece), "v"(uint32_t(lane) * 16u), "s"(src_piece)
      : "memory", "m0");
}

template <int KS, int T, int C, int TH>
__global__ void __launch_bounds__(32 * TH) __attribute__((amdgpu_waves_per_eu(kWide<KS, T, C> ? 1 : 2)))
k_render_bf16(const float *__restrict__ img, const uint16_t *__restrict__ beta,
              const uint16_t *__restrict__ psi /*[NTP][2][32][KPP]*/, float *__restrict__ out,
              int H, int W) {
  using G = PairGeom<T, TH, KS * 16, C>;
  constexpr int KB = KS * 16, R = G::R, SH = G::SH, SW = G::SW, SWH = G::SWH, RSR = G::RSR, CH = G::CH;
  constexpr int NPX = G::NPX, NP = G::NP, NTP = G::NTP, KPP = G::KPP, GB = G::GB, NCH = G::NCH, NS = G::NS;
  constexpr int NW = TH / 2, CPW = (NCH + NW - 1) / NW;   // waves, copies per wave and group
  extern __shared__ float smem[];
  uint32_t *tile = reinterpret_cast<uint32_t *>(smem);     // [C][SH][RSR] image samples
  int *ltab = reinterpret_cast<int *>(tile + C * CH);      // NTP * 32 lane bases
  char *ring = reinterpret_cast<char *>(smem) + G::BASE;   // NS groups of the basis
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * 16;
  const float *imf = img + size_t(f) * C * H * W;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pn = lane & 31, g = lane >> 5;
  // group tp goes to ring stage tp % NS; wave w copies pieces w, w + NW, ...
  // (a wave past the last piece repeats it: same bytes to the same place),
  // groups past the last one repeat it into the stage that was just freed
  const uint32_t ring_lds = uint32_t(reinterpret_cast<uintptr_t>(ring));
  auto stage_in = [&](int tp) {
    const char *src = reinterpret_cast<const char *>(psi) + size_t(min(tp, NTP - 1)) * GB;
    const uint32_t dst = ring_lds + uint32_t((tp % NS) * GB);
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int piece = min(w + k * NW, NCH - 1);
      copy_to_lds(src + piece * 1024, dst + uint32_t(piece * 1024), lane);
    }
  };
  stage_in(0);
  stage_in(1);
  // A operand: beta of pixel pn of the wave (rows 2w, 2w + 1 of the block)
  uint4 b[KS];
  {
    const int py = 2 * w + (pn >> 4), px = pn & 15;
    const int y = ty0 + py, x = tx0 + px;
    const bool ok = (y < H) && (x < W);
    const uint16_t *bp = beta + ((size_t(f) * H + (ok ? y : 0)) * W + (ok ? x : 0)) * KB + 8 * g;
#pragma unroll
    for (int s = 0; s < KS; ++s) b[s] = ok ? ld_frag(bp + 16 * s) : make_uint4(0u, 0u, 0u, 0u);
  }
  // tile column q of row sy holds I(ty0 + sy - R, tx0 + q - R) (clamped), at
  // parity q % 2, index q / 2; all of a thread's samples are requested
  // before the first is written
  {
    constexpr int NE = C * SH * SW, NIT = (NE + 32 * TH - 1) / (32 * TH);
    const char *imb = reinterpret_cast<const char *>(imf);   // a frame spans < 4 GiB
    float v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = min(int(threadIdx.x) + it * 32 * TH, NE - 1);
      const int c = e / (SH * SW);
      const int rem = e - c * (SH * SW);
      const int sy = rem / SW, q = rem - sy * SW;
      const int gy = min(max(ty0 + sy - R, 0), H - 1);
      const int gx = min(max(tx0 + q - R, 0), W - 1);
      v[it] = *reinterpret_cast<const float *>(imb + uint32_t(4u * uint32_t((c * H + gy) * W + gx)));
    }
    float *tf = reinterpret_cast<float *>(tile);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = threadIdx.x + it * 32 * TH;
      if (e < NE) {
        const int c = e / (SH * SW);
        const int rem = e - c * (SH * SW);
        const int sy = rem / SW, q = rem - sy * SW;
        tf[c * CH + sy * RSR + (q & 1) * SWH + (q >> 1)] = v[it];
      }
    }
  }
  // lane base of tap pair j = (uy, i): the left tap (uy, 2i) of pixel (py,
  // px) reads tile row py + 2R - uy, column px + 2R - 2i, the right tap the
  // column before; padding pairs (j >= NP, zero psi) point at harmless
  // in-tile words
  for (int j = threadIdx.x; j < NTP * 32; j += 32 * TH) {
    const int uy = j / NPX, i = j - uy * NPX;
    ltab[j] = j < NP ? (2 * R - uy) * RSR + R - i : 0;
  }
  const int wbase = 2 * w * RSR + 2 * g;
  __syncthreads();

  float sum[C][16];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) sum[c][r] = 0.f;
  // accumulator row r = 4 run + j holds pixel py = 2w + run / 2, px = px0 +
  // j with px0 = 8 (run % 2) + 4g: the left tap reads column q0 + j, q0 =
  // px0 + 2R - 2i (even), the right tap column q0 + j - 1.  The run's five
  // columns q0 - 1 .. q0 + 3 are words k0 = q0 / 2 and k0 + 1 of the even
  // half and k0 - 1 .. k0 + 1 of the odd half, k0 = (lane base) + 4 (run % 2)
  // one base per channel, kept opaque so that every read folds its
  // compile-time offset (< 256 words) into the LDS instruction; the bases of
  // the group to be applied next are formed a group early
  auto bases = [&](int tp, int (&cb)[C]) {
    cb[0] = wbase + ltab[32 * min(tp, NTP - 1) + pn];
#pragma unroll
    for (int c = 1; c < C; ++c) {
      cb[c] = cb[0] + c * CH;
      asm volatile("" : "+v"(cb[c]));
    }
  };
  auto apply = [&](const f32x16 &xl, const f32x16 &xr, const int (&cb)[C]) {
    const float *tf = reinterpret_cast<const float *>(tile);
#pragma unroll
    for (int run = 0; run < 4; ++run) {
      const int ro = (run >> 1) * RSR + 4 * (run & 1);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const float *t0 = tf + cb[c] + ro;
        const float sm[5] = {t0[SWH - 1], t0[0], t0[SWH], t0[1], t0[SWH + 1]};   // columns q0 - 1 .. q0 + 3
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 4 * run + j;
          sum[c][r] = fmaf(xl[r], sm[j + 1], sum[c][r]);
          sum[c][r] = fmaf(xr[r], sm[j], sum[c][r]);
        }
      }
    }
  };
  // B operand from the ring: psi^T column = tap pair pn, k-slice 8g..8g+7.
  // A group's left fragments are read one step before its products, its
  // right fragments at the start of its own step (needed only after the
  // seven left products), so no product waits for LDS.
  const char *frag = ring + (pn * KPP + 8 * g) * 2;
  auto read_left = [&](int tp, uint4 (&fl)[KS]) {
    const char *st = frag + (tp % NS) * GB;
#pragma unroll
    for (int s = 0; s < KS; ++s) fl[s] = *reinterpret_cast<const uint4 *>(st + 32 * s);
  };
  uint4 fr[KS];
  auto read_right = [&](int tp) {
    const char *st = frag + (tp % NS) * GB + 32 * KPP * 2;
#pragma unroll
    for (int s = 0; s < KS; ++s) fr[s] = *reinterpret_cast<const uint4 *>(st + 32 * s);
  };
  // each matrix-core instruction is followed by three LDS reads of image
  // samples and seven FMAs of the previous group's application
  auto interleave = [&]() {
#pragma unroll
    for (int i = 0; i < 2 * KS; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 7, 0);
    }
  };
  // step tp: meet the other waves (group tp + 1 has landed: this wave's
  // copies of it are its only ones in flight; every read of group tp - 1's
  // stage is done), refill that stage with group tp + 2, read fragments,
  // multiply group tp and apply group tp - 1
  auto step = [&](int tp, f32x16 &al, f32x16 &ar, uint4 (&fl)[KS], uint4 (&fln)[KS], bool next,
                  const f32x16 &pl_, const f32x16 &pr_, int (&cp)[C], bool prev) {
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" : : : "memory");
    stage_in(tp + 2);
    read_right(tp);
    if (next) read_left(tp + 1, fln);
    __builtin_amdgcn_sched_barrier(0);
    al = f32x16{};
    ar = f32x16{};
#pragma unroll
    for (int s = 0; s < KS; ++s) al = mfma_bf16(b[s], fl[s], al);
#pragma unroll
    for (int s = 0; s < KS; ++s) ar = mfma_bf16(b[s], fr[s], ar);
    if (prev) {
      apply(pl_, pr_, cp);
      bases(tp + 1, cp);
      interleave();
    }
  };
  f32x16 al, ar, bl, br;
  int ca[C], cbb[C];
  uint4 fla[KS], flb[KS];
  bases(0, ca);
  bases(1, cbb);
  read_left(0, fla);
  step(0, al, ar, fla, flb, NTP > 1, bl, br, cbb, false);
  // steps 1, 2, ... in pairs while both read a next group; the rest resolved at compile time
  constexpr int TS = 1 + 2 * (NTP > 2 ? (NTP - 2) / 2 : 0);
  for (int tp = 1; tp < TS; tp += 2) {
    step(tp, bl, br, flb, fla, true, al, ar, ca, true);
    step(tp + 1, al, ar, fla, flb, true, bl, br, cbb, true);
  }
  if constexpr (NTP - TS >= 1) step(TS, bl, br, flb, fla, TS + 1 < NTP, al, ar, ca, true);
  if constexpr (NTP - TS >= 2) step(TS + 1, al, ar, fla, flb, TS + 2 < NTP, bl, br, cbb, true);
  if constexpr (((NTP - 1) & 1) != 0) {
    apply(bl, br, cbb);
  } else {
    apply(al, ar, ca);
  }
  // the copies issued for groups past the last one are still in flight
  asm volatile("s_waitcnt vmcnt(0)" : : : "memory");
  // the 32 lanes of a half hold partial sums of the same 16 pixels: halve the
  // set of rows each lane keeps at every exchange (keep the rows selected by
  // the lane's bit, send the others), so after lane bits 16, 8, 4, 2 a lane
  // holds row r = 8 b16 + 4 b8 + 2 b4 + b2; bit 1 completes the sum
  float v[C][8];
  {
    const bool hi = pn & 16;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float send = hi ? sum[c][k] : sum[c][k + 8];
        const float keep = hi ? sum[c][k + 8] : sum[c][k];
        v[c][k] = keep + __shfl_xor(send, 16, 64);
      }
  }
#pragma unroll
  for (int bit = 8, n = 4; bit >= 2; bit >>= 1, n >>= 1) {
    const bool hi = pn & bit;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const float send = hi ? v[c][k] : v[c][k + n];
        const float keep = hi ? v[c][k + n] : v[c][k];
        v[c][k] = keep + __shfl_xor(send, bit, 64);
      }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) v[c][0] += __shfl_xor(v[c][0], 1, 64);
  if ((pn & 1) == 0) {
    const int r = 8 * ((pn >> 4) & 1) + 4 * ((pn >> 3) & 1) + 2 * ((pn >> 2) & 1) + ((pn >> 1) & 1);
    const int y = ty0 + 2 * w + (r >> 3), x = tx0 + 8 * ((r >> 2) & 1) + (r & 3) + 4 * g;
    if (y < H && x < W) {
      float *of = out + size_t(f) * C * H * W + size_t(y) * W + x;
      const size_t pl = size_t(H) * W;
#pragma unroll
      for (int c = 0; c < C; ++c) of[c * pl] = v[c][0];
    }
  }
}

// The plain form's blur on the 16-bit matrix cores at FP32 accuracy
// (v_mfma_f32_32x32x16_f16), with the block/wave/lane layout of the BF16
// kernel: htilde^T[32 taps][32 px] = psi x beta^T per 32-tap block, then the
// taps applied to the image tile with FP32 FMAs.  The FP32 matrix
// instructions would run at the FP32 vector rate; instead every operand is
// split into FP16 x = x_hi + x_lo (x_lo = fp16(x - x_hi)) and each 16-wide
// k-step is three products, psi_hi beta_hi + psi_hi beta_lo +
// psi_lo beta_hi, in three FP32 accumulators (the dropped psi_lo beta_lo
// and the rounding of the parts are each below 2^-22 of |psi beta|).  beta
// is scaled by 2^12 and psi by 2^10 into FP16's normal range; the sums are
// scaled back by 2^-22 at the end.  A lane's beta (its pixel, constant over
// the taps) is split once; psi_hi and psi_lo of each tap block come split
// from the plan table in fragment order and are staged in LDS for the
// block's waves (two tile rows of 16 pixels each) by asynchronous copies,
// one block ahead, in a ring of two stages.
constexpr float kRBetaScale = 4096.f;                   // 2^12
constexpr float kROutScale = 1.f / (4096.f * 1024.f);   // 2^-22

template <int KS, int T, int TH_ = 8>
struct H3Geom {
  static constexpr int TH = TH_, TW = 16, R = (T - 1) / 2;
  static constexpr int NW = TH / 2, NTHR = 64 * NW;  // waves (two tile rows each), threads
  static constexpr int SH = TH + T - 1, SW = TW + T - 1, PLANE = SH * SW;
  static constexpr int NT = (T * T + 31) / 32;   // tap blocks
  static constexpr int GB = KS * 2 * 1024;        // bytes of one block's fragments: [KS][hi, lo][64 lanes][16 B]
  static constexpr int NCH = GB / 1024;           // 1 KB wave copies per block
  static constexpr int NS = 2;                    // ring stages: block tb + 1 in flight
  static size_t lds(int C) { return size_t(C) * PLANE * sizeof(float) + NS * size_t(GB); }
};

__device__ __forceinline__ f32x16 mfma_f16(const uint4 &a, const uint4 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                0, 0);
}

template <int KS, int T, int C, int TH_>
__global__ void __launch_bounds__(32 * TH_)
k_render_h3(const float *__restrict__ img, const float *__restrict__ beta,
            const uint16_t *__restrict__ psi /*[NT][KS][2][64][8] f16*/, float *__restrict__ out, int H, int W,
            int K) {
  using G = H3Geom<KS, T, TH_>;
  constexpr int TH = G::TH, TW = G::TW, R = G::R, SW = G::SW, PLANE = G::PLANE, NT = G::NT;
  constexpr int NW = G::NW, NTHR = G::NTHR;
  constexpr int GB = G::GB, NCH = G::NCH, CPW = (NCH + NW - 1) / NW, NS = G::NS;
  static_assert(CPW <= 15, "copies per wave fit the counted wait");
  extern __shared__ __attribute__((aligned(16))) float tile[];  // [C][PLANE] image samples, then the psi ring
  __shared__ __attribute__((aligned(16))) short offtab[NT * 32];
  const int f = blockIdx.z;
  const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
  const float *imf = img + size_t(f) * C * H * W;
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  char *ring = reinterpret_cast<char *>(tile + C * PLANE);
  // tap block tb goes to ring stage tb % 2; wave w copies pieces w, w + NW,
  // ... (a wave past the last piece repeats it: same bytes to the same place)
  const uint32_t ring_lds = uint32_t(reinterpret_cast<uintptr_t>(ring));
  auto stage_in = [&](int tb) {
    const char *src = reinterpret_cast<const char *>(psi) + size_t(tb) * GB;
    const uint32_t dst = ring_lds + uint32_t((tb % NS) * GB);
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
      const int piece = min(w + NW * k, NCH - 1);
      copy_to_lds(src + piece * 1024, dst + uint32_t(piece * 1024), lane);
    }
  };
  stage_in(0);
  // tile loads in batches of eight per thread, all requested before any is
  // stored (a frame spans < 4 GiB)
  {
    const char *imb = reinterpret_cast<const char *>(imf);
    const int NE = C * PLANE;
    for (int e0 = 0; e0 < NE; e0 += 8 * NTHR) {
      float v[8];
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int e = min(e0 + it * NTHR + int(threadIdx.x), NE - 1);
        const int c = e / PLANE;
        const int rem = e - c * PLANE;
        const int sy = rem / SW, sx = rem - sy * SW;
        const int gy = min(max(ty0 + sy - R, 0), H - 1);
        const int gx = min(max(tx0 + sx - R, 0), W - 1);
        v[it] = *reinterpret_cast<const float *>(imb + uint32_t(4u * uint32_t((c * H + gy) * W + gx)));
      }
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int e = e0 + it * NTHR + int(threadIdx.x);
        if (e < NE) tile[e] = v[it];
      }
    }
  }
  for (int e = threadIdx.x; e < NT * 32; e += NTHR) {
    const int uy = e / T - R, ux = e % T - R;
    offtab[e] = (e < T * T) ? uy * SW + ux : 0;
  }
  const int g = lane >> 5, pn = lane & 31;
  const int py = 2 * w + (pn >> 4), px = pn & 15;
  const int y = ty0 + py, x = tx0 + px;
  const bool ok = (y < H) && (x < W);
  // B operand: this pixel's beta, k-slice 16 q + 8 g + 0..7 of step q, as
  // FP16 hi and lo
  uint4 bhi[KS], blo[KS];
  {
    const float *bp = beta + ((size_t(f) * H + (ok ? y : 0)) * W + (ok ? x : 0)) * K;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      f32x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * q + 8 * g + e;
        v[e] = (ok && k < K) ? bp[k] : 0.f;
      }
      v *= kRBetaScale;
      const f16x8 hi = __builtin_convertvector(v, f16x8);
      const f16x8 lo = __builtin_convertvector(v - __builtin_convertvector(hi, f32x8), f16x8);
      bhi[q] = __builtin_bit_cast(uint4, hi);
      blo[q] = __builtin_bit_cast(uint4, lo);
    }
  }
  const int pbase = (py + R) * SW + px + R;
  const int mrow = 4 * g;
  float sc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sc[c] = 0.f;
  const char *frag = ring + lane * 16;
  // products of tap block tb: x1 = psi_hi beta_hi, x2 = psi_hi beta_lo +
  // psi_lo beta_hi.  This wave's only copies in flight are block tb's
  // (issued at step tb - 1); past the barrier every wave's copies of it have
  // landed, and every wave is done with stage (tb + 1) % 2 (read at step
  // tb - 1), which the copies of block tb + 1 then fill.  The fragments are
  // read from LDS next to their products.  Before the first block the
  // barrier also completes the tile and the offset table.
  auto products = [&](int tb, f32x16 &x1, f32x16 &x2) {
    __builtin_amdgcn_s_waitcnt(7 << 4);  // vmcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    if (tb + 1 < NT) stage_in(tb + 1);
    const char *st = frag + (tb % NS) * GB;
    x1 = f32x16{};
    x2 = f32x16{};
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const uint4 ahi = *reinterpret_cast<const uint4 *>(st + (2 * q) * 1024);
      const uint4 alo = *reinterpret_cast<const uint4 *>(st + (2 * q + 1) * 1024);
      x1 = mfma_f16(ahi, bhi[q], x1);
      x2 = mfma_f16(ahi, blo[q], x2);
      x2 = mfma_f16(alo, bhi[q], x2);
    }
  };
  // the taps of block tb applied to the image tile: the lane's 16 tap
  // offsets in four 8-byte reads, then every sample read before its FMA
  // (no branch in between, so the reads go out together)
  auto apply = [&](int tb, const f32x16 &x1, const f32x16 &x2) {
    const short *ot = offtab + 32 * tb + mrow;
    int idx[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const s16x4 o = *reinterpret_cast<const s16x4 *>(ot + 8 * i);
#pragma unroll
      for (int j = 0; j < 4; ++j) idx[4 * i + j] = pbase - o[j];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = x1[r] + x2[r];
#pragma unroll
      for (int c = 0; c < C; ++c) sc[c] = fmaf(v, tile[c * PLANE + idx[r]], sc[c]);
    }
  };
  // block tb's products are issued before block tb - 1's application, so
  // the matrix cores work while the image samples are read and applied (the
  // compiler's own schedule of the two measured faster than a forced
  // one-by-one interleave)
  f32x16 p1, p2, q1, q2;
  products(0, p1, p2);
  int tb = 1;
  for (; tb + 1 < NT; tb += 2) {
    products(tb, q1, q2);
    apply(tb - 1, p1, p2);
    products(tb + 1, p1, p2);
    apply(tb, q1, q2);
  }
  if (tb < NT) {
    products(tb, q1, q2);
    apply(tb - 1, p1, p2);
    apply(tb, q1, q2);
  } else {
    apply(tb - 1, p1, p2);
  }
#pragma unroll
  for (int c = 0; c < C; ++c) sc[c] += __shfl_xor(sc[c], 32);
  if (lane < 32 && ok) {
    float *of = out + size_t(f) * C * H * W + size_t(y) * W + x;
    const size_t pl = size_t(H) * W;
#pragma unroll
    for (int c = 0; c < C; ++c) of[c * pl] = sc[c] * kROutScale;
  }
}

// Dynamic LDS of the image tile (plus, for T > 0, the FP32 kernel's static
// offset table); tiles above 64 KB need the device's larger workgroup limit,
// checked here and raised on the kernel.
template <typename Kern>
int prepare_lds(Kern kern, size_t lds, int T) {
  const size_t stat = T > 0 ? sizeof(short) * size_t((T * T + 31) / 32 * 32) : 0;
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

template <int KS, int T, int C, int TH>
int launch_ks_tch(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta, float *out,
                  hipStream_t s) {
  using G = PairGeom<T, TH, KS * 16, C>;
  const int H = pl->H, W = pl->W;
  if (size_t(C) * H * W * sizeof(float) >= (size_t(1) << 32)) return TSIM_EUNSUPPORTED;
  if (pl->KP != KS * 16) return TSIM_EINVAL;
  dim3 grid((W + 15) / 16, (H + TH - 1) / TH, frames);
  const int st = prepare_lds(k_render_bf16<KS, T, C, TH>, G::LDS, 0);
  if (st != TSIM_OK) return st;
  hipLaunchKernelGGL((k_render_bf16<KS, T, C, TH>), grid, dim3(32 * TH), G::LDS, s, img, beta, pl->d_basis_bf,
                     out, H, W);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

// The 65-tap tile leaves LDS for one block per CU: 16 output rows (8 waves)
// keep two waves per SIMD there; other kernels use 8-row blocks, and the
// widest forms 4-row blocks where an 8-row tile and the basis ring would not
// fit the LDS.
template <int KS, int T, int C>
int launch_ks_tc(const tsim_plan *pl, int frames, const float *img, const uint16_t *beta, float *out,
                 hipStream_t s) {
  constexpr int KP = KS * 16;
  if constexpr (T == 65 && !kWide<KS, T, C> && PairGeom<T, 16, KP, C>::kFits)
    return launch_ks_tch<KS, T, C, 16>(pl, frames, img, beta, out, s);
  else if constexpr (PairGeom<T, 8, KP, C>::kFits)
    return launch_ks_tch<KS, T, C, 8>(pl, frames, img, beta, out, s);
  else if constexpr (PairGeom<T, 4, KP, C>::kFits)
    return launch_ks_tch<KS, T, C, 4>(pl, frames, img, beta, out, s);
  else
    return TSIM_EUNSUPPORTED;
}

// Whether one of the block heights above fits the LDS for this shape.
template <int KS, int T, int C>
constexpr bool bf16_shape_fits() {
  constexpr int KP = KS * 16;
  return (T == 65 && !kWide<KS, T, C> && PairGeom<T, 16, KP, C>::kFits) || PairGeom<T, 8, KP, C>::kFits ||
         PairGeom<T, 4, KP, C>::kFits;
}

template <int KS, int T>
constexpr bool bf16_fits_c(int C) {
  return C == 1 ? bf16_shape_fits<KS, T, 1>()
       : C == 2 ? bf16_shape_fits<KS, T, 2>()
       : C == 3 ? bf16_shape_fits<KS, T, 3>()
       : C == 4 ? bf16_shape_fits<KS, T, 4>()
                : false;
}

template <int KS>
constexpr bool bf16_fits_tc(int T, int C) {
  return T == 65 ? bf16_fits_c<KS, 65>(C)
       : T == 33 ? bf16_fits_c<KS, 33>(C)
       : T == 21 ? bf16_fits_c<KS, 21>(C)
       : T == 15 ? bf16_fits_c<KS, 15>(C)
                 : false;
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

namespace {

// tiles of 8 rows (four waves) at T = 33; at T = 65 the tile is mostly
// halo and one block fills a CU's LDS, so 16 rows (eight waves) per block
template <int KS, int T>
int launch_h3(const tsim_plan *pl, int frames, const float *img, const float *beta, float *out, hipStream_t s) {
  constexpr int TH = T == 65 ? 16 : 8;
  using G = H3Geom<KS, T, TH>;
  const int H = pl->H, W = pl->W, C = pl->C;
  dim3 grid((W + G::TW - 1) / G::TW, (H + G::TH - 1) / G::TH, frames);
  const size_t lds = G::lds(C);
  int st = TSIM_OK;
  switch (C) {
    case 1: st = prepare_lds(k_render_h3<KS, T, 1, TH>, lds, T); break;
    case 2: st = prepare_lds(k_render_h3<KS, T, 2, TH>, lds, T); break;
    case 3: st = prepare_lds(k_render_h3<KS, T, 3, TH>, lds, T); break;
    case 4: st = prepare_lds(k_render_h3<KS, T, 4, TH>, lds, T); break;
    default: return TSIM_EUNSUPPORTED;
  }
  if (st != TSIM_OK) return st;
  TraceScope tr("k_render_fp32", s);
#define TSIM_H3(CC)                                                                                            \
  hipLaunchKernelGGL((k_render_h3<KS, T, CC, TH>), grid, dim3(G::NTHR), lds, s, img, beta, pl->d_basis_h3r, out, \
                     H, W, pl->K)
  switch (C) {
    case 1: TSIM_H3(1); break;
    case 2: TSIM_H3(2); break;
    case 3: TSIM_H3(3); break;
    default: TSIM_H3(4); break;
  }
#undef TSIM_H3
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

template <int KS>
int launch_h3_ks(const tsim_plan *pl, int frames, const float *img, const float *beta, float *out,
                 hipStream_t s) {
  if (pl->T == 33) return launch_h3<KS, 33>(pl, frames, img, beta, out, s);
  if (pl->T == 65) return launch_h3<KS, 65>(pl, frames, img, beta, out, s);
  return TSIM_EUNSUPPORTED;
}

}  // namespace

int launch_render_f32_mfma(const tsim_plan *pl, int frames, const float *img, const float *beta,
                           float *out, hipStream_t s) {
  if (!pl->d_basis_h3r || pl->C > 4) return TSIM_EUNSUPPORTED;
  if (size_t(pl->C) * pl->H * pl->W * sizeof(float) >= (size_t(1) << 32)) return TSIM_EUNSUPPORTED;
  switch (pl->KP) {
    case 32: return launch_h3_ks<2>(pl, frames, img, beta, out, s);
    case 64: return launch_h3_ks<4>(pl, frames, img, beta, out, s);
    case 112: return launch_h3_ks<7>(pl, frames, img, beta, out, s);
    case 128: return launch_h3_ks<8>(pl, frames, img, beta, out, s);
    default: return TSIM_EUNSUPPORTED;
  }
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

bool render_bf16_supported(int KP, int T, int C) {
  switch (KP) {
    case 32: return bf16_fits_tc<2>(T, C);
    case 64: return bf16_fits_tc<4>(T, C);
    case 112: return bf16_fits_tc<7>(T, C);
    case 128: return bf16_fits_tc<8>(T, C);
    default: return false;
  }
}
