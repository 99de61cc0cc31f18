// DF-P2S Zernike-field sampler (Sec. III-A circulant sampling, Sec. III-C
// two-step generation, Eq. (9)).
//
// Pass 1 (k_sampler_cols): for field q (Noll modes 2+2q, 3+2q in its real
// and imaginary parts) and NC/2 pairs of Hermitian-mirror frequency columns
// (kx, Gw - kx), the white noise is drawn in registers from Philox once per
// bin pair, coloured by the square-root spectra at both bins, and
// inverse-transformed along ky in LDS; rows y < H of the result are written
// to the workspace V[f][q][y][slot], columns in mirror-pair slot order.  A
// block serves every frame of the launch in turn, so the spectra and the
// draws' LDS positions are read and formed once.
// Pass 2 (k_sampler_rows_mix): one block per output row y inverse-transforms
// V[f][q][y][:] along kx for every field, keeps columns x < W, and mixes the
// N unit-variance fields at each pixel with (D/r0)^{5/6} L before writing
// the N coefficient planes (N = 35 modes by default, Noll 2..N+1) (only L's structurally non-zero entries, each
// output plane written once its last field is in).  Only rows y < H survive pass 1 and only columns
// x < W pass 2 (crop of the top-left corner of the periodic grid).
#include <algorithm>

#include "common.cuh"
#include "internal.h"

namespace {

using namespace tsim;

// Complex samples per pass-1 block (32 KB): four 1024-point columns, so
// four 512-thread blocks (the 32-wave limit of a CU) fit in its LDS; never
// fewer than one mirror pair of columns.
constexpr int kLdsFloat2 = 4096;
constexpr int kMaxFramesPerLaunch = 64;

struct FrameScales {
  float s[kMaxFramesPerLaunch];
};

// Subharmonic compensation of the tilt fields (Noll 2, 3): for level p (0-
// based here, 1-based in the counter) and half-plane cell c of (m, n) =
// (1,0), (1,1), (0,1), (-1,1), the wave A cos t + B sin t with t = pi x
// fx[p] m + pi y fy[p] n, fx[p] = 2/(Gw 3^(p+1)), fy[p] = 2/(Gh 3^(p+1));
// (A2, B2, A3, B3) = amp times the Gaussians of the Philox call with counter
// (c, p + 1, frame, kTagSubharmonic).
constexpr uint32_t kTagSubharmonic = 5u;
constexpr int kSubhMaxLevels = 4;
struct SubhArgs {
  float amp[2][kSubhMaxLevels][4];
  float fx[kSubhMaxLevels], fy[kSubhMaxLevels];
  int levels;
  uint32_t key0, key1, frame_base;
};

// Column slots of the intermediate: slots 2p and 2p + 1 hold the Hermitian
// mirror columns kx = p and Gw - p (1 <= p < Gw/2); slots 0 and 1 hold the
// self-mirror columns 0 and Gw/2.  A pass-1 block owns whole slot pairs, so
// every noise draw serves a bin and its mirror, and writes NC adjacent slots.
__device__ __forceinline__ int slot_col(int c, int Gw) {
  const int p = c >> 1;
  if (p == 0) return (c & 1) ? (Gw >> 1) : 0;
  return (c & 1) ? Gw - p : p;
}

// Position and colour of one noise draw of a pass-1 block (work item e):
// LDS positions of bin A and its Hermitian mirror B (posB < 0 when A is
// self-conjugate), the canonical bin's counter, the sign that turns the
// canonical draw into A's noise, and the square-root spectra of the two
// modes at A's quarter-table bin.  None of it depends on the frame.
struct DrawItem {
  int posA, posB;
  uint32_t canon;
  float sg, sa, sb;
};

__device__ __forceinline__ DrawItem draw_item(int e, const float *__restrict__ sqrtS, int Gh, int Gw, int log2h,
                                              int s0, int ysh, int ma, int mb, bool has_b) {
  const bool zero_pair = s0 == 0;
  int slotA, slotB, kyA, kyB, kx;
  bool self_conj = false;
  if (zero_pair && e < Gh + 2) {
    const int half = Gh / 2 + 1;
    const int c = e < half ? 0 : 1;
    kyA = e < half ? e : e - half;   // 0..Gh/2
    kx = c ? (Gw >> 1) : 0;
    kyB = (Gh - kyA) & (Gh - 1);
    slotA = slotB = c;
    self_conj = kyA == kyB;
  } else {
    const int e2 = zero_pair ? e - 2 : e;
    const int pp = e2 >> log2h;     // pair within the block
    kyA = e2 & (Gh - 1);
    kx = (s0 >> 1) + pp;            // >= 1 here
    kyB = (Gh - kyA) & (Gh - 1);
    slotA = 2 * pp;
    slotB = 2 * pp + 1;
  }
  // bin A = (kyA, kx); its mirror B = (kyB, -kx mod Gw); canonical = smaller linear index
  const uint32_t linA = uint32_t(kyA) * Gw + kx;
  const uint32_t linB = uint32_t(kyB) * Gw + ((Gw - kx) & (Gw - 1));
  DrawItem d;
  d.canon = linA <= linB ? linA : linB;
  d.sg = linA <= linB ? 1.f : -1.f;
  const int qh = Gh / 2 + 1, qw = Gw / 2 + 1;
  const int kyq = kyA < qh ? kyA : Gh - kyA;   // kx <= Gw/2 for every bin A
  d.sa = sqrtS[(size_t(ma) * qw + kx) * qh + kyq];
  d.sb = has_b ? sqrtS[(size_t(mb) * qw + kx) * qh + kyq] : 0.f;
  d.posA = slotA * Gh + lds_swz(bitrev(uint32_t(kyA), log2h), slotA << ysh);
  d.posB = self_conj ? -1 : slotB * Gh + lds_swz(bitrev(uint32_t(kyB), log2h), slotB << ysh);
  return d;
}

// The coloured noise of one draw for one frame, into the block's LDS lines.
__device__ __forceinline__ void draw_noise(float2 *lds, const DrawItem &d, int q, uint32_t frame, uint32_t key0,
                                           uint32_t key1) {
  const float rs2 = 0.70710678118654752f;
  u32x4 r = philox4x32_10(u32x4{d.canon, uint32_t(q), frame, 0u}, key0, key1);
  const float2 g01 = box_muller_hw(r.x, r.y);
  const float2 g23 = box_muller_hw(r.z, r.w);
  if (d.posB < 0) {
    // U = sa g0 + i sb g2 (real noise at self-conjugate bins)
    lds[d.posA] = make_float2(d.sa * g01.x, d.sb * g23.x);
  } else {
    // noise of A: W (canonical) or conj(W); B takes the conjugate
    const float2 wa = make_float2(g01.x * rs2, d.sg * g01.y * rs2);
    const float2 wb = make_float2(g23.x * rs2, d.sg * g23.y * rs2);
    // U = sa Wa + i sb Wb at A, and sa conj(Wa) + i sb conj(Wb) at B
    lds[d.posA] = make_float2(d.sa * wa.x - d.sb * wb.y, d.sa * wa.y + d.sb * wb.x);
    lds[d.posB] = make_float2(d.sa * wa.x + d.sb * wb.y, -d.sa * wa.y + d.sb * wb.x);
  }
}

// One block per (slot group, field) for all frames of the launch: the
// twiddles, the draws' LDS positions and their square-root spectra are set
// up once and kept (IPT draws per thread, in registers), then each frame
// draws its noise, transforms and writes out.  The self-mirror pair of the
// first block has two draws more than IPT x 512; threads 0 and 1 take them.
template <int IPT>
__global__ void __launch_bounds__(512)
k_sampler_cols(const float *__restrict__ sqrtS, const float2 *__restrict__ tw, float2 *__restrict__ V,
               int Gh, int Gw, int log2h, int H, int NC, uint32_t key0, uint32_t key1,
               uint32_t frame_base, int nf, int nmodes) {
  extern __shared__ float2 lds[];  // [NC][Gh] in the lds_swz layout, slot-major; then the twiddles
  float2 *tws = lds + NC * Gh;
  load_twiddles(tws, tw, Gh, log2h);
  // line term: the read-out below visits 2^ysh rows of each of NC slots per
  // 32 lanes, so the slot number goes to bank bits ysh and up
  const int log2nc = __builtin_ctz(NC);
  const int ysh = log2nc < 5 ? 5 - log2nc : 0;
  const int q = blockIdx.y;
  // XCD-aware order: consecutive blocks go to different XCDs (round robin over
  // 8), so give the blocks of one XCD adjacent slot groups; their row
  // segments then share 128-byte lines in that XCD's L2.
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int grp = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int s0 = grp * NC;          // first slot of this block
  const int ma = 2 * q, mb = 2 * q + 1;  // 0-based mode indices (Noll 2+2q, 3+2q)
  const bool has_b = mb < nmodes;
  // (NC / 2) Gh = IPT x 512 draws, plus two in the self-mirror pair
  const int tail = (s0 == 0 && threadIdx.x < 2) ? IPT * 512 + threadIdx.x : -1;
  DrawItem it[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k)
    it[k] = draw_item(threadIdx.x + k * 512, sqrtS, Gh, Gw, log2h, s0, ysh, ma, mb, has_b);
  DrawItem itt = it[0];
  if (tail >= 0) itt = draw_item(tail, sqrtS, Gh, Gw, log2h, s0, ysh, ma, mb, has_b);
  const float norm = rsqrtf(float(Gh) * float(Gw));
  // read-out item e: row bits 0..ysh-1 from its low bits, then the slot,
  // then the remaining row bits (a wave writes 64/NC rows of the NC slots)
  const int ym = (1 << ysh) - 1;
  const int ritems = ((H + ym) >> ysh) << (ysh + log2nc);
  for (int fl = 0; fl < nf; ++fl) {
    const uint32_t frame = frame_base + uint32_t(fl);
#pragma unroll
    for (int k = 0; k < IPT; ++k) draw_noise(lds, it[k], q, frame, key0, key1);
    if (tail >= 0) draw_noise(lds, itt, q, frame, key0, key1);
    __syncthreads();
    lds_fft_dit(lds, Gh, log2h, NC, ysh, tws, 1.f);
    float2 *Vout = V + (size_t(fl) * gridDim.y + q) * size_t(H) * Gw + s0;
    for (int e = threadIdx.x; e < ritems; e += blockDim.x) {
      const int c = (e >> ysh) & (NC - 1);
      const int y = (e & ym) | ((e >> (ysh + log2nc)) << ysh);
      if (y < H) {
        const float2 v = lds[c * Gh + lds_swz(y, c << ysh)];
        Vout[size_t(y) * Gw + c] = make_float2(v.x * norm, v.y * norm);
      }
    }
    __syncthreads();  // the next frame's draws overwrite the lines
  }
}

// Structure of the mixing matrix.  L (lower Cholesky factor of the Noll
// matrix in Noll order) is non-zero only inside the (|m|, parity) groups of
// modes: mode k feeds output t iff both have the same |m| (and, for m != 0,
// the same parity of the Noll index) and k <= t.  Field q carries modes
// 2q and 2q + 1 (0-based, Noll 2 + 2q and 3 + 2q).  For the 35 modes of the
// default plan the mix is fused into the row pass: fields are transformed
// in the order below, chosen so that at most 9 outputs have received some
// but not all of their terms at any point, and each output is written as
// soon as its last field is mixed in: few accumulators stay live per pixel.
// Plans with more modes write the unit fields and mix them afterwards, group
// by group (k_mix_groups).
template <int N>
struct MixPlan {
  static constexpr int NF = (N + 1) / 2;
  bool nz[N][N];   // L[t][k] structurally non-zero
  int order[NF];   // fields in transform order
  int first[N];    // position in `order` of output t's first term
  int first_k[N];  // mode of that first term
  int last[N];     // position in `order` of output t's last field
};

constexpr int kFieldOrder35[18] = {10, 4, 16, 8, 15, 9, 1, 17, 14, 3, 7, 5, 2, 11, 0, 6, 13, 12};

constexpr int noll_abs_m(int j) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 < j) ++n;
  const int p = j - (n * (n + 1) / 2 + 1);
  return (n % 2 == 0) ? 2 * ((p + 1) / 2) : 2 * (p / 2) + 1;
}

constexpr int mix_group(int t) {  // t = 0-based mode index (Noll t + 2)
  const int j = t + 2, m = noll_abs_m(j);
  return m == 0 ? 0 : 2 * m - 1 + (j & 1);
}

template <int N>
constexpr MixPlan<N> make_mix_plan() {
  static_assert(N == 35, "the fused mix is built for the 35-mode plan");
  constexpr int NF = (N + 1) / 2;
  MixPlan<N> mp{};
  for (int t = 0; t < N; ++t) {
    mp.first[t] = mp.first_k[t] = mp.last[t] = -1;
    for (int k = 0; k < N; ++k) mp.nz[t][k] = k <= t && mix_group(k) == mix_group(t);
  }
  for (int i = 0; i < NF; ++i) mp.order[i] = kFieldOrder35[i];
  for (int i = 0; i < NF; ++i) {
    const int q = mp.order[i];
    for (int t = 0; t < N; ++t) {
      const bool a = mp.nz[t][2 * q];
      const bool b = 2 * q + 1 < N && mp.nz[t][2 * q + 1];
      if ((a || b) && mp.first[t] < 0) {
        mp.first[t] = i;
        mp.first_k[t] = a ? 2 * q : 2 * q + 1;
      }
      if (a || b) mp.last[t] = i;
    }
  }
  return mp;
}

template <int N>
struct Mix {
  static constexpr MixPlan<N> plan = make_mix_plan<N>();
};

struct RowArgs {
  float2 *lds;      // RW lines of Gw samples in the lds_swz layout (line term 0 and 1)
  const float2 *V;  // this frame's rows: V[q][y][:] at V + (q * H + y) * Gw
  const float2 *tws;  // LDS twiddle table
  const float *Lmat;
  float *out;       // this frame and first row: plane t at out + t * H * W
  int Gw, log2w, H, W, y0, nrows;
  float sc;
};

// The block's RW rows of field position I: GPT = Gw / NT samples per thread
// and row, read into registers (GPT > 0), or straight into LDS (GPT = 0).
template <int N, int I, int NT, int RW, int GPT>
__device__ __forceinline__ void read_field(const RowArgs &a, float2 (&pre)[RW][GPT > 0 ? GPT : 1]) {
  constexpr int q = Mix<N>::plan.order[I];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const float2 *row = a.V + (size_t(q) * a.H + a.y0 + (r < a.nrows ? r : 0)) * size_t(a.Gw);
#pragma unroll
    for (int j = 0; j < GPT; ++j) pre[r][j] = row[threadIdx.x + j * NT];
  }
}

// Field at position I of the transform order for the block's RW rows: inverse
// transform of the rows (one LDS pass over all RW lines), then the field's
// terms of the mix; outputs whose last field this is are written.  With
// GPT > 0 the field's samples arrive in registers, read while the previous
// field was transformed, and the next field's are requested here.
template <int N, int I, int PX, int NT, int RW, int GPT>
__device__ __forceinline__ void mix_field(const RowArgs &a, float (&acc)[N][RW][PX],
                                          float2 (&pre)[RW][GPT > 0 ? GPT : 1]) {
  constexpr MixPlan<N> kMix = Mix<N>::plan;
  constexpr int q = kMix.order[I];
  constexpr int ta = 2 * q, tb = 2 * q + 1;
  if constexpr (GPT > 0) {
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int j = 0; j < GPT; ++j) {
        const int c = threadIdx.x + j * NT;
        a.lds[r * a.Gw + lds_swz(bitrev(uint32_t(slot_col(c, a.Gw)), a.log2w), r)] = pre[r][j];
      }
    if constexpr (I + 1 < MixPlan<N>::NF) read_field<N, I + 1, NT, RW, GPT>(a, pre);
  } else {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const float2 *row = a.V + (size_t(q) * a.H + a.y0 + (r < a.nrows ? r : 0)) * size_t(a.Gw);
      for (int c = threadIdx.x; c < a.Gw; c += NT)
        a.lds[r * a.Gw + lds_swz(bitrev(uint32_t(slot_col(c, a.Gw)), a.log2w), r)] = row[c];
    }
  }
  __syncthreads();
  lds_fft_dit(a.lds, a.Gw, a.log2w, RW, 0, a.tws, 1.f);
  float ya[RW][PX], yb[RW][PX];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int x = threadIdx.x + k * NT;
      const float2 z = (x < a.W) ? a.lds[r * a.Gw + lds_swz(x, r)] : make_float2(0.f, 0.f);
      ya[r][k] = z.x;
      yb[r][k] = z.y;
    }
  __syncthreads();  // lds is overwritten by the next field
#pragma unroll
  for (int t = 0; t < N; ++t) {
    if (kMix.nz[t][ta]) {
      const float la = a.Lmat[t * N + ta];
      const bool init = kMix.first[t] == I && kMix.first_k[t] == ta;
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int k = 0; k < PX; ++k) acc[t][r][k] = init ? la * ya[r][k] : fmaf(la, ya[r][k], acc[t][r][k]);
    }
    if (tb < N && kMix.nz[t][tb]) {
      const float lb = a.Lmat[t * N + tb];
      const bool init = kMix.first[t] == I && kMix.first_k[t] == tb;
#pragma unroll
      for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int k = 0; k < PX; ++k) acc[t][r][k] = init ? lb * yb[r][k] : fmaf(lb, yb[r][k], acc[t][r][k]);
    }
    if (kMix.last[t] == I) {
      // opaque plane size: keeps the compiler from forming all N plane
      // addresses at kernel entry and holding them in registers
      size_t plane = size_t(a.H) * a.W;
      asm volatile("" : "+s"(plane));
      float *po = a.out + size_t(t) * plane;
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        if (r >= a.nrows) break;
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          const int x = threadIdx.x + k * NT;
          if (x < a.W) po[size_t(r) * a.W + x] = acc[t][r][k] * a.sc;
        }
      }
    }
  }
}

template <int N, int I, int PX, int NT, int RW, int GPT>
struct FieldSteps {
  __device__ __forceinline__ static void run(const RowArgs &a, float (&acc)[N][RW][PX],
                                             float2 (&pre)[RW][GPT > 0 ? GPT : 1]) {
    if constexpr (I < MixPlan<N>::NF) {
      mix_field<N, I, PX, NT, RW, GPT>(a, acc, pre);
      FieldSteps<N, I + 1, PX, NT, RW, GPT>::run(a, acc, pre);
    }
  }
};

// One block per RW consecutive output rows (the last block may hold fewer).
// GPT = Gw / NT (field samples per thread and row, read one field ahead) or 0.
template <int N, int PX, int NT, int RW, int GPT>
__global__ void __launch_bounds__(NT)
k_sampler_rows_mix(const float2 *__restrict__ V, const float2 *__restrict__ tw,
                   const float *__restrict__ Lmat, float *__restrict__ zern, int Gw, int log2w,
                   int H, int W, FrameScales scales, int frame_out0) {
  extern __shared__ float2 lds[];
  const int y0 = blockIdx.x * RW;
  const int fl = blockIdx.y;
  RowArgs a;
  a.lds = lds;
  a.V = V + size_t(fl) * MixPlan<N>::NF * H * size_t(Gw);
  a.tws = lds + RW * Gw;
  load_twiddles(lds + RW * Gw, tw, Gw, log2w);
  a.Lmat = Lmat;
  a.out = zern + size_t(frame_out0 + fl) * N * size_t(H) * W + size_t(y0) * W;
  a.Gw = Gw;
  a.log2w = log2w;
  a.H = H;
  a.W = W;
  a.y0 = y0;
  a.nrows = min(RW, H - y0);
  a.sc = scales.s[fl];
  float acc[N][RW][PX];  // each output starts at its first term
  float2 pre[RW][GPT > 0 ? GPT : 1];
  if constexpr (GPT > 0) read_field<N, 0, NT, RW, GPT>(a, pre);
  FieldSteps<N, 0, PX, NT, RW, GPT>::run(a, acc, pre);
}

// Row pass without the mix (plans with more than 35 modes): one block per
// RW output rows inverse-transforms every field's rows and writes its real
// and imaginary parts, cropped to W columns, as the unit fields of modes
// 2q and 2q + 1 (planes of zern, unscaled); k_mix_groups then mixes them.
template <int PX, int NT, int RW>
__global__ void __launch_bounds__(NT)
k_sampler_rows_unit(const float2 *__restrict__ V, const float2 *__restrict__ tw, float *__restrict__ zern, int Gw,
                    int log2w, int H, int W, int nmodes, int frame_out0) {
  extern __shared__ float2 lds[];
  const int y0 = blockIdx.x * RW;
  const int fl = blockIdx.y;
  const int nfields = (nmodes + 1) / 2;
  const int nrows = min(RW, H - y0);
  float2 *tws = lds + RW * Gw;
  load_twiddles(tws, tw, Gw, log2w);
  const float2 *Vf = V + size_t(fl) * nfields * H * size_t(Gw);
  const size_t plane = size_t(H) * W;
  float *out = zern + size_t(frame_out0 + fl) * nmodes * plane + size_t(y0) * W;
  for (int q = 0; q < nfields; ++q) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const float2 *row = Vf + (size_t(q) * H + y0 + (r < nrows ? r : 0)) * size_t(Gw);
      for (int c = threadIdx.x; c < Gw; c += NT)
        lds[r * Gw + lds_swz(bitrev(uint32_t(slot_col(c, Gw)), log2w), r)] = row[c];
    }
    __syncthreads();
    lds_fft_dit(lds, Gw, log2w, RW, 0, tws, 1.f);
    const bool has_b = 2 * q + 1 < nmodes;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      if (r >= nrows) break;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        const int x = threadIdx.x + k * NT;
        if (x < W) {
          const float2 z = lds[r * Gw + lds_swz(x, r)];
          out[size_t(2 * q) * plane + size_t(r) * W + x] = z.x;
          if (has_b) out[size_t(2 * q + 1) * plane + size_t(r) * W + x] = z.y;
        }
      }
    }
    __syncthreads();  // lds is overwritten by the next field
  }
}

// The mix of Eq. (9) in place on unit fields, a = (D/r0)^{5/6} L ybar, one
// (|m|, parity) group of modes at a time (L is block-diagonal on the groups):
// a group's members (at most kMaxGroup, listed in Noll order) are read at a
// pixel, their lower-triangular block of L applied, the outputs written.
// One thread per pixel, grid (ceil(H W / 256), frames).
constexpr int kMaxGroup = 6;   // modes per group up to radial order 10
constexpr int kMaxGroups = 21; // m = 0 and two parities for m = 1..10
struct MixGroups {
  int count;
  int member[kMaxGroups][kMaxGroup];            // 0-based mode index, -1 beyond the group
  float L[kMaxGroups][kMaxGroup][kMaxGroup];    // the group's block of L
};

__global__ void __launch_bounds__(256)
k_mix_groups(float *__restrict__ zern, size_t plane, int nmodes, FrameScales scales, int frame_out0,
             MixGroups g) {
  const size_t e = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= plane) return;
  const int fl = blockIdx.y;
  float *z = zern + size_t(frame_out0 + fl) * nmodes * plane + e;
  const float sc = scales.s[fl];
  for (int gi = 0; gi < g.count; ++gi) {
    float y[kMaxGroup];
#pragma unroll
    for (int i = 0; i < kMaxGroup; ++i) y[i] = g.member[gi][i] >= 0 ? z[size_t(g.member[gi][i]) * plane] : 0.f;
#pragma unroll
    for (int i = 0; i < kMaxGroup; ++i) {
      if (g.member[gi][i] < 0) break;
      float a = 0.f;
#pragma unroll
      for (int k = 0; k <= i; ++k) a = fmaf(g.L[gi][i][k], y[k], a);
      z[size_t(g.member[gi][i]) * plane] = a * sc;
    }
  }
}

// Subharmonic waves of the tilt fields, added after the mix: the waves w2,
// w3 belong to the unit fields of Noll 2 and 3, so output t gains
// s_f (L[t][0] w2 + L[t][1] w3), non-zero only for the outputs of the two
// tilt groups (|m| = 1).  One thread per pixel, grid (ceil(W/256), H,
// frames); the first 4 * levels threads draw the frame's wave amplitudes.
__global__ void __launch_bounds__(256)
k_subharmonic_add(float *__restrict__ zern, const float *__restrict__ Lmat, int H, int W, int N,
                  FrameScales scales, SubhArgs sub, int frame_out0) {
  __shared__ float coef[kSubhMaxLevels * 16];  // [level][cell][A2, B2, A3, B3]
  const int fl = blockIdx.z;
  if (int(threadIdx.x) < 4 * sub.levels) {
    const int p = threadIdx.x >> 2, c = threadIdx.x & 3;
    const u32x4 r = philox4x32_10(
        u32x4{uint32_t(c), uint32_t(p + 1), sub.frame_base + uint32_t(fl), kTagSubharmonic}, sub.key0, sub.key1);
    const float2 g01 = box_muller_hw(r.x, r.y);
    const float2 g23 = box_muller_hw(r.z, r.w);
    float *o = coef + (p * 4 + c) * 4;
    o[0] = sub.amp[0][p][c] * g01.x;
    o[1] = sub.amp[0][p][c] * g01.y;
    o[2] = sub.amp[1][p][c] * g23.x;
    o[3] = sub.amp[1][p][c] * g23.y;
  }
  __syncthreads();
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= W) return;
  float w2 = 0.f, w3 = 0.f;
  for (int p = 0; p < sub.levels; ++p) {
    float sa, ca, sb, cb;
    sincospif(float(x) * sub.fx[p], &sa, &ca);
    sincospif(float(y) * sub.fy[p], &sb, &cb);
    const float cd = ca * cb - sa * sb, sd = sa * cb + ca * sb;  // cell (1, 1): alpha + beta
    const float ce = ca * cb + sa * sb, se = ca * sb - sa * cb;  // cell (-1, 1): beta - alpha
    const float *c = coef + p * 16;
    w2 += c[0] * ca + c[1] * sa + c[4] * cd + c[5] * sd + c[8] * cb + c[9] * sb + c[12] * ce + c[13] * se;
    w3 += c[2] * ca + c[3] * sa + c[6] * cd + c[7] * sd + c[10] * cb + c[11] * sb + c[14] * ce + c[15] * se;
  }
  const float sc = scales.s[fl];
  const size_t plane = size_t(H) * W;
  float *out = zern + size_t(frame_out0 + fl) * N * plane + size_t(y) * W + x;
  // L[t][0] and L[t][1] are exactly zero outside the two tilt groups
  for (int t = 0; t < N; ++t) {
    const float l0 = Lmat[t * N], l1 = Lmat[t * N + 1];
    if (l0 != 0.f || l1 != 0.f) {
      float d = 0.f;
      if (l0 != 0.f) d = fmaf(l0, w2, d);
      if (l1 != 0.f) d = fmaf(l1, w3, d);
      out[size_t(t) * plane] += sc * d;
    }
  }
}

// Temporal auto-regression on the mixed fields, in place over a chunk of
// frames: a_f = mul_f a_{f-1} + c a_f^new (mul_f = alpha s_f / s_{f-1}); the
// frame before the chunk comes from `prev` (NULL at the start of a sequence:
// frame 0 keeps its own draw).  One thread per (mode, pixel) element, frames
// in order; every access is a coalesced stream over the planes.
struct ArCoefs {
  float mul[kMaxFramesPerLaunch];
};

__global__ void __launch_bounds__(256)
k_ar_scan(float *__restrict__ zern, const float *__restrict__ prev, size_t plane, int nf, ArCoefs co,
          float c) {
  constexpr int FB = 8;  // frames loaded ahead: their loads are in flight together
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < plane;
       e += size_t(gridDim.x) * blockDim.x) {
    float a = prev ? prev[e] : 0.f;
    for (int f0 = 0; f0 < nf; f0 += FB) {
      float nw[FB];
#pragma unroll
      for (int i = 0; i < FB; ++i)
        if (f0 + i < nf) nw[i] = zern[size_t(f0 + i) * plane + e];
#pragma unroll
      for (int i = 0; i < FB; ++i) {
        const int f = f0 + i;
        if (f < nf) {
          const float v = (f == 0 && !prev) ? nw[i] : fmaf(co.mul[f], a, c * nw[i]);
          zern[size_t(f) * plane + e] = v;
          a = v;
        }
      }
    }
  }
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

int frames_per_chunk(const tsim_plan *pl, int frames) {
  // bound the pass-1 intermediate to ~2 GB and the launch's scale table
  size_t per = size_t(pl->NF) * pl->H * size_t(pl->Gw) * sizeof(float2);
  size_t cap = size_t(2) << 30;
  int n = int(std::max<size_t>(1, cap / per));
  n = std::min(n, kMaxFramesPerLaunch);
  return std::min(n, frames);
}

}  // namespace

size_t sampler_ws_bytes(const tsim_plan *pl, int frames) {
  if (frames < 1) return 0;
  int n = frames_per_chunk(pl, frames);
  return size_t(n) * pl->NF * pl->H * size_t(pl->Gw) * sizeof(float2);
}

// pass 2 with the per-thread sample count Gw / NT as a compile-time constant
// where it is 2, 4 or 8 (the samples of the next field are then read one
// field ahead), without the look-ahead otherwise, for the 1024-thread
// blocks (whose extra registers would halve the blocks resident per CU)
template <int N, int PX, int NT, int RW>
void launch_rows(dim3 grid, size_t lds, hipStream_t s, const float2 *V, const float2 *tw, const float *L,
                 float *zern, int Gw, int log2w, int H, int W, FrameScales sc, int f0) {
  if constexpr (NT > 256) {
    hipLaunchKernelGGL((k_sampler_rows_mix<N, PX, NT, RW, 0>), grid, dim3(NT), lds, s, V, tw, L, zern, Gw, log2w,
                       H, W, sc, f0);
  } else {
    switch (Gw / NT) {
      case 2:
        hipLaunchKernelGGL((k_sampler_rows_mix<N, PX, NT, RW, 2>), grid, dim3(NT), lds, s, V, tw, L, zern, Gw,
                           log2w, H, W, sc, f0);
        break;
      case 4:
        hipLaunchKernelGGL((k_sampler_rows_mix<N, PX, NT, RW, 4>), grid, dim3(NT), lds, s, V, tw, L, zern, Gw,
                           log2w, H, W, sc, f0);
        break;
      case 8:
        hipLaunchKernelGGL((k_sampler_rows_mix<N, PX, NT, RW, 8>), grid, dim3(NT), lds, s, V, tw, L, zern, Gw,
                           log2w, H, W, sc, f0);
        break;
      default:
        hipLaunchKernelGGL((k_sampler_rows_mix<N, PX, NT, RW, 0>), grid, dim3(NT), lds, s, V, tw, L, zern, Gw,
                           log2w, H, W, sc, f0);
    }
  }
}

// The row pass's form: 1 = two rows per 256-thread block with the fewest
// outputs per thread covering W (up to W = 1024), 2 = the same with twice
// the outputs per thread (W <= 512), 3 = one row per 1024-thread block
// (four outputs per thread, any W <= 4096).  Every form computes the same
// transforms and sums; they differ only in how the work is spread.
int pass2_default(const tsim_plan *pl) { return pl->W <= 1024 ? 1 : 3; }

int pass2_form(const tsim_plan *pl) { return pl->tune_rows ? pl->tune_rows : pass2_default(pl); }

bool pass2_valid(const tsim_plan *pl, int form) {
  if (form == 1) return pl->W <= 1024;
  if (form == 2) return pl->W <= 512;
  return form == 3;
}

// Pass-1 columns per block: NC columns of Gh points in LDS, (NC / 2) Gh =
// 512 IPT draws with IPT = 2, 4 or 8; the built-in choice fills 32 KB.
int pass1_default(const tsim_plan *pl) { return std::min(std::max(2, std::min(kLdsFloat2 / pl->Gh, 32)), pl->Gw); }

bool pass1_valid(const tsim_plan *pl, int nc) {
  if (nc < 2 || nc > pl->Gw || (nc & (nc - 1)) != 0) return false;
  const long ipt = long(nc / 2) * pl->Gh / 512;
  return (ipt == 2 || ipt == 4 || ipt == 8) && (long(nc / 2) * pl->Gh) % 512 == 0;
}

int pass1_nc(const tsim_plan *pl) { return pl->tune_nc ? pl->tune_nc : pass1_default(pl); }

// pass 2 (with the mix for 35 modes; unit fields and k_mix_groups beyond)
// and the subharmonic waves
int launch_rows_n(const tsim_plan *pl, int nf, int f0, const float2 *V, float *zern, const FrameScales &sc,
                  const SubhArgs &sub, hipStream_t s) {
  const int Gw = pl->Gw, H = pl->H, W = pl->W, log2w = ilog2(Gw);
  {
    TraceScope tr("k_sampler_rows_mix", s);
    // two rows per block (one LDS transform pass and one barrier set for both)
    // up to 1024 columns; 1024-thread blocks over single rows beyond
    const size_t lds2 = (2 * size_t(Gw) + fft_twiddle_count(log2w)) * sizeof(float2);
    const size_t lds1 = (size_t(Gw) + fft_twiddle_count(log2w)) * sizeof(float2);
    dim3 g2((H + 1) / 2, nf), g1r(H, nf);
    // outputs per thread of the two-row form: the least that covers W, or
    // twice that (form 2); the one-row form takes four per thread
    int px = W <= 256 ? 1 : W <= 512 ? 2 : 4;
    const int form = pass2_form(pl);
    if (form == 2) px *= 2;
    if (form == 3 || px > 4) px = 0;  // one row per 1024-thread block
    if (pl->N == 35) {
      if (px == 1)
        launch_rows<35, 1, 256, 2>(g2, lds2, s, V, pl->d_tw_w, pl->d_L, zern, Gw, log2w, H, W, sc, f0);
      else if (px == 2)
        launch_rows<35, 2, 256, 2>(g2, lds2, s, V, pl->d_tw_w, pl->d_L, zern, Gw, log2w, H, W, sc, f0);
      else if (px == 4)
        launch_rows<35, 4, 256, 2>(g2, lds2, s, V, pl->d_tw_w, pl->d_L, zern, Gw, log2w, H, W, sc, f0);
      else
        launch_rows<35, 4, 1024, 1>(g1r, lds1, s, V, pl->d_tw_w, pl->d_L, zern, Gw, log2w, H, W, sc, f0);
    } else {
      const int N = pl->N;
      if (px == 1)
        hipLaunchKernelGGL((k_sampler_rows_unit<1, 256, 2>), g2, dim3(256), lds2, s, V, pl->d_tw_w, zern, Gw, log2w,
                           H, W, N, f0);
      else if (px == 2)
        hipLaunchKernelGGL((k_sampler_rows_unit<2, 256, 2>), g2, dim3(256), lds2, s, V, pl->d_tw_w, zern, Gw, log2w,
                           H, W, N, f0);
      else if (px == 4)
        hipLaunchKernelGGL((k_sampler_rows_unit<4, 256, 2>), g2, dim3(256), lds2, s, V, pl->d_tw_w, zern, Gw, log2w,
                           H, W, N, f0);
      else
        hipLaunchKernelGGL((k_sampler_rows_unit<4, 1024, 1>), g1r, dim3(1024), lds1, s, V, pl->d_tw_w, zern, Gw,
                           log2w, H, W, N, f0);
    }
  }
  if (pl->N != 35) {
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
    // the groups of modes sharing (|m|, parity), members in Noll order
    MixGroups g{};
    int gid[kMaxModes];
    for (int t = 0; t < pl->N; ++t) gid[t] = -1;
    for (int t = 0; t < pl->N; ++t) {
      if (gid[t] >= 0) continue;
      if (g.count >= kMaxGroups) return TSIM_EUNSUPPORTED;
      int n = 0;
      for (int k = t; k < pl->N; ++k)
        if (mix_group(k) == mix_group(t)) {
          if (n >= kMaxGroup) return TSIM_EUNSUPPORTED;
          gid[k] = g.count;
          g.member[g.count][n++] = k;
        }
      for (int i = n; i < kMaxGroup; ++i) g.member[g.count][i] = -1;
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < kMaxGroup; ++k)
          g.L[g.count][i][k] =
              k <= i && k < n ? float(pl->L[size_t(g.member[g.count][i]) * pl->N + g.member[g.count][k]]) : 0.f;
      ++g.count;
    }
    const size_t plane = size_t(H) * W;
    TraceScope tr("k_mix_groups", s);
    hipLaunchKernelGGL(k_mix_groups, dim3(unsigned((plane + 255) / 256), nf), dim3(256), 0, s, zern, plane, pl->N, sc,
                       f0, g);
  }
  if (sub.levels > 0) {
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
    TraceScope tr("k_subharmonic_add", s);
    hipLaunchKernelGGL(k_subharmonic_add, dim3((W + 255) / 256, H, nf), dim3(256), 0, s, zern, pl->d_L, H, W, pl->N,
                       sc, sub, f0);
  }
  return TSIM_OK;
}

namespace {

// pass 1 over nf frames (frame counters fb, fb + 1, ...) into V
int launch_pass1(const tsim_plan *pl, int nf, uint32_t fb, uint32_t key0, uint32_t key1, float2 *V,
                 hipStream_t s) {
  const int Gh = pl->Gh, Gw = pl->Gw, H = pl->H;
  const int log2h = ilog2(Gh);
  const int NC = pass1_nc(pl);
  if (!pass1_valid(pl, NC)) return TSIM_EUNSUPPORTED;
  // NC columns plus the twiddle table: 2 x 4096 + 1365 samples (75 KB) at
  // Gh = 4096, above the default 64 KB of dynamic LDS; the device limit is
  // checked and raised once (only the 8-draw form reaches it)
  const size_t lds1 = (size_t(NC) * Gh + fft_twiddle_count(log2h)) * sizeof(float2);
  if (lds1 > 64 * 1024) {
    static size_t raised = 0;
    if (lds1 > raised) {
      int dev = 0, max_lds = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return TSIM_EDEVICE;
      if (lds1 > size_t(max_lds)) return TSIM_EUNSUPPORTED;
      if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_sampler_cols<8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds1)) != hipSuccess)
        return TSIM_EDEVICE;
      raised = lds1;
    }
  }
  // draws per thread of a pass-1 block: (NC / 2) Gh / 512 = 2, 4 or 8
  const int ipt = (NC / 2) * Gh / 512;
  dim3 g1(Gw / NC, pl->NF);
  TraceScope tr("k_sampler_cols", s);
  if (ipt == 2)
    hipLaunchKernelGGL(k_sampler_cols<2>, g1, dim3(512), lds1, s, pl->d_sqrtS, pl->d_tw_h, V, Gh, Gw, log2h, H, NC,
                       key0, key1, fb, nf, pl->N);
  else if (ipt == 4)
    hipLaunchKernelGGL(k_sampler_cols<4>, g1, dim3(512), lds1, s, pl->d_sqrtS, pl->d_tw_h, V, Gh, Gw, log2h, H, NC,
                       key0, key1, fb, nf, pl->N);
  else
    hipLaunchKernelGGL(k_sampler_cols<8>, g1, dim3(512), lds1, s, pl->d_sqrtS, pl->d_tw_h, V, Gh, Gw, log2h, H, NC,
                       key0, key1, fb, nf, pl->N);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

// pass 2 (and the subharmonic waves) of nf frames with scales scale[0..nf)
// into zern frames f0 .. f0 + nf - 1 of the call
int launch_pass2(const tsim_plan *pl, int nf, int f0, const float *scale, uint32_t fb, uint32_t key0,
                 uint32_t key1, const float2 *V, float *zern, hipStream_t s) {
  const int Gh = pl->Gh, Gw = pl->Gw;
  FrameScales sc;
  for (int i = 0; i < kMaxFramesPerLaunch; ++i) sc.s[i] = 0.f;
  for (int i = 0; i < nf; ++i) sc.s[i] = scale[i];
  SubhArgs sub{};
  sub.levels = pl->p.subharmonic_levels;
  for (int p = 0; p < kSubhMaxLevels; ++p) {
    const double r = std::pow(3.0, p + 1);
    sub.fx[p] = float(2.0 / (Gw * r));
    sub.fy[p] = float(2.0 / (Gh * r));
    for (int c = 0; c < 4; ++c)
      for (int t = 0; t < 2; ++t) sub.amp[t][p][c] = float(pl->subh[(t * 4 + p) * 4 + c]);
  }
  sub.key0 = key0;
  sub.key1 = key1;
  sub.frame_base = fb;
  const int st = launch_rows_n(pl, nf, f0, V, zern, sc, sub, s);
  if (st != TSIM_OK) return st;
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}

}  // namespace

int launch_sampler(const tsim_plan *pl, int frames, const float *scale_host, uint64_t seed,
                   uint64_t frame0, float *zern, void *ws, hipStream_t s) {
  const uint32_t key0 = uint32_t(seed & 0xffffffffu), key1 = uint32_t(seed >> 32);
  float2 *V = static_cast<float2 *>(ws);
  const int chunk = frames_per_chunk(pl, frames);
  for (int f0 = 0; f0 < frames; f0 += chunk) {
    const int nf = std::min(chunk, frames - f0);
    const uint32_t fb = uint32_t(frame0 + uint64_t(f0));
    int st = launch_pass1(pl, nf, fb, key0, key1, V, s);
    if (st != TSIM_OK) return st;
    st = launch_pass2(pl, nf, f0, scale_host + f0, fb, key0, key1, V, zern, s);
    if (st != TSIM_OK) return st;
  }
  return TSIM_OK;
}

int sampler_chunk_frames(const tsim_plan *pl, int frames) { return frames_per_chunk(pl, frames); }

int sampler_pass1_forms(const tsim_plan *pl, int *nc) {
  const int d = pass1_default(pl);
  int n = 0;
  for (int c : {d, d / 2, d * 2})
    if (pass1_valid(pl, c)) nc[n++] = c;
  return n;
}

int sampler_pass2_forms(const tsim_plan *pl, int *form) {
  const int d = pass2_default(pl);
  int n = 0;
  form[n++] = d;
  for (int f = 1; f <= 3; ++f)
    if (f != d && pass2_valid(pl, f)) form[n++] = f;
  return n;
}

bool sampler_form_valid(const tsim_plan *pl, int nc, int rows) {
  return (nc == 0 || pass1_valid(pl, nc)) && (rows == 0 || pass2_valid(pl, rows));
}

int launch_sampler_pass(const tsim_plan *pl, int pass, int frames, float *zern, void *ws, hipStream_t s) {
  if (frames < 1 || frames > frames_per_chunk(pl, frames)) return TSIM_EINVAL;
  float scale[kMaxFramesPerLaunch];
  for (int i = 0; i < frames; ++i) scale[i] = 1.f;
  float2 *V = static_cast<float2 *>(ws);
  return pass == 1 ? launch_pass1(pl, frames, 0, 0, 0, V, s)
                   : launch_pass2(pl, frames, 0, scale, 0, 0, 0, V, zern, s);
}

int launch_sampler_ar(const tsim_plan *pl, int frames, const float *scale_host, float alpha,
                      const float *zern_prev, float scale_prev, uint64_t seed, uint64_t frame0,
                      float *zern, void *ws, hipStream_t s) {
  int st = launch_sampler(pl, frames, scale_host, seed, frame0, zern, ws, s);
  if (st != TSIM_OK) return st;
  const size_t plane = size_t(pl->N) * pl->H * pl->W;
  const float c = sqrtf(fmaxf(0.f, 1.f - alpha * alpha));
  const unsigned blocks = unsigned(std::min<size_t>((plane + 255) / 256, size_t(1) << 20));
  for (int f0 = 0; f0 < frames; f0 += kMaxFramesPerLaunch) {
    const int nf = std::min(kMaxFramesPerLaunch, frames - f0);
    ArCoefs co;
    for (int i = 0; i < kMaxFramesPerLaunch; ++i) co.mul[i] = 0.f;
    for (int i = 0; i < nf; ++i) {
      const int g = f0 + i;
      const float sp = g > 0 ? scale_host[g - 1] : scale_prev;
      co.mul[i] = (g > 0 || zern_prev) ? alpha * scale_host[g] / sp : 0.f;
    }
    const float *prev = f0 > 0 ? zern + size_t(f0 - 1) * plane : zern_prev;
    TraceScope tr("k_ar_scan", s);
    hipLaunchKernelGGL(k_ar_scan, dim3(blocks), dim3(256), 0, s, zern + size_t(f0) * plane, prev, plane, nf,
                       co, c);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  return TSIM_OK;
}
