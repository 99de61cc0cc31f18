// Spatial tilt statistics (Sec. IV-B): the tilt correlation E[a(0) a(theta)]
// and the differential tilt variance E[(a(0) - a(theta))^2] of the Noll 2 and
// Noll 3 coefficient planes, as functions of the pixel lag d = 0..L along x
// and along y, over all frames and every pixel pair inside the frame.
//
// k_tilt_stats_rows: one 256-thread block per (row y, frame).  Row y of both
// tilt planes is staged in LDS.  Each wave takes every fourth lag and sums,
// along the row, the products and squared differences with the pixel d
// columns to the right (from LDS) and d rows below (coalesced reads of that
// row), reduces the 8 sums (mode, axis, product / squared difference) over
// its lanes in a fixed order and writes them as FP32 partials
// part[frame][y][8][L + 1].
// k_tilt_stats_sum adds the partials of all rows and frames in FP64, one
// block per output, again in a fixed order: the result is deterministic.
#include "common.cuh"
#include "internal.h"

namespace {

constexpr int kStatsThreads = 256;

__global__ void __launch_bounds__(kStatsThreads)
k_tilt_stats_rows(const float *__restrict__ zern, int H, int W, int L, int nmodes, float *__restrict__ part) {
  extern __shared__ float row[];  // [2][W] tilt rows
  const int y = blockIdx.x, f = blockIdx.y;
  const size_t plane = size_t(H) * W;
  const float *a = zern + size_t(f) * nmodes * plane;  // Noll 2; Noll 3 at + plane
  for (int x = threadIdx.x; x < W; x += kStatsThreads) {
    row[x] = a[size_t(y) * W + x];
    row[W + x] = a[plane + size_t(y) * W + x];
  }
  __syncthreads();
  float *out = part + (size_t(f) * H + y) * 8 * size_t(L + 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each wave owns the lags d = wave, wave + 4, ...: its lanes stride over
  // the row and a shuffle tree sums them, so no lag waits on a block barrier
  for (int d = wave; d <= L; d += kStatsThreads / 64) {
    // v[(m * 2 + axis) * 2 + stat]: m = Noll 2 / 3, axis = x / y, stat = product / squared difference
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const bool ylag = y + d < H;
    for (int x = lane; x < W; x += 64) {
      const float u2 = row[x], u3 = row[W + x];
      if (x + d < W) {
        const float p2 = row[x + d], p3 = row[W + x + d];
        v[0] = fmaf(u2, p2, v[0]);
        v[1] = fmaf(u2 - p2, u2 - p2, v[1]);
        v[4] = fmaf(u3, p3, v[4]);
        v[5] = fmaf(u3 - p3, u3 - p3, v[5]);
      }
      if (ylag) {
        const float q2 = a[size_t(y + d) * W + x];
        const float q3 = a[plane + size_t(y + d) * W + x];
        v[2] = fmaf(u2, q2, v[2]);
        v[3] = fmaf(u2 - q2, u2 - q2, v[3]);
        v[6] = fmaf(u3, q3, v[6]);
        v[7] = fmaf(u3 - q3, u3 - q3, v[7]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    if (lane < 8) {
      float r = v[0];
#pragma unroll
      for (int i = 1; i < 8; ++i) r = lane == i ? v[i] : r;
      out[size_t(lane) * (L + 1) + d] = r;
    }
  }
}

__global__ void __launch_bounds__(kStatsThreads)
k_tilt_stats_sum(const float *__restrict__ part, size_t rows, int n_out, double *__restrict__ out) {
  __shared__ double red[kStatsThreads];
  const int o = blockIdx.x;
  double acc = 0.0;
  for (size_t r = threadIdx.x; r < rows; r += kStatsThreads) acc += double(part[r * n_out + o]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kStatsThreads / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[o] = red[0];
}

// Second moments of the coefficient vectors, for the aperture statistics
// (the structure function is a quadratic form in them): one block per tile
// of 256 pixels of one frame, its 35 x 256 coefficients staged in LDS; the
// 630 pairs j <= k are shared out over the threads, each summing a_j a_k
// over the tile into an FP32 partial part[frame][tile][630].
constexpr int kPairs = TSIM_N_MODES * (TSIM_N_MODES + 1) / 2;
struct PairTable {
  unsigned char j[kPairs], k[kPairs];
};
constexpr PairTable make_pairs() {
  PairTable t{};
  int q = 0;
  for (int j = 0; j < TSIM_N_MODES; ++j)
    for (int k = j; k < TSIM_N_MODES; ++k) {
      t.j[q] = static_cast<unsigned char>(j);
      t.k[q] = static_cast<unsigned char>(k);
      ++q;
    }
  return t;
}
__constant__ PairTable kPairTable = make_pairs();

__global__ void __launch_bounds__(kStatsThreads)
k_moments_tiles(const float *__restrict__ zern, size_t plane, int tiles, float *__restrict__ part) {
  __shared__ float tile[TSIM_N_MODES][kStatsThreads + 1];
  const int f = blockIdx.y, ti = blockIdx.x;
  const size_t p = size_t(ti) * kStatsThreads + threadIdx.x;
  const float *a = zern + size_t(f) * TSIM_N_MODES * plane;
  for (int j = 0; j < TSIM_N_MODES; ++j) tile[j][threadIdx.x] = p < plane ? a[size_t(j) * plane + p] : 0.f;
  __syncthreads();
  float *out = part + (size_t(f) * tiles + ti) * kPairs;
  for (int q = threadIdx.x; q < kPairs; q += kStatsThreads) {
    const int j = kPairTable.j[q], k = kPairTable.k[q];
    float acc = 0.f;
    for (int i = 0; i < kStatsThreads; ++i) acc = fmaf(tile[j][i], tile[k][i], acc);
    out[q] = acc;
  }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t tilt_stats_ws_bytes(const tsim_plan *pl, int frames, int max_lag) {
  const size_t n_out = 8 * size_t(max_lag + 1);
  return align256(size_t(frames) * pl->H * n_out * sizeof(float)) + align256(n_out * sizeof(double));
}

int launch_tilt_stats(const tsim_plan *pl, int frames, const float *zern, int max_lag, double *host_out,
                      void *ws, hipStream_t s) {
  const int H = pl->H, W = pl->W, L = max_lag;
  const int n_out = 8 * (L + 1);
  float *part = static_cast<float *>(ws);
  double *sums = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                            align256(size_t(frames) * H * n_out * sizeof(float)));
  {
    TraceScope tr("k_tilt_stats_rows", s);
    const size_t lds = 2 * size_t(W) * sizeof(float);
    hipLaunchKernelGGL(k_tilt_stats_rows, dim3(H, frames), dim3(kStatsThreads), lds, s, zern, H, W, L, pl->N, part);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  {
    TraceScope tr("k_tilt_stats_sum", s);
    hipLaunchKernelGGL(k_tilt_stats_sum, dim3(n_out), dim3(kStatsThreads), 0, s, part,
                       size_t(frames) * H, n_out, sums);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  std::vector<double> h(n_out);
  TSIM_HIP_CHECK(hipMemcpyAsync(h.data(), sums, n_out * sizeof(double), hipMemcpyDeviceToHost, s));
  TSIM_HIP_CHECK(hipStreamSynchronize(s));
  // means over the pairs: H (W - d) per frame for an x lag, (H - d) W for a y lag
  for (int i = 0; i < 8; ++i) {
    const int axis = (i >> 1) & 1;
    for (int d = 0; d <= L; ++d) {
      const double pairs = double(frames) * (axis == 0 ? double(H) * (W - d) : double(H - d) * W);
      host_out[i * (L + 1) + d] = h[size_t(i) * (L + 1) + d] / pairs;
    }
  }
  return TSIM_OK;
}

size_t moments_ws_bytes(const tsim_plan *pl, int frames) {
  const size_t tiles = (size_t(pl->H) * pl->W + kStatsThreads - 1) / kStatsThreads;
  return align256(size_t(frames) * tiles * kPairs * sizeof(float)) + align256(kPairs * sizeof(double));
}

int launch_moments(const tsim_plan *pl, int frames, const float *zern, double *host_out, void *ws,
                   hipStream_t s) {
  const size_t plane = size_t(pl->H) * pl->W;
  const int tiles = int((plane + kStatsThreads - 1) / kStatsThreads);
  float *part = static_cast<float *>(ws);
  double *sums = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                            align256(size_t(frames) * tiles * kPairs * sizeof(float)));
  {
    TraceScope tr("k_moments_tiles", s);
    hipLaunchKernelGGL(k_moments_tiles, dim3(tiles, frames), dim3(kStatsThreads), 0, s, zern, plane, tiles, part);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  {
    TraceScope tr("k_tilt_stats_sum", s);
    hipLaunchKernelGGL(k_tilt_stats_sum, dim3(kPairs), dim3(kStatsThreads), 0, s, part, size_t(frames) * tiles,
                       kPairs, sums);
    if (hipGetLastError() != hipSuccess) return TSIM_EDEVICE;
  }
  std::vector<double> h(kPairs);
  TSIM_HIP_CHECK(hipMemcpyAsync(h.data(), sums, kPairs * sizeof(double), hipMemcpyDeviceToHost, s));
  TSIM_HIP_CHECK(hipStreamSynchronize(s));
  const double n = double(frames) * double(plane);
  const PairTable pt = make_pairs();
  for (int q = 0; q < kPairs; ++q) {
    const int j = pt.j[q], k = pt.k[q];
    host_out[j * TSIM_N_MODES + k] = host_out[k * TSIM_N_MODES + j] = h[q] / n;
  }
  return TSIM_OK;
}

int launch_partial_sum(const float *part, size_t rows, int n_out, double *out, hipStream_t s) {
  TraceScope tr("k_tilt_stats_sum", s);
  hipLaunchKernelGGL(k_tilt_stats_sum, dim3(n_out), dim3(kStatsThreads), 0, s, part, rows, n_out, out);
  return hipGetLastError() == hipSuccess ? TSIM_OK : TSIM_EDEVICE;
}
