// PSF basis of Eq. (7) by PCA over a database of exact PSFs (Sec. II-C: the
// basis is learned by principal component analysis on a PSF database).
//
// Device: draw n Zernike vectors a = (D/r0)^{5/6} L g (g ~ N(0, I_35) from
// Philox counters (i, w, 0, 1), D/r0 uniform in [lo, hi] from word 0 of
// (i, 9, 0, 1)), their exact PSFs (k_psf64), and the FP64 Gram matrix
// G = H^T H of the (n, T*T) PSF matrix.  Host: the top-K eigenvectors of G
// by block subspace iteration with Rayleigh-Ritz (Jacobi on the small
// projected matrix).  The eigenvectors of H^T H are the right singular
// vectors of H, i.e. an uncentred PCA.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.cuh"
#include "internal.h"

namespace {

using namespace tsim;

// Coefficient vectors of the PSF database, N modes: g ~ N(0, I_N) from
// the Gaussians of Philox calls (i, w, 0, 1), w < ceil(N/4), and D/r0 from
// word 0 of call (i, ceil(N/4), 0, 1); a = (D/r0)^{5/6} L g.
__global__ void k_basis_draws(const float *__restrict__ Lmat, float *__restrict__ zvec, int n, int N,
                              uint32_t key0, uint32_t key1, float lo, float hi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float g[4 * ((kMaxModes + 3) / 4)];
  const int calls = (N + 3) / 4;
#pragma unroll
  for (int w = 0; w < (kMaxModes + 3) / 4; ++w) {
    if (w >= calls) break;
    u32x4 r = philox4x32_10(u32x4{uint32_t(i), uint32_t(w), 0u, 1u}, key0, key1);
    float2 a = box_muller(r.x, r.y), b = box_muller(r.z, r.w);
    g[4 * w + 0] = a.x;
    g[4 * w + 1] = a.y;
    g[4 * w + 2] = b.x;
    g[4 * w + 3] = b.y;
  }
  u32x4 r = philox4x32_10(u32x4{uint32_t(i), uint32_t(calls), 0u, 1u}, key0, key1);
  const float dr = lo + (hi - lo) * u01(r.x);
  const float sc = powf(dr, 5.0f / 6.0f);
  for (int j = 0; j < N; ++j) {
    float s = 0.f;
    for (int k = 0; k <= j; ++k) s = fmaf(Lmat[j * N + k], g[k], s);
    zvec[size_t(i) * N + j] = s * sc;
  }
}

// G[a][b] = sum_i h[i][a] h[i][b] in FP64, upper-triangle 32 x 32 tiles.
__global__ void __launch_bounds__(256)
k_gram(const float *__restrict__ h, double *__restrict__ G, int n, int T2) {
  const int ta = blockIdx.y, tb = blockIdx.x;
  if (tb < ta) return;
  __shared__ double As[32][33];
  __shared__ double Bs[32][33];
  const int a0 = ta * 32, b0 = tb * 32;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;  // 16 x 16 threads, 2 x 2 outputs each
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int i0 = 0; i0 < n; i0 += 32) {
    for (int e = threadIdx.x; e < 32 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      const int i = i0 + r;
      As[r][c] = (i < n && a0 + c < T2) ? double(h[size_t(i) * T2 + a0 + c]) : 0.0;
      Bs[r][c] = (i < n && b0 + c < T2) ? double(h[size_t(i) * T2 + b0 + c]) : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 32; ++r) {
      const double x0 = As[r][ty], x1 = As[r][ty + 16];
      const double y0 = Bs[r][tx], y1 = Bs[r][tx + 16];
      acc[0][0] = fma(x0, y0, acc[0][0]);
      acc[0][1] = fma(x0, y1, acc[0][1]);
      acc[1][0] = fma(x1, y0, acc[1][0]);
      acc[1][1] = fma(x1, y1, acc[1][1]);
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int a = a0 + ty + 16 * u, b = b0 + tx + 16 * v;
      if (a < T2 && b < T2) {
        G[size_t(a) * T2 + b] = acc[u][v];
        G[size_t(b) * T2 + a] = acc[u][v];
      }
    }
}

// ---------------------------------------------------------------- host ----
// Y = G Q for G (n x n, row-major) and Q (n x p, row-major), multithreaded.
void gemm_gq(const std::vector<double> &G, const std::vector<double> &Q, std::vector<double> &Y,
             int n, int p) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      double *y = &Y[size_t(r) * p];
      std::fill(y, y + p, 0.0);
      const double *g = &G[size_t(r) * n];
      for (int k = 0; k < n; ++k) {
        const double gk = g[k];
        const double *q = &Q[size_t(k) * p];
        for (int c = 0; c < p; ++c) y[c] += gk * q[c];
      }
    }
  };
  std::vector<std::thread> th;
  int chunk = (n + int(nt) - 1) / int(nt);
  for (unsigned i = 0; i < nt; ++i) {
    int a = int(i) * chunk, b = std::min(n, a + chunk);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto &t : th) t.join();
}

// Orthonormalise the columns of Q (n x p, row-major): modified Gram-Schmidt,
// applied twice.
void orthonormalise(std::vector<double> &Q, int n, int p) {
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = 0; c < p; ++c) {
      for (int d = 0; d < c; ++d) {
        double dot = 0.0;
        for (int r = 0; r < n; ++r) dot += Q[size_t(r) * p + c] * Q[size_t(r) * p + d];
        for (int r = 0; r < n; ++r) Q[size_t(r) * p + c] -= dot * Q[size_t(r) * p + d];
      }
      double nrm = 0.0;
      for (int r = 0; r < n; ++r) nrm += Q[size_t(r) * p + c] * Q[size_t(r) * p + c];
      nrm = std::sqrt(nrm);
      const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
      for (int r = 0; r < n; ++r) Q[size_t(r) * p + c] *= inv;
    }
  }
}

// Cyclic Jacobi eigen-decomposition of the symmetric p x p matrix B
// (destroyed); eigenvectors in the columns of V.
void jacobi_eig(std::vector<double> &B, std::vector<double> &V, std::vector<double> &w, int p) {
  V.assign(size_t(p) * p, 0.0);
  for (int i = 0; i < p; ++i) V[size_t(i) * p + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        double v = B[size_t(i) * p + j] * B[size_t(i) * p + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int i = 0; i < p - 1; ++i) {
      for (int j = i + 1; j < p; ++j) {
        const double bij = B[size_t(i) * p + j];
        if (bij == 0.0) continue;
        const double bii = B[size_t(i) * p + i], bjj = B[size_t(j) * p + j];
        const double theta = (bjj - bii) / (2.0 * bij);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < p; ++k) {  // columns i, j
          const double bki = B[size_t(k) * p + i], bkj = B[size_t(k) * p + j];
          B[size_t(k) * p + i] = c * bki - s * bkj;
          B[size_t(k) * p + j] = s * bki + c * bkj;
        }
        for (int k = 0; k < p; ++k) {  // rows i, j
          const double bik = B[size_t(i) * p + k], bjk = B[size_t(j) * p + k];
          B[size_t(i) * p + k] = c * bik - s * bjk;
          B[size_t(j) * p + k] = s * bik + c * bjk;
        }
        for (int k = 0; k < p; ++k) {
          const double vki = V[size_t(k) * p + i], vkj = V[size_t(k) * p + j];
          V[size_t(k) * p + i] = c * vki - s * vkj;
          V[size_t(k) * p + j] = s * vki + c * vkj;
        }
      }
    }
  }
  w.resize(p);
  for (int i = 0; i < p; ++i) w[i] = B[size_t(i) * p + i];
}

// Top-K eigenpairs of the symmetric positive semi-definite G (n x n).
int top_eigen(const std::vector<double> &G, int n, int K, std::vector<double> &vecs /*K x n*/,
              std::vector<double> &vals) {
  const int p = std::min(n, K + 32);
  std::vector<double> Q(size_t(n) * p), Y(size_t(n) * p), B(size_t(p) * p), V, w;
  uint64_t st = 0x243F6A8885A308D3ull;  // SplitMix64 start vectors
  for (auto &q : Q) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    q = double(z >> 11) * 0x1.0p-53 - 0.5;
  }
  orthonormalise(Q, n, p);
  std::vector<double> prev(K, 0.0);
  for (int it = 0; it < 400; ++it) {
    gemm_gq(G, Q, Y, n, p);
    // Rayleigh-Ritz: B = Q^T G Q, rotate Q onto the Ritz vectors, then
    // advance the subspace with the product already formed.
    for (int a = 0; a < p; ++a)
      for (int b = 0; b < p; ++b) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) s += Q[size_t(r) * p + a] * Y[size_t(r) * p + b];
        B[size_t(a) * p + b] = s;
      }
    for (int a = 0; a < p; ++a)
      for (int b = a + 1; b < p; ++b) {
        double m = 0.5 * (B[size_t(a) * p + b] + B[size_t(b) * p + a]);
        B[size_t(a) * p + b] = B[size_t(b) * p + a] = m;
      }
    jacobi_eig(B, V, w, p);
    std::vector<int> order(p);
    for (int i = 0; i < p; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });
    bool conv = it > 2;
    for (int k = 0; k < K; ++k) {
      const double v = w[order[k]];
      if (std::fabs(v - prev[k]) > 1e-13 * std::fabs(w[order[0]])) conv = false;
      prev[k] = v;
    }
    // Ritz vectors X = Q V (sorted), and the next block Q <- orth(G X) = orth(Y V)
    std::vector<double> X(size_t(n) * p), Z(size_t(n) * p);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < p; ++c) {
        double sx = 0.0, sz = 0.0;
        for (int k = 0; k < p; ++k) {
          const double v = V[size_t(k) * p + order[c]];
          sx += Q[size_t(r) * p + k] * v;
          sz += Y[size_t(r) * p + k] * v;
        }
        X[size_t(r) * p + c] = sx;
        Z[size_t(r) * p + c] = sz;
      }
    if (conv || it == 399) {
      vecs.assign(size_t(K) * n, 0.0);
      vals.assign(K, 0.0);
      for (int k = 0; k < K; ++k) {
        vals[k] = w[order[k]];
        for (int r = 0; r < n; ++r) vecs[size_t(k) * n + r] = X[size_t(r) * p + k];
      }
      return conv ? TSIM_OK : TSIM_EARTEFACT;
    }
    Q.swap(Z);
    orthonormalise(Q, n, p);
  }
  return TSIM_EARTEFACT;
}

int basis_build_impl(const tsim_plan *pl, int n_psf, uint64_t seed, double dr_lo, double dr_hi,
                     double *basis_out, double *eig_out) {
  if (!pl || !basis_out || n_psf < 1 || n_psf > (1 << 22)) return TSIM_EINVAL;
  if (!(dr_lo > 0.0) || !(dr_hi >= dr_lo) || !std::isfinite(dr_hi)) return TSIM_EINVAL;
  const int T2 = pl->T * pl->T, K = pl->K;
  if (K > T2 || K > n_psf) return TSIM_EINVAL;
  float *d_z = nullptr, *d_h = nullptr;
  double *d_G = nullptr;
  int st = TSIM_OK;
  std::vector<double> G(size_t(T2) * T2), vecs, vals;
  if (hipMalloc(&d_z, size_t(n_psf) * pl->N * sizeof(float)) != hipSuccess ||
      hipMalloc(&d_h, size_t(n_psf) * T2 * sizeof(float)) != hipSuccess ||
      hipMalloc(&d_G, size_t(T2) * T2 * sizeof(double)) != hipSuccess) {
    st = TSIM_ENOMEM;
    goto done;
  }
  hipLaunchKernelGGL(k_basis_draws, dim3((n_psf + 255) / 256), dim3(256), 0, 0, pl->d_L, d_z, n_psf, pl->N,
                     uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32), float(dr_lo), float(dr_hi));
  if (hipGetLastError() != hipSuccess) {
    st = TSIM_EDEVICE;
    goto done;
  }
  if ((st = launch_psf_exact(pl, n_psf, d_z, d_h, 0)) != TSIM_OK) goto done;
  {
    const int nt = (T2 + 31) / 32;
    hipLaunchKernelGGL(k_gram, dim3(nt, nt), dim3(256), 0, 0, d_h, d_G, n_psf, T2);
  }
  if (hipGetLastError() != hipSuccess ||
      hipMemcpy(G.data(), d_G, G.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    st = TSIM_EDEVICE;
    goto done;
  }
  st = top_eigen(G, T2, K, vecs, vals);
  if (st != TSIM_OK) goto done;
  for (int k = 0; k < K; ++k) {
    double *v = &vecs[size_t(k) * T2];
    double sum = 0.0, big = 0.0;
    int ibig = 0;
    for (int t = 0; t < T2; ++t) {
      sum += v[t];
      if (std::fabs(v[t]) > big) {
        big = std::fabs(v[t]);
        ibig = t;
      }
    }
    const bool flip = (std::fabs(sum) < 1e-9) ? (v[ibig] < 0) : (sum < 0);
    for (int t = 0; t < T2; ++t) basis_out[size_t(k) * T2 + t] = flip ? -v[t] : v[t];
    if (eig_out) eig_out[k] = vals[k];
  }
done:
  if (d_z) (void)hipFree(d_z);
  if (d_h) (void)hipFree(d_h);
  if (d_G) (void)hipFree(d_G);
  return st;
}

}  // namespace

extern "C" int tsim_basis_build(const tsim_plan *pl, int n_psf, uint64_t seed, double dr_lo,
                                double dr_hi, double *basis_out, double *eig_out) {
  return note_status("tsim_basis_build", basis_build_impl(pl, n_psf, seed, dr_lo, dr_hi, basis_out, eig_out));
}
