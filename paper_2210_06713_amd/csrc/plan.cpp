// Host-side FP64 plan tables and the plan half of the C ABI.
//
// Everything here runs once per plan on the CPU in float64 and is uploaded
// to the device as float32:
//   * the Noll covariance A_0 of the Zernike coefficients at one pixel
//     (Sec. II-B; Sec. III-B: the s = 0 slice of the tensor of Eq. (6)) and
//     its lower Cholesky factor L (Sec. III-C, Eq. (9): L L^T = A_0);
//   * per-mode lattice spectra of the homogeneous autocovariances A_ii
//     (Sec. III-B/III-C), square-rooted, stored as a quarter table;
//   * the Zernike pupil table for the exact PSFs of Eq. (2);
//   * the PSF basis of Eq. (7).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>

#include "internal.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- Noll ----
void noll_nm(int j, int *n_out, int *m_out) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 < j) ++n;
  int k = j - n * (n + 1) / 2;  // 1..n+1 inside the radial order
  int m = (n % 2 == 0) ? 2 * (k / 2) : 2 * ((k - 1) / 2) + 1;
  *n_out = n;
  *m_out = m;
}

// Phase-spectrum constant for Phi(f) = c r0^{-5/3} f^{-11/3}, f in cycles per
// metre, chosen so the structure function is Eq. (4)'s 6.88 (r/r0)^{5/3} with
// 6.88 = 2[(24/5) Gamma(6/5)]^{5/6}.
double kolmogorov_c() {
  double bracket = 4.8 * std::tgamma(1.2);
  return std::tgamma(11.0 / 6.0) * std::tgamma(11.0 / 6.0) / (2.0 * std::pow(kPi, 11.0 / 3.0)) *
         std::pow(bracket, 5.0 / 6.0);
}

// Noll's closed form: the Zernike filters of a Kolmogorov screen integrate to
// Gamma-function ratios (Weber-Schafheitlin, exponent 14/3).
double noll_entry(int j, int jp, double kc) {
  int n, m, np, mp;
  noll_nm(j, &n, &m);
  noll_nm(jp, &np, &mp);
  if (m != mp) return 0.0;
  if (m != 0 && (j % 2) != (jp % 2)) return 0.0;
  double sign = (((n + np - 2 * m) / 2) % 2 == 0) ? 1.0 : -1.0;
  double g = std::tgamma((n + np - 5.0 / 3.0) / 2.0) /
             (std::tgamma((n - np + 17.0 / 3.0) / 2.0) * std::tgamma((np - n + 17.0 / 3.0) / 2.0) *
              std::tgamma((n + np + 23.0 / 3.0) / 2.0));
  return kc * sign * std::sqrt(double((n + 1) * (np + 1))) * g;
}

bool cholesky(const std::vector<double> &A, std::vector<double> &L, int n) {
  L.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = A[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) s -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[size_t(i) * n + i] = std::sqrt(s);
      } else {
        L[size_t(i) * n + j] = s / L[size_t(j) * n + j];
      }
    }
  }
  return true;
}

// ------------------------------------------------------------- Bessel ----
// J_0..J_nmax(x) for x >= 0 by Miller's downward recurrence
//   J_{k-1} = (2k/x) J_k - J_{k+1},
// started well above max(x, nmax) and normalised with the Neumann identity
// J_0 + 2 sum_k J_{2k} = 1.  One pass gives every order needed by a
// frequency sample.
void bessel_j_orders(double x, int nmax, double *out) {
  if (x < 1e-8) {
    out[0] = 1.0;
    for (int k = 1; k <= nmax; ++k) out[k] = 0.0;
    // leading term (x/2)^k / k! keeps tiny-frequency spectra exact
    double t = 1.0;
    for (int k = 1; k <= nmax; ++k) {
      t *= 0.5 * x / k;
      out[k] = t;
    }
    return;
  }
  int start = int(std::max(x, double(nmax))) + 30 + int(12.0 * std::cbrt(x));
  if (start & 1) ++start;
  double jp1 = 0.0, j = 1e-300, norm = 0.0;
  for (int k = start; k >= 1; --k) {
    double jm1 = (2.0 * k / x) * j - jp1;
    jp1 = j;
    j = jm1;  // now J_{k-1}
    int km1 = k - 1;
    if (km1 <= nmax) out[km1] = j;
    if (km1 % 2 == 0 && km1 > 0) norm += 2.0 * j;
    if (std::fabs(j) > 1e250) {  // rescale to stay in range
      j *= 1e-250;
      jp1 *= 1e-250;
      norm *= 1e-250;
      for (int q = km1; q <= nmax; ++q) out[q] *= 1e-250;
    }
  }
  norm += j;  // J_0
  double inv = 1.0 / norm;
  for (int k = 0; k <= nmax; ++k) out[k] *= inv;
}

// Spectrum of mode j (without its constant): f^{-11/3} |Q_j(f)|^2 with
// |Q_j|^2 = (n+1) [2 J_{n+1}(pi f)/(pi f)]^2 Theta_j(phi), f in cycles per D.
// `jb` holds J_0..J_11(pi f).  cos(m phi), sin(m phi) come from the caller.
inline double mode_spectrum(int n, int m, int kind, double f, const double *jb, double cm,
                            double sm) {
  double x = kPi * f;
  double r = 2.0 * jb[n + 1] / x;
  double ang = (kind == 0) ? 1.0 : (kind == 1 ? 2.0 * cm * cm : 2.0 * sm * sm);
  return std::pow(f, -11.0 / 3.0) * (n + 1) * r * r * ang;
}

struct ModeInfo {
  int n, m, kind;  // kind 0: m = 0, 1: cosine (even j), 2: sine (odd j)
};

// Spectra of all modes at (fx0, fy0) cycles per D, summed over the lattice
// aliases (fx0 + lx/ds, fy0 + ly/ds), |lx|, |ly| <= A.
void folded_spectra(const ModeInfo *mi, int N, double fx0, double fy0, double ds, int A, double *acc) {
  double jb[12];
  double cm[11], sm[11];
  for (int t = 0; t < N; ++t) acc[t] = 0.0;
  for (int lx = -A; lx <= A; ++lx) {
    for (int ly = -A; ly <= A; ++ly) {
      double fx = fx0 + lx / ds;
      double fy = fy0 + ly / ds;
      double f = std::hypot(fx, fy);
      if (f == 0.0) continue;
      bessel_j_orders(kPi * f, 11, jb);
      double c1 = fx / f, s1 = fy / f;
      cm[0] = 1.0;
      sm[0] = 0.0;
      for (int q = 1; q < 11; ++q) {
        cm[q] = cm[q - 1] * c1 - sm[q - 1] * s1;
        sm[q] = sm[q - 1] * c1 + cm[q - 1] * s1;
      }
      for (int t = 0; t < N; ++t)
        acc[t] += mode_spectrum(mi[t].n, mi[t].m, mi[t].kind, f, jb, cm[mi[t].m], sm[mi[t].m]);
    }
  }
}

void build_spectra(tsim_plan *pl) {
  const int Gh = pl->Gh, Gw = pl->Gw;
  const int qh = Gh / 2 + 1, qw = Gw / 2 + 1;
  const int A = pl->p.alias_fold;
  const double ds = pl->ds;
  const int N = pl->N;
  ModeInfo mi[kMaxModes];
  for (int t = 0; t < N; ++t) {
    int j = t + 2, n, m;
    noll_nm(j, &n, &m);
    mi[t] = {n, m, m == 0 ? 0 : (j % 2 == 0 ? 1 : 2)};
  }
  // quarter table S[mode][kx'][ky'] in float64
  std::vector<double> S(size_t(N) * qw * qh, 0.0);
  auto work = [&](int kx0, int kx1) {
    for (int kx = kx0; kx < kx1; ++kx) {
      for (int ky = 0; ky < qh; ++ky) {
        if (kx == 0 && ky == 0) continue;  // DC removed
        double acc[kMaxModes];
        folded_spectra(mi, N, double(kx) / (Gw * ds), double(ky) / (Gh * ds), ds, A, acc);
        for (int t = 0; t < N; ++t) S[(size_t(t) * qw + kx) * qh + ky] = acc[t];
      }
    }
  };
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  int chunk = (qw + nt - 1) / nt;
  for (unsigned i = 0; i < nt; ++i) {
    int a = int(i) * chunk, b = std::min(qw, a + chunk);
    if (a < b) th.emplace_back(work, a, b);
  }
  for (auto &t : th) t.join();
  // Subharmonic cells of the tilt modes (t = 0, 1): level p, half-plane
  // cell (m, n) at (m/(Gw ds), n/(Gh ds))/3^p; a level-p cell has 1/9^p of a
  // bin's area, and each half-plane cell stands for itself and its mirror.
  const int levels = pl->p.subharmonic_levels;
  static const int kCell[4][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}};
  double cellS[2][4][4] = {};
  double cellW[2] = {0.0, 0.0};
  for (int p = 1; p <= levels; ++p) {
    const double r = std::pow(3.0, p);
    for (int c = 0; c < 4; ++c) {
      double acc[kMaxModes];
      folded_spectra(mi, N, kCell[c][0] / (Gw * ds * r), kCell[c][1] / (Gh * ds * r), ds, A, acc);
      for (int t = 0; t < 2; ++t) {
        cellS[t][p - 1][c] = acc[t];
        cellW[t] += 2.0 * acc[t] / (r * r);
      }
    }
  }
  pl->subh.assign(2 * 4 * 4, 0.0);
  // unit mean over the full Gh x Gw grid (plus, for the tilt modes, the
  // subharmonic cells): interior quarter bins stand for two mirror bins per
  // axis, the DC and Nyquist rows/columns for one.
  pl->sqrtS.assign(S.size(), 0.0);
  for (int t = 0; t < N; ++t) {
    double tot = t < 2 ? cellW[t] : 0.0;
    for (int kx = 0; kx < qw; ++kx) {
      double wx = (kx == 0 || kx == Gw / 2) ? 1.0 : 2.0;
      for (int ky = 0; ky < qh; ++ky) {
        double wy = (ky == 0 || ky == Gh / 2) ? 1.0 : 2.0;
        tot += wx * wy * S[(size_t(t) * qw + kx) * qh + ky];
      }
    }
    double scale = double(Gh) * Gw / tot;
    for (size_t i = size_t(t) * qw * qh; i < size_t(t + 1) * qw * qh; ++i)
      pl->sqrtS[i] = std::sqrt(S[i] * scale);
    // wave amplitude: variance of the cell and its mirror, 2 S scale / (Gh Gw 9^p)
    if (t < 2)
      for (int p = 1; p <= levels; ++p)
        for (int c = 0; c < 4; ++c)
          pl->subh[(t * 4 + (p - 1)) * 4 + c] =
              std::sqrt(2.0 * cellS[t][p - 1][c] * scale / (double(Gh) * Gw * std::pow(9.0, p)));
  }
}

// Zernike Z_j(rho, theta), Noll normalisation (mean square 1 on the disc).
double zernike(int j, double rho, double theta) {
  int n, m;
  noll_nm(j, &n, &m);
  double r = 0.0;
  for (int s = 0; s <= (n - m) / 2; ++s) {
    double c = std::tgamma(n - s + 1.0) /
               (std::tgamma(s + 1.0) * std::tgamma((n + m) / 2 - s + 1.0) *
                std::tgamma((n - m) / 2 - s + 1.0));
    r += ((s % 2) ? -c : c) * std::pow(rho, n - 2 * s);
  }
  r *= std::sqrt(double(n + 1));
  if (m == 0) return r;
  return (j % 2 == 0) ? r * std::sqrt(2.0) * std::cos(m * theta)
                      : r * std::sqrt(2.0) * std::sin(m * theta);
}

// IEEE half precision of a double, nearest with ties to even (subnormals
// kept, overflow to infinity), and the exact value of a half
uint16_t f16_rn(double x) {
  const uint16_t sign = std::signbit(x) ? 0x8000 : 0;
  const double a = std::fabs(x);
  if (a == 0.0) return sign;
  int e;
  (void)std::frexp(a, &e);                         // a = f 2^e, f in [0.5, 1)
  const int q = std::max(e - 11, -24);             // weight of the last kept bit
  const double v = std::ldexp(std::nearbyint(std::ldexp(a, -q)), q);  // ties to even
  if (v >= 65520.0) return sign | 0x7c00;
  if (v < std::ldexp(1.0, -14)) return sign | uint16_t(std::ldexp(v, 24));  // subnormal
  int ev;
  const double fr = std::frexp(v, &ev);            // v = fr 2^ev, fr in [0.5, 1)
  const uint16_t man = uint16_t(uint32_t(std::ldexp(fr, 11)) & 0x3ffu);
  return uint16_t(sign | uint16_t((ev + 14) << 10) | man);
}

double f16_value(uint16_t h) {
  const int e = (h >> 10) & 0x1f, m = h & 0x3ff;
  const double v = e == 0 ? std::ldexp(double(m), -24) : std::ldexp(double(1024 + m), e - 25);
  return (h & 0x8000) ? -v : v;
}

template <class T>
int upload(T **dst, const T *src, size_t n) {
  if (hipMalloc(dst, n * sizeof(T)) != hipSuccess) {
    *dst = nullptr;
    return TSIM_ENOMEM;
  }
  if (hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return TSIM_EDEVICE;
  return TSIM_OK;
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int validate(const tsim_params *p) {
  if (!p) return TSIM_EINVAL;
  if (p->H < 1 || p->W < 1 || p->H > 4096 || p->W > 4096) return TSIM_EINVAL;
  if (p->C < 1 || p->C > 4) return TSIM_EINVAL;
  if (!pow2(p->Gh) || !pow2(p->Gw) || p->Gh < 64 || p->Gw < 64 || p->Gh > 4096 || p->Gw > 4096)
    return TSIM_EINVAL;
  if (p->Gh < p->H || p->Gw < p->W) return TSIM_EINVAL;
  if (!modes_supported(p->n_modes)) return TSIM_EINVAL;
  // the network's input layer is 35 wide
  if (p->p2s_mode == TSIM_P2S_LEARNED && p->n_modes != TSIM_N_MODES) return TSIM_EUNSUPPORTED;
  if (p->alias_fold < 0 || p->alias_fold > 4) return TSIM_EINVAL;
  if (!(p->pixel_pitch_over_d > 0.0) || !std::isfinite(p->pixel_pitch_over_d)) {
    if (!(p->aperture_d_m > 0.0) || !(p->wavelength_m > 0.0) || !(p->path_length_m > 0.0))
      return TSIM_EINVAL;
  }
  if (p->pupil_n != 64 && p->pupil_n != 128) return TSIM_EUNSUPPORTED;
  if (p->psf_t < 3 || (p->psf_t % 2) == 0 || p->psf_t > p->pupil_n / 2 + 1) return TSIM_EINVAL;
  if (p->basis_k < 1 || p->basis_k > 128) return TSIM_EINVAL;
  if (p->p2s_mode != TSIM_P2S_EXACT && p->p2s_mode != TSIM_P2S_LEARNED) return TSIM_EINVAL;
  if (p->precision != TSIM_FP32 && p->precision != TSIM_BF16) return TSIM_EINVAL;
  if (p->subharmonic_levels < 0 || p->subharmonic_levels > 4) return TSIM_EINVAL;
  // the exact path (plain form, basis build, training pairs, and the learned
  // form's fallback) must exist for the plan's PSF support, and so must the
  // BF16 blur in BF16 plans
  if (!psf_size_supported(p->pupil_n, p->psf_t, p->n_modes)) return TSIM_EUNSUPPORTED;
  const int kp = p->basis_k <= 32 ? 32 : p->basis_k <= 64 ? 64 : p->basis_k <= 112 ? 112 : 128;
  if (p->precision == TSIM_BF16 && !render_bf16_supported(kp, p->psf_t, p->C)) return TSIM_EUNSUPPORTED;
  return TSIM_OK;
}

void free_plan(tsim_plan *pl) {
  if (!pl) return;
  void *ptrs[] = {pl->d_sqrtS, pl->d_tw_h, pl->d_tw_w, pl->d_L, pl->d_zcheb, pl->d_basis, pl->d_basis_h3, pl->d_basis_h3r,
                  pl->d_basis_t, pl->d_basis_bf, pl->d_mlp_w, pl->d_mlp_f};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  delete pl;
}

}  // namespace

// Phase structure function over the aperture from the coefficients' second
// moments C[j][k] = mean a_j a_k (Noll 2..36): on a 64 x 64 pupil grid with
// the aperture 32 samples across (points strictly inside), D(r) = mean over
// the pairs (p, p + r x) inside of (sum_j a_j (Z_j(p) - Z_j(p + r x)))^2,
// whose mean over pixels is sum_jk C_jk M_jk(r), M_jk(r) = mean over the
// pairs of dZ_j dZ_k.  r = 0..30 samples.  M depends on nothing but the grid
// and is built once per process.
namespace {

std::vector<double> build_sf_pair_moments() {
  constexpr int P = kSfPupil, N = TSIM_N_MODES;
  const double rad = P / 4.0;
  std::vector<double> Z(size_t(N) * P * P, 0.0);
  std::vector<char> in(size_t(P) * P, 0);
  for (int y = 0; y < P; ++y)
    for (int x = 0; x < P; ++x) {
      const double X = (x - P / 2) / rad, Y = (y - P / 2) / rad, rho = std::hypot(X, Y);
      if (!(rho < 1.0)) continue;
      in[size_t(y) * P + x] = 1;
      for (int t = 0; t < N; ++t) Z[(size_t(t) * P + y) * P + x] = zernike(t + 2, rho, std::atan2(Y, X));
    }
  std::vector<double> M(size_t(kSfLags) * N * N, 0.0);
  std::vector<double> dz(N);
  for (int r = 1; r < kSfLags; ++r) {
    double *m = M.data() + size_t(r) * N * N;
    long pairs = 0;
    for (int y = 0; y < P; ++y)
      for (int x = 0; x + r < P; ++x) {
        if (!in[size_t(y) * P + x] || !in[size_t(y) * P + x + r]) continue;
        for (int t = 0; t < N; ++t) dz[t] = Z[(size_t(t) * P + y) * P + x] - Z[(size_t(t) * P + y) * P + x + r];
        for (int j = 0; j < N; ++j)
          for (int k = 0; k < N; ++k) m[j * N + k] += dz[j] * dz[k];
        ++pairs;
      }
    if (pairs)
      for (int i = 0; i < N * N; ++i) m[i] /= double(pairs);
  }
  return M;
}

}  // namespace

void structure_function_from_moments(const double *C, double *out) {
  constexpr int N = TSIM_N_MODES;
  static const std::vector<double> M = build_sf_pair_moments();  // thread-safe, once
  for (int r = 0; r < kSfLags; ++r) {
    const double *m = M.data() + size_t(r) * N * N;
    double acc = 0.0;
    for (int i = 0; i < N * N; ++i) acc += C[i] * m[i];
    out[r] = acc;
  }
}

extern "C" {

const char *tsim_status_string(int s) {
  switch (s) {
    case TSIM_OK: return "ok";
    case TSIM_EINVAL: return "invalid argument";
    case TSIM_ENOMEM: return "out of memory";
    case TSIM_EDEVICE: return "device or HIP runtime error";
    case TSIM_EARTEFACT: return "basis or network weights missing or malformed";
    case TSIM_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// Host half of plan creation: validated parameters -> FP64 tables.
int build_host(const tsim_params *p, tsim_plan *pl) {
  pl->p = *p;
  pl->p.basis = nullptr;
  pl->Gh = p->Gh;
  pl->Gw = p->Gw;
  pl->H = p->H;
  pl->W = p->W;
  pl->C = p->C;
  pl->P = p->pupil_n;
  pl->T = p->psf_t;
  pl->K = p->basis_k;
  pl->KP = p->basis_k <= 32 ? 32 : p->basis_k <= 64 ? 64 : p->basis_k <= 112 ? 112 : 128;
  pl->ds = (p->pixel_pitch_over_d > 0.0)
               ? p->pixel_pitch_over_d
               : p->path_length_m * p->wavelength_m / (2.0 * p->aperture_d_m * p->aperture_d_m);
  pl->N = p->n_modes;
  pl->NF = (p->n_modes + 1) / 2;
  pl->NCH = cheb_terms(p->n_modes);
  // Noll matrix and its Cholesky factor
  const int N = pl->N;
  double c = kolmogorov_c();
  double kc = 8.0 * c * std::pow(kPi, 8.0 / 3.0) * std::tgamma(14.0 / 3.0) / std::pow(2.0, 14.0 / 3.0);
  pl->A0.assign(size_t(N) * N, 0.0);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) pl->A0[size_t(a) * N + b] = noll_entry(a + 2, b + 2, kc);
  if (!cholesky(pl->A0, pl->L, N)) return TSIM_EINVAL;
  build_spectra(pl);
  return TSIM_OK;
}

int copy_table(const tsim_plan *pl, int what, double *host_out, size_t count) {
  const std::vector<double> *src = nullptr;
  switch (what) {
    case 0: src = &pl->A0; break;
    case 1: src = &pl->L; break;
    case 2: src = &pl->sqrtS; break;
    case 4: src = &pl->subh; break;
    case 3:
      if (count < 1) return TSIM_EINVAL;
      host_out[0] = pl->ds;
      return TSIM_OK;
    default: return TSIM_EINVAL;
  }
  if (count < src->size()) return TSIM_EINVAL;
  std::memcpy(host_out, src->data(), src->size() * sizeof(double));
  return TSIM_OK;
}

int host_tables_impl(const tsim_params *p, int what, double *host_out, size_t count);
int plan_create_impl(const tsim_params *p, tsim_plan **out);

}  // namespace

extern "C" {

int tsim_host_tables(const tsim_params *p, int what, double *host_out, size_t count) {
  return note_status("tsim_host_tables", host_tables_impl(p, what, host_out, count));
}

int tsim_plan_create(const tsim_params *p, tsim_plan **out) {
  return note_status("tsim_plan_create", plan_create_impl(p, out));
}

int tsim_plan_destroy(tsim_plan *pl) {
  free_plan(pl);
  return TSIM_OK;
}

int tsim_plan_table(const tsim_plan *pl, int what, double *host_out, size_t count) {
  if (!pl || !host_out) return note_status("tsim_plan_table", TSIM_EINVAL);
  return note_status("tsim_plan_table", copy_table(pl, what, host_out, count));
}

}  // extern "C"

namespace {

int host_tables_impl(const tsim_params *p, int what, double *host_out, size_t count) {
  if (!host_out) return TSIM_EINVAL;
  int st = validate(p);
  if (st != TSIM_OK) return st;
  tsim_plan *pl = new (std::nothrow) tsim_plan();
  if (!pl) return TSIM_ENOMEM;
  st = build_host(p, pl);
  if (st == TSIM_OK) st = copy_table(pl, what, host_out, count);
  delete pl;
  return st;
}

int plan_create_impl(const tsim_params *p, tsim_plan **out) {
  if (!out) return TSIM_EINVAL;
  *out = nullptr;
  int st = validate(p);
  if (st != TSIM_OK) return st;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return TSIM_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TSIM_EDEVICE;

  tsim_plan *pl = new (std::nothrow) tsim_plan();
  if (!pl) return TSIM_ENOMEM;
  if ((st = build_host(p, pl)) != TSIM_OK) {
    free_plan(pl);
    return st;
  }
  // device tables
  std::vector<float> f32(pl->sqrtS.begin(), pl->sqrtS.end());
  if ((st = upload(&pl->d_sqrtS, f32.data(), f32.size())) != TSIM_OK) goto fail;
  {
    std::vector<float2> tw(static_cast<size_t>(pl->Gh / 2));
    for (int k = 0; k < pl->Gh / 2; ++k)
      tw[k] = make_float2(float(std::cos(2 * kPi * k / pl->Gh)), float(std::sin(2 * kPi * k / pl->Gh)));
    if ((st = upload(&pl->d_tw_h, tw.data(), tw.size())) != TSIM_OK) goto fail;
    std::vector<float2> tw2(static_cast<size_t>(pl->Gw / 2));
    for (int k = 0; k < pl->Gw / 2; ++k)
      tw2[k] = make_float2(float(std::cos(2 * kPi * k / pl->Gw)), float(std::sin(2 * kPi * k / pl->Gw)));
    if ((st = upload(&pl->d_tw_w, tw2.data(), tw2.size())) != TSIM_OK) goto fail;
    std::vector<float> Lf(pl->L.begin(), pl->L.end());
    if ((st = upload(&pl->d_L, Lf.data(), Lf.size())) != TSIM_OK) goto fail;
  }
  {
    // Phase of modes 4..N+1 as 2D Chebyshev series over the aperture square:
    // Z_j(x, y) = sum_{p,q < NCH} E[j][p][q] T_p(x) T_q(y) exactly (a mode of
    // radial order n is a polynomial of degree <= n in x and in y, and NCH
    // is the plan's highest order plus one), with E by interpolation at the
    // NCH x NCH Chebyshev nodes.  Coordinates are normalised to the aperture
    // radius (P/4 samples), so the table does not depend on P.  Stored
    // [j][p][q].
    const int NZ = pl->N - 2, NP = pl->NCH;
    // zero padded to the kernels' 33 (8 terms) or 63 (11 terms) modes
    const int NZP = NP == 8 ? 33 : 63;
    std::vector<float> zc(size_t(NZP) * NP * NP, 0.0f);
    for (int t = 0; t < NZ; ++t) {
      double f[11][11];
      for (int k = 0; k < NP; ++k)
        for (int l = 0; l < NP; ++l) {
          const double x = std::cos(kPi * (k + 0.5) / NP), y = std::cos(kPi * (l + 0.5) / NP);
          f[k][l] = zernike(t + 4, std::hypot(x, y), std::atan2(y, x));
        }
      for (int p = 0; p < NP; ++p)
        for (int q = 0; q < NP; ++q) {
          double c = 0.0;
          for (int k = 0; k < NP; ++k)
            for (int l = 0; l < NP; ++l)
              c += f[k][l] * std::cos(p * kPi * (k + 0.5) / NP) * std::cos(q * kPi * (l + 0.5) / NP);
          c *= (p == 0 ? 1.0 : 2.0) * (q == 0 ? 1.0 : 2.0) / (NP * NP);
          zc[(size_t(t) * NP + p) * NP + q] = float(c);
        }
    }
    if ((st = upload(&pl->d_zcheb, zc.data(), zc.size())) != TSIM_OK) goto fail;
  }
  if (p->basis) {
    const int T2 = pl->T * pl->T, K = pl->K, KP = pl->KP;
    pl->basis.assign(p->basis, p->basis + size_t(K) * T2);
    for (double v : pl->basis)
      if (!std::isfinite(v)) {
        st = TSIM_EARTEFACT;
        goto fail;
      }
    std::vector<float> b(size_t(K) * T2), bt(size_t(KP) * T2, 0.0f);
    for (int k = 0; k < K; ++k)
      for (int t = 0; t < T2; ++t) {
        b[size_t(k) * T2 + t] = float(pl->basis[size_t(k) * T2 + t]);
        bt[size_t(t) * KP + k] = float(pl->basis[size_t(k) * T2 + t]);
      }
    if ((st = upload(&pl->d_basis, b.data(), b.size())) != TSIM_OK) goto fail;
    if ((st = upload(&pl->d_basis_t, bt.data(), bt.size())) != TSIM_OK) goto fail;
    // BF16 copy for the matrix-core blur in groups of 32 horizontal tap
    // pairs: [group][side][pair][KP + 8], pair j = (uy, i) = (j / NPX, j %
    // NPX) covers taps (uy, 2i) (side 0) and (uy, 2i + 1) (side 1); taps past
    // the kernel edge, pairs past the last one and the row pads are zero
    const int T = pl->T, NPX = (T + 1) / 2, NPR = T * NPX, NTP = (NPR + 31) / 32, KPP = KP + 8;
    std::vector<uint16_t> bb(size_t(NTP) * 64 * KPP, 0);
    for (int j = 0; j < NPR; ++j)
      for (int h = 0; h < 2; ++h) {
        const int uy = j / NPX, ux = 2 * (j % NPX) + h;
        if (ux >= T) continue;
        const size_t row = (size_t(j / 32) * 2 + h) * 32 + j % 32;
        for (int k = 0; k < K; ++k) {
          float f = float(pl->basis[size_t(k) * T2 + uy * T + ux]);
          uint32_t u;
          std::memcpy(&u, &f, 4);
          bb[row * KPP + k] = uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
        }
      }
    if ((st = upload(&pl->d_basis_bf, bb.data(), bb.size())) != TSIM_OK) goto fail;
    // the projection's operand: psi x 2^10 split into FP16 (hi, lo), in
    // fragment order [chunk of 32 taps][step][output tile][lane][hi, lo][8]:
    // lane l holds output 32 tile + l % 32, taps 32 chunk + 16 step +
    // 8 (l / 32) + 0..7; zero past K and T*T, and to a whole number of
    // 64-tap chunks (the kernel takes two of these chunks at a time)
    {
      const int NCHK = (T2 + 63) / 64 * 2, NTL = (KP + 31) / 32;
      std::vector<uint16_t> h3(size_t(NCHK) * 2 * NTL * 64 * 2 * 8, 0);
      for (int c = 0; c < NCHK; ++c)
        for (int st2 = 0; st2 < 2; ++st2)
          for (int j = 0; j < NTL; ++j)
            for (int l = 0; l < 64; ++l)
              for (int e = 0; e < 8; ++e) {
                const int o = 32 * j + l % 32, t = 32 * c + 16 * st2 + 8 * (l / 32) + e;
                const double x = (o < K && t < T2) ? std::ldexp(pl->basis[size_t(o) * T2 + t], 10) : 0.0;
                const uint16_t hi = f16_rn(x);
                const uint16_t lo = f16_rn(x - f16_value(hi));
                const size_t at = ((((size_t(c) * 2 + st2) * NTL + j) * 64 + l) * 2) * 8 + e;
                h3[at] = hi;
                h3[at + 8] = lo;
              }
      if ((st = upload(&pl->d_basis_h3, h3.data(), h3.size())) != TSIM_OK) goto fail;
    }
    // the plain blur's operand: psi x 2^10 split into FP16 (hi, lo), in
    // fragment order [tap block of 32][k-step of 16][hi, lo][lane][8]: lane l
    // holds tap 32 block + l % 32, coefficients 16 step + 8 (l / 32) + 0..7;
    // zero past K and T*T
    {
      const int NTB = (T2 + 31) / 32, KSR = KP / 16;
      std::vector<uint16_t> r3(size_t(NTB) * KSR * 2 * 64 * 8, 0);
      for (int tb = 0; tb < NTB; ++tb)
        for (int q = 0; q < KSR; ++q)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int t = 32 * tb + l % 32, k = 16 * q + 8 * (l / 32) + e;
              const double x = (t < T2 && k < K) ? std::ldexp(pl->basis[size_t(k) * T2 + t], 10) : 0.0;
              const uint16_t hi = f16_rn(x);
              const uint16_t lo = f16_rn(x - f16_value(hi));
              r3[(((size_t(tb) * KSR + q) * 2 + 0) * 64 + l) * 8 + e] = hi;
              r3[(((size_t(tb) * KSR + q) * 2 + 1) * 64 + l) * 8 + e] = lo;
            }
      if ((st = upload(&pl->d_basis_h3r, r3.data(), r3.size())) != TSIM_OK) goto fail;
    }
  }
  // device address of the allocation-free sampler's scratch array, looked
  // up now (once per device) so that its calls do no set-up work
  if ((st = noalloc_scratch_init()) != TSIM_OK) goto fail;
  *out = pl;
  return TSIM_OK;
fail:
  free_plan(pl);
  return st;
}

}  // namespace
