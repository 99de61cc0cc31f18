"""Zernike modes, their Fourier transforms and the Noll covariance (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II-B, Eq. (5) expands the aperture phase at each pixel on Zernike
functions Z_j with Noll's single index j; the paper keeps N = 36 modes.  The
correlation tensor of Eq. (6) at zero displacement is Noll's covariance
matrix (Sec. II-B, last paragraph; Sec. III-B).  Noll's closed form is cited,
not printed, so it is derived here from the Kolmogorov phase spectrum fixed by
Eq. (4) (see ``spectra.kolmogorov_c``) and the Weber-Schafheitlin integral;
tests pin it against direct numerical quadrature of that spectrum.
"""
import math
import numpy as np
from scipy import special

N_MODES = 35          # Noll j = 2..36 (piston dropped, it moves no pixel)
J_FIRST = 2
J_LAST = 36


def noll_nm(j):
    """Noll index j >= 1 -> (n, m).  m rises with j inside radial order n."""
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2          # 1 .. n+1 inside the order
    if n % 2 == 0:
        m = 2 * (k // 2)
    else:
        m = 2 * ((k - 1) // 2) + 1
    return n, m


def noll_kind(j):
    """'c' (cosine, even j), 's' (sine, odd j) or '0' (m = 0)."""
    n, m = noll_nm(j)
    if m == 0:
        return '0'
    return 'c' if j % 2 == 0 else 's'


def radial(n, m, rho):
    """Zernike radial polynomial R_n^m(rho) (explicit finite sum)."""
    rho = np.asarray(rho, dtype=np.float64)
    out = np.zeros_like(rho)
    for s in range((n - m) // 2 + 1):
        coef = ((-1) ** s * math.factorial(n - s)
                / (math.factorial(s) * math.factorial((n + m) // 2 - s)
                   * math.factorial((n - m) // 2 - s)))
        out = out + coef * rho ** (n - 2 * s)
    return out


def zernike(j, rho, theta):
    """Orthonormal Zernike Z_j(rho, theta) on the unit disc (Noll's norm:
    the mean of Z_j^2 over the disc is 1)."""
    n, m = noll_nm(j)
    r = math.sqrt(n + 1) * radial(n, m, rho)
    kind = noll_kind(j)
    if kind == '0':
        return r
    if kind == 'c':
        return r * math.sqrt(2.0) * np.cos(m * theta)
    return r * math.sqrt(2.0) * np.sin(m * theta)


def zernike_ft(j, fr, fphi):
    """Fourier transform of Z_j over the unit-radius disc, normalised by the
    disc area, at radial frequency ``fr`` in cycles per *diameter* and polar
    angle ``fphi`` (forward transform, kernel exp(-2 pi i f.r)).

    Q_j(f) = sqrt(n+1) * 2 J_{n+1}(pi f)/(pi f) * (-i)^m * (-1)^{(n-m)/2}
             * {sqrt2 cos(m phi), sqrt2 sin(m phi), 1}  -- with the sign of the
    (-i)^m factor following the forward-kernel convention.  The tests check
    this against direct numerical integration of Z_j over the disc.
    """
    n, m = noll_nm(j)
    fr = np.asarray(fr, dtype=np.float64)
    x = np.pi * fr
    with np.errstate(divide='ignore', invalid='ignore'):
        radial_part = np.where(x > 0, 2.0 * special.jv(n + 1, x) / np.where(x > 0, x, 1.0),
                               1.0 if n == 0 else 0.0)
    pref = math.sqrt(n + 1) * ((-1) ** ((n - m) // 2)) * ((-1j) ** m)
    kind = noll_kind(j)
    if kind == '0':
        ang = 1.0
    elif kind == 'c':
        ang = math.sqrt(2.0) * np.cos(m * fphi)
    else:
        ang = math.sqrt(2.0) * np.sin(m * fphi)
    return pref * radial_part * ang


def noll_constant():
    """K_c in A_0[j,j'] = K_c (D/r0)^{5/3} (-1)^{(n+n'-2m)/2} sqrt((n+1)(n'+1))
    Gamma((n+n'-5/3)/2) / [Gamma((n-n'+17/3)/2) Gamma((n'-n+17/3)/2)
    Gamma((n+n'+23/3)/2)].

    Derivation: A_0[j,j'] = c (D/r0)^{5/3} \\int f^{-11/3} Q_j Q_j'^* d^2 f with f
    in cycles per D and c the phase-spectrum constant fixed by Eq. (4).  The
    angular integral gives 2 pi (1 for m=0 pairs), the radial one is a
    Weber-Schafheitlin integral with lambda = 14/3, giving
    K_c = 8 c pi^{8/3} Gamma(14/3) / 2^{14/3}.
    """
    from .spectra import kolmogorov_c
    c = kolmogorov_c()
    return 8.0 * c * np.pi ** (8.0 / 3.0) * special.gamma(14.0 / 3.0) / 2.0 ** (14.0 / 3.0)


def _noll_pair(j, jp, kc):
    n, m = noll_nm(j)
    npp, mp = noll_nm(jp)
    if m != mp:
        return 0.0
    if m != 0 and (j % 2) != (jp % 2):
        return 0.0
    sign = (-1) ** ((n + npp - 2 * m) // 2)
    g = (special.gamma((n + npp - 5.0 / 3.0) / 2.0)
         / (special.gamma((n - npp + 17.0 / 3.0) / 2.0)
            * special.gamma((npp - n + 17.0 / 3.0) / 2.0)
            * special.gamma((n + npp + 23.0 / 3.0) / 2.0)))
    return kc * sign * math.sqrt((n + 1) * (npp + 1)) * g


def noll_matrix(d_over_r0=1.0, j_first=J_FIRST, j_last=J_LAST):
    """A_0 for Noll modes j_first..j_last (Sec. II-B: [A]_{0,i,j} is Noll's
    covariance), in rad^2, scaled by (D/r0)^{5/3}."""
    kc = noll_constant()
    js = list(range(j_first, j_last + 1))
    A = np.zeros((len(js), len(js)))
    for a, j in enumerate(js):
        for b, jp in enumerate(js):
            A[a, b] = _noll_pair(j, jp, kc)
    return A * float(d_over_r0) ** (5.0 / 3.0)


def noll_order_variance(n):
    """Diagonal A_0 value shared by every mode of radial order n (D/r0 = 1)."""
    kc = noll_constant()
    return kc * (n + 1) * (special.gamma(n - 5.0 / 6.0)
                           / (special.gamma(17.0 / 6.0) ** 2 * special.gamma(n + 23.0 / 6.0)))


def noll_residual(J, n_max=200000):
    """Noll residual Delta_J = sum_{j > J} A_0[j,j] (D/r0 = 1).

    Each radial order n holds n+1 modes of equal variance, so the infinite sum
    is taken order by order up to n_max and the tail is closed with the
    asymptotic n^{-8/3} law of the order totals."""
    n = np.arange(1, n_max + 1, dtype=np.float64)
    kc = noll_constant()
    logv = (np.log(kc) + np.log(n + 1) + special.gammaln(n - 5.0 / 6.0)
            - 2 * special.gammaln(17.0 / 6.0) - special.gammaln(n + 23.0 / 6.0))
    per_mode = np.exp(logv)
    per_order = per_mode * (n + 1)
    total = per_order.sum()
    # tail: per_order ~ C n^{-8/3};  sum_{n>N} ~ C N^{-5/3} / (5/3)
    C = per_order[-1] * n_max ** (8.0 / 3.0)
    total += C * n_max ** (-5.0 / 3.0) / (5.0 / 3.0)
    # subtract modes j = 2..J
    s = 0.0
    for j in range(2, J + 1):
        nn, _ = noll_nm(j)
        s += per_mode[nn - 1]
    return total - s


def cholesky_lower(A0):
    """Lower-triangular L with L L^T = A_0 in Noll order (Sec. III-C, Eq. (9);
    the mixing matrix is obtained by Cholesky decomposition, Fig. 5)."""
    return np.linalg.cholesky(A0)


def mixing_groups(j_first=J_FIRST, j_last=J_LAST):
    """Noll modes grouped by (m, parity); A_0 and L are block-diagonal on
    these groups (m = 0 modes form one group)."""
    groups = {}
    for j in range(j_first, j_last + 1):
        n, m = noll_nm(j)
        key = (m, 0 if m == 0 else j % 2)
        groups.setdefault(key, []).append(j)
    return groups
