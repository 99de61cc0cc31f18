"""Homogeneous per-mode spectra (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. III-C step 1 draws, for every mode i, a unit-variance field whose
autocovariance is the diagonal slice A_ii of the tensor of Eq. (6); Sec. III-B
notes each such slice is a function of the displacement s = (x - x')/D only,
so it has a spectrum and FFT colouring (Sec. III-A) applies.  The paper defers
the form of A_ii to the multi-aperture model it cites; the reading used here
is one collapsed Kolmogorov screen seen by apertures displaced by s*D, which
makes the spectrum of mode j

    S_j(f) = f^{-11/3} |Q_j(f)|^2,   f in cycles per D,

with |Q_j|^2 = (n+1) [2 J_{n+1}(pi f)/(pi f)]^2 Theta_j(phi_f) and
Theta_j = 2cos^2(m phi), 2sin^2(m phi) or 1.  Its constant (and D/r0) drop
out after normalising to unit variance.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy import special

from .zernike import noll_nm, noll_kind, J_FIRST, J_LAST


def kolmogorov_c():
    """Constant c of the phase spectrum Phi(f) = c r0^{-5/3} f^{-11/3} (f in
    cycles per metre) for which the structure function is Eq. (4)'s
    6.88 (r/r0)^{5/3}; 6.88 is 2 [(24/5) Gamma(6/5)]^{5/6} rounded.

    D(r) = 2 \\int Phi(f) (1 - cos 2 pi f.r) d^2 f; the integral
    \\int_0^inf u^{-8/3}(1 - J0(u)) du has a closed form that gives
    c = Gamma(11/6)^2 / (2 pi^{11/3}) [(24/5) Gamma(6/5)]^{5/6}.
    Tests check D(r) by quadrature against Eq. (4)."""
    bracket = (24.0 / 5.0) * special.gamma(6.0 / 5.0)
    return special.gamma(11.0 / 6.0) ** 2 / (2.0 * np.pi ** (11.0 / 3.0)) * bracket ** (5.0 / 6.0)


def kolmogorov_structure_constant():
    """The Eq. (4) constant before rounding: 2 [(24/5) Gamma(6/5)]^{5/6}."""
    return 2.0 * ((24.0 / 5.0) * special.gamma(6.0 / 5.0)) ** (5.0 / 6.0)


def mode_spectrum(j, fx, fy):
    """Continuous S_j(f) at frequencies (fx, fy) in cycles per D; 0 at f = 0."""
    n, m = noll_nm(j)
    fx = np.asarray(fx, dtype=np.float64)
    fy = np.asarray(fy, dtype=np.float64)
    fr = np.hypot(fx, fy)
    phi = np.arctan2(fy, fx)
    x = np.pi * fr
    safe = np.where(fr > 0, fr, 1.0)
    xs = np.pi * safe
    radial = (n + 1) * (2.0 * special.jv(n + 1, xs) / xs) ** 2
    kind = noll_kind(j)
    if kind == '0':
        ang = 1.0
    elif kind == 'c':
        ang = 2.0 * np.cos(m * phi) ** 2
    else:
        ang = 2.0 * np.sin(m * phi) ** 2
    out = safe ** (-11.0 / 3.0) * radial * ang
    return np.where(fr > 0, out, 0.0)


def signed_index(G):
    """Signed FFT bin index k' for k = 0..G-1 (k' = k - G for k >= G/2)."""
    k = np.arange(G)
    return np.where(k < G // 2, k, k - G)


def discrete_spectrum(j, Gh, Gw, ds, fold=2):
    """Folded, DC-free, unit-mean discrete spectrum Sbar_j on a Gh x Gw grid.

    Bin k sits at f_k = (k'_x/(Gw ds), k'_y/(Gh ds)) cycles per D, where ds is
    the pixel pitch in units of D (s = (x - x')/D, Sec. III-B footnote).  The
    lattice spectrum folds the aliases f_k + l/ds for |l_x|, |l_y| <= fold;
    the DC bin is set to 0; the table is scaled to mean 1 so every field has
    unit variance (Sec. III-C step 1) and the s = 0 covariance is exactly A_0.
    Layout [ky][kx] (row = y)."""
    kx = signed_index(Gw) / (Gw * ds)
    ky = signed_index(Gh) / (Gh * ds)
    FX, FY = np.meshgrid(kx, ky)
    S = np.zeros((Gh, Gw))
    for lx in range(-fold, fold + 1):
        for ly in range(-fold, fold + 1):
            S += mode_spectrum(j, FX + lx / ds, FY + ly / ds)
    S[0, 0] = 0.0
    S *= (Gh * Gw) / S.sum()
    return S


def discrete_correlation(Sbar):
    """rho_bar = Re IFFT(Sbar): the exact lattice autocorrelation of a field
    coloured by Sbar (Sec. III-A circulant sampling); rho_bar[0,0] = 1."""
    return np.real(np.fft.ifft2(Sbar))


# Subharmonic compensation of the low frequencies (the remedy the paper
# names for the low-frequency deficit of FFT screens, Sec. IV-B), for the two
# tilt modes only.  Level p = 1..levels refines the grid's central frequency
# cell 3^p times per axis: its 3 x 3 cells of size (dfx, dfy) / 3^p, the
# centre excluded (it is the next level's), sit at (m dfx, n dfy) / 3^p with
# dfx = 1/(Gw ds), dfy = 1/(Gh ds).  The four half-plane cells below stand
# for the eight (the spectrum is even in each axis).
SUBH_MODES = (2, 3)
SUBH_CELLS = ((1, 0), (1, 1), (0, 1), (-1, 1))
SUBH_MAX_LEVELS = 4


def folded_spectrum(j, fx, fy, ds, fold):
    """S_j summed over the lattice aliases f + l/ds, |l_x|, |l_y| <= fold (the
    same fold as the grid bins)."""
    out = 0.0
    for lx in range(-fold, fold + 1):
        for ly in range(-fold, fold + 1):
            out = out + mode_spectrum(j, fx + lx / ds, fy + ly / ds)
    return out


def subharmonic_cell_spectra(j, Gh, Gw, ds, fold, levels):
    """(levels, 4) array: folded S_j at the half-plane cells of each level."""
    out = np.zeros((levels, len(SUBH_CELLS)))
    for p in range(1, levels + 1):
        for c, (m, n) in enumerate(SUBH_CELLS):
            fx = m / (Gw * ds * 3.0 ** p)
            fy = n / (Gh * ds * 3.0 ** p)
            out[p - 1, c] = folded_spectrum(j, fx, fy, ds, fold)
    return out


def subharmonic_weight(j, Gh, Gw, ds, fold, levels):
    """The cells' share of the normalising sum, in grid-bin units: a level-p
    cell has 1/9^p of a bin's area, and each half-plane cell stands for two
    cells (f and -f)."""
    cs = subharmonic_cell_spectra(j, Gh, Gw, ds, fold, levels)
    w = 9.0 ** -np.arange(1, levels + 1)
    return float(2.0 * (cs.sum(axis=1) * w).sum())


def subharmonic_amplitudes(Gh, Gw, ds, fold, levels):
    """(2, levels, 4) amplitudes for the tilt modes: a level-p half-plane cell
    adds A cos(theta) + B sin(theta) to the unit field, A, B ~ N(0, amp^2),
    theta = 2 pi (m x / (Gw 3^p) + n y / (Gh 3^p)) at pixel (x, y).  amp^2 =
    2 C_j S_j(f) / (Gh Gw 9^p): the power of cells f and -f under the same
    normalisation C_j as the grid bins (``all_spectra`` with these levels),
    so the field keeps unit variance."""
    amps = np.zeros((len(SUBH_MODES), levels, len(SUBH_CELLS)))
    if levels == 0:
        return amps
    kx = signed_index(Gw) / (Gw * ds)
    ky = signed_index(Gh) / (Gh * ds)
    FX, FY = np.meshgrid(kx, ky)
    for t, j in enumerate(SUBH_MODES):
        grid = folded_spectrum(j, FX, FY, ds, fold)
        grid[0, 0] = 0.0
        total = grid.sum() + subharmonic_weight(j, Gh, Gw, ds, fold, levels)
        cj = Gh * Gw / total
        cs = subharmonic_cell_spectra(j, Gh, Gw, ds, fold, levels)
        w = 9.0 ** -np.arange(1, levels + 1)
        amps[t] = np.sqrt(2.0 * cj * cs * w[:, None] / (Gh * Gw))
    return amps


def all_spectra(Gh, Gw, ds, fold=2, j_first=J_FIRST, j_last=J_LAST, subharmonic_levels=0):
    """Stack of ``discrete_spectrum`` for modes j_first..j_last.  Same sums as
    calling it per mode; the radial factor (one Bessel order per radial order
    n) is evaluated once per alias and shared by the modes of that order.
    With subharmonic levels, the tilt modes' normalising sum also counts the
    subharmonic cells (their unit variance is then shared with them)."""
    js = list(range(j_first, j_last + 1))
    kx = signed_index(Gw) / (Gw * ds)
    ky = signed_index(Gh) / (Gh * ds)
    FX, FY = np.meshgrid(kx, ky)
    orders = sorted({noll_nm(j)[0] for j in js})

    def alias_term(l):
        lx, ly = l
        fx = FX + lx / ds
        fy = FY + ly / ds
        fr = np.hypot(fx, fy)
        phi = np.arctan2(fy, fx)
        safe = np.where(fr > 0, fr, 1.0)
        xs = np.pi * safe
        base = np.where(fr > 0, safe ** (-11.0 / 3.0), 0.0)
        rad = {n: (n + 1) * (2.0 * special.jv(n + 1, xs) / xs) ** 2 * base for n in orders}
        part = np.zeros((len(js), Gh, Gw))
        for t, j in enumerate(js):
            n, m = noll_nm(j)
            kind = noll_kind(j)
            if kind == '0':
                part[t] = rad[n]
            elif kind == 'c':
                part[t] = rad[n] * 2.0 * np.cos(m * phi) ** 2
            else:
                part[t] = rad[n] * 2.0 * np.sin(m * phi) ** 2
        return part

    aliases = [(lx, ly) for lx in range(-fold, fold + 1) for ly in range(-fold, fold + 1)]
    workers = min(len(aliases), os.cpu_count() or 1, 16)
    S = np.zeros((len(js), Gh, Gw))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for part in ex.map(alias_term, aliases):   # summed in alias order
            S += part
    S[:, 0, 0] = 0.0
    total = S.sum(axis=(1, 2))
    if subharmonic_levels:
        for t, j in enumerate(js):
            if j in SUBH_MODES:
                total[t] += subharmonic_weight(j, Gh, Gw, ds, fold, subharmonic_levels)
    S *= (Gh * Gw) / total[:, None, None]
    return S


def model_correlation(j, Gh, Gw, ds, fold, levels, dx, dy):
    """Covariance of the unit field of mode j at a lag of (dx, dy) pixels, as
    the sampler draws it: the grid bins' exact lattice correlation plus the
    subharmonic waves' amp^2 cos(2 pi f . lag)."""
    S = all_spectra(Gh, Gw, ds, fold, j, j, subharmonic_levels=levels)[0]
    rho = discrete_correlation(S)[dy % Gh, dx % Gw]
    if levels and j in SUBH_MODES:
        amps = subharmonic_amplitudes(Gh, Gw, ds, fold, levels)[SUBH_MODES.index(j)]
        for p in range(1, levels + 1):
            for c, (m, n) in enumerate(SUBH_CELLS):
                rho += amps[p - 1, c] ** 2 * np.cos(2.0 * np.pi * (m * dx / (Gw * 3.0 ** p) +
                                                                   n * dy / (Gh * 3.0 ** p)))
    return rho


def continuous_correlation(j, sx, sy, fmax=200.0, n_r=20000):
    """Unit-normalised continuous autocorrelation rho_j(s) of mode j at
    displacement (sx, sy) in units of D, by Hankel-transform quadrature of
    S_j (independent of the FFT route).  Uses 2cos^2(m phi) = 1 + cos(2 m phi)
    and the Jacobi-Anger integral over the angle."""
    n, m = noll_nm(j)
    kind = noll_kind(j)
    # radial grid, geometric near 0 (integrable singularity f^{-5/3} for n=1)
    f = np.concatenate([np.geomspace(1e-7, 1e-2, 4000, endpoint=False),
                        np.linspace(1e-2, fmax, n_r)])
    x = np.pi * f
    Sr = f ** (-11.0 / 3.0) * (n + 1) * (2.0 * special.jv(n + 1, x) / x) ** 2
    s = np.hypot(sx, sy)
    psi = np.arctan2(sy, sx)
    z = 2.0 * np.pi * f * s
    if kind == '0':
        ang = special.jv(0, z)
    else:
        sgn = 1.0 if kind == 'c' else -1.0
        ang = special.jv(0, z) + sgn * ((-1) ** m) * special.jv(2 * m, z) * np.cos(2 * m * psi)
    num = np.trapezoid(f * Sr * ang, f)
    den = np.trapezoid(f * Sr, f)
    return num / den
