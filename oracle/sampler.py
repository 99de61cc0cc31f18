"""DF-P2S Zernike-field sampler (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. III-C gives the method in two steps, which this module follows in order:

1. draw N independent unit-variance homogeneous fields, field i coloured by
   its autocovariance A_ii, by the circulant/FFT route of Sec. III-A
   (y = F^{-1}(S^{1/2} F(e)));
2. mix them per pixel with L, L L^T = A_0 (the Noll matrix), giving the
   approximate tensor A~ = L blockdiag(A_11..A_NN) L^T of Eq. (9).

Readings of the paper used here, where it leaves the choice open:
white noise is drawn directly in the frequency domain as Hermitian complex
Gaussian noise (same law as F(e)); two modes share one complex inverse FFT
(real and imaginary parts); the field is cropped from the top-left corner of
a zero-padded periodic grid; the L factor is the lower Cholesky factor in Noll
order; modes are Noll j = 2..36 by default, 2..J for n_modes = J - 1
(Sec. II-B keeps N = 36 and notes that N can be raised at some cost).
"""
import numpy as np

from . import philox
from .zernike import noll_matrix, cholesky_lower, N_MODES, J_FIRST
from .spectra import (all_spectra, discrete_correlation, subharmonic_amplitudes, SUBH_MODES,
                      SUBH_CELLS)

N_FIELDS = (N_MODES + 1) // 2      # 18 complex fields carry 35 real modes


def field_modes(q, n_modes=N_MODES):
    """Noll modes carried by complex field q: real part 2+2q, imaginary part
    3+2q (absent for the last field when n_modes is odd)."""
    a = J_FIRST + 2 * q
    b = a + 1
    return a, (b if b <= J_FIRST + n_modes - 1 else None)


def hermitian_noise(Gh, Gw, q, frame, seed, tag=philox.TAG_SAMPLER):
    """Two independent Hermitian white-noise spectra (Wa, Wb), E|W|^2 = 1.

    Bin k and its mirror -k share one Philox call at the canonical bin (the
    smaller linear index ky*Gw + kx); the canonical bin takes (g0 + i g1)/sqrt2
    and (g2 + i g3)/sqrt2, the mirror their conjugates; self-conjugate bins
    (k = -k) take the real values g0 and g2."""
    ky, kx = np.meshgrid(np.arange(Gh), np.arange(Gw), indexing='ij')
    lin = ky * Gw + kx
    lin_m = ((-ky) % Gh) * Gw + ((-kx) % Gw)
    canon = np.minimum(lin, lin_m)
    g0, g1, g2, g3 = philox.gaussians4(canon, q, frame, tag, seed)
    s = 1.0 / np.sqrt(2.0)
    Wa = (g0 + 1j * g1) * s
    Wb = (g2 + 1j * g3) * s
    mirror = lin > lin_m
    Wa = np.where(mirror, np.conj(Wa), Wa)
    Wb = np.where(mirror, np.conj(Wb), Wb)
    selfc = lin == lin_m
    Wa = np.where(selfc, g0 + 0j, Wa)
    Wb = np.where(selfc, g2 + 0j, Wb)
    return Wa, Wb


def subharmonic_waves(amps, H, W, Gh, Gw, frame, seed, rows=None):
    """Low-frequency part of the tilt fields (2, H, W) for one frame: for
    level p and half-plane cell (m, n), A cos(theta) + B sin(theta) per tilt
    mode, theta = 2 pi (m x / (Gw 3^p) + n y / (Gh 3^p)) at pixel (x, y).
    (A, B) of Noll 2 and of Noll 3 are the four Gaussians of the Philox call
    with counter (cell, p, frame, TAG_SUBHARMONIC), scaled by ``amps``.
    ``rows``: evaluate only these rows y (then the result has len(rows) rows)."""
    levels = amps.shape[1]
    ys = np.arange(H, dtype=np.float64) if rows is None else np.asarray(rows, dtype=np.float64)
    out = np.zeros((len(SUBH_MODES), len(ys), W))
    yy, xx = np.meshgrid(ys, np.arange(W, dtype=np.float64), indexing='ij')
    for p in range(1, levels + 1):
        for c, (m, n) in enumerate(SUBH_CELLS):
            g = philox.gaussians4(np.array([c]), p, frame, philox.TAG_SUBHARMONIC, seed)
            g = [float(v[0]) for v in g]
            theta = 2.0 * np.pi * (m * xx / (Gw * 3.0 ** p) + n * yy / (Gh * 3.0 ** p))
            ct, st = np.cos(theta), np.sin(theta)
            for t in range(len(SUBH_MODES)):
                a = amps[t, p - 1, c]
                out[t] += a * g[2 * t] * ct + a * g[2 * t + 1] * st
    return out


def unit_fields(spectra, H, W, frame, seed, subharmonics=None):
    """Step 1: the 35 independent unit-variance fields ybar[j-2] (H x W).

    ``spectra`` is the (35, Gh, Gw) stack of discrete spectra Sbar_j.
    U = sqrt(Sbar_a) Wa + i sqrt(Sbar_b) Wb; z = unitary inverse DFT of U;
    ybar_a = Re z, ybar_b = Im z, cropped to rows [0,H), columns [0,W).
    ``subharmonics``: the (2, levels, 4) amplitudes of
    ``subharmonic_amplitudes`` (spectra built with the same levels); their
    waves are added to the tilt fields."""
    n_modes, Gh, Gw = spectra.shape
    y = np.zeros((n_modes, H, W))
    for q in range((n_modes + 1) // 2):
        a, b = field_modes(q, n_modes)
        Wa, Wb = hermitian_noise(Gh, Gw, q, frame, seed)
        U = np.sqrt(spectra[a - J_FIRST]) * Wa
        if b is not None:
            U = U + 1j * np.sqrt(spectra[b - J_FIRST]) * Wb
        z = np.fft.ifft2(U) * np.sqrt(Gh * Gw)
        y[a - J_FIRST] = z.real[:H, :W]
        if b is not None:
            y[b - J_FIRST] = z.imag[:H, :W]
    if subharmonics is not None and subharmonics.shape[1] > 0:
        waves = subharmonic_waves(subharmonics, H, W, Gh, Gw, frame, seed)
        for t, j in enumerate(SUBH_MODES):
            y[j - J_FIRST] += waves[t]
    return y


def mix(y, L, d_over_r0):
    """Step 2: a_x = (D/r0)^{5/6} L ybar_x at every pixel (Sec. III-C)."""
    return float(d_over_r0) ** (5.0 / 6.0) * np.einsum('ij,jyx->iyx', L, y)


def sample_zernike(H, W, Gh, Gw, ds, d_over_r0, seed, frame, fold=2, spectra=None, L=None,
                   subharmonic_levels=0, n_modes=N_MODES):
    """Full oracle sampler for one frame: returns a (n_modes, H, W) float64
    array zern[j-2, y, x] (Noll 2..n_modes + 1).  ``subharmonic_levels`` > 0
    adds the tilt modes' subharmonic waves (``spectra``, if given, must be
    built with the same levels and modes)."""
    if spectra is None:
        spectra = all_spectra(Gh, Gw, ds, fold, j_last=J_FIRST + n_modes - 1,
                              subharmonic_levels=subharmonic_levels)
    if L is None:
        L = cholesky_lower(noll_matrix(1.0, j_last=J_FIRST + n_modes - 1))
    amps = (subharmonic_amplitudes(Gh, Gw, ds, fold, subharmonic_levels)
            if subharmonic_levels else None)
    y = unit_fields(spectra, H, W, frame, seed, subharmonics=amps)
    return mix(y, L, d_over_r0)


def sample_sequence_ar(H, W, Gh, Gw, ds, d_over_r0s, seed, frame0, alpha, y_prev=None, fold=2,
                       spectra=None, L=None, subharmonic_levels=0, n_modes=N_MODES):
    """Temporally correlated frames by an auto-regressive process (the
    workaround the paper gives for spatio-temporal correlation, Sec. III-E):
    the unit-variance fields follow ybar_t = alpha ybar_{t-1} +
    sqrt(1 - alpha^2) w_t, where w_t are frame (frame0 + t)'s own independent
    unit fields, and frame t is mixed with its own (D/r0)^{5/6} L.  Each field
    keeps its spatial correlation and unit variance, and fields of frames
    t and t + k correlate by alpha^k.  ``y_prev`` holds the unit fields of the
    frame before the first (None: the sequence starts from its first draw,
    which is already stationary).  With subharmonic levels, each frame's
    own draw w_t carries its subharmonic waves (``spectra``, if given, built
    with the same levels).  Returns (frames (F, 35, H, W), the last frame's
    unit fields)."""
    if spectra is None:
        spectra = all_spectra(Gh, Gw, ds, fold, j_last=J_FIRST + n_modes - 1,
                              subharmonic_levels=subharmonic_levels)
    if L is None:
        L = cholesky_lower(noll_matrix(1.0, j_last=J_FIRST + n_modes - 1))
    amps = (subharmonic_amplitudes(Gh, Gw, ds, fold, subharmonic_levels)
            if subharmonic_levels else None)
    c = np.sqrt(1.0 - alpha * alpha)
    y = y_prev
    out = []
    for t, dr in enumerate(d_over_r0s):
        w = unit_fields(spectra, H, W, frame0 + t, seed, subharmonics=amps)
        y = w if y is None else alpha * y + c * w
        out.append(mix(y, L, dr))
    return np.stack(out), y


# ----------------------------------------------------------------------------
# Exact covariance of the sampler (Eq. (9)) and the full tensor on tiny grids
# ----------------------------------------------------------------------------

def approx_tensor(spectra, L, d_over_r0, offsets):
    """A~_s = (D/r0)^{5/3} L diag(rho_bar_k[s]) L^T for each lattice offset s
    in ``offsets`` (list of (dy, dx)); Eq. (9) with correlation (unit-variance)
    diagonal blocks.  Returns (len(offsets), 35, 35)."""
    rho = np.stack([discrete_correlation(S) for S in spectra])
    Gh, Gw = spectra.shape[1:]
    out = []
    for dy, dx in offsets:
        r = rho[:, dy % Gh, dx % Gw]
        out.append(L @ np.diag(r) @ L.T)
    return np.array(out) * float(d_over_r0) ** (5.0 / 3.0)


def full_tensor_spectral(Gh, Gw, ds, fold=2, j_first=J_FIRST, j_last=J_FIRST + N_MODES - 1):
    """Cross-spectra of the full multi-aperture tensor A on a periodic lattice.

    S_ij[k] = sum_l f^{-11/3} Q_i(f) Q_j(f)^*  at f = f_k + l/ds, DC set to 0.
    The lattice cross-covariance is A_ij[d] = (D/r0)^{5/3} kappa IFFT(S_ij)[d];
    kappa is fixed per mode pair by A_ii[0] = A_0[i,i] (geometric mean for
    i != j), i.e. the s = 0 slice reproduces the Noll variances.
    Returns the complex array (nm, nm, Gh, Gw) of IFFT(S_ij) after scaling."""
    from .zernike import zernike_ft
    from .spectra import signed_index
    js = list(range(j_first, j_last + 1))
    kx = signed_index(Gw) / (Gw * ds)
    ky = signed_index(Gh) / (Gh * ds)
    FX, FY = np.meshgrid(kx, ky)
    nm = len(js)
    S = np.zeros((nm, nm, Gh, Gw), dtype=np.complex128)
    for lx in range(-fold, fold + 1):
        for ly in range(-fold, fold + 1):
            fx = FX + lx / ds
            fy = FY + ly / ds
            fr = np.hypot(fx, fy)
            ph = np.arctan2(fy, fx)
            w = np.where(fr > 0, np.where(fr > 0, fr, 1.0) ** (-11.0 / 3.0), 0.0)
            Q = np.stack([zernike_ft(j, fr, ph) for j in js])
            S += w[None, None] * Q[:, None] * np.conj(Q[None, :])
    S[:, :, 0, 0] = 0.0
    C = np.fft.ifft2(S, axes=(2, 3))
    A0 = noll_matrix(1.0, j_first, j_last)
    diag0 = np.real(np.array([C[i, i, 0, 0] for i in range(nm)]))
    scale = np.sqrt(np.diag(A0) / diag0)
    C = C * scale[:, None, None, None] * scale[None, :, None, None]
    return C


def full_tensor_matrix(C, ph, pw, d_over_r0):
    """Dense covariance over a ph x pw pixel patch: index (mode i, y, x).

    [A]_{(i,x),(j,x')} = E[a_{x,i} a_{x',j}] = Re C_ij[x' - x] (Eq. (6)); with
    the forward-kernel Q_j, C_ij[d] = IFFT(S_ij)[d] is E[a_i(x) a_j(x + d)]."""
    nm = C.shape[0]
    Gh, Gw = C.shape[2:]
    ys, xs = np.meshgrid(np.arange(ph), np.arange(pw), indexing='ij')
    ys = ys.ravel()
    xs = xs.ravel()
    dy = (ys[None, :] - ys[:, None]) % Gh
    dx = (xs[None, :] - xs[:, None]) % Gw
    p = ph * pw
    A = np.zeros((nm * p, nm * p))
    for i in range(nm):
        for j in range(nm):
            A[i * p:(i + 1) * p, j * p:(j + 1) * p] = np.real(C[i, j][dy, dx])
    return A * float(d_over_r0) ** (5.0 / 3.0)


def approx_matrix(spectra, L, ph, pw, d_over_r0):
    """Dense A~ over a ph x pw patch, same (mode, y, x) indexing as
    ``full_tensor_matrix``: [A~]_{(i,x),(j,x')} = sum_k L_ik L_jk rho_k[x-x']."""
    rho = np.stack([discrete_correlation(S) for S in spectra])
    Gh, Gw = spectra.shape[1:]
    ys, xs = np.meshgrid(np.arange(ph), np.arange(pw), indexing='ij')
    ys = ys.ravel()
    xs = xs.ravel()
    dy = (ys[:, None] - ys[None, :]) % Gh
    dx = (xs[:, None] - xs[None, :]) % Gw
    nm = L.shape[0]
    p = ph * pw
    R = rho[:, dy, dx]                                # (nm, p, p)
    A = np.einsum('ik,jk,kab->iajb', L, L, R).reshape(nm * p, nm * p)
    return A * float(d_over_r0) ** (5.0 / 3.0)


def cholesky_sample(A, n_samples, seed, tag=philox.TAG_BASIS + 10):
    """Draw y = chol(A) e with e ~ N(0, I) (Sec. III-A, small-grid route)."""
    Lf = np.linalg.cholesky(A + 1e-12 * np.trace(A) / A.shape[0] * np.eye(A.shape[0]))
    e = philox.gaussian_vectors(n_samples, A.shape[0], 0, tag, seed)
    return e @ Lf.T


def energy_functions(C, spectra, L, ds, s_max, n_bins, i0=2):
    """E(s), E~(s), E^(-)(s) of Eqs. (10)-(12) on the lattice.

    The integral over displacements up to radius s becomes a sum over lattice
    offsets with |d| ds <= s, weighted by the cell area ds^2.  Modes below
    index ``i0`` of the 35-vector (Noll 2 and 3, the tilts) are excluded, as
    the paper excludes piston and tilts from its plot.  Returns
    (s_edges, E, E_tilde, E_minus)."""
    nm = C.shape[0]
    Gh, Gw = C.shape[2:]
    rho = np.stack([discrete_correlation(S) for S in spectra])
    R = int(np.ceil(s_max / ds))
    s_edges = np.linspace(0.0, s_max, n_bins + 1)
    e = np.zeros(n_bins + 1)
    et = np.zeros(n_bins + 1)
    em = np.zeros(n_bins + 1)
    sel = slice(i0, nm)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            s = np.hypot(dy, dx) * ds
            if s > s_max:
                continue
            A = np.real(C[:, :, dy % Gh, dx % Gw])[sel, sel]
            At = (L @ np.diag(rho[:, dy % Gh, dx % Gw]) @ L.T)[sel, sel]
            fa = np.sum(A * A)
            ft = np.sum(At * At)
            mask = s_edges >= s
            e[mask] += fa * ds * ds
            et[mask] += ft * ds * ds
            em[mask] += abs(fa - ft) * ds * ds
    return s_edges, e, et, em
