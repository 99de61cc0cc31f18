"""Spatial tilt statistics of Sec. IV-B (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper validates the generated fields by the tilt correlation
E[alpha(0) alpha(theta)] and the differential tilt variance (DTV)
E[(alpha(0) - alpha(theta))^2], the latter also written as
2 (E[alpha^2(0)] - E[alpha(0) alpha(theta)]).  Here both are estimated from
coefficient planes for the two tilt modes (Noll 2 and 3) at pixel lags
d = 0..max_lag along x and along y, averaging over all frames and over every
pixel pair inside the frame (no wrap-around): H (W - d) pairs per frame for
an x lag, (H - d) W for a y lag.
"""
import numpy as np

TILT_MODES = (2, 3)


def tilt_statistics(zern, max_lag):
    """zern: (F, 35, H, W) coefficient planes, mode j at index j - 2.
    Returns (corr, dtv), each (2 modes, 2 axes, max_lag + 1) float64: the mean
    product and the mean squared difference of the pairs at each lag; axis 0
    is the x (column) lag, axis 1 the y (row) lag."""
    z = np.asarray(zern, dtype=np.float64)
    F, _, H, W = z.shape
    corr = np.zeros((2, 2, max_lag + 1))
    dtv = np.zeros((2, 2, max_lag + 1))
    for m, j in enumerate(TILT_MODES):
        a = z[:, j - 2]
        for d in range(max_lag + 1):
            u, v = a[:, :, :W - d], a[:, :, d:]
            corr[m, 0, d] = np.mean(u * v)
            dtv[m, 0, d] = np.mean((u - v) ** 2)
            u, v = a[:, :H - d, :], a[:, d:, :]
            corr[m, 1, d] = np.mean(u * v)
            dtv[m, 1, d] = np.mean((u - v) ** 2)
    return corr, dtv


# Aperture statistics of Sec. IV-B: the phase structure function, whose
# Kolmogorov form is Eq. (4), D(r) = 6.88 (r / r0)^{5/3}.
SF_PUPIL = 64          # pupil grid of the structure function: aperture 32 samples across


def structure_function(zern, P=SF_PUPIL):
    """Direct estimate from coefficient planes (F, 35, H, W): at every pixel
    the phase phi = sum_{j=2}^{36} a_j Z_j on the P x P pupil grid of
    ``psf.pupil_grid`` (aperture diameter P/2 samples), then the mean of
    (phi(p) - phi(p + r x))^2 over the pupil-point pairs with both points
    inside the aperture, for r = 0..P/2 - 2 samples (r / D = 2 r / P; the
    points strictly inside the aperture span P/2 - 2 samples), and the mean
    over pixels and frames.  Returns D[r], float64."""
    from .psf import pupil_grid
    from .zernike import zernike
    rho, theta, mask = pupil_grid(P)
    Z = np.stack([np.where(mask, zernike(j, rho, theta), 0.0) for j in range(2, 37)])  # [35][P][P]
    a = np.asarray(zern, dtype=np.float64)
    a = a.transpose(0, 2, 3, 1).reshape(-1, 35)                    # [pixels][35]
    out = np.zeros(P // 2 - 1)
    for r in range(1, P // 2 - 1):
        pairs = mask[:, :P - r] & mask[:, r:]
        dZ = (Z[:, :, :P - r] - Z[:, :, r:])[:, pairs]             # [35][pairs]
        dphi = a @ dZ                                              # [pixels][pairs]
        out[r] = np.mean(dphi ** 2)
    return out


# The optical transfer functions of Sec. IV-B.  One realisation's OTF is the
# autocorrelation of the generalised pupil G = P(xi) exp(-j phi(xi)):
# H(xi) = sum_x G(x) conj(G(x - xi)); the long-exposure (LE) OTF is its
# expectation over realisations, the short-exposure (SE) OTF the same with
# the tilt-corrected phase phi - alpha^T xi, alpha the plane of best fit.
# Readings: the realisations are the per-pixel coefficient vectors (every
# pixel of every frame is one aperture's phase); the plane of best fit over
# the aperture is the Zernike tilt, so the SE phase omits Noll 2 and 3; the
# pupil grid is that of the PSFs (P x P, aperture P/2 samples, points
# strictly inside), and H is normalised by H(0) = the number of aperture
# samples, so H(0) = 1.  Lags xi run over the P x P grid with xi = 0 at
# index (P/2, P/2); the aperture autocorrelation vanishes at |xi| >= P/2, so
# the circular lags of the grid hold it without wrap-around.


def _otf_pupil(P, tilt_removed, n_modes=35):
    from .psf import pupil_grid
    from .zernike import zernike
    rho, theta, mask = pupil_grid(P)
    first = 4 if tilt_removed else 2
    Z = np.stack([np.where(mask, zernike(j, rho, theta), 0.0) if j >= first else np.zeros((P, P))
                  for j in range(2, n_modes + 2)])                 # [N][P][P]
    return Z, mask


def otf_mean(zvecs, P, tilt_removed=False):
    """Sample mean of the OTF over coefficient vectors ``zvecs`` (n, N),
    Noll 2..N+1.  Each realisation's autocorrelation is taken with the
    autocorrelation theorem, H = IFFT2(|FFT2(G)|^2) on the P x P grid.
    Returns a complex (P, P) array, zero lag at (P/2, P/2)."""
    A = np.asarray(zvecs, dtype=np.float64)
    A = A.reshape(-1, A.shape[-1])
    Z, mask = _otf_pupil(P, tilt_removed, A.shape[1])
    acc = np.zeros((P, P))
    for a in A:
        G = np.where(mask, np.exp(-1j * np.tensordot(a, Z, axes=1)), 0.0)
        acc += np.abs(np.fft.fft2(G)) ** 2
    H = np.fft.ifft2(acc / len(A))
    return np.fft.fftshift(H) / mask.sum()


def otf_direct(a, P, tilt_removed=False):
    """One realisation's OTF by the definition, sum over aperture points x of
    G(x) conj(G(x - xi)), for small grids (brute force)."""
    a = np.asarray(a, dtype=np.float64)
    Z, mask = _otf_pupil(P, tilt_removed, a.size)
    phi = np.tensordot(a, Z, axes=1)
    G = np.where(mask, np.exp(-1j * phi), 0.0)
    H = np.zeros((P, P), dtype=complex)
    c = P // 2
    for dy in range(-c, c):
        for dx in range(-c, c):
            s = 0j
            for y in range(P):
                for x in range(P):
                    yy, xx = y - dy, x - dx
                    if 0 <= yy < P and 0 <= xx < P:
                        s += G[y, x] * np.conj(G[yy, xx])
            H[dy + c, dx + c] = s
    return H / mask.sum()


def otf_gaussian(C, P, tilt_removed=False):
    """Expectation of the OTF for Gaussian coefficients a ~ N(0, C) (C the
    N x N covariance, Noll 2..N+1): E[exp(-j (phi(x) - phi(x - xi)))] =
    exp(-D(x, x - xi) / 2) with D the phase structure function of the pair,
    (Z(x) - Z(x'))^T C (Z(x) - Z(x')).  Real, (P, P), zero lag at (P/2, P/2)."""
    Z, mask = _otf_pupil(P, tilt_removed, C.shape[0])
    pts = np.argwhere(mask)
    Zp = Z[:, mask]                                                # [35][n_ap], same order as pts
    index = -np.ones((P, P), dtype=np.int64)
    index[mask] = np.arange(len(pts))
    H = np.zeros((P, P))
    c = P // 2
    for dy in range(-c, c):
        for dx in range(-c, c):
            ys, xs = pts[:, 0] - dy, pts[:, 1] - dx
            ok = (ys >= 0) & (ys < P) & (xs >= 0) & (xs < P)
            j = np.where(ok, index[np.clip(ys, 0, P - 1), np.clip(xs, 0, P - 1)], -1)
            ok &= j >= 0
            if not ok.any():
                continue
            dZ = Zp[:, ok] - Zp[:, j[ok]]
            D = np.einsum('ip,ij,jp->p', dZ, C, dZ)
            H[dy + c, dx + c] = np.exp(-0.5 * D).sum()
    return H / mask.sum()
