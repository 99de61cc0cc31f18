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
