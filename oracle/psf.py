"""Exact PSFs, the PCA PSF basis and exact projection (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. (2): h_x = |Fourier{P(xi) exp(-j phi_x(xi))}|^2 up to constants, with
phi_x expanded on Zernike modes (Eq. (5)).  Eq. (7): h_x = sum_m beta_{x,m}
varphi_m with a basis obtained by PCA over a database of PSFs (Sec. II-C).

Readings where the paper leaves the choice open: the pupil is sampled on a P x P grid
whose aperture spans P/2 samples (Nyquist-sampled PSF, so one PSF sample is
one image pixel); the aperture is centred on sample P/2 and contains the
samples strictly inside the unit circle; the forward DFT is used; the PSF is
fftshift-ed so frequency 0 sits at index P/2, cropped to T x T around it and
normalised to unit sum.  Tilt modes (Noll 2, 3) are left out of the PSF by
default because the renderer applies them as a warp.
"""
import numpy as np

from . import philox
from .zernike import zernike, noll_matrix, cholesky_lower, J_FIRST


def pupil_grid(P):
    """(rho, theta, mask) on the P x P pupil grid; x = column, y = row."""
    idx = np.arange(P, dtype=np.float64)
    rad = P / 4.0                                  # aperture diameter P/2
    X, Y = np.meshgrid((idx - P / 2) / rad, (idx - P / 2) / rad)
    rho = np.hypot(X, Y)
    theta = np.arctan2(Y, X)
    mask = rho < 1.0
    return rho, theta, mask


def zernike_stack(P, modes):
    rho, theta, mask = pupil_grid(P)
    return np.stack([zernike(j, rho, theta) for j in modes]), mask


def phase(a, P, modes=range(4, 37), zstack=None):
    """phi(xi) = sum_j a_j Z_j(xi) on the pupil grid (Eq. (5)); ``a`` is the
    vector of Noll 2.. coefficients (35 of them for Noll 2..36)."""
    modes = list(modes)
    if zstack is None:
        zstack, _ = zernike_stack(P, modes)
    coeffs = np.array([a[j - J_FIRST] for j in modes])
    return np.tensordot(coeffs, zstack, axes=1)


def psf_full(a, P, modes=range(4, 37), zstack=None):
    """Un-cropped, un-normalised |FFT2(P exp(-i phi))|^2, fftshift-ed so the
    zero frequency is at index (P/2, P/2) (Eq. (2))."""
    rho, theta, mask = pupil_grid(P)
    phi = phase(a, P, modes, zstack)
    field = np.where(mask, np.exp(-1j * phi), 0.0)
    h = np.abs(np.fft.fft2(field)) ** 2
    return np.fft.fftshift(h)


def crop(h_full, T):
    P = h_full.shape[0]
    r = (T - 1) // 2
    c = P // 2
    return h_full[c - r:c + r + 1, c - r:c + r + 1]


def psf_exact(a, P, T, modes=range(4, 37), zstack=None):
    """T x T unit-sum PSF of one Zernike vector (Eq. (2) with the crop and
    normalisation readings)."""
    h = crop(psf_full(a, P, modes, zstack), T)
    return h / h.sum()


def psf_batch(A, P, T, modes=range(4, 37)):
    """PSFs for a batch of Zernike vectors, shape (n, T, T)."""
    modes = list(modes)
    zstack, _ = zernike_stack(P, modes)
    return np.stack([psf_exact(a, P, T, modes, zstack) for a in A])


def basis_draws(n, seed, dr_lo=0.5, dr_hi=5.0, tag=philox.TAG_BASIS, n_modes=35):
    """Zernike vectors for the PSF database: a = (D/r0)^{5/6} L g with
    g ~ N(0, I_N) from Philox counters (i, w, 0, tag), w = 0..ceil(N/4) - 1
    (0..8 for N = 35), and D/r0 = lo + (hi - lo) u with u from word 0 of call
    (i, ceil(N/4), 0, tag); tag 1 for the basis database, tag 2 for network
    training pairs."""
    L = cholesky_lower(noll_matrix(1.0, j_last=J_FIRST + n_modes - 1))
    g = philox.gaussian_vectors(n, n_modes, 0, tag, seed)
    u = philox.uniforms_extra(n, (n_modes + 3) // 4, 0, tag, seed)
    dr = dr_lo + (dr_hi - dr_lo) * u
    return (g @ L.T) * (dr ** (5.0 / 6.0))[:, None], dr


def pca_basis(psfs, K):
    """Uncentred PCA (Eq. (7) has no mean term): the top-K right singular
    vectors of the (n, T*T) PSF matrix.  Signs: each vector has a
    non-negative sum; a vector with |sum| < 1e-9 gets its largest-magnitude
    entry positive.  Returns (Psi (K, T*T), singular values)."""
    X = psfs.reshape(psfs.shape[0], -1)
    _, s, Vt = np.linalg.svd(X, full_matrices=False)
    Psi = Vt[:K].copy()
    for m in range(K):
        tot = Psi[m].sum()
        if abs(tot) < 1e-9:
            if Psi[m][np.argmax(np.abs(Psi[m]))] < 0:
                Psi[m] = -Psi[m]
        elif tot < 0:
            Psi[m] = -Psi[m]
    return Psi, s


def project(psfs, Psi):
    """beta_x = Psi h_x (exact projection onto the orthonormal basis)."""
    X = psfs.reshape(psfs.shape[0], -1)
    return X @ Psi.T


def psf_field(zern, P, T, Psi, modes=None):
    """Plain-form P2S for a whole field: zern (N, H, W) -> beta (H, W, K);
    the PSF takes modes 4..N+1 unless ``modes`` says otherwise."""
    n, H, W = zern.shape
    if modes is None:
        modes = range(4, n + 2)
    A = zern.reshape(n, -1).T
    h = psf_batch(A, P, T, modes)
    return project(h, Psi).reshape(H, W, -1)
