"""Pins for the oracle's exact PSFs (Eq. (2)), PCA basis and projection
(Eq. (7)), basis blur (Eq. (8)), gather blur (Eq. (1)) and tilt warp.

Pins: closed-form special cases (Airy symmetry, exact integer tilt shift,
on-axis defocus intensity), library routines that compute the same thing by
another route (scipy.ndimage.convolve and shift), and invariants
(orthonormality, linearity).
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import psf, render, zernike

P, T = 64, 33


def test_airy_pattern_symmetry():
    """a = 0 gives the diffraction-limited pattern of a centred circular
    aperture: invariant under 90-degree rotation and both flips, unit sum."""
    a = np.zeros(35)
    h = psf.psf_exact(a, P, T)
    np.testing.assert_allclose(h, np.rot90(h), atol=1e-15)
    np.testing.assert_allclose(h, h[::-1, :], atol=1e-15)
    np.testing.assert_allclose(h, h[:, ::-1], atol=1e-15)
    assert abs(h.sum() - 1) < 1e-14 and h.min() >= 0
    assert np.unravel_index(np.argmax(h), h.shape) == (T // 2, T // 2)


@pytest.mark.parametrize("k", [1, 2, -3])
def test_integer_tilt_is_exact_circular_shift(k):
    """Eq. (2) with exp(-j phi) and a forward DFT: Z_2 = 2x with x = (i - P/2)
    / (P/4) gives phi = a_2 (i - P/2)/8, a linear phase of 4 a_2/pi bins, so
    a_2 = k pi/4 moves the PSF by exactly -k samples along x (columns); Z_3
    does the same along y (rows)."""
    a = np.zeros(35)
    h0 = psf.psf_full(a, P, modes=range(2, 37))
    a2 = a.copy()
    a2[0] = k * np.pi / 4
    h2 = psf.psf_full(a2, P, modes=range(2, 37))
    np.testing.assert_allclose(h2, np.roll(h0, -k, axis=1), atol=1e-9 * h0.max())
    a3 = a.copy()
    a3[1] = k * np.pi / 4
    h3 = psf.psf_full(a3, P, modes=range(2, 37))
    np.testing.assert_allclose(h3, np.roll(h0, -k, axis=0), atol=1e-9 * h0.max())


@pytest.mark.parametrize("a4", [0.3, 0.8, 1.5])
def test_defocus_on_axis_intensity(a4):
    """On-axis intensity of pure defocus relative to a = 0:
    |int_0^1 exp(-i sqrt3 a4 (2 rho^2 - 1)) 2 rho drho|^2 = sinc^2(sqrt3 a4)
    (closed form).  The sampled pupil approximates the disc with an error
    that falls like 1/P (boundary samples), so the closed form is asserted on a
    fine pupil and the error must shrink as the pupil is refined."""
    x = math.sqrt(3) * a4
    want = (math.sin(x) / x) ** 2
    errs = []
    for Pp in (64, 256):
        a = np.zeros(35)
        a[2] = a4
        h = psf.psf_full(a, Pp)
        h0 = psf.psf_full(np.zeros(35), Pp)
        errs.append(abs(h[Pp // 2, Pp // 2] / h0[Pp // 2, Pp // 2] - want))
    assert errs[1] < 1.5e-3
    assert errs[0] < 1.2e-2
    assert errs[1] < errs[0] / 3


def test_marechal_small_aberration():
    """Strehl ~ exp(-sigma^2) for a small random aberration (Marechal), with
    sigma^2 the variance of the sampled phase over the pupil; the neglected
    terms are O(sigma^4)."""
    rng = np.random.default_rng(4)
    a = np.zeros(35)
    a[2:] = rng.standard_normal(33) * 0.03
    _, _, mask = psf.pupil_grid(P)
    sigma2 = np.var(psf.phase(a, P)[mask])
    assert abs(sigma2 - np.sum(a[2:] ** 2)) < 0.1 * np.sum(a[2:] ** 2)
    h = psf.psf_full(a, P)
    h0 = psf.psf_full(np.zeros(35), P)
    S = h[P // 2, P // 2] / h0[P // 2, P // 2]
    assert abs(S - math.exp(-sigma2)) < sigma2 ** 2


def test_pupil_sampling():
    rho, th, mask = psf.pupil_grid(P)
    n = int(mask.sum())
    assert abs(n - math.pi * (P / 4) ** 2) < 0.02 * math.pi * (P / 4) ** 2
    ys, xs = np.nonzero(mask)
    # support fits a 31 x 31 window centred on sample P/2
    assert xs.min() == P // 2 - 15 and xs.max() == P // 2 + 15
    assert ys.min() == P // 2 - 15 and ys.max() == P // 2 + 15


def test_pca_basis_orthonormal_and_projection():
    A, dr = psf.basis_draws(300, seed=11)
    assert np.all(dr >= 0.5) and np.all(dr <= 5.0)
    H = psf.psf_batch(A, P, T)
    Psi, s = psf.pca_basis(H, 40)
    np.testing.assert_allclose(Psi @ Psi.T, np.eye(40), atol=1e-12)
    assert np.all(np.diff(s) <= 1e-12)
    assert np.all(Psi.sum(1) >= 0)
    # beta(psi_m) = e_m
    np.testing.assert_allclose(psf.project(Psi.reshape(40, T, T), Psi), np.eye(40), atol=1e-12)
    # the basis captures most PSF energy
    b = psf.project(H, Psi)
    rec = b @ Psi
    err = np.linalg.norm(rec - H.reshape(300, -1), axis=1) / np.linalg.norm(H.reshape(300, -1), axis=1)
    assert np.median(err) < 0.1


def test_basis_draws_have_noll_covariance():
    A, dr = psf.basis_draws(20000, seed=3)
    cov = (A / (dr ** (5 / 6))[:, None]).T @ (A / (dr ** (5 / 6))[:, None]) / A.shape[0]
    A0 = zernike.noll_matrix(1.0)
    scale = np.sqrt(np.outer(np.diag(A0), np.diag(A0)))
    assert np.max(np.abs(cov - A0) / scale) < 5 / math.sqrt(20000) * 2


# ---------------------------------------------------------------- render ---
def _basis(K=12, Tt=9, seed=0):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((Tt * Tt, K))
    Q, _ = np.linalg.qr(M)
    return Q.T.copy()


def test_constant_beta_equals_library_convolution():
    """With beta constant over the image, Eq. (8) is one spatially invariant
    convolution; scipy.ndimage.convolve(mode='nearest') computes it."""
    Tt, K = 9, 12
    Psi = _basis(K, Tt)
    rng = np.random.default_rng(1)
    img = rng.random((20, 23))
    b = rng.standard_normal(K)
    beta = np.broadcast_to(b, (20, 23, K))
    out = render.render_basis(img, beta, Psi, Tt)
    kern = (b @ Psi).reshape(Tt, Tt)
    ref = ndimage.convolve(img, kern, mode='nearest')
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_basis_blur_equals_gather_blur():
    """Linearity: sum_m beta_m (psi_m conv I) = (sum_m beta_m psi_m) conv I at
    each pixel (Eq. (8) = Eq. (1) with the projected PSF)."""
    Tt, K = 7, 10
    Psi = _basis(K, Tt, 2)
    rng = np.random.default_rng(2)
    img = rng.random((15, 11))
    beta = rng.standard_normal((15, 11, K))
    out = render.render_basis(img, beta, Psi, Tt)
    psfs = (beta @ Psi).reshape(15, 11, Tt, Tt)
    ref = render.render_gather(img, psfs, Tt)
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_delta_image_reproduces_psf():
    """A true convolution of a delta at p gives B(p + u) = h(u)."""
    Tt, K = 7, 5
    Psi = _basis(K, Tt, 3)
    img = np.zeros((21, 21))
    img[10, 10] = 1.0
    b = np.arange(1, K + 1, dtype=float)
    beta = np.broadcast_to(b, (21, 21, K))
    out = render.render_basis(img, beta, Psi, Tt)
    h = (b @ Psi).reshape(Tt, Tt)
    np.testing.assert_allclose(out[7:14, 7:14], h, atol=1e-12)


def test_warp_identity_integer_and_subpixel():
    rng = np.random.default_rng(5)
    img = rng.random((17, 19))
    z = np.zeros((17, 19))
    np.testing.assert_array_equal(render.warp(img, z, z), img)
    # integer shift with clamping: O(x) = B(clamp(x - t))
    out = render.warp(img, z + 2, z - 3)
    ys, xs = np.meshgrid(np.arange(17), np.arange(19), indexing='ij')
    np.testing.assert_allclose(out, img[np.clip(ys + 3, 0, 16), np.clip(xs - 2, 0, 18)], atol=1e-15)
    # constant sub-pixel shift equals scipy's order-1 spline shift
    for tx, ty in [(0.3, -0.7), (-1.25, 2.5)]:
        out = render.warp(img, z + tx, z + ty)
        ref = ndimage.shift(img, (ty, tx), order=1, mode='nearest')
        np.testing.assert_allclose(out, ref, atol=1e-12)


def test_warp_sign_matches_psf_tilt():
    """The warp displacement for a_2 equals the shift that the same a_2 gives
    the Eq. (2) PSF: a PSF kept with its tilt and a tilt-free PSF followed by
    the warp move the image the same way."""
    k = 2
    a2 = k * np.pi / 4
    tx, ty = render.tilt_shift(np.array([[[a2]], [[0.0]]]))
    assert abs(tx[0, 0] - (-k)) < 1e-12 and ty[0, 0] == 0
    a = np.zeros(35)
    a[0] = a2
    h = psf.crop(psf.psf_full(a, P, modes=range(2, 37)), T)
    peak = np.unravel_index(np.argmax(h), h.shape)
    assert peak == (T // 2, T // 2 - k)


def test_render_at_constant_beta_and_delta():
    """Eq. (8) at listed pixels: with beta constant it is one spatially
    invariant convolution (scipy.ndimage.convolve, nearest), clamped borders
    included; a delta image at p returns B(p + u) = h(u)."""
    Tt, K = 9, 12
    Psi = _basis(K, Tt, 7)
    rng = np.random.default_rng(8)
    img = rng.random((20, 23))
    b = rng.standard_normal(K)
    ys, xs = np.meshgrid(np.arange(20), np.arange(23), indexing='ij')
    ys, xs = ys.ravel(), xs.ravel()
    got = render.render_at(img, np.broadcast_to(b, (len(ys), K)), Psi, Tt, ys, xs)
    ref = ndimage.convolve(img, (b @ Psi).reshape(Tt, Tt), mode='nearest')
    np.testing.assert_allclose(got, ref.ravel(), atol=1e-12)
    d = np.zeros((21, 21))
    d[10, 10] = 1.0
    py, px = np.meshgrid(np.arange(6, 15), np.arange(6, 15), indexing='ij')
    got = render.render_at(d, np.broadcast_to(b, (81, K)), Psi, Tt, py.ravel(), px.ravel())
    np.testing.assert_allclose(got.reshape(9, 9), (b @ Psi).reshape(Tt, Tt), atol=1e-12)


def test_render_at_per_pixel_weights_match_gather():
    """With per-pixel weights, each listed pixel equals the gather form
    Eq. (1) with the projected PSF sum_m beta_m psi_m (linearity)."""
    Tt, K = 7, 10
    Psi = _basis(K, Tt, 9)
    rng = np.random.default_rng(10)
    img = rng.random((15, 11))
    beta = rng.standard_normal((15, 11, K))
    ref = render.render_gather(img, (beta @ Psi).reshape(15, 11, Tt, Tt), Tt)
    ys = np.array([0, 0, 14, 14, 7, 3])
    xs = np.array([0, 10, 0, 10, 5, 9])
    got = render.render_at(img, beta[ys, xs], Psi, Tt, ys, xs)
    np.testing.assert_allclose(got, ref[ys, xs], atol=1e-12)


def test_warp_at_matches_library_shift():
    """The bilinear warp at listed pixels against scipy.ndimage.shift
    (order 1, nearest) for a constant displacement, borders included."""
    rng = np.random.default_rng(11)
    img = rng.random((17, 19))
    ys, xs = np.meshgrid(np.arange(17), np.arange(19), indexing='ij')
    for tx, ty in [(0.3, -0.7), (-1.25, 2.5), (3.0, -2.0)]:
        got = render.warp_at(img, np.full(ys.size, tx), np.full(ys.size, ty), ys.ravel(), xs.ravel())
        ref = ndimage.shift(img, (ty, tx), order=1, mode='nearest')
        np.testing.assert_allclose(got, ref.ravel(), atol=1e-12)
