"""Pins of the oracle's spatial tilt statistics (Sec. IV-B): closed forms on
ramps and constants, and the sampler's own fields against the exact model
covariance by Monte Carlo (which also fixes which axis is which)."""
import numpy as np
import pytest

from oracle import sampler as osamp
from oracle import spectra as ospec
from oracle import stats as ostats
from oracle import zernike as ozern


def _planes(F, H, W):
    return np.zeros((F, 35, H, W))


def test_ramp_closed_forms():
    F, H, W, L = 2, 9, 13, 6
    z = _planes(F, H, W)
    x = np.arange(W, dtype=np.float64)
    y = np.arange(H, dtype=np.float64)
    z[:, 0] = x[None, None, :]          # Noll 2 = column index
    z[:, 1] = y[None, :, None]          # Noll 3 = row index
    corr, dtv = ostats.tilt_statistics(z, L)
    for d in range(L + 1):
        n = W - d
        s1, s2 = n * (n - 1) / 2.0, (n - 1) * n * (2 * n - 1) / 6.0
        assert np.isclose(corr[0, 0, d], (s2 + d * s1) / n)          # mean x (x + d)
        assert np.isclose(dtv[0, 0, d], d * d)
        assert np.isclose(dtv[0, 1, d], 0.0)                         # rows are identical
        assert np.isclose(corr[0, 1, d], (W - 1) * (2 * W - 1) / 6.0)  # mean x^2
        assert np.isclose(dtv[1, 1, d], d * d)
        assert np.isclose(dtv[1, 0, d], 0.0)


def test_constant_field():
    z = _planes(3, 5, 7)
    z[:, 0] = 1.5
    z[:, 1] = -2.0
    corr, dtv = ostats.tilt_statistics(z, 4)
    assert np.allclose(corr[0], 2.25) and np.allclose(corr[1], 4.0)
    assert np.allclose(dtv, 0.0)


def test_sampler_fields_match_model_covariance():
    """200 frames of the oracle sampler at D/r0 = 1 (a_2 = L_00 ybar_2):
    the mean products equal A_0[2,2] rho(d) of the sampled field's exact
    covariance, and the DTV 2 A_0[2,2] (1 - rho(d)), within 15% of the
    variance (about 5 standard errors).  Along x and along y the x-tilt's
    correlation differs by far more than that (longitudinal vs transverse)."""
    H = W = 32
    G = 64
    S = ospec.all_spectra(G, G, 0.125, 2)
    L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    z = np.stack([osamp.sample_zernike(H, W, G, G, 0.125, 1.0, 3, f, spectra=S, L=L) for f in range(200)])
    corr, dtv = ostats.tilt_statistics(z, 8)
    A0 = ozern.noll_matrix(1.0)
    for m, j in enumerate((2, 3)):
        var = A0[j - 2, j - 2]
        for axis in (0, 1):
            for d in (0, 2, 4, 8):
                rho = ospec.model_correlation(j, G, G, 0.125, 2, 0, d * (axis == 0), d * (axis == 1))
                assert abs(corr[m, axis, d] - var * rho) < 0.15 * var, (j, axis, d)
                assert abs(dtv[m, axis, d] - 2 * var * (1 - rho)) < 0.3 * var, (j, axis, d)
    # longitudinal (x lag of the x-tilt) and transverse correlations differ
    assert corr[0, 1, 8] - corr[0, 0, 8] > 0.3 * A0[0, 0]


def test_structure_function_pure_tilt():
    """phi = c Z_2 = 2 c x (x in aperture radii): D(r) = 4 c^2 (r / R)^2 with
    R = P/4 samples, whichever pairs are inside."""
    z = _planes(1, 2, 3)
    z[:, 0] = 0.7
    D = ostats.structure_function(z)
    R = ostats.SF_PUPIL / 4.0
    r = np.arange(ostats.SF_PUPIL // 2 - 1)
    np.testing.assert_allclose(D, 4 * 0.49 * (r / R) ** 2, rtol=1e-12, atol=1e-15)


def test_structure_function_matches_kolmogorov():
    """Coefficient vectors drawn from N(0, A_0) at D/r0 = 1: the 35-mode phase
    follows Eq. (4)'s 6.88 (r/r0)^{5/3} within 8% for r >= D/4 (the modes
    above Noll 36 carry the missing power at small separations, where the
    truncated structure function must fall below Eq. (4))."""
    A0 = ozern.noll_matrix(1.0)
    Lc = ozern.cholesky_lower(A0)
    g = np.random.default_rng(5).standard_normal((35, 6000))
    z = (Lc @ g).T.reshape(6000, 1, 1, 35).transpose(0, 3, 1, 2)   # (F, 35, 1, 1)
    D = ostats.structure_function(z)
    P = ostats.SF_PUPIL
    for r in (8, 16, 24):
        kol = 6.88 * (2.0 * r / P) ** (5.0 / 3.0)
        assert abs(D[r] / kol - 1.0) < 0.08, (r, D[r], kol)
    assert D[2] < 0.85 * 6.88 * (4.0 / P) ** (5.0 / 3.0)


# ---- optical transfer functions (Sec. IV-B: LE and SE OTFs) ----

def _shift_overlap(mask, dy, dx):
    """Number of aperture samples x with x - (dy, dx) also in the aperture."""
    P = mask.shape[0]
    a = np.zeros((3 * P, 3 * P), bool)
    a[P:2 * P, P:2 * P] = mask
    b = np.zeros_like(a)
    b[P + dy:2 * P + dy, P + dx:2 * P + dx] = mask
    return int((a & b).sum())


@pytest.mark.parametrize("tilt_removed", [False, True])
def test_otf_fft_route_equals_definition(tilt_removed):
    """The autocorrelation theorem route of otf_mean equals the double sum of
    the definition, realisation by realisation (brute force, 16 x 16 grid)."""
    rng = np.random.default_rng(31)
    for _ in range(3):
        a = rng.normal(size=35) * 0.4
        H = ostats.otf_mean(a[None], 16, tilt_removed)
        Hd = ostats.otf_direct(a, 16, tilt_removed)
        assert np.abs(H - Hd).max() < 1e-12


def test_otf_diffraction_limited():
    """a = 0: the OTF is the aperture's overlap with its shifted copy over the
    aperture size (counted by integer shifts of the mask), real, 1 at zero
    lag, and close to the continuous disc's (2/pi)(acos u - u sqrt(1 - u^2)),
    u = |xi| / D."""
    from oracle.psf import pupil_grid
    P = 64
    H = ostats.otf_mean(np.zeros((1, 35)), P)
    _, _, mask = pupil_grid(P)
    n = mask.sum()
    c = P // 2
    assert abs(H[c, c] - 1) < 1e-12 and np.abs(H.imag).max() < 1e-12
    for dy, dx in [(0, 1), (3, -7), (-12, 5), (20, 20), (0, 31), (-31, 0), (16, -16)]:
        assert abs(H[c + dy, c + dx].real - _shift_overlap(mask, dy, dx) / n) < 1e-12
    yy, xx = np.mgrid[-c:c, -c:c]
    u = np.minimum(np.hypot(yy, xx) / (P / 2), 1.0)
    cont = 2 / np.pi * (np.arccos(u) - u * np.sqrt(1 - u * u))
    assert np.abs(H.real - cont).max() < 0.05


def test_otf_symmetry_and_tilt_removal():
    """H(-xi) = conj H(xi) for each realisation; a pure tilt is a linear
    phase (|H| is the diffraction OTF) that the short-exposure OTF removes
    exactly; the SE OTF of any vector is the LE OTF of the vector without
    its tilt coefficients."""
    P = 32
    rng = np.random.default_rng(5)
    a = rng.normal(size=35) * 0.5
    H = ostats.otf_mean(a[None], P)
    i = np.arange(P)
    Hm = H[np.ix_((P - i) % P, (P - i) % P)]
    assert np.abs(Hm - np.conj(H)).max() < 1e-12
    H0 = ostats.otf_mean(np.zeros((1, 35)), P)
    tilt = np.zeros(35)
    tilt[:2] = [0.9, -0.6]
    Ht = ostats.otf_mean(tilt[None], P)
    assert np.abs(np.abs(Ht) - H0.real).max() < 1e-12 and np.abs(Ht - H0).max() > 0.1
    assert np.abs(ostats.otf_mean(tilt[None], P, tilt_removed=True) - H0).max() < 1e-12
    b = a.copy()
    b[:2] = 0
    assert np.abs(ostats.otf_mean(a[None], P, True) - ostats.otf_mean(b[None], P)).max() < 1e-12


@pytest.mark.parametrize("tilt_removed", [False, True])
def test_otf_monte_carlo_matches_gaussian_expectation(tilt_removed):
    """For a ~ N(0, (D/r0)^{5/3} A_0) the sample mean of the OTF tends to
    exp(-D(x, x') / 2) averaged over the aperture pairs (Gaussian phase):
    2000 draws at D/r0 = 1.5 agree with otf_gaussian within 5 standard
    errors (batch means) plus 1e-3 at every lag."""
    P = 32
    dr = 1.5
    A0 = ozern.noll_matrix(1.0)
    L = ozern.cholesky_lower(A0)
    C = dr ** (5 / 3) * A0
    rng = np.random.default_rng(77)
    g = rng.standard_normal((2000, 35))
    a = dr ** (5 / 6) * g @ L.T
    means = np.stack([ostats.otf_mean(a[k::20], P, tilt_removed) for k in range(20)])
    m = means.mean(0)
    se_re = means.real.std(0, ddof=1) / np.sqrt(20)
    se_im = means.imag.std(0, ddof=1) / np.sqrt(20)
    ref = ostats.otf_gaussian(C, P, tilt_removed)
    assert abs(ref[P // 2, P // 2] - 1) < 1e-12
    assert np.all(np.abs(m.real - ref) <= 5 * se_re + 1e-3)
    assert np.all(np.abs(m.imag) <= 5 * se_im + 1e-3)
    # the mean OTF at mid lags lies clearly below the diffraction OTF
    H0 = ostats.otf_mean(np.zeros((1, 35)), P).real
    assert ref[P // 2, P // 2 + 8] < 0.9 * H0[P // 2, P // 2 + 8]
