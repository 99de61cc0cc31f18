"""Pins of the oracle's spatial tilt statistics (Sec. IV-B): closed forms on
ramps and constants, and the sampler's own fields against the exact model
covariance by Monte Carlo (which also fixes which axis is which)."""
import numpy as np

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
