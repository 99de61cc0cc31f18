"""Pins of the oracle's subharmonic compensation of the tilt fields (the
low-frequency remedy named in Sec. IV-B), each against something other than
the oracle's own formulas:

* the cells' weights against a 2-D quadrature of the folded spectrum over
  the frequency region they stand for;
* the model covariance of the tilt fields against the continuous correlation
  (an independent Hankel-transform quadrature), at lags up to half the grid;
* unit variance with the subharmonic cells in the normalisation;
* the drawn waves' covariance against the analytic one, by Monte Carlo.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import philox
from oracle import sampler as osamp
from oracle import spectra as ospec

GH = GW = 128
DS = 0.125
FOLD = 2


def _quadrature_central_region(j, levels):
    """Integral of the folded S_j over the central bin minus the central
    cell of the last level (the region the levels' cells stand for)."""
    dfx, dfy = 1.0 / (GW * DS), 1.0 / (GH * DS)

    def square(a, b):
        v, _ = integrate.dblquad(lambda y, x: ospec.folded_spectrum(j, x, y, DS, FOLD), 0, a, 0, b,
                                 epsabs=1e-10, epsrel=1e-8)
        return 4.0 * v
    r = 3.0 ** levels
    return square(dfx / 2, dfy / 2) - square(dfx / 2 / r, dfy / 2 / r)


@pytest.mark.parametrize("j,levels", [(2, 1), (3, 3)])
def test_cell_weights_match_quadrature(j, levels):
    """Level-p cells weigh S at their centres by 1/9^p of a bin's area; over
    the region they cover this midpoint rule must come within 15% of the
    exact integral (a dropped mirror factor gives 45%, 3^p instead of 9^p
    several times too much)."""
    dfx, dfy = 1.0 / (GW * DS), 1.0 / (GH * DS)
    w = ospec.subharmonic_weight(j, GH, GW, DS, FOLD, levels) * dfx * dfy
    exact = _quadrature_central_region(j, levels)
    assert 0.85 < w / exact < 1.0


def test_unit_variance_and_other_modes_unchanged():
    for levels in (1, 2, 3, 4):
        for j in (2, 3):
            assert abs(ospec.model_correlation(j, GH, GW, DS, FOLD, levels, 0, 0) - 1.0) < 1e-12
    S0 = ospec.all_spectra(GH, GW, DS, FOLD, j_first=4, j_last=9)
    S3 = ospec.all_spectra(GH, GW, DS, FOLD, j_first=4, j_last=9, subharmonic_levels=3)
    np.testing.assert_array_equal(S0, S3)
    assert ospec.subharmonic_amplitudes(GH, GW, DS, FOLD, 0).size == 0


@pytest.mark.parametrize("j,axis", [(2, 0), (3, 1), (2, 1)])
def test_long_lag_correlation_approaches_continuous(j, axis):
    """On a 16 D grid the FFT field misses the tilt's low frequencies, so its
    correlation at lags of 1-4 D falls well below the continuous one.  Each
    added level must bring it closer, and three levels must remove more than
    half of the error."""
    lags = (8, 16, 32)
    cont = [ospec.continuous_correlation(j, d * DS * (axis == 0), d * DS * (axis == 1)) for d in lags]
    errs = []
    for levels in range(4):
        model = [ospec.model_correlation(j, GH, GW, DS, FOLD, levels, d * (axis == 0), d * (axis == 1))
                 for d in lags]
        errs.append(np.abs(np.array(model) - np.array(cont)))
    for a, b in zip(errs, errs[1:]):
        assert (b < a).all()
    assert (errs[3] < 0.5 * errs[0]).all()


def test_wave_draws_match_their_covariance():
    """Monte Carlo over frames of the drawn waves alone: variance and lag
    covariance of both tilt modes against sum amp^2 cos(2 pi f . lag)."""
    Gh = Gw = 64
    levels = 2
    amps = ospec.subharmonic_amplitudes(Gh, Gw, DS, FOLD, levels)
    n = 3000
    lag = 40
    vals = np.zeros((n, 2, 2))   # frame, mode, pixel (x = 0 and x = lag on row 0; y lag for mode 3)
    for f in range(n):
        w = osamp.subharmonic_waves(amps, lag + 1, lag + 1, Gh, Gw, f, 11)
        vals[f, 0] = w[0, 0, 0], w[0, 0, lag]
        vals[f, 1] = w[1, 0, 0], w[1, lag, 0]
    for t, (dx, dy) in enumerate([(lag, 0), (0, lag)]):
        var = (amps[t] ** 2).sum()
        cov = sum(amps[t, p - 1, c] ** 2 * np.cos(2 * np.pi * (m * dx / (Gw * 3.0 ** p) + n_ * dy / (Gh * 3.0 ** p)))
                  for p in range(1, levels + 1) for c, (m, n_) in enumerate(ospec.SUBH_CELLS))
        v = vals[:, t]
        assert abs(np.mean(v[:, 0] ** 2) - var) < 4 * var * np.sqrt(2.0 / n)
        assert abs(np.mean(v[:, 0] * v[:, 1]) - cov) < 4 * var * np.sqrt(2.0 / n)


def test_sampler_levels_zero_is_the_plain_sampler():
    z0 = osamp.sample_zernike(8, 12, 64, 64, DS, 2.0, 5, 1)
    z = osamp.sample_zernike(8, 12, 64, 64, DS, 2.0, 5, 1, subharmonic_levels=0)
    np.testing.assert_array_equal(z0, z)
    # the waves use their own Philox tag
    assert philox.TAG_SUBHARMONIC not in (philox.TAG_SAMPLER, philox.TAG_BASIS, philox.TAG_MLP_DATA,
                                          philox.TAG_MLP_INIT, philox.TAG_IMAGE)


def test_stored_4096_amplitudes_match_oracle_cells():
    """The stored 4096^2 amplitudes (tests/golden, written from the oracle)
    against the oracle's cell spectra: squared-amplitude ratios do not
    depend on the normalising sum, so they are checked in full, and the
    first cell of each mode sets the scale for the rest."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "subharmonic_amplitudes_G4096.txt")
    amps = np.loadtxt(path).reshape(2, 3, 4)
    for t, j in enumerate(ospec.SUBH_MODES):
        cs = ospec.subharmonic_cell_spectra(j, 4096, 4096, DS, FOLD, 3)
        w = 9.0 ** -np.arange(1, 4)
        model = cs * w[:, None]
        ref = amps[t, 0, 0] ** 2 / model[0, 0] if j == 2 else amps[t, 0, 2] ** 2 / model[0, 2]
        np.testing.assert_allclose(amps[t] ** 2, ref * model, rtol=1e-10)
