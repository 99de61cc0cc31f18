"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/tsim.h declares, validates arguments, and its host plan builder
(FP64 Noll matrix, Cholesky factor, folded lattice spectra) agrees with the
independent oracle.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import spectra as ospec
from oracle import zernike as ozern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def t():
    import paper_2210_06713_amd as t
    return t


def test_library_exports_every_declared_symbol(t):
    hdr = open(os.path.join(ROOT, "include", "tsim.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(tsim_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    lib = ctypes.CDLL(t.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared <= set(t.EXPORTED)


def test_status_strings(t):
    for code in (0, -1, -2, -3, -4, -5):
        assert t._lib_status(code)
    assert t._lib_status(-99) == b"unknown status"


@pytest.mark.parametrize("field,value", [
    ("H", 0), ("Gh", 96), ("Gw", 32), ("n_modes", 36), ("psf_t", 32), ("psf_t", 1),
    ("basis_k", 0), ("basis_k", 200), ("alias_fold", 7), ("C", 0), ("precision", 5),
    ("subharmonic_levels", -1), ("subharmonic_levels", 5)])
def test_invalid_parameters_rejected(t, field, value):
    p = t.make_params(64, 64, 1, 128, 128)
    setattr(p, field, value)
    with pytest.raises(t.TsimError) as e:
        t.host_tables(p, 0)
    assert e.value.status == t.EINVAL


@pytest.mark.parametrize("P,T,C,K,precision", [
    (64, 17, 1, 100, 0),     # no exact-PSF kernel for this support
    (128, 31, 1, 100, 0),
    (64, 9, 1, 100, 1),      # BF16 blur: T in {15, 21, 33, 65} only
    (128, 65, 4, 120, 1),    # BF16 blur: image tile + basis staging exceed the LDS
])
def test_unbuilt_kernel_shapes_rejected_at_plan_creation(t, P, T, C, K, precision):
    """A plan whose exact-PSF or BF16-blur shape has no kernel is refused
    when it is made, not when a later call would launch it."""
    p = t.make_params(64, 64, C, 128, 128, pupil_n=P, psf_t=T, basis_k=K, precision=precision)
    with pytest.raises(t.TsimError) as e:
        t.host_tables(p, 0)
    assert e.value.status == t.EUNSUPPORTED


@pytest.mark.parametrize("P,T,C,K,precision", [
    (128, 65, 4, 120, 0),    # FP32: the vector-ALU blur takes any shape
    (128, 65, 4, 112, 1),
    (64, 15, 4, 128, 1),
    (64, 9, 2, 10, 0),
])
def test_built_kernel_shapes_accepted(t, P, T, C, K, precision):
    p = t.make_params(64, 64, C, 128, 128, pupil_n=P, psf_t=T, basis_k=K, precision=precision)
    assert t.host_tables(p, 3) == 0.125


def test_last_error_names_the_failing_call(t):
    t.last_error()                                  # clear
    p = t.make_params(64, 64, 1, 128, 128)
    p.C = 0
    with pytest.raises(t.TsimError):
        t.host_tables(p, 0)
    st, msg = t.last_error()
    assert st == t.EINVAL and msg == "tsim_host_tables: invalid argument"
    assert t.last_error() == (0, "")                # reading clears it
    p.C = 1
    t.host_tables(p, 3)                             # a successful call leaves it clear
    assert t.last_error() == (0, "")


def test_grid_smaller_than_image_rejected(t):
    p = t.make_params(200, 64, 1, 128, 128)
    with pytest.raises(t.TsimError):
        t.host_tables(p, 0)


def test_pitch_from_optics(t):
    p = t.make_params(64, 64, 1, 128, 128, pixel_pitch_over_d=0.0, aperture_d_m=0.1,
                      wavelength_m=0.5e-6, path_length_m=5000.0)
    assert abs(t.host_tables(p, 3) - 0.125) < 1e-15
    p = t.make_params(64, 64, 1, 128, 128, pixel_pitch_over_d=0.0)
    with pytest.raises(t.TsimError):
        t.host_tables(p, 0)


def test_noll_and_cholesky_match_oracle(t):
    p = t.make_params(64, 64, 1, 128, 128)
    A0 = t.host_tables(p, 0)
    L = t.host_tables(p, 1)
    ref = ozern.noll_matrix(1.0)
    np.testing.assert_allclose(A0, ref, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(L, ozern.cholesky_lower(ref), rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("Gh,Gw,ds,fold", [(128, 128, 0.125, 2), (64, 256, 0.25, 1), (256, 128, 0.125, 3)])
def test_spectra_match_oracle(t, Gh, Gw, ds, fold):
    p = t.make_params(32, 32, 1, Gh, Gw, pixel_pitch_over_d=ds, alias_fold=fold)
    sq = t.host_tables(p, 2)                 # [35][Gw/2+1][Gh/2+1]
    for j in [2, 3, 4, 7, 12, 20, 36]:
        S = ospec.discrete_spectrum(j, Gh, Gw, ds, fold)   # [ky][kx]
        quarter = np.sqrt(S[:Gh // 2 + 1, :Gw // 2 + 1]).T  # [kx][ky]
        np.testing.assert_allclose(sq[j - 2], quarter, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("Gh,Gw,ds,fold,levels", [(128, 128, 0.125, 2, 3), (64, 256, 0.25, 1, 4),
                                                 (256, 128, 0.125, 2, 1)])
def test_subharmonic_tables_match_oracle(t, Gh, Gw, ds, fold, levels):
    """With subharmonic levels the tilt spectra share their normalisation with
    the subharmonic cells, and table 4 holds the wave amplitudes."""
    p = t.make_params(32, 32, 1, Gh, Gw, pixel_pitch_over_d=ds, alias_fold=fold,
                      subharmonic_levels=levels)
    sq = t.host_tables(p, 2)
    S = ospec.all_spectra(Gh, Gw, ds, fold, subharmonic_levels=levels)
    for j in [2, 3, 4, 8, 36]:
        quarter = np.sqrt(S[j - 2, :Gh // 2 + 1, :Gw // 2 + 1]).T
        np.testing.assert_allclose(sq[j - 2], quarter, rtol=1e-11, atol=1e-14)
    amp = t.host_tables(p, 4)                # [2][4][4]
    ref = ospec.subharmonic_amplitudes(Gh, Gw, ds, fold, levels)
    np.testing.assert_allclose(amp[:, :levels], ref, rtol=1e-11, atol=1e-15)
    assert not amp[:, levels:].any()
    # levels 0: the table is all zero and the spectra are the plain ones
    p0 = t.make_params(32, 32, 1, Gh, Gw, pixel_pitch_over_d=ds, alias_fold=fold)
    assert not t.host_tables(p0, 4).any()


# ---- more than 35 modes (Sec. II-B: N can be raised at some cost) ----

@pytest.mark.parametrize("n_modes", [44, 54, 65])
def test_noll_cholesky_and_spectra_match_oracle_more_modes(t, n_modes):
    """Plans of 44, 54 and 65 modes (complete radial orders up to 8, 9, 10):
    A_0, L and the folded spectra of every mode equal the oracle's."""
    jl = n_modes + 1
    p = t.make_params(32, 32, 1, 64, 128, pixel_pitch_over_d=0.125, n_modes=n_modes)
    A0 = t.host_tables(p, 0)
    assert A0.shape == (n_modes, n_modes)
    ref = ozern.noll_matrix(1.0, j_last=jl)
    np.testing.assert_allclose(A0, ref, rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(t.host_tables(p, 1), ozern.cholesky_lower(ref), rtol=1e-10, atol=1e-14)
    sq = t.host_tables(p, 2)
    S = ospec.all_spectra(64, 128, 0.125, 2, j_last=jl)
    for j in range(2, jl + 1):
        quarter = np.sqrt(S[j - 2, :33, :65]).T
        np.testing.assert_allclose(sq[j - 2], quarter, rtol=1e-11, atol=1e-14, err_msg=f"j={j}")


@pytest.mark.parametrize("n_modes,kw,status", [
    (36, {}, "EINVAL"), (50, {}, "EINVAL"), (66, {}, "EINVAL"),
    (65, dict(psf_t=31), "EUNSUPPORTED"),            # exact PSFs with more modes: T = 33 (P = 64)
    (44, dict(p2s_mode=1, basis_k=100), "EUNSUPPORTED"),   # the network takes 35 inputs
])
def test_mode_counts_checked_at_plan_creation(t, n_modes, kw, status):
    p = t.make_params(32, 32, 1, 64, 64, n_modes=n_modes, **kw)
    with pytest.raises(t.TsimError) as e:
        t.host_tables(p, 0)
    assert e.value.status == getattr(t, status)


def test_mode_counts_accepted(t):
    for n in (35, 44, 54, 65):
        for P, T in ((64, 33), (128, 65), (128, 33)):
            p = t.make_params(32, 32, 1, 64, 64, n_modes=n, pupil_n=P, psf_t=T)
            assert t.host_tables(p, 3) == 0.125
