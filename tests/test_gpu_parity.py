"""GPU parity: every hot-path call through the C ABI against the FP64 oracle
on the same seeded inputs.

Bar (FP32 paths): per coefficient plane, PSF, weight array and image, both
the relative L2 error ||gpu - oracle|| / ||oracle|| and the largest element
error max|gpu - oracle| / max|oracle| are <= 1e-5 (``parity.err``); the FP32
kernels accumulate a few dozen rounding steps (two FFT passes, a 33-term
phase sum, 1089-term projections), each ~6e-8 relative.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle import sampler as osamp  # noqa: E402
from oracle import spectra as ospec  # noqa: E402
from oracle import zernike as ozern  # noqa: E402
import synthetic  # noqa: E402
from parity import err  # noqa: E402

TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()




@pytest.fixture(scope="module")
def t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_06713_amd as t
    return t


@pytest.fixture(scope="module")
def basis33():
    A, _ = opsf.basis_draws(1500, seed=2024)
    H = opsf.psf_batch(A, 64, 33)
    Psi, _ = opsf.pca_basis(H, 100)
    return Psi


def _sample(t, plan, d_over_r0, seed, frame0, frames):
    dev = torch.device("cuda")
    zern = torch.empty((frames, 35, plan.H, plan.W), dtype=torch.float32, device=dev)
    ws = plan.workspace(frames)
    plan.sample_zernike(d_over_r0, seed, frame0, zern, ws)
    torch.cuda.synchronize()
    return zern


@pytest.mark.parametrize("H,W,Gh,Gw,seed,frame0,dr", [
    (64, 64, 128, 128, 0, 0, 2.0),             # 64 x 64 workload, G = 128
    (48, 80, 128, 256, 2 ** 40 + 77, 5, 3.3),  # ragged, non-square, 64-bit seed
    (64, 64, 64, 64, 11, 0, 1.0),              # grid equal to the image
    # row pass with the next field read ahead: samples per thread and row
    # Gw / 256 = 2, 4 and 8, for 1, 2 and 4 output columns per thread, odd
    # row counts (a last block with one row)
    (13, 200, 64, 512, 3, 1, 2.0),
    (9, 256, 64, 1024, 8, 0, 2.5),
    (7, 1000, 64, 1024, 7, 0, 2.5),
    (11, 130, 64, 2048, 4, 0, 1.5),
    (9, 400, 64, 2048, 5, 0, 2.5),
    (7, 1000, 64, 2048, 6, 0, 2.5),
    # degenerate frames: a single row, a single column
    (1, 64, 64, 64, 12, 0, 2.0),
    (64, 1, 64, 64, 13, 0, 2.0),
])
def test_sampler_matches_oracle(t, H, W, Gh, Gw, seed, frame0, dr):
    say(f"sampler H={H} W={W} G={Gh}x{Gw} seed={seed} frame0={frame0}")
    plan = t.Plan(H, W, 1, Gh, Gw, pixel_pitch_over_d=0.125)
    frames = 2
    zern = _sample(t, plan, [dr, 0.5 * dr], seed, frame0, frames).cpu().numpy()
    S = ospec.all_spectra(Gh, Gw, 0.125, 2)
    L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    for f in range(frames):
        ref = osamp.sample_zernike(H, W, Gh, Gw, 0.125, [dr, 0.5 * dr][f], seed, frame0 + f,
                                   spectra=S, L=L)
        errs = [err(zern[f, j], ref[j]) for j in range(35)]
        assert max(errs) < TOL, (f, int(np.argmax(errs)), max(errs))


@pytest.mark.parametrize("H,W,Gh,Gw,levels,seed,frame0", [
    (64, 64, 128, 128, 3, 5, 2),
    (48, 80, 128, 256, 4, 2 ** 40 + 77, 5),   # ragged, non-square, 64-bit seed
    (13, 200, 64, 512, 1, 3, 1),
    (7, 1000, 64, 1024, 2, 6, 0),
])
def test_sampler_subharmonics_match_oracle(t, H, W, Gh, Gw, levels, seed, frame0):
    """Subharmonic compensation of the tilt fields: every plane against the
    oracle, which adds the same Philox-drawn waves to its unit fields."""
    say(f"sampler subharmonics levels={levels} H={H} W={W} G={Gh}x{Gw}")
    plan = t.Plan(H, W, 1, Gh, Gw, pixel_pitch_over_d=0.125, subharmonic_levels=levels)
    drs = [2.0, 3.0]
    zern = _sample(t, plan, drs, seed, frame0, 2).cpu().numpy()
    S = ospec.all_spectra(Gh, Gw, 0.125, 2, subharmonic_levels=levels)
    L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    np.testing.assert_allclose(plan.table(4)[:, :levels],
                               ospec.subharmonic_amplitudes(Gh, Gw, 0.125, 2, levels), rtol=1e-11)
    for f in range(2):
        ref = osamp.sample_zernike(H, W, Gh, Gw, 0.125, drs[f], seed, frame0 + f, spectra=S, L=L,
                                   subharmonic_levels=levels)
        errs = [err(zern[f, j], ref[j]) for j in range(35)]
        assert max(errs) < TOL, (f, int(np.argmax(errs)), max(errs))


def test_sampler_ar_with_subharmonics_matches_oracle(t):
    """Auto-regressive sequence on a plan with two subharmonic levels: each
    frame's fresh draw carries its own waves, then the recursion."""
    say("sampler AR + subharmonics 40x56 G=128")
    H, W, G, levels = 40, 56, 128, 2
    plan = t.Plan(H, W, 1, G, G, pixel_pitch_over_d=0.125, subharmonic_levels=levels)
    drs = [1.0, 2.0, 3.5, 2.5]
    ref, _ = osamp.sample_sequence_ar(H, W, G, G, 0.125, drs, 13, 7, 0.8, subharmonic_levels=levels)
    zern = torch.empty((4, 35, H, W), dtype=torch.float32, device="cuda")
    plan.sample_zernike_ar(drs, 13, 7, 0.8, zern, plan.workspace(4))
    torch.cuda.synchronize()
    got = zern.cpu().numpy()
    for f in range(4):
        errs = [err(got[f, j], ref[f, j]) for j in range(35)]
        assert max(errs) < TOL, (f, int(np.argmax(errs)), max(errs))


@pytest.mark.slow
def test_sampler_full_size_frame(t):
    """512 x 512 frame on the 1024 x 1024 grid, the benchmark's launch shape."""
    say("sampler full size 512x512 G=1024")
    H = W = 512
    plan = t.Plan(H, W, 3, 1024, 1024, pixel_pitch_over_d=0.125)
    zern = _sample(t, plan, [2.0, 4.0], 0, 0, 2).cpu().numpy()
    ref = osamp.sample_zernike(H, W, 1024, 1024, 0.125, 4.0, 0, 1)
    errs = [err(zern[1, j], ref[j]) for j in range(35)]
    assert max(errs) < TOL, max(errs)


def test_plan_tables_match_oracle(t):
    plan = t.Plan(64, 64, 1, 128, 128)
    np.testing.assert_allclose(plan.table(0), ozern.noll_matrix(1.0), rtol=1e-12, atol=1e-16)


def test_psf_exact_matches_oracle(t):
    say("psf exact, 300 vectors, P=64 T=33")
    plan = t.Plan(64, 64, 1, 128, 128, psf_t=33)
    A, _ = opsf.basis_draws(300, seed=77)
    A[:5] *= 0.0                     # diffraction-limited
    A[5:10] *= 3.0                   # strong turbulence (D/r0 up to ~10)
    z = torch.tensor(A, dtype=torch.float32, device="cuda")
    out = torch.empty((300, 33 * 33), dtype=torch.float32, device="cuda")
    plan.psf_exact(z, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(300, 33, 33)
    ref = opsf.psf_batch(A.astype(np.float32).astype(np.float64), 64, 33)
    errs = [err(got[i], ref[i]) for i in range(300)]
    assert max(errs) < TOL, (int(np.argmax(errs)), max(errs))
    np.testing.assert_allclose(got.sum(axis=(1, 2)), 1.0, atol=1e-5)


@pytest.mark.parametrize("T", [15, 21])
def test_psf_exact_smaller_crops(t, T):
    plan = t.Plan(64, 64, 1, 128, 128, psf_t=T)
    A, _ = opsf.basis_draws(40, seed=5)
    z = torch.tensor(A, dtype=torch.float32, device="cuda")
    out = torch.empty((40, T * T), dtype=torch.float32, device="cuda")
    plan.psf_exact(z, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(40, T, T)
    ref = opsf.psf_batch(A.astype(np.float32).astype(np.float64), 64, T)
    assert max(err(got[i], ref[i]) for i in range(40)) < TOL


def test_p2s_exact_matches_oracle(t, basis33):
    say("p2s exact 64x64x2 frames K=100")
    H = W = 64
    plan = t.Plan(H, W, 1, 128, 128, basis=basis33, psf_t=33)
    # the oracle's own fields (D/r0 = 2 and 5) are the common input
    z32 = np.stack([osamp.sample_zernike(H, W, 128, 128, 0.125, dr, 3, f)
                    for f, dr in enumerate([2.0, 5.0])]).astype(np.float32)
    z = z32.astype(np.float64)
    beta = torch.empty((2, H, W, 100), dtype=torch.float32, device="cuda")
    plan.p2s(torch.tensor(z32, device="cuda"), beta, plan.workspace(2))
    torch.cuda.synchronize()
    got = beta.cpu().numpy()
    for f in range(2):
        ref = opsf.psf_field(z[f], 64, 33, basis33)
        assert err(got[f], ref) < TOL, f


# the FP32-accurate blur's kernel forms: K = 20, 60, 120 (2, 4 and 8
# matrix-core k-steps), C = 1, 2, 4, T = 33 (8-row tiles) and T = 65
# (16-row tiles), ragged images; the basis is any K x T^2 matrix with unit
# rows (Eq. (8) is linear in it)
@pytest.mark.parametrize("T,C,K,H,W", [(33, 1, 20, 19, 37), (33, 2, 60, 24, 33), (33, 4, 120, 17, 48),
                                       (65, 1, 120, 18, 21), (65, 2, 20, 33, 40), (65, 4, 60, 17, 35)])
def test_render_fp32_kernel_shapes(t, T, C, K, H, W):
    say(f"render fp32 T={T} C={C} K={K} {H}x{W}")
    rng = np.random.default_rng(T * 1000 + C * 100 + K)
    basis = rng.standard_normal((K, T * T))
    basis /= np.linalg.norm(basis, axis=1, keepdims=True)
    plan = t.Plan(H, W, C, 64, 64, basis=basis, psf_t=T, pupil_n=64 if T == 33 else 128)
    img = synthetic.test_image(C, H, W, 4, seed=T + C)[None]
    beta = (rng.standard_normal((1, H, W, K)) * 0.1).astype(np.float32)
    out = torch.full((1, C, H, W), float("nan"), dtype=torch.float32, device="cuda")
    plan.render(torch.tensor(img, device="cuda"), torch.tensor(beta, device="cuda"), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    for c in range(C):
        ref = orender.render_basis(img[0, c].astype(np.float64), beta[0].astype(np.float64), basis, T)
        assert err(got[c], ref) < TOL, c
    plan.close()


def test_render_matches_oracle(t, basis33):
    say("render fp32 C=3 40x72")
    H, W, C = 40, 72, 3
    plan = t.Plan(H, W, C, 128, 128, basis=basis33, psf_t=33)
    img = synthetic.test_image(C, H, W, 8, seed=1)[None]
    rng = np.random.default_rng(3)
    beta = (rng.standard_normal((1, H, W, 100)) * 0.05).astype(np.float32)
    beta[..., 0] += 1.0
    out = torch.empty((1, C, H, W), dtype=torch.float32, device="cuda")
    plan.render(torch.tensor(img, device="cuda"), torch.tensor(beta, device="cuda"), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    for c in range(C):
        ref = orender.render_basis(img[0, c].astype(np.float64), beta[0].astype(np.float64),
                                   basis33, 33)
        assert err(got[c], ref) < TOL, c


@pytest.mark.parametrize("F,H,W,C", [
    (1, 50, 70, 2),
    (2, 64, 300, 3),    # two frames, a ragged last 256-pixel row segment
])
def test_warp_matches_oracle(t, F, H, W, C):
    say(f"warp F={F} C={C} {H}x{W}")
    plan = t.Plan(H, W, C, 128, 512)
    img = np.stack([synthetic.test_image(C, H, W, 4, seed=2 + f) for f in range(F)])
    rng = np.random.default_rng(9)
    zern = np.zeros((F, 35, H, W), dtype=np.float32)
    zern[:, 0] = rng.standard_normal((F, H, W)) * 3.0
    zern[:, 1] = rng.standard_normal((F, H, W)) * 3.0
    out = torch.empty((F, C, H, W), dtype=torch.float32, device="cuda")
    plan.warp(torch.tensor(img, device="cuda"), torch.tensor(zern, device="cuda"), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for f in range(F):
        tx, ty = orender.tilt_shift(zern[f].astype(np.float64))
        for c in range(C):
            ref = orender.warp(img[f, c].astype(np.float64), tx, ty)
            assert err(got[f, c], ref) < TOL, (f, c)


def test_end_to_end_small_workload(t, basis33):
    """64 x 64 grayscale, D/r0 = 2, G = 128, seed 0: sample -> exact P2S ->
    render -> warp, against the oracle chain on the same inputs."""
    say("end-to-end 64x64")
    H = W = 64
    plan = t.Plan(H, W, 1, 128, 128, basis=basis33, psf_t=33)
    img = synthetic.test_image(1, H, W, 8, seed=0)[None]
    zern = _sample(t, plan, [2.0], 0, 0, 1)
    beta = torch.empty((1, H, W, 100), dtype=torch.float32, device="cuda")
    ws = plan.workspace(1)
    plan.p2s(zern, beta, ws)
    blur = torch.empty((1, 1, H, W), dtype=torch.float32, device="cuda")
    out = torch.empty_like(blur)
    plan.render(torch.tensor(img, device="cuda"), beta, blur)
    plan.warp(blur, zern, out)
    torch.cuda.synchronize()
    zr = osamp.sample_zernike(H, W, 128, 128, 0.125, 2.0, 0, 0)
    br = opsf.psf_field(zr, 64, 33, basis33)
    ref = orender.render_frame(img[0].astype(np.float64), zr, br, basis33, 33)
    assert err(zern.cpu().numpy()[0], zr) < TOL
    assert err(out.cpu().numpy()[0], ref) < TOL


def test_argument_errors(t, basis33):
    plan = t.Plan(32, 32, 1, 64, 64, basis=basis33, psf_t=33)
    x = torch.zeros((1, 1, 32, 32), dtype=torch.float32, device="cuda")
    z = torch.zeros((1, 35, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(t.TsimError) as e:
        plan.warp(x, z, x)              # in place
    assert e.value.status == t.EINVAL
    with pytest.raises(t.TsimError):
        plan.sample_zernike([float("nan")], 0, 0, z, plan.workspace(1))
    with pytest.raises(t.TsimError):
        plan.sample_zernike([-1.0], 0, 0, z, plan.workspace(1))
    big = torch.zeros(1024 + 64, dtype=torch.float32, device="cuda")
    mis = big[1:1 + 32 * 32].view(1, 1, 32, 32)   # 4-byte offset: misaligned
    with pytest.raises(t.TsimError):
        plan.warp(mis, z, x)
    nobasis = t.Plan(32, 32, 1, 64, 64)
    with pytest.raises(t.TsimError) as e:
        nobasis.render(x, torch.zeros((1, 32, 32, 1), device="cuda"), torch.empty_like(x))
    assert e.value.status == t.EARTEFACT
    # empty calls (no frames) are rejected before any launch
    z0 = torch.zeros((0, 35, 32, 32), dtype=torch.float32, device="cuda")
    x0 = torch.zeros((0, 1, 32, 32), dtype=torch.float32, device="cuda")
    ws = plan.workspace(1)
    for call in (lambda: plan.sample_zernike([], 0, 0, z0, ws),
                 lambda: plan.warp(x0, z0, torch.empty_like(x0)),
                 lambda: plan.tilt_stats(z0, 4, ws=ws),
                 lambda: plan.structure_function(z0, ws=ws)):
        with pytest.raises(t.TsimError) as e:
            call()
        assert e.value.status == t.EINVAL


def test_repeat_run_is_bit_identical(t):
    plan = t.Plan(64, 64, 1, 128, 128)
    a = _sample(t, plan, [2.0], 9, 3, 1)
    b = _sample(t, plan, [2.0], 9, 3, 1)
    assert torch.equal(a, b)


def test_basis_build_matches_oracle_pca(t):
    """The library's PCA basis (device PSFs, FP64 Gram, host subspace
    iteration) against the oracle's SVD of the same PSF database: the
    eigenvalues agree, and every eigenvector whose eigenvalue is separated
    from its neighbours by > 5% agrees (signs fixed by the same rule); the
    rest of the subspace is checked through orthonormality and the energy
    it captures."""
    say("basis build n=3000 K=40")
    plan = t.Plan(32, 32, 1, 64, 64, psf_t=33, basis_k=40)
    Psi_g, eig_g = plan.basis_build(3000, seed=21, dr_lo=0.5, dr_hi=5.0)
    A, _ = opsf.basis_draws(3000, seed=21)
    H = opsf.psf_batch(A, 64, 33)
    Psi_o, s = opsf.pca_basis(H, 40)
    lam = s[:41] ** 2
    np.testing.assert_allclose(eig_g, lam[:40], rtol=2e-5)
    np.testing.assert_allclose(Psi_g @ Psi_g.T, np.eye(40), atol=1e-10)
    gaps = np.minimum(np.abs(lam[:40] - np.r_[np.inf, lam[:39]]), np.abs(lam[:40] - lam[1:41])) / lam[:40]
    checked = 0
    for k in range(40):
        if gaps[k] > 0.05:
            assert float(Psi_g[k] @ Psi_o[k]) > 1 - 1e-5, (k, float(Psi_g[k] @ Psi_o[k]))
            checked += 1
    assert checked >= 5
    X = H.reshape(3000, -1)
    cap_g = np.linalg.norm(X @ Psi_g.T) ** 2
    cap_o = np.linalg.norm(X @ Psi_o.T) ** 2
    assert abs(cap_g - cap_o) / cap_o < 1e-8


def test_sampler_ar_matches_oracle(t):
    """Auto-regressive sequence (alpha = 0.9, per-frame D/r0): five frames from
    a fresh start, then three more continuing from the oracle's own last
    frame, against the oracle's recursion on the unit fields."""
    say("sampler AR 40x56 G=128")
    H, W, G = 40, 56, 128
    plan = t.Plan(H, W, 1, G, G, pixel_pitch_over_d=0.125)
    S = ospec.all_spectra(G, G, 0.125, 2)
    L = ozern.cholesky_lower(ozern.noll_matrix(1.0))
    drs = [1.0, 2.0, 3.5, 2.5, 4.0]
    ref, ylast = osamp.sample_sequence_ar(H, W, G, G, 0.125, drs, 7, 20, 0.9, spectra=S, L=L)
    zern = torch.empty((5, 35, H, W), dtype=torch.float32, device="cuda")
    ws = plan.workspace(5)
    plan.sample_zernike_ar(drs, 7, 20, 0.9, zern, ws)
    torch.cuda.synchronize()
    got = zern.cpu().numpy()
    for f in range(5):
        errs = [err(got[f, j], ref[f, j]) for j in range(35)]
        assert max(errs) < TOL, (f, int(np.argmax(errs)), max(errs))
    drs2 = [1.5, 3.0, 2.0]
    ref2, _ = osamp.sample_sequence_ar(H, W, G, G, 0.125, drs2, 7, 25, 0.9, y_prev=ylast, spectra=S, L=L)
    prev = torch.tensor(ref[-1].astype(np.float32), device="cuda")
    zern2 = torch.empty((3, 35, H, W), dtype=torch.float32, device="cuda")
    plan.sample_zernike_ar(drs2, 7, 25, 0.9, zern2, ws, zern_prev=prev, d_over_r0_prev=drs[-1])
    torch.cuda.synchronize()
    got2 = zern2.cpu().numpy()
    for f in range(3):
        errs = [err(got2[f, j], ref2[f, j]) for j in range(35)]
        assert max(errs) < TOL, (f, int(np.argmax(errs)), max(errs))
    with pytest.raises(t.TsimError) as e:
        plan.sample_zernike_ar(drs2, 7, 25, 1.5, zern2, ws)
    assert e.value.status == t.EINVAL
    with pytest.raises(t.TsimError) as e:   # previous frame inside the output range
        plan.sample_zernike_ar(drs2[:2], 7, 25, 0.9, zern2[1:], ws, zern_prev=zern2[1], d_over_r0_prev=1.0)
    assert e.value.status == t.EINVAL


def test_p2s_exact_k120_matches_oracle(t):
    """K = 120 takes the projection's eight-tile variant (K > 112)."""
    say("p2s exact 24x40 K=120")
    A, _ = opsf.basis_draws(400, seed=120)
    Psi, _ = opsf.pca_basis(opsf.psf_batch(A, 64, 33), 120)
    H, W = 24, 40
    plan = t.Plan(H, W, 1, 64, 64, basis=Psi, psf_t=33)
    z32 = osamp.sample_zernike(H, W, 64, 64, 0.125, 2.5, 9, 0).astype(np.float32)
    beta = torch.empty((1, H, W, 120), dtype=torch.float32, device="cuda")
    plan.p2s(torch.tensor(z32[None], device="cuda"), beta, plan.workspace(1))
    torch.cuda.synchronize()
    ref = opsf.psf_field(z32.astype(np.float64), 64, 33, Psi)
    assert err(beta.cpu().numpy()[0], ref) < TOL


def test_binding_rejects_mismatched_buffers(t, basis33):
    """The binding checks every buffer's shape, element type, device and
    size against the plan before calling the library (the C ABI cannot see
    extents): each mismatch raises ValueError and launches nothing."""
    say("binding buffer checks")
    H, W, C = 32, 48, 2
    dev = torch.device("cuda")
    plan = t.Plan(H, W, C, 64, 64, basis=basis33, psf_t=33)
    bplan = t.Plan(H, W, C, 64, 64, basis=basis33, psf_t=33, p2s_mode=t.P2S_LEARNED, precision=t.BF16)
    z = torch.zeros((2, 35, H, W), device=dev)
    img = torch.zeros((2, C, H, W), device=dev)
    out = torch.empty_like(img)
    beta = torch.zeros((2, H, W, 100), device=dev)
    ws = plan.workspace(2)
    bad = [
        lambda: plan.sample_zernike([1.0, 2.0], 0, 0, z[:, :34].contiguous(), ws),        # 34 planes
        lambda: plan.sample_zernike([1.0, 2.0], 0, 0, z.double(), ws),                    # float64
        lambda: plan.sample_zernike([1.0, 2.0], 0, 0, z, plan.workspace(1)[:1024]),       # small workspace
        lambda: plan.sample_zernike([1.0], 0, 0, z, ws),                                  # D/r0 count
        lambda: plan.p2s(z, beta[:1], ws),                                                # frame count
        lambda: plan.p2s(z, torch.zeros((2, H, W, 112), device=dev), ws),                 # K
        lambda: bplan.p2s(z, beta, ws),                                                   # f32 for a BF16 plan
        lambda: bplan.render(img, torch.zeros((2, H, W, 100), dtype=torch.bfloat16, device=dev), out),  # KP
        lambda: plan.render(img, beta, out[:1]),                                          # out frames
        lambda: plan.render(img[:, :1].contiguous(), beta[:, :, :, :], out),              # channels
        lambda: plan.warp(img, z[:1], out),                                               # zern frames
        lambda: plan.warp(img.cpu(), z, out),                                             # host tensor
        lambda: plan.warp(img, z.transpose(2, 3), out),                                   # layout
        lambda: plan.psf_exact(z[0, 0, :4, :35], torch.empty((4, 33 * 33), device=dev)),  # not contiguous
        lambda: plan.psf_exact(torch.zeros((4, 35), device=dev), torch.empty((4, 32 * 32), device=dev)),
    ]
    out.fill_(3.0)
    for i, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    torch.cuda.synchronize()
    assert bool(torch.all(out == 3.0))


def test_sync_and_last_error_on_device(t):
    """A failing call on the device path is named by tsim_last_error; a
    clean stream synchronises with TSIM_OK."""
    plan = t.Plan(32, 32, 1, 64, 64)
    z = torch.zeros((1, 35, 32, 32), device="cuda")
    t.last_error()
    with pytest.raises(t.TsimError):
        plan.sample_zernike([-1.0], 0, 0, z, plan.workspace(1))
    assert t.last_error() == (t.EINVAL, "tsim_sample_zernike: invalid argument")
    plan.sample_zernike([1.0], 0, 0, z, plan.workspace(1))
    t.sync()
    assert t.last_error() == (0, "")
