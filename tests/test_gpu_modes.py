"""Plans with more than 35 modes (Sec. II-B: the expansion keeps N = 36
modes, and N can be raised at some cost in speed): 44, 54 and 65 modes,
i.e. Noll 2..45, 2..55, 2..66, complete radial orders up to 8, 9 and 10.

The sampler (unit fields by the row pass, then the group mix, and the
subharmonic waves), the exact PSFs and projection (phase series of 11
Chebyshev terms), the warp and the statistics against the oracle with the
same mode count, at the FP32 bound of the other parity tests (relative L2
and largest element error over the largest reference magnitude, both
<= 1e-5); the allocation-free sampler and a batch with such a plan against
their workspace and call-by-call forms; the calls that take 35 modes only
refuse such plans before any launch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle import sampler as osamp  # noqa: E402
from oracle import stats as ostats  # noqa: E402
from oracle import zernike as ozern  # noqa: E402
import synthetic  # noqa: E402
from parity import err, maxrel, rel  # noqa: E402

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


def _coeffs(n_modes, shape, dr, seed):
    """Seeded coefficient vectors with the per-mode variances of A_0 at D/r0 = dr
    (float32, modes last)."""
    sd = np.sqrt(np.diag(ozern.noll_matrix(dr, j_last=n_modes + 1)))
    return (synthetic.random_coefficients(tuple(shape) + (n_modes,), 1.0, seed) * sd).astype(np.float32)


@pytest.mark.parametrize("N,H,W,Gh,Gw,levels", [(44, 40, 72, 64, 128, 0), (54, 64, 64, 128, 128, 2),
                                                (65, 20, 1030, 64, 2048, 0), (65, 50, 300, 64, 512, 1)])
def test_sampler_more_modes_matches_oracle(t, N, H, W, Gh, Gw, levels):
    say(f"sampler N={N} {H}x{W} on {Gh}x{Gw}, subharmonic levels {levels}")
    plan = t.Plan(H, W, 1, Gh, Gw, pixel_pitch_over_d=0.125, subharmonic_levels=levels, n_modes=N)
    zern = torch.empty((2, N, H, W), dtype=torch.float32, device="cuda")
    plan.sample_zernike([2.0, 0.7], 9, 3, zern, plan.workspace(2))
    torch.cuda.synchronize()
    got = zern.cpu().numpy()
    S = osamp.all_spectra(Gh, Gw, 0.125, 2, j_last=N + 1, subharmonic_levels=levels)
    for f, dr in enumerate((2.0, 0.7)):
        ref = osamp.sample_zernike(H, W, Gh, Gw, 0.125, dr, 9, 3 + f, spectra=S, subharmonic_levels=levels,
                                   n_modes=N)
        for j in range(N):
            assert err(got[f, j], ref[j]) < TOL, (f, j + 2, rel(got[f, j], ref[j]), maxrel(got[f, j], ref[j]))


@pytest.mark.parametrize("P,T", [(64, 33), (128, 65)])
def test_psf_and_projection_more_modes(t, P, T):
    """Exact PSFs with modes 4..66 in the phase, and the projected weights
    of a whole small field."""
    say(f"exact PSFs and P2S with 65 modes, P={P} T={T}")
    N = 65
    A, _ = opsf.basis_draws(200 if P == 64 else 120, seed=66, n_modes=N)
    assert A.shape[1] == N
    basis, _ = opsf.pca_basis(opsf.psf_batch(A, P, T, modes=range(4, N + 2)), 40)
    H, W = (12, 20) if P == 64 else (4, 6)
    plan = t.Plan(H, W, 1, 64, 64, pupil_n=P, psf_t=T, basis=basis, n_modes=N)
    z = _coeffs(N, (H * W,), 2.0, 67)
    psf = torch.empty((H * W, T * T), dtype=torch.float32, device="cuda")
    plan.psf_exact(torch.tensor(z, device="cuda"), psf)
    torch.cuda.synchronize()
    ref = opsf.psf_batch(z.astype(np.float64), P, T, modes=range(4, N + 2)).reshape(H * W, -1)
    got = psf.cpu().numpy()
    for i in range(0, H * W, 7):
        assert err(got[i], ref[i]) < TOL, (i, rel(got[i], ref[i]), maxrel(got[i], ref[i]))
    zern = torch.tensor(np.ascontiguousarray(z.reshape(H, W, N).transpose(2, 0, 1))[None], device="cuda")
    beta = torch.empty((1, H, W, 40), dtype=torch.float32, device="cuda")
    plan.p2s(zern, beta, plan.workspace(1))
    torch.cuda.synchronize()
    bref = opsf.psf_field(zern[0].cpu().numpy().astype(np.float64), P, T, basis)
    assert err(beta[0].cpu().numpy(), bref) < TOL


def test_render_and_warp_more_modes(t):
    """Blur and warp of a 65-mode plan: the warp reads the tilt planes of
    [frames][65][H][W] coefficients."""
    say("sample -> exact P2S -> render -> warp with 65 modes, 2 frames of 24 x 36")
    N, H, W = 65, 24, 36
    A, _ = opsf.basis_draws(150, seed=70, n_modes=N)
    basis, _ = opsf.pca_basis(opsf.psf_batch(A, 64, 33, modes=range(4, N + 2)), 30)
    plan = t.Plan(H, W, 2, 64, 64, basis=basis, n_modes=N)
    img = synthetic.test_image(2, H, W, 6, 71)
    zern = torch.empty((2, N, H, W), dtype=torch.float32, device="cuda")
    beta = torch.empty((2, H, W, 30), dtype=torch.float32, device="cuda")
    blur = torch.empty((2, 2, H, W), dtype=torch.float32, device="cuda")
    out = torch.empty_like(blur)
    ws = plan.workspace(2)
    plan.sample_zernike([3.0, 1.5], 4, 0, zern, ws)
    plan.p2s(zern, beta, ws)
    plan.render(torch.tensor(np.repeat(img[None], 2, 0), device="cuda"), beta, blur)
    plan.warp(blur, zern, out)
    torch.cuda.synchronize()
    for f in range(2):
        zr = zern[f].cpu().numpy().astype(np.float64)
        br = opsf.psf_field(zr, 64, 33, basis)
        ref = orender.render_frame(img.astype(np.float64), zr, br, basis, 33)
        got = out[f].cpu().numpy()
        for c in range(2):
            assert err(got[c], ref[c]) < TOL, (f, c, rel(got[c], ref[c]), maxrel(got[c], ref[c]))


def test_statistics_more_modes(t):
    """Tilt statistics and the OTFs on 65-mode planes; the structure function
    (35-mode moments) refuses them."""
    say("tilt statistics and OTFs with 65 modes")
    N, F, H, W = 65, 2, 11, 13
    z = np.ascontiguousarray(_coeffs(N, (F, H, W), 1.5, 72).transpose(0, 3, 1, 2))
    plan = t.Plan(H, W, 1, 64, 64, n_modes=N)
    zt = torch.tensor(z, device="cuda")
    corr, dtv = plan.tilt_stats(zt, 5)
    rc, rd = ostats.tilt_statistics(z, 5)
    np.testing.assert_allclose(corr, rc, rtol=1e-5, atol=1e-6 * np.abs(rc).max())
    np.testing.assert_allclose(dtv, rd, rtol=1e-5, atol=1e-6 * np.abs(rd).max())
    for short in (False, True):
        got = plan.otf(zt, short_exposure=short)
        ref = ostats.otf_mean(z.transpose(0, 2, 3, 1).reshape(-1, N).astype(np.float64), 64, short)
        d = np.abs(got - ref)
        assert np.linalg.norm(d) / np.linalg.norm(ref) < TOL and d.max() / np.abs(ref).max() < TOL
    with pytest.raises(t.TsimError) as e:
        plan.structure_function(zt)
    assert e.value.status == t.EUNSUPPORTED


def test_noalloc_and_batch_more_modes(t):
    """The allocation-free sampler and a batch item of a 54-mode plan equal
    the workspace form and the calls one by one."""
    say("noalloc sampler and batch with 54 modes")
    N, H, W = 54, 30, 50
    A, _ = opsf.basis_draws(120, seed=73, n_modes=N)
    basis, _ = opsf.pca_basis(opsf.psf_batch(A, 64, 33, modes=range(4, N + 2)), 20)
    plan = t.Plan(H, W, 3, 64, 128, basis=basis, n_modes=N)
    ref = torch.empty((3, N, H, W), dtype=torch.float32, device="cuda")
    got = torch.full_like(ref, float("nan"))
    plan.sample_zernike([1.0, 2.0, 3.0], 5, 11, ref, plan.workspace(3))
    plan.sample_zernike_noalloc([1.0, 2.0, 3.0], 5, 11, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    img = torch.tensor(np.repeat(synthetic.test_image(3, H, W, 8, 74)[None], 2, 0), device="cuda")
    it = dict(plan=plan, d_over_r0=[1.5, 2.5], frame0=0, img=img,
              zern=torch.empty((2, N, H, W), device="cuda"), beta=torch.empty((2, H, W, 20), device="cuda"),
              blur=torch.empty((2, 3, H, W), device="cuda"), out=torch.empty((2, 3, H, W), device="cuda"),
              ws=plan.workspace(2))
    z2, b2, bl2, o2 = (torch.empty_like(it[k]) for k in ("zern", "beta", "blur", "out"))
    plan.sample_zernike([1.5, 2.5], 5, 0, z2, it["ws"])
    plan.p2s(z2, b2, it["ws"])
    plan.render(img, b2, bl2)
    plan.warp(bl2, z2, o2)
    b = t.Batch([it], 5)
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(it["out"], o2) and torch.equal(it["zern"], z2)
    b.close()


def test_network_calls_refuse_more_modes(t):
    say("network calls refuse plans with more than 35 modes")
    plan = t.Plan(16, 16, 1, 64, 64, basis_k=8, n_modes=44)
    with pytest.raises(t.TsimError) as e:
        t.Mlp(plan, batch=64)
    assert e.value.status == t.EUNSUPPORTED
