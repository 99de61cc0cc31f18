"""GPU parity of the spatial tilt statistics (tsim_tilt_stats, Sec. IV-B)
against the FP64 oracle on the same planes: seeded random planes of ragged
sizes, the sampler's own 512 x 512 output at the benchmark's lag range, the
lag edge cases, and argument checks."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import stats as ostats  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_06713_amd as t
    return t


def _check(corr, dtv, ref_corr, ref_dtv, scale):
    # FP32 row sums, FP64 totals: well inside 1e-5 of the planes' variance
    np.testing.assert_allclose(corr, ref_corr, rtol=1e-5, atol=1e-6 * scale)
    np.testing.assert_allclose(dtv, ref_dtv, rtol=1e-5, atol=1e-6 * scale)


@pytest.mark.parametrize("F,H,W,L", [(2, 37, 53, 20), (1, 64, 64, 63), (3, 1, 300, 0),
                                     (2, 200, 17, 16), (1, 9, 4096, 8)])
def test_tilt_stats_random_planes(t, F, H, W, L):
    say(f"tilt stats random F={F} H={H} W={W} L={L}")
    rng = np.random.default_rng(H * 1000 + W)
    z = rng.standard_normal((F, 35, H, W)).astype(np.float32)
    plan = t.Plan(H, W, 1, 64 if H <= 64 else 256, 4096 if W > 1024 else 1024 if W > 256 else 512,
                  pixel_pitch_over_d=0.125)
    corr, dtv = plan.tilt_stats(torch.tensor(z, device="cuda"), L)
    ref_corr, ref_dtv = ostats.tilt_statistics(z, L)
    _check(corr, dtv, ref_corr, ref_dtv, 1.0)
    assert np.all(dtv[:, :, 0] == 0.0)


def test_tilt_stats_sampler_512(t):
    """The benchmark's shape: four 512 x 512 frames from the sampler, lags to 64."""
    say("tilt stats sampler 512 L=64")
    plan = t.Plan(512, 512, 1, 1024, 1024, pixel_pitch_over_d=0.125, subharmonic_levels=3)
    z = torch.empty((4, 35, 512, 512), dtype=torch.float32, device="cuda")
    plan.sample_zernike([1.0, 2.0, 4.0, 1.0], 0, 0, z, plan.workspace(4))
    corr, dtv = plan.tilt_stats(z, 64)
    ref_corr, ref_dtv = ostats.tilt_statistics(z.cpu().numpy(), 64)
    _check(corr, dtv, ref_corr, ref_dtv, float(ref_corr[:, :, 0].max()))


def test_tilt_stats_rejects_bad_lags(t):
    plan = t.Plan(16, 24, 1, 64, 64, pixel_pitch_over_d=0.125)
    z = torch.zeros((1, 35, 16, 24), dtype=torch.float32, device="cuda")
    for L in (16, -1, 257):
        with pytest.raises(t.TsimError) as e:
            plan.tilt_stats(z, L)
        assert e.value.status == t.EINVAL
