"""The allocation-free sampling entry point, tsim_sample_zernike_noalloc,
against tsim_sample_zernike (which takes a caller workspace): two calls in a
row, the second on a smaller plan, each bit-identical to the workspace
form's fields (the same kernels run on the same counters, only the
intermediate's buffer differs).  The first call spans two chunks of the
fixed scratch array; the second reuses the array the first left filled.
Plans whose single-frame intermediate exceeds the array are refused before
any launch, with a reason from tsim_last_error."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_06713_amd as t
    return t


def _both(t, plan, d, seed, frame0):
    F = len(d)
    ref = torch.empty((F, 35, plan.H, plan.W), dtype=torch.float32, device="cuda")
    got = torch.full_like(ref, float("nan"))
    plan.sample_zernike(d, seed, frame0, ref, plan.workspace(F))
    plan.sample_zernike_noalloc(d, seed, frame0, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


def test_noalloc_sampler_matches_workspace_form_twice(t):
    scratch = 256 << 20
    # call 1: 512 x 512 on a 1024 grid, 75.5 MB of intermediate per frame,
    # so 3 frames per chunk of the array and 5 frames take two chunks
    say("noalloc sampler: 5 frames of 512x512 on 1024^2")
    p1 = t.Plan(512, 512, 3, 1024, 1024, pixel_pitch_over_d=0.125)
    assert 18 * 512 * 1024 * 8 * 3 <= scratch < 18 * 512 * 1024 * 8 * 4
    got, ref = _both(t, p1, [1.0, 2.0, 4.0, 1.5, 3.0], 11, 7)
    assert np.isfinite(got).all()
    np.testing.assert_array_equal(got, ref)
    # call 2: a smaller, ragged plan with subharmonic levels, other seed and frames
    say("noalloc sampler: 2 frames of 40x72 on 64x128, 2 subharmonic levels")
    p2 = t.Plan(40, 72, 1, 64, 128, pixel_pitch_over_d=0.2, subharmonic_levels=2)
    got, ref = _both(t, p2, [0.7, 2.5], 3, 1000)
    assert np.isfinite(got).all()
    np.testing.assert_array_equal(got, ref)


def test_noalloc_sampler_refuses_plans_beyond_the_scratch(t):
    say("noalloc sampler: 1024x1024 on 2048^2 is refused (302 MB > 256 MiB)")
    t.last_error()
    p = t.Plan(1024, 1024, 1, 2048, 2048, pixel_pitch_over_d=0.125)
    z = torch.zeros((1, 35, 1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(t.TsimError) as e:
        p.sample_zernike_noalloc([1.0], 0, 0, z)
    assert e.value.status == t.EUNSUPPORTED
    st, msg = t.last_error()
    assert st == t.EUNSUPPORTED and "scratch" in msg, msg
    torch.cuda.synchronize()
    assert not z.any()                      # nothing was launched
    # a bad D/r0 is refused before any launch as well
    p2 = t.Plan(64, 64, 1, 128, 128)
    z2 = torch.zeros((2, 35, 64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(t.TsimError) as e:
        p2.sample_zernike_noalloc([1.0, -1.0], 0, 0, z2)
    assert e.value.status == t.EINVAL
    torch.cuda.synchronize()
    assert not z2.any()
