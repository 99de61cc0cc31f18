"""The sampler's launch forms (tsim_plan_set_tuning / tsim_plan_tuning /
tsim_plan_autotune): every form the plan's shape allows gives the same
fields, bit for bit, as the built-in form, so tuning changes only the time;
the autotuner keeps an allowed form; forms the shape does not allow are
refused before any launch.  The built-in form itself is checked against the
oracle by the sampler parity tests."""
import sys

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


SHAPES = [(40, 72, 64, 128, 0), (64, 64, 128, 128, 2), (48, 96, 128, 256, 0), (200, 520, 256, 1024, 1),
          (20, 1030, 64, 2048, 0)]


def _fields(plan, frames, ws):
    zern = torch.full((frames, plan.N, plan.H, plan.W), float("nan"), device="cuda")
    plan.sample_zernike([1.0 + 0.5 * f for f in range(frames)], 11, 2, zern, ws)
    torch.cuda.synchronize()
    return zern


@pytest.mark.parametrize("H,W,Gh,Gw,levels", SHAPES)
def test_every_allowed_form_gives_the_same_fields(t, H, W, Gh, Gw, levels):
    plan = t.Plan(H, W, 1, Gh, Gw, pixel_pitch_over_d=0.125, subharmonic_levels=levels)
    ws = plan.workspace(3)
    plan.set_tuning(0, 0)
    nc0, rows0 = plan.tuning()
    ref = _fields(plan, 3, ws)
    assert not torch.isnan(ref).any()
    tried = 0
    for nc in (nc0 // 2, nc0, 2 * nc0):
        for rows in (1, 2, 3):
            try:
                plan.set_tuning(nc, rows)
            except t.TsimError as e:
                assert e.status == t.EINVAL
                continue
            assert plan.tuning() == (nc, rows)
            say(f"{H}x{W} on {Gh}x{Gw}: pass-1 columns {nc}, pass-2 form {rows}")
            got = _fields(plan, 3, ws)
            assert torch.equal(got, ref), (nc, rows)
            tried += 1
    assert tried >= 2
    plan.close()


def test_autotune_keeps_an_allowed_form_and_the_fields(t):
    plan = t.Plan(64, 64, 1, 128, 128, pixel_pitch_over_d=0.125)
    ws = plan.workspace(4)
    ref = _fields(plan, 4, ws)
    scratch = torch.empty_like(ref)
    nc, rows = plan.autotune(4, scratch, ws)
    say(f"autotune chose pass-1 columns {nc}, pass-2 form {rows}")
    plan.set_tuning(nc, rows)          # the choice is an allowed form
    assert torch.equal(_fields(plan, 4, ws), ref)
    plan.close()


def test_disallowed_forms_rejected(t):
    plan = t.Plan(20, 1030, 1, 64, 2048, pixel_pitch_over_d=0.125)
    for nc, rows in ((3, 0), (1, 0), (0, 1), (0, 2), (0, 4), (-1, 0)):
        with pytest.raises(t.TsimError) as e:
            plan.set_tuning(nc, rows)
        assert e.value.status == t.EINVAL
    plan.close()
