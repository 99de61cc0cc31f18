"""The one-call path (tsim_frame): fields, weights, blur and warp group by
group of frames with the group's intermediates in the workspace.

For every group size (one frame, a ragged split, all frames at once, the
default) the outputs and the kept fields equal the four individual calls
bit for bit, in the exact FP32 form (also with subharmonics) and in the
learned BF16 form; the last frame of the exact form also equals the oracle's
whole frame (relative L2 and largest element error over the largest
reference magnitude both <= 1e-5, the FP32 path's tolerance).  Bad arguments
are refused before any launch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle import sampler as osamp  # noqa: E402
import synthetic  # noqa: E402
from parity import err, maxrel, rel  # noqa: E402

TOL = 1e-5
SEED = 9
F, H, W, GH, GW, FRAME0 = 5, 48, 96, 128, 256, 3
DR = [1.0, 2.5, 0.8, 4.0, 1.7]


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
def basis():
    A, _ = opsf.basis_draws(400, seed=17)
    return opsf.pca_basis(opsf.psf_batch(A, 64, 33), 100)[0]


def _image():
    img = synthetic.test_image(3, H, W, 8, 21)
    return torch.tensor(np.stack([np.roll(img, 3 * f, axis=2) for f in range(F)]), device="cuda")


def _calls(p, img, kb, bt):
    zern = torch.empty((F, p.N, H, W), device="cuda")
    beta = torch.empty((F, H, W, kb), dtype=bt, device="cuda")
    blur = torch.empty_like(img)
    out = torch.empty_like(img)
    ws = p.workspace(F)
    p.sample_zernike(DR, SEED, FRAME0, zern, ws)
    p.p2s(zern, beta, ws)
    p.render(img, beta, blur)
    p.warp(blur, zern, out)
    torch.cuda.synchronize()
    return zern, out


def _frame_calls(p, img, ref_zern, ref_out):
    for group in (1, 2, F, None):
        g = p.frame_group() if group is None else group
        say(f"  group {g}")
        ws = p.frame_workspace(g)
        out = torch.full_like(img, float("nan"))
        zern = torch.full((F, p.N, H, W), float("nan"), device="cuda")
        p.frame(DR, SEED, FRAME0, img, out, ws, group=g, zern_out=zern)
        torch.cuda.synchronize()
        assert torch.equal(zern, ref_zern), g
        assert torch.equal(out, ref_out), g
        # without kept fields: the same images
        out2 = torch.full_like(img, float("nan"))
        p.frame(DR, SEED, FRAME0, img, out2, ws, group=g)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref_out), g


@pytest.mark.parametrize("levels", [0, 2])
def test_frame_exact_form_equals_calls_and_oracle(t, basis, levels):
    say(f"tsim_frame, exact FP32 form, {F} frames of {H}x{W}x3, subharmonic levels {levels}")
    p = t.Plan(H, W, 3, GH, GW, basis=basis, pixel_pitch_over_d=0.125, subharmonic_levels=levels)
    img = _image()
    ref_zern, ref_out = _calls(p, img, 100, torch.float32)
    _frame_calls(p, img, ref_zern, ref_out)
    if levels == 0:
        f = F - 1
        say(f"  oracle frame {f}")
        zr = osamp.sample_zernike(H, W, GH, GW, 0.125, DR[f], SEED, FRAME0 + f)
        br = opsf.psf_field(zr, 64, 33, basis)
        ref = orender.render_frame(img[f].cpu().numpy().astype(np.float64), zr, br, basis, 33)
        go = ref_out[f].cpu().numpy()
        for c in range(3):
            say(f"  channel {c}: rel {rel(go[c], ref[c]):.2e} maxrel {maxrel(go[c], ref[c]):.2e}")
            assert err(go[c], ref[c]) < TOL, c
    p.close()


def test_frame_learned_form_equals_calls(t, basis):
    say("tsim_frame, learned BF16 form")
    p = t.Plan(H, W, 3, GH, GW, basis=basis, pixel_pitch_over_d=0.125, p2s_mode=t.P2S_LEARNED,
               precision=t.BF16)
    net = t.Mlp(p, batch=64, seed=6)
    t.plan_set_mlp(p, net)
    img = _image()
    ref_zern, ref_out = _calls(p, img, p.KP, torch.bfloat16)
    _frame_calls(p, img, ref_zern, ref_out)
    net.close()
    p.close()


def test_frame_group_and_workspace(t, basis):
    p = t.Plan(512, 512, 3, 1024, 1024, basis=basis, pixel_pitch_over_d=0.125, p2s_mode=t.P2S_LEARNED,
               precision=t.BF16)
    g = p.frame_group()
    per = 512 * 512 * (35 * 4 + p.KP * 2 + 3 * 4)
    say(f"512^2 BF16 plan: default group {g}, workspace {p.frame_workspace_bytes(g) / 2**20:.0f} MiB")
    assert g == (1 << 30) // per
    assert p.frame_workspace_bytes(1) < p.frame_workspace_bytes(2) < p.frame_workspace_bytes(g)
    p.close()


def test_frame_rejects_bad_arguments(t, basis):
    say("tsim_frame: argument checks")
    p = t.Plan(H, W, 3, GH, GW, basis=basis, pixel_pitch_over_d=0.125)
    img = _image()
    out = torch.empty_like(img)
    ws = p.frame_workspace(2)
    for g in (0, -1, 65536):
        with pytest.raises(t.TsimError) as e:
            p.frame(DR, SEED, FRAME0, img, out, ws, group=g)
        assert e.value.status == t.EINVAL
    with pytest.raises(t.TsimError) as e:
        p.frame(DR, SEED, FRAME0, img, img, ws, group=2)           # img and out must differ
    assert e.value.status == t.EINVAL
    with pytest.raises(t.TsimError) as e:
        p.frame([1.0, -1.0, 1.0, 1.0, 1.0], SEED, FRAME0, img, out, ws, group=2)
    assert e.value.status == t.EINVAL
    with pytest.raises(ValueError):
        p.frame(DR, SEED, FRAME0, img, out, p.frame_workspace(1), group=2)   # workspace too small
    nb = t.Plan(H, W, 3, GH, GW, pixel_pitch_over_d=0.125)
    with pytest.raises(t.TsimError) as e:
        nb.frame(DR, SEED, FRAME0, img, out, nb.frame_workspace(2), group=2)
    assert e.value.status == t.EARTEFACT
    nb.close()
    p.close()


def test_frame_large_learned_frames_equal_calls(t, basis):
    """Two 768 x 1024 x 3 frames on the 2048^2 grid (the batch workload's
    largest size) in the learned form, one frame per group: equal to the
    individual calls bit for bit."""
    Hl, Wl, Fl = 768, 1024, 2
    say(f"tsim_frame, learned BF16 form, {Fl} frames of {Hl}x{Wl}x3 on 2048^2, group 1")
    p = t.Plan(Hl, Wl, 3, 2048, 2048, basis=basis, pixel_pitch_over_d=0.125, p2s_mode=t.P2S_LEARNED,
               precision=t.BF16)
    net = t.Mlp(p, batch=64, seed=8)
    t.plan_set_mlp(p, net)
    img = torch.tensor(np.repeat(synthetic.test_image(3, Hl, Wl, 16, 5)[None], Fl, 0), device="cuda")
    dr = [1.5, 3.5]
    zern = torch.empty((Fl, p.N, Hl, Wl), device="cuda")
    beta = torch.empty((Fl, Hl, Wl, p.KP), dtype=torch.bfloat16, device="cuda")
    blur = torch.empty_like(img)
    ref = torch.empty_like(img)
    ws = p.workspace(Fl)
    p.sample_zernike(dr, SEED, 40, zern, ws)
    p.p2s(zern, beta, ws)
    p.render(img, beta, blur)
    p.warp(blur, zern, ref)
    del ws, beta, blur
    out = torch.full_like(img, float("nan"))
    p.frame(dr, SEED, 40, img, out, p.frame_workspace(1), group=1)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    net.close()
    p.close()
