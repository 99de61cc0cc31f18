"""GPU parity of the learned phase-to-space path (BF16 matrix cores, FP32
accumulation) against the oracle's BF16-mirrored network, and of the BF16
blur against Eq. (8) on the same BF16-rounded operands.

Tolerances: the oracle rounds every GEMM operand to bfloat16 at the same
points as the kernels, so the remaining differences come from FP32 versus
FP64 accumulation (~1e-6 relative) and from the rare elements where that
difference flips a bfloat16 rounding (one unit, 2^-8, in a small fraction
of elements): relative L2 <= 1e-3 for gradients and network outputs.  The
BF16 blur accumulates in FP32 on exactly rounded operands: <= 1e-5.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from oracle import mlp as omlp  # noqa: E402
from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle import philox  # noqa: E402
import synthetic  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def t():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_06713_amd as t
    return t


@pytest.fixture(scope="module")
def basis():
    A, _ = opsf.basis_draws(800, seed=99)
    Psi, _ = opsf.pca_basis(opsf.psf_batch(A, 64, 33), 100)
    return Psi


def _random_net(t, net, seed):
    layers = []
    for l in range(4):
        i, o = net.dims[l], net.dims[l + 1]
        W = synthetic.random_coefficients((o, i), 1.0 / np.sqrt(i), seed + l)
        b = synthetic.random_coefficients((o,), 0.1, seed + 10 + l)
        layers.append((W, b))
    net.set(0, net.pack(layers))
    return [(W.astype(np.float64), b.astype(np.float64)) for W, b in layers]


def _inv_s(seed):
    v = np.abs(synthetic.random_coefficients((35,), 1.0, seed)) + 0.5
    v[:2] = 0.0
    return v.astype(np.float32)


def test_mlp_gradients_match_bf16_mirror(t):
    say("mlp gradients B=192 K=24")
    plan = t.Plan(32, 32, 1, 64, 64, basis_k=24)
    net = t.Mlp(plan, batch=192, seed=1)
    params = _random_net(t, net, 100)
    inv = _inv_s(7)
    net.set(2, inv)
    z = synthetic.random_coefficients((192, 35), 0.7, 3)
    tgt = synthetic.random_coefficients((192, 24), 1.0, 4)
    loss = net.grad(torch.tensor(z, device="cuda"), torch.tensor(tgt, device="cuda"))
    g = net.unpack(net.get(1))
    x = omlp.to_bf16(z.astype(np.float64) * inv.astype(np.float64))
    ref_loss, ref = omlp.loss_and_grads(params, x, tgt.astype(np.float64), bf16=True)
    assert abs(loss - ref_loss) / ref_loss < 1e-4
    for l in range(4):
        assert rel(g[l][0], ref[l][0]) < 1e-3, ("dW", l, rel(g[l][0], ref[l][0]))
        assert rel(g[l][1], ref[l][1]) < 1e-3, ("db", l, rel(g[l][1], ref[l][1]))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mlp_inference_matches_bf16_mirror(t, basis, precision):
    say(f"mlp inference {precision}")
    H, W = 24, 40
    prec = t.FP32 if precision == "fp32" else t.BF16
    plan = t.Plan(H, W, 1, 64, 64, basis=basis, p2s_mode=t.P2S_LEARNED, precision=prec)
    net = t.Mlp(plan, batch=64, seed=2)
    params = _random_net(t, net, 200)
    inv = _inv_s(8)
    net.set(2, inv)
    mu = synthetic.random_coefficients((100,), 0.05, 9)
    net.set(3, mu)
    net.set(4, [0.3])
    t.plan_set_mlp(plan, net)
    zern = synthetic.random_coefficients((2, 35, H, W), 0.6, 11)
    KB = 100 if precision == "fp32" else 112
    dt = torch.float32 if precision == "fp32" else torch.bfloat16
    beta = torch.zeros((2, H, W, KB), dtype=dt, device="cuda")
    plan.p2s(torch.tensor(zern, device="cuda"), beta, plan.workspace(2))
    torch.cuda.synchronize()
    got = beta.float().cpu().numpy().reshape(-1, KB)
    a = zern.transpose(0, 2, 3, 1).reshape(-1, 35).astype(np.float64)
    x = omlp.to_bf16(a * inv.astype(np.float64))
    y, _ = omlp.forward(params, x, bf16=True)
    ref = 0.3 * y + mu.astype(np.float64)
    if precision == "bf16":
        ref = omlp.to_bf16(ref)
        assert np.all(got[:, 100:] == 0)
    assert rel(got[:, :100], ref) < 2e-3


def test_render_bf16_matches_eq8_on_rounded_operands(t, basis):
    say("render bf16 C=3 40x72")
    H, W, C = 40, 72, 3
    plan = t.Plan(H, W, C, 128, 128, basis=basis, p2s_mode=t.P2S_LEARNED, precision=t.BF16)
    img = synthetic.test_image(C, H, W, 8, seed=4)[None]
    b = synthetic.random_coefficients((1, H, W, 100), 0.05, 5)
    b[..., 0] += 1.0
    bpad = np.zeros((1, H, W, 112), dtype=np.float32)
    bpad[..., :100] = b
    bt = torch.tensor(bpad, device="cuda").to(torch.bfloat16)
    out = torch.empty((1, C, H, W), dtype=torch.float32, device="cuda")
    plan.render(torch.tensor(img, device="cuda"), bt, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    br = omlp.to_bf16(b[0].astype(np.float64))
    Pr = omlp.to_bf16(basis)
    for c in range(C):
        ref = orender.render_basis(img[0, c].astype(np.float64), br, Pr, 33)
        assert rel(got[c], ref) < 1e-5, c


@pytest.mark.parametrize("T,C,K,H,W", [(15, 1, 20, 19, 37), (21, 2, 60, 24, 33), (33, 4, 120, 17, 48),
                                       (65, 2, 100, 21, 35)])
def test_render_bf16_kernel_shapes(t, T, C, K, H, W):
    """Every (kernel size, channel count, padded basis size) form of the
    BF16 blur on ragged frames: 32, 64 and 128-wide bases, 4 to 68 groups of
    tap pairs (steady-state loop and its compile-time tail), 8- and 16-row
    blocks."""
    say(f"render bf16 T={T} C={C} K={K} {H}x{W}")
    P = 128 if T == 65 else 64
    A, _ = opsf.basis_draws(max(300, 2 * K), seed=40 + T)
    Psi = opsf.pca_basis(opsf.psf_batch(A, P, T), K)[0]
    plan = t.Plan(H, W, C, 64, 64, psf_t=T, pupil_n=P, basis=Psi, p2s_mode=t.P2S_LEARNED, precision=t.BF16)
    KP = 32 if K <= 32 else 64 if K <= 64 else 112 if K <= 112 else 128
    img = synthetic.test_image(C, H, W, 4, seed=T)[None]
    b = synthetic.random_coefficients((1, H, W, K), 0.05, T + 1)
    b[..., 0] += 1.0
    bpad = np.zeros((1, H, W, KP), dtype=np.float32)
    bpad[..., :K] = b
    out = torch.empty((1, C, H, W), dtype=torch.float32, device="cuda")
    plan.render(torch.tensor(img, device="cuda"), torch.tensor(bpad, device="cuda").to(torch.bfloat16), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[0]
    br, Pr = omlp.to_bf16(b[0].astype(np.float64)), omlp.to_bf16(Psi)
    for c in range(C):
        ref = orender.render_basis(img[0, c].astype(np.float64), br, Pr, T)
        assert rel(got[c], ref) < 1e-5, c


def test_render_bf16_unsupported_shape_is_rejected(t):
    """The one BF16 shape whose image tile and basis staging exceed the LDS
    (K > 112, C = 4, T = 65) returns TSIM_EUNSUPPORTED before any launch and
    leaves the output untouched."""
    say("render bf16 K=120 C=4 T=65: rejected")
    H, W, C, K, T = 20, 24, 4, 120, 65
    rng = np.random.default_rng(9)
    Psi = np.linalg.qr(rng.standard_normal((T * T, K)))[0].T.copy()
    plan = t.Plan(H, W, C, 64, 64, psf_t=T, pupil_n=128, basis=Psi, p2s_mode=t.P2S_LEARNED, precision=t.BF16)
    img = torch.ones((1, C, H, W), dtype=torch.float32, device="cuda")
    beta = torch.zeros((1, H, W, 128), dtype=torch.bfloat16, device="cuda")
    out = torch.full((1, C, H, W), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(t.TsimError) as e:
        plan.render(img, beta, out)
    assert e.value.status == t.EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))


def test_training_pairs_match_oracle(t, basis):
    say("training pairs n=2000")
    plan = t.Plan(32, 32, 1, 64, 64, basis=basis)
    z, b = t.make_training_data(plan, 2000, seed=5)
    torch.cuda.synchronize()
    A, _ = opsf.basis_draws(2000, seed=5, tag=philox.TAG_MLP_DATA)
    assert rel(z.cpu().numpy(), A) < 1e-6
    ref = opsf.project(opsf.psf_batch(A.astype(np.float32).astype(np.float64), 64, 33), basis)
    assert rel(b.cpu().numpy(), ref) < 1e-5


def test_training_reduces_loss(t, basis):
    say("training 400 steps")
    plan = t.Plan(32, 32, 1, 64, 64, basis=basis)
    z, b = t.make_training_data(plan, 65536, seed=6)
    net = t.Mlp(plan, batch=1024, seed=3)
    bn = b.cpu().numpy()
    net.set(3, bn.mean(0))
    net.set(4, [float(np.sqrt(((bn - bn.mean(0)) ** 2).mean()))])
    losses = net.train(z, b, 400, lr_max=2e-3, lr_min=1e-4)
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.2 * losses[:5].mean(), (losses[:5], losses[-5:])
