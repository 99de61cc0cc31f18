"""GPU parity of the learned phase-to-space path (BF16 matrix cores, FP32
accumulation) against the oracle's BF16-mirrored network, and of the BF16
blur against Eq. (8) on the same BF16-rounded operands.

Tolerances: the oracle rounds every GEMM operand to bfloat16 at the same
points as the kernels, so the remaining differences come from FP32 versus
FP64 accumulation (~1e-6 relative) and from the rare elements where that
difference flips a bfloat16 rounding (one unit, 2^-8, in a small fraction
of elements): relative L2 <= 1e-3 for gradients and <= 2e-3 for network
outputs (which are themselves rounded to bfloat16), and the largest element
error over the largest reference magnitude <= 1e-2 (one bfloat16 unit of the
largest output is 2^-8 of it).  The BF16 blur accumulates in FP32 on exactly
rounded operands: <= 1e-5 in both measures.
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
from parity import err, maxrel, rel  # noqa: E402


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


@pytest.mark.parametrize("B", [192, 2048])
def test_mlp_gradients_match_bf16_mirror(t, B):
    """B = 192 reduces each weight gradient in one block per tile; B = 2048
    splits the batch over 8 blocks per tile (the split-K path of training
    batches), whose partial products are added in a fixed order."""
    say(f"mlp gradients B={B} K=24")
    plan = t.Plan(32, 32, 1, 64, 64, basis_k=24)
    net = t.Mlp(plan, batch=B, seed=1)
    params = _random_net(t, net, 100)
    inv = _inv_s(7)
    net.set(2, inv)
    z = synthetic.random_coefficients((B, 35), 0.7, 3)
    tgt = synthetic.random_coefficients((B, 24), 1.0, 4)
    loss = net.grad(torch.tensor(z, device="cuda"), torch.tensor(tgt, device="cuda"))
    g = net.unpack(net.get(1))
    x = omlp.to_bf16(z.astype(np.float64) * inv.astype(np.float64))
    ref_loss, ref = omlp.loss_and_grads(params, x, tgt.astype(np.float64), bf16=True)
    assert abs(loss - ref_loss) / ref_loss < 1e-4
    for l in range(4):
        for k, name in ((0, "dW"), (1, "db")):
            say(f"  {name}{l}: rel {rel(g[l][k], ref[l][k]):.2e} maxrel {maxrel(g[l][k], ref[l][k]):.2e}")
            assert rel(g[l][k], ref[l][k]) < 1e-3, (name, l, rel(g[l][k], ref[l][k]))
            assert maxrel(g[l][k], ref[l][k]) < 1e-2, (name, l, maxrel(g[l][k], ref[l][k]))


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
    say(f"  rel {rel(got[:, :100], ref):.2e} maxrel {maxrel(got[:, :100], ref):.2e}")
    assert rel(got[:, :100], ref) < 2e-3
    assert maxrel(got[:, :100], ref) < 1e-2


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
        assert err(got[c], ref) < 1e-5, (c, rel(got[c], ref), maxrel(got[c], ref))


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
        assert err(got[c], ref) < 1e-5, (c, rel(got[c], ref), maxrel(got[c], ref))


def test_render_bf16_unsupported_shape_is_rejected(t):
    """The one BF16 shape whose image tile and basis staging exceed the LDS
    (K > 112, C = 4, T = 65) is refused at plan creation, with the call
    named by tsim_last_error."""
    say("render bf16 K=120 C=4 T=65: rejected")
    H, W, C, K, T = 20, 24, 4, 120, 65
    rng = np.random.default_rng(9)
    Psi = np.linalg.qr(rng.standard_normal((T * T, K)))[0].T.copy()
    t.last_error()
    with pytest.raises(t.TsimError) as e:
        t.Plan(H, W, C, 64, 64, psf_t=T, pupil_n=128, basis=Psi, p2s_mode=t.P2S_LEARNED, precision=t.BF16)
    assert e.value.status == t.EUNSUPPORTED
    assert t.last_error() == (t.EUNSUPPORTED, "tsim_plan_create: unsupported configuration")


def test_training_pairs_match_oracle(t, basis):
    say("training pairs n=2000")
    plan = t.Plan(32, 32, 1, 64, 64, basis=basis)
    z, b = t.make_training_data(plan, 2000, seed=5)
    torch.cuda.synchronize()
    A, _ = opsf.basis_draws(2000, seed=5, tag=philox.TAG_MLP_DATA)
    assert err(z.cpu().numpy(), A) < 1e-6
    ref = opsf.project(opsf.psf_batch(A.astype(np.float32).astype(np.float64), 64, 33), basis)
    assert err(b.cpu().numpy(), ref) < 1e-5


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


def _cosine_lr(i, steps, lr_max, lr_min):
    prog = i / (steps - 1) if steps > 1 else 1.0
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + np.cos(np.pi * prog))


def test_training_steps_match_oracle_adamw(t):
    """Three steps of tsim_mlp_train at batch 1024 (split-K weight
    gradients, 4 blocks per tile), one call per step, against the oracle.
    Before each step the network's gradient at its current parameters on
    that step's batch (the batch the step counter selects) is compared with
    the oracle's BF16-mirrored gradient; the step itself must then equal
    ``oracle.mlp.adamw_step`` applied to that gradient and to the moments
    the network held, at the cosine learning rate of the step (schedule
    length 3).  That update is computed in FP32 on the device and in FP64
    by the oracle, so parameters and moments agree to a few FP32 roundings
    element by element.  (Chaining three oracle steps on the oracle's own
    gradients instead is not a parity test of the optimiser: AdamW moves
    every parameter by about lr whatever its gradient's size, so elements
    whose gradient is within FP32-accumulation rounding of zero may move
    by lr in opposite directions.)  The gradient the step used is the one
    the gradient call returned, bit for bit, and the packed layout's
    padding stays 0."""
    say("mlp train 3 steps B=1024 vs oracle AdamW")
    B, K, steps, lr_max, lr_min = 1024, 24, 3, 2e-3, 2e-4
    plan = t.Plan(32, 32, 1, 64, 64, basis_k=K)
    net = t.Mlp(plan, batch=B, seed=1)
    _random_net(t, net, 500)
    inv = _inv_s(17)
    net.set(2, inv)
    mu = synthetic.random_coefficients((K,), 0.1, 18)
    net.set(3, mu)
    net.set(4, [0.5])
    z = synthetic.random_coefficients((steps * B, 35), 0.7, 19)
    tgt = synthetic.random_coefficients((steps * B, K), 1.0, 20)
    zd, td = torch.tensor(z, device="cuda"), torch.tensor(tgt, device="cuda")
    x_all = omlp.to_bf16(z.astype(np.float64) * inv.astype(np.float64))
    t_all = (tgt.astype(np.float64) - mu.astype(np.float32).astype(np.float64)) * np.float64(np.float32(1 / 0.5))
    pad = np.ones(net.n_params, bool)
    for l in range(4):
        pad[net.off_w[l]:net.off_w[l] + net.dims[l] * net.dims[l + 1]] = False
        pad[net.off_b[l]:net.off_b[l] + net.dims[l + 1]] = False
    eps32 = 2.0 ** -24
    for i in range(steps):
        sl = slice(i * B, (i + 1) * B)
        p0 = net.get(0).astype(np.float64)
        m0 = net.get(5).astype(np.float64)
        v0 = net.get(6).astype(np.float64)
        loss_g = net.grad(zd[sl], td[sl])
        g = net.get(1)
        # the gradient against the oracle at the network's own parameters
        cur = [(W.astype(np.float64), b.astype(np.float64)) for W, b in net.unpack(p0)]
        ref_loss, ref_g = omlp.loss_and_grads(cur, x_all[sl], t_all[sl], bf16=True)
        assert abs(loss_g - ref_loss) / ref_loss < 1e-4
        gg = net.unpack(g)
        for l in range(4):
            for k in range(2):
                assert rel(gg[l][k], ref_g[l][k]) < 1e-3, (i, l, k, rel(gg[l][k], ref_g[l][k]))
                assert maxrel(gg[l][k], ref_g[l][k]) < 1e-2, (i, l, k, maxrel(gg[l][k], ref_g[l][k]))
        # one optimiser step at global step i of a 3-step schedule
        net.set(7, [i, steps])
        loss_t = net.train(zd, td, 1, lr_max=lr_max, lr_min=lr_min)[0]
        assert abs(loss_t - loss_g) <= 1e-5 * loss_g     # the loss sum is atomic: order may vary
        np.testing.assert_array_equal(net.get(1), g)     # same batch, same gradient, bit for bit
        lr = _cosine_lr(i, steps, lr_max, lr_min)
        sh = lambda f: [(f[net.off_w[l]:net.off_w[l] + net.dims[l] * net.dims[l + 1]],
                         f[net.off_b[l]:net.off_b[l] + net.dims[l + 1]]) for l in range(4)]
        ref_p, (ti, ref_m, ref_v) = omlp.adamw_step(sh(p0), sh(g.astype(np.float64)),
                                                    (i, sh(m0), sh(v0)), lr)
        assert ti == i + 1
        got_p, got_m, got_v = net.get(0).astype(np.float64), net.get(5), net.get(6)
        # bounds: a few FP32 roundings of each term of the moment sums (which
        # may cancel), and for the parameters one rounding of the result plus
        # 1e-5 of the step size (the update's relative error is a few FP32
        # roundings of m_hat, sqrt(v_hat) and the quotient)
        g64 = g.astype(np.float64)
        tol_p = 8 * eps32 * np.abs(np.concatenate([np.ravel(a) for pr in ref_p for a in pr])) + 1e-5 * lr
        tol_m = 8 * eps32 * (0.9 * np.abs(m0) + 0.1 * np.abs(g64)) + 1e-30
        tol_v = 8 * eps32 * (0.999 * v0 + 1e-3 * g64 * g64) + 1e-30
        flat = lambda parts: np.concatenate([np.ravel(a) for pr in parts for a in pr])
        keep = flat(sh(np.arange(net.n_params))).astype(np.int64)
        for name, r, q, tol in (("params", flat(ref_p), got_p[keep], tol_p),
                                ("m", flat(ref_m), got_m[keep], tol_m[keep]),
                                ("v", flat(ref_v), got_v[keep], tol_v[keep])):
            excess = np.abs(q - r) - tol
            assert np.all(excess <= 0), (i, name, int((excess > 0).sum()), float(excess.max()))
        upd = got_p - p0
        say(f"  step {i}: lr {lr:.3e}, loss {loss_t:.6f} (oracle {ref_loss:.6f}), "
            f"mean |update| / lr {np.abs(upd[~pad]).mean() / lr:.3f}")
        assert not got_p[pad].any()
    np.testing.assert_array_equal(net.get(7), [steps, steps])


def test_training_checkpoint_resumes_bit_identically(t):
    """Six steps in one run versus three steps, a checkpoint (parameters,
    AdamW moments, step counter, schedule length) restored into a fresh
    network, and three more: the parameters are bit-identical, because the
    batches, learning rates and bias corrections follow the step counter and
    the split-K gradient sums run in a fixed order."""
    say("mlp checkpoint / resume B=2048")
    B, K = 2048, 24
    plan = t.Plan(32, 32, 1, 64, 64, basis_k=K)
    z = torch.tensor(synthetic.random_coefficients((4 * B, 35), 0.7, 21), device="cuda")
    tgt = torch.tensor(synthetic.random_coefficients((4 * B, K), 1.0, 22), device="cuda")
    a = t.Mlp(plan, batch=B, seed=3)
    a.set(7, [0, 6])
    a.train(z, tgt, 6, lr_max=2e-3, lr_min=1e-4)
    b = t.Mlp(plan, batch=B, seed=3)
    b.set(7, [0, 6])
    b.train(z, tgt, 3, lr_max=2e-3, lr_min=1e-4)
    ck = b.checkpoint()
    b.close()
    c = t.Mlp(plan, batch=B, seed=99)          # different initialisation, overwritten
    c.restore(ck)
    c.train(z, tgt, 3, lr_max=2e-3, lr_min=1e-4)
    np.testing.assert_array_equal(c.get(0), a.get(0))
    np.testing.assert_array_equal(c.get(5), a.get(5))
    np.testing.assert_array_equal(c.get(7), [6, 6])
    # and a repeat of the whole run is bit-identical
    d = t.Mlp(plan, batch=B, seed=3)
    d.set(7, [0, 6])
    d.train(z, tgt, 6, lr_max=2e-3, lr_min=1e-4)
    np.testing.assert_array_equal(d.get(0), a.get(0))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_learned_plan_without_network_falls_back_to_exact(t, basis, precision):
    """A learned plan that holds no network runs the exact path (Eq. (2)
    PSFs projected by Eq. (7)), says so through tsim_p2s_form, and writes
    the plan's weight layout: float32 [F][H][W][K], or bfloat16 [F][H][W][KP]
    with zero padding, each weight the FP32 projection rounded once."""
    say(f"learned plan without network: exact fallback ({precision})")
    H, W = 24, 40
    bf = precision == "bf16"
    plan = t.Plan(H, W, 1, 64, 64, basis=basis, p2s_mode=t.P2S_LEARNED,
                  precision=t.BF16 if bf else t.FP32)
    assert plan.p2s_form() == t.P2S_EXACT
    z32 = synthetic.random_coefficients((1, 35, H, W), 0.5, 23)
    KB = 112 if bf else 100
    beta = torch.zeros((1, H, W, KB), dtype=torch.bfloat16 if bf else torch.float32, device="cuda")
    plan.p2s(torch.tensor(z32, device="cuda"), beta, plan.workspace(1))
    torch.cuda.synchronize()
    got = beta.float().cpu().numpy()[0]
    ref = opsf.psf_field(z32[0].astype(np.float64), 64, 33, basis)
    if bf:
        assert np.all(got[..., 100:] == 0)
        got = got[..., :100]
        # round to nearest bfloat16: within half a unit (2^-9 relative) of
        # the FP32 value, itself within 1e-5 of the oracle
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())
    else:
        assert err(got, ref) < 1e-5
    net = t.Mlp(plan, batch=64, seed=5)
    t.plan_set_mlp(plan, net)
    assert plan.p2s_form() == t.P2S_LEARNED
