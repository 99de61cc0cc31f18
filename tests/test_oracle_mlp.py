"""Pins for the oracle's P2S network: back-propagated gradients against
central finite differences in float64, the erf-GELU against its closed
forms, bfloat16 rounding against exhaustive definitions, and AdamW against
a hand-computed first step."""
import numpy as np

from oracle import mlp


def _params(rng, dims):
    return [(rng.standard_normal((o, i)) / np.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(dims[:-1], dims[1:])]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    dims = [7, 12, 9, 11, 5]
    params = _params(rng, dims)
    x = rng.standard_normal((6, 7))
    tgt = rng.standard_normal((6, 5))
    _, grads = mlp.loss_and_grads(params, x, tgt)
    h = 1e-6
    for li in range(len(params)):
        W, b = params[li]
        for (a, c) in [(0, 0), (2, 3), (W.shape[0] - 1, W.shape[1] - 1)]:
            Wp = W.copy(); Wp[a, c] += h
            Wm = W.copy(); Wm[a, c] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (mlp.loss_and_grads(pp, x, tgt)[0] - mlp.loss_and_grads(pm, x, tgt)[0]) / (2 * h)
            assert abs(fd - grads[li][0][a, c]) < 1e-7 * max(1.0, abs(fd)), (li, a, c)
        for a in [0, b.shape[0] - 1]:
            bp = b.copy(); bp[a] += h
            bm = b.copy(); bm[a] -= h
            pp = list(params); pp[li] = (W, bp)
            pm = list(params); pm[li] = (W, bm)
            fd = (mlp.loss_and_grads(pp, x, tgt)[0] - mlp.loss_and_grads(pm, x, tgt)[0]) / (2 * h)
            assert abs(fd - grads[li][1][a]) < 1e-7 * max(1.0, abs(fd)), (li, a)


def test_gelu_closed_forms():
    # GELU(0) = 0, GELU(z) - GELU(-z) = z, GELU'(0) = 1/2, large-z limits
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-14)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15
    np.testing.assert_allclose(mlp.gelu(np.array([30.0])), [30.0], rtol=1e-15)
    # derivative against a central difference
    h = 1e-6
    np.testing.assert_allclose((mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), mlp.gelu_grad(z), atol=1e-8)


def test_bf16_rounding():
    # exactly representable values are kept; halfway cases round to even
    x = np.array([1.0, -2.5, 0.0, 1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.0e38])
    got = mlp.to_bf16(x)
    assert got[0] == 1.0 and got[1] == -2.5 and got[2] == 0.0
    assert got[3] == 1.0 + 2 ** -7          # representable (7 mantissa bits)
    assert got[4] == 1.0                    # tie -> even (mantissa 0)
    assert got[5] == 1.0 + 2 ** -6          # tie -> even (mantissa 2)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(10000)
    err = np.abs(mlp.to_bf16(v) - v) / np.abs(v)
    assert err.max() <= 2 ** -8 * (1 + 1e-6)


def test_adamw_first_step():
    """After one step with zero moments, AdamW moves each weight by
    -lr * g/(|g| + eps) (bias correction makes m_hat = g, v_hat = g^2)."""
    rng = np.random.default_rng(2)
    params = _params(rng, [3, 4, 2])
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    new, state = mlp.adamw_step(params, grads, mlp.init_state(params), lr=1e-2)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        np.testing.assert_allclose(W1 - W, -1e-2 * gW / (np.abs(gW) + 1e-8), rtol=1e-9)
        np.testing.assert_allclose(b1 - b, -1e-2 * gb / (np.abs(gb) + 1e-8), rtol=1e-9)
    assert state[0] == 1


def test_bf16_mirror_close_to_fp64():
    rng = np.random.default_rng(3)
    params = _params(rng, [35, 64, 64, 64, 20])
    x = rng.standard_normal((32, 35))
    y64, _ = mlp.forward(params, x)
    y16, _ = mlp.forward(params, x, bf16=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 3e-2
