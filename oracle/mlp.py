"""The P2S network: forward and backward in float64 (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II-C: a small neural network maps each pixel's Zernike vector a_x to its
PSF-basis weights beta_x.  The paper gives no architecture; the reading used
here is a multilayer perceptron 35 -> 256 -> 256 -> 256 -> K with the exact
(erf) GELU, GELU(z) = z Phi(z), on standardised inputs (the two tilt slots
zeroed: tilt is applied as a warp), trained by mean squared error on the
weights (equal to the L2 error of the reconstructed PSF because the basis is
orthonormal).

``bf16=True`` mirrors a BF16 implementation: every GEMM operand (inputs,
activations, weights, back-propagated gradients) is rounded to bfloat16 at
the same points as the GPU kernels, with products accumulated exactly
(float64 here, float32 on the GPU) and biases, pre-activations and the
loss kept in full precision.
"""
import numpy as np
from scipy import special

LAYERS = 4


def to_bf16(x):
    """Round to bfloat16 (nearest, ties to even) via binary32, as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return z * 0.5 * (1.0 + special.erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)


def forward(params, x, bf16=False):
    """params: list of (W [out, in], b [out]); x [B, in].  Returns the output
    [B, out] and the cache for backward.  GELU after every layer but the
    last."""
    r = to_bf16 if bf16 else (lambda v: v)
    acts = [r(x)]
    zs = []
    h = acts[0]
    for i, (W, b) in enumerate(params):
        z = h @ r(W).T + b
        zs.append(z)
        if i < len(params) - 1:
            h = r(gelu(z))
            acts.append(h)
        else:
            h = z
    return h, (acts, zs)


def loss_and_grads(params, x, target, bf16=False):
    """MSE = mean over batch and outputs of (y - target)^2 and its gradients
    [(dW, db)] by back-propagation."""
    r = to_bf16 if bf16 else (lambda v: v)
    y, (acts, zs) = forward(params, x, bf16)
    B, K = y.shape
    diff = y - target
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / (B * K)
    grads = [None] * len(params)
    for i in reversed(range(len(params))):
        W, _ = params[i]
        dzr = r(dz)
        grads[i] = (dzr.T @ acts[i], dz.sum(axis=0))
        if i > 0:
            da = dzr @ r(W)
            dz = da * gelu_grad(zs[i - 1])
    return loss, grads


def adamw_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update of FP64 master weights; ``state`` holds (t, m, v)."""
    t, m, v = state
    t += 1
    new_params, new_m, new_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        out = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** t)
            vh = vv / (1 - beta2 ** t)
            p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
            out.append((p, mm, vv))
        new_params.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_params, (t, new_m, new_v)


def init_state(params):
    z = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    return 0, z, [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
