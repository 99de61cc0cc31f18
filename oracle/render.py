"""Image formation: basis blur, gather-form blur and tilt warp (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Eq. (8): I(x) = sum_m beta_{x,m} (varphi_m conv I_g)(x) -- K spatially
invariant convolutions and a per-pixel weighted sum.  Eq. (1): the gather form
I(x) = (h_x conv I_g)(x) keeping only the centre pixel.  Readings: a true
convolution (kernel flipped), offsets u in [-r, r]^2 with r = (T-1)/2, image
boundary replicated (clamped); the tilt modes (Noll 2, 3) act as a bilinear
backward warp applied after the blur, with displacement t = -(4/pi)(a_2, a_3)
pixels: a pure tilt a_2 moves the Eq. (2) PSF by -4 a_2/pi samples along x,
and one PSF sample is one pixel.
"""
import numpy as np
from scipy import signal

TILT_PIX_PER_RAD = -4.0 / np.pi


def basis_convolutions(img, Psi, T):
    """(varphi_m conv I)(x) for every m, replicate boundary: (K, H, W)."""
    r = (T - 1) // 2
    pad = np.pad(img, r, mode='edge')
    out = []
    for m in range(Psi.shape[0]):
        k = Psi[m].reshape(T, T)
        out.append(signal.fftconvolve(pad, k, mode='valid'))
    return np.stack(out)


def render_basis(img, beta, Psi, T):
    """Eq. (8) for one channel: img (H, W), beta (H, W, K) -> (H, W)."""
    conv = basis_convolutions(img, Psi, T)
    return np.einsum('hwk,khw->hw', beta, conv)


def render_gather(img, psfs, T):
    """Eq. (1) literally: every output pixel x uses its own T x T PSF h_x
    (psfs (H, W, T, T), h_x[r + uy, r + ux] is the weight of offset u) and
    I(x) = sum_u h_x(u) I_g(clamp(x - u))."""
    H, W = img.shape
    r = (T - 1) // 2
    out = np.zeros((H, W))
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    for uy in range(-r, r + 1):
        for ux in range(-r, r + 1):
            yy = np.clip(ys - uy, 0, H - 1)
            xx = np.clip(xs - ux, 0, W - 1)
            out += psfs[:, :, r + uy, r + ux] * img[yy, xx]
    return out


def tilt_shift(zern):
    """Per-pixel displacement (tx, ty) in pixels from Noll 2 (x) and 3 (y)."""
    return TILT_PIX_PER_RAD * zern[0], TILT_PIX_PER_RAD * zern[1]


def warp(img, tx, ty):
    """O(x) = bilinear(B, x - t_x), the four taps clamped to the image."""
    H, W = img.shape
    ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing='ij')
    px = xs - tx
    py = ys - ty
    x0 = np.floor(px)
    y0 = np.floor(py)
    fx = px - x0
    fy = py - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    x0c = np.clip(x0, 0, W - 1)
    x1c = np.clip(x0 + 1, 0, W - 1)
    y0c = np.clip(y0, 0, H - 1)
    y1c = np.clip(y0 + 1, 0, H - 1)
    return ((1 - fy) * ((1 - fx) * img[y0c, x0c] + fx * img[y0c, x1c])
            + fy * ((1 - fx) * img[y1c, x0c] + fx * img[y1c, x1c]))


def render_at(img, beta_px, Psi, T, ys, xs):
    """Eq. (8) at the listed pixels only, for frames too large to blur whole:
    I(x) = sum_m beta_{x,m} sum_u varphi_m(u) I_g(clamp(x - u)).
    img (H, W); beta_px (n, K) holds the weights of pixel (ys[i], xs[i])."""
    H, W = img.shape
    r = (T - 1) // 2
    u = np.arange(-r, r + 1)
    out = np.empty(len(ys))
    for i, (y, x) in enumerate(zip(ys, xs)):
        yy = np.clip(y - u, 0, H - 1)[:, None]
        xx = np.clip(x - u, 0, W - 1)[None, :]
        patch = img[yy, xx].reshape(-1)          # I(x - u), u row-major like varphi_m
        conv = Psi @ patch                        # (varphi_m conv I)(x) for every m
        out[i] = float(np.dot(beta_px[i], conv))
    return out


def warp_at(img, tx_px, ty_px, ys, xs):
    """The bilinear backward warp at the listed pixels; tx_px, ty_px are the
    displacements of those pixels."""
    H, W = img.shape
    px = np.asarray(xs, np.float64) - tx_px
    py = np.asarray(ys, np.float64) - ty_px
    x0 = np.floor(px)
    y0 = np.floor(py)
    fx = px - x0
    fy = py - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    x0c = np.clip(x0, 0, W - 1)
    x1c = np.clip(x0 + 1, 0, W - 1)
    y0c = np.clip(y0, 0, H - 1)
    y1c = np.clip(y0 + 1, 0, H - 1)
    return ((1 - fy) * ((1 - fx) * img[y0c, x0c] + fx * img[y0c, x1c])
            + fy * ((1 - fx) * img[y1c, x0c] + fx * img[y1c, x1c]))


def render_frame(img, zern, beta, Psi, T):
    """Blur then warp for a multi-channel frame: img (C, H, W)."""
    tx, ty = tilt_shift(zern)
    out = []
    for c in range(img.shape[0]):
        b = render_basis(img[c], beta, Psi, T)
        out.append(warp(b, tx, ty))
    return np.stack(out)
