"""Writes batch_768x1024_frame.txt: the oracle's coefficient vector and
output pixel values (blur of Eq. (8) with exact projected PSFs, then the
tilt warp) at sampled pixels of one 768 x 1024 x 3 frame on a 2048 x 2048
sampling grid (the largest frame size of the mixed-size batch), for the
batch test's inputs: seed 5, frame counter 20, D/r0 2.5, pixel pitch D/8,
the test's 100-vector basis of 33 x 33 PSFs from 600 seeded draws, and
image ``synthetic.test_image(3, 768, 1024, 16, 768)``.  Calls only
``oracle/`` (and ``synthetic`` for the inputs); the 2048^2 spectra of every
mode take about a minute in numpy, which is why the GPU test reads this
file.

    python tests/golden/make_batch_768x1024.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import psf as opsf  # noqa: E402
from oracle import render as orender  # noqa: E402
from oracle import sampler as osamp  # noqa: E402
import synthetic  # noqa: E402

H, W, G, DS, DR, SEED, FRAME, T, P = 768, 1024, 2048, 0.125, 2.5, 5, 20, 33, 64


def test_basis():
    A, _ = opsf.basis_draws(600, seed=31)
    return opsf.pca_basis(opsf.psf_batch(A, P, T), 100)[0]


def sampled_pixels():
    rng = np.random.default_rng(768)
    pts = {(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (0, W // 2), (H - 1, W // 2),
           (H // 2, W - 1), (1, 1), (383, 511), (384, 512), (255, 767), (511, 256)}
    pts |= {(int(y), int(x)) for y, x in zip(rng.integers(0, H, 40), rng.integers(0, W, 40))}
    return np.array(sorted(pts)).T


def main():
    Psi = test_basis()
    img = synthetic.test_image(3, H, W, 16, 768).astype(np.float64)
    zern = osamp.sample_zernike(H, W, G, G, DS, DR, SEED, FRAME)          # (35, H, W)
    ys, xs = sampled_pixels()
    tx, ty = orender.tilt_shift(zern)
    # the warp reads the blurred frame at the four bilinear taps of each
    # sampled pixel; the blur there needs only that tap's own weights
    taps = set()
    for y, x in zip(ys, xs):
        py, px = y - ty[y, x], x - tx[y, x]
        y0, x0 = int(np.floor(py)), int(np.floor(px))
        for yy in (y0, y0 + 1):
            for xx in (x0, x0 + 1):
                taps.add((min(max(yy, 0), H - 1), min(max(xx, 0), W - 1)))
    ty_, tx_ = np.array(sorted(taps)).T
    beta = opsf.project(opsf.psf_batch(zern[:, ty_, tx_].T, P, T), Psi)
    out = np.empty((3, len(ys)))
    for c in range(3):
        blur = np.zeros((H, W))
        blur[ty_, tx_] = orender.render_at(img[c], beta, Psi, T, ty_, tx_)
        out[c] = orender.warp_at(blur, tx[ys, xs], ty[ys, xs], ys, xs)
    rows = np.column_stack([ys, xs, zern[:, ys, xs].T, out.T])
    header = (f"oracle values at sampled pixels of one {H}x{W}x3 frame, grid {G}x{G}, pitch {DS} D, "
              f"D/r0 {DR}, seed {SEED}, frame {FRAME}, K=100 T={T} P={P}\n"
              "columns: y, x, zern Noll 2..36 (35), out channels 0..2 (3)\n"
              "written by tests/golden/make_batch_768x1024.py from oracle/")
    np.savetxt(os.path.join(HERE, "batch_768x1024_frame.txt"), rows, fmt="%.17e", header=header)


if __name__ == "__main__":
    main()
