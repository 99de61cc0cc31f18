"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds none of the renderer's arithmetic: it only makes input
images and per-frame turbulence strengths.  The paper's photographs,
heat-chamber frames and 4K test image are not available, so images are a
seeded mix of uniform noise and a checkerboard (edges at every scale the blur
acts on), and D/r0 values are drawn from the ranges the workloads name.
"""
import numpy as np


def test_image(C, H, W, square, seed):
    """I = 0.5 U[0,1) + 0.5 checker, float32 (C, H, W).

    The checkerboard has ``square``-pixel cells and a seeded phase offset;
    the noise is numpy's PCG64 stream for ``seed``."""
    rng = np.random.default_rng(seed)
    oy, ox = rng.integers(0, 2 * square, size=2)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing='ij')
    checker = (((ys + oy) // square + (xs + ox) // square) % 2).astype(np.float64)
    noise = rng.random((C, H, W))
    return (0.5 * noise + 0.5 * checker[None]).astype(np.float32)


def d_over_r0_uniform(n, lo, hi, seed):
    """Per-frame turbulence strengths D/r0 ~ U[lo, hi), float32."""
    rng = np.random.default_rng(seed + 7919)
    return (lo + (hi - lo) * rng.random(n)).astype(np.float32)


def random_coefficients(n, scale, seed):
    """Generic N(0, scale^2) float32 array of shape n (weights, test betas)."""
    rng = np.random.default_rng(seed + 104729)
    return (scale * rng.standard_normal(n)).astype(np.float32)


def index_map(H, W, n, seed):
    """Seeded int64 map (H, W) of row indices into an n-row table: gives a
    full-size frame of per-pixel inputs (weights, coefficient vectors) from a
    small random table."""
    rng = np.random.default_rng(seed + 15485863)
    return rng.integers(0, n, size=(H, W))
