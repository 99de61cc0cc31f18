"""Philox4x32-10 and Gaussian white noise (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper draws white noise e ~ N(0, I) and colours it (Sec. III-A).  It does
not fix a generator, so this project uses the counter-based Philox4x32-10 of
Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
(SC'11), implemented here from that paper's description: a 4x32-bit counter
and a 2x32-bit key; each round multiplies counter words 0 and 2 by two fixed
constants, takes the 64-bit products' high and low halves, and recombines them
with the other two words and the key by XOR; the key is bumped by two Weyl
constants between rounds.  The GPU implements the same published definition
independently, so both sides draw identical 32-bit words.

Project conventions (shared *definitions*, not code):

* key = (seed & 0xffffffff, seed >> 32).
* counter = (c0, c1, c2, c3); the sampler uses c0 = canonical linear bin index,
  c1 = field index q, c2 = frame index, c3 = stream tag.
* uniform from a 32-bit word x: u = ((x >> 9) + 0.5) * 2**-23, in (0, 1) and
  exactly representable in binary32, so both sides start Box-Muller from the
  same number.
* Box-Muller: r = sqrt(-2 ln u0), g0 = r cos(2 pi u1), g1 = r sin(2 pi u1);
  words (x2, x3) give (g2, g3) the same way.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

TAG_SAMPLER = 0
TAG_BASIS = 1
TAG_MLP_DATA = 2
TAG_MLP_INIT = 3
TAG_IMAGE = 4
TAG_SUBHARMONIC = 5


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on broadcastable uint32 counter arrays.

    Returns four uint32 arrays.  Arithmetic is carried in uint64 so that the
    32x32 -> 64 bit products are exact.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform(x):
    """Map uint32 words to (0, 1): ((x >> 9) + 0.5) * 2^-23, in float64."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def box_muller(x0, x1):
    """Two standard normals from two uint32 words (float64 arithmetic)."""
    u0 = uniform(x0)
    u1 = uniform(x1)
    r = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * np.pi * u1
    return r * np.cos(ang), r * np.sin(ang)


def gaussians4(c0, c1, c2, c3, seed):
    """Four N(0,1) arrays (g0, g1, g2, g3) for the given counters."""
    k0, k1 = seed_key(seed)
    x0, x1, x2, x3 = philox4x32_10(c0, c1, c2, c3, k0, k1)
    g0, g1 = box_muller(x0, x1)
    g2, g3 = box_muller(x2, x3)
    return g0, g1, g2, g3


def gaussian_vectors(n_vec, n_dim, c2, tag, seed):
    """n_vec independent N(0, I_n_dim) vectors, shape (n_vec, n_dim).

    Vector i uses counters (i, w, c2, tag) for w = 0 .. ceil(n_dim/4)-1;
    component 4w+t is the t-th Gaussian of call w.  Used for per-sample draws
    (basis database, MLP training pairs).
    """
    n_call = (n_dim + 3) // 4
    i = np.arange(n_vec, dtype=np.uint64)[:, None]
    w = np.arange(n_call, dtype=np.uint64)[None, :]
    g = gaussians4(i, w, c2, tag, seed)
    out = np.stack(g, axis=-1).reshape(n_vec, n_call * 4)
    return out[:, :n_dim]


def uniforms_extra(n_vec, word_index, c2, tag, seed):
    """Per-vector uniform in (0,1) from word 0 of call (i, word_index, c2, tag)."""
    k0, k1 = seed_key(seed)
    i = np.arange(n_vec, dtype=np.uint64)
    x0, _, _, _ = philox4x32_10(i, word_index, c2, tag, k0, k1)
    return uniform(x0)
