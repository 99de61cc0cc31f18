"""Error measures shared by the GPU parity tests.

rel    : relative L2 error ||got - ref|| / ||ref|| of one array (a coefficient
         plane, a PSF, a weight array, an image).
maxrel : largest element error relative to the largest reference magnitude,
         max |got - ref| / max |ref|.  A single wrong pixel (a halo, seam or
         ragged-edge defect) that the L2 norm averages away shows up here.
err    : the larger of the two; FP32 parity bounds apply to both at once.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def err(a, b):
    return max(rel(a, b), maxrel(a, b))
