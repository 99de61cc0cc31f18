"""FP64 CPU oracle for the dense-field phase-to-space (DF-P2S) renderer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark use it.  The oracle shares no code, tables or constants with the GPU
path: every quantity is recomputed here from the paper's definitions in
float64 with numpy/scipy.

Modules (each function cites the passage of the paper it follows):

* ``philox``   -- Philox4x32-10 counter-based generator (Salmon et al., SC'11)
                  and the Box-Muller mapping; the white noise e ~ N(0, I) of
                  Sec. III-A.
* ``zernike``  -- Noll indexing, Zernike polynomials (Sec. II-B, Eq. (5)),
                  their Fourier transforms and the Noll covariance A_0
                  (Sec. II-B, Eq. (6) at s = 0; Sec. III-B).
* ``spectra``  -- per-mode homogeneous spectra of the autocovariances A_ii
                  (Sec. III-B, III-C) and the Kolmogorov constant of Eq. (4).
* ``sampler``  -- DF-P2S field generation: FFT colouring of N unit-variance
                  fields followed by per-pixel mixing with L, L L^T = A_0
                  (Sec. III-A, III-C, Eq. (9)); full-tensor sampling on tiny
                  grids and the energy functions of Eqs. (10)-(12).
* ``psf``      -- exact pupil-FFT PSFs (Eq. (2)), the PCA PSF basis (Eq. (7))
                  and exact projection onto it.
* ``render``   -- basis-weighted blur (Eq. (8)), gather-form spatially varying
                  convolution (Eq. (1)) and the tilt warp.
* ``mlp``      -- FP64 forward/backward of the P2S network (Sec. II-C).
* ``stats``    -- validation statistics of Sec. IV-B: tilt correlation
                  and differential tilt variance against pixel lag; the
                  phase structure function over the aperture (Eq. (4)).
"""
