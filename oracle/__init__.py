"""CPU FP64 oracle for the dilated differentiable Gaussian-splat rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it and shares no code with it; a missing HIP build must fail loudly and
never fall back to anything in here.

Everything is plain PyTorch on the CPU in float64, written to be read against
the paper (Turbo-GS, arXiv 2412.13547):

* ``sh``          real spherical-harmonic basis, degree 0..3 (colour model, Sec. 3)
* ``preprocess``  3D covariance, EWA projection, low-pass, radius, colour
                  (Sec. 3 Eq. 1; Sec. 4.1 on the original focal length)
* ``binning``     downsampled centres / radii, tile rectangles, (tile | depth)
                  keys, stable sort, per-tile ranges (Sec. 4.1 Eq. 3-4)
* ``raster``      front-to-back compositing of Sec. 3 Eq. 2 on the dilated
                  pixel set (Sec. 4.1 Eq. 5 and the offset scheme of Fig. 2)
* ``loss``        L1 loss against the full-resolution pixels that were rendered
* ``backward``    gradients by reverse-mode differentiation of the forward,
                  and the per-Gaussian densification statistics of Sec. 4.3
* ``pipeline``    the stages chained end to end

Readings of passages that the paper leaves open are listed in the module that
implements them.  No function here has "parity unpinned" status: each is pinned
by the CPU tests (closed forms, library routines, brute force, invariants and
central finite differences).
"""

from . import sh, preprocess, binning, raster, loss, backward, pipeline  # noqa: F401
