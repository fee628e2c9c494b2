"""Dilated differentiable Gaussian-splat rasterizer for AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library ``libtgs.so`` built from ``csrc/`` (HIP).
``api`` is its thin Python binding; ``scenes`` draws seeded synthetic inputs.
Importing the package loads nothing; the library is loaded on first use of
``api`` and a missing build raises instead of falling back to anything else.
"""
__all__ = ["api", "autotune", "scenes"]
