"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds only input generation: random-ellipse and Gaussian-blob
phantoms, their closed-form line integrals (the physics the tomography
operator approximates, Sec. 2), and Beer-Lambert / Poisson measurement noise.
It contains none of the sparse Fubini-Radon arithmetic, and it imports neither
the oracle nor the GPU package.
"""

from .phantoms import (  # noqa: F401
    PIXEL_UNIT_DISK,
    ellipse_params,
    rasterize_ellipses,
    ellipse_sinogram,
    gaussian_blobs_image,
    gaussian_blobs_sinogram,
    poisson_log_sinogram,
    phantom_stack,
    slice_rng,
)
