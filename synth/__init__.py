"""Seeded synthetic microscopy-like inputs shared by the tests, the benchmark
and the smoke check.

This module holds none of the deconvolution arithmetic: it renders objects
(points, Gaussian blobs, tubular filaments), samples Gaussian PSFs and draws
photon and read noise.  Blurring an object is left to the caller (the oracle
in tests, the library in the benchmark), which passes the blurred image to
`add_noise`.

Shapes are (z, y, x), C order, x contiguous.  The paper's own test images are
not used: these inputs stand in for them with the paper's shapes, value ranges
and structure (point sources, blobs and filaments on a dim background, blurred
by Gaussian PSFs, with photon and read noise).
"""
from .volumes import (CONFIGS, PAPER_2D, SWEEP_PSFS, VolumeConfig, add_noise, batched_configs, crossing_lines,
                      flat_start, gaussian_factors, gaussian_noise, gaussian_psf, make_objects, piecewise_image,
                      psf_for, stable_seed)

__all__ = ["CONFIGS", "PAPER_2D", "SWEEP_PSFS", "VolumeConfig", "add_noise", "batched_configs", "crossing_lines",
           "flat_start", "gaussian_factors", "gaussian_noise", "gaussian_psf", "make_objects", "piecewise_image",
           "psf_for", "stable_seed"]
