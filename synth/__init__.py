"""Seeded synthetic inputs for the PSF-library operator.

This package only *generates data*: coronagraph-like off-axis PSF cubes,
radial sample offsets and exozodi/planet scenes.  It contains none of the
operator's arithmetic (no radial interpolation, no rotation, no products),
so the FP64 oracle and the HIP path can both be fed from it without sharing
any of the method.
"""
from .inputs import (  # noqa: F401
    SEED_ROOT, STREAM_ABERR, STREAM_DISK, STREAM_PLANETS, STREAM_NOISE,
    STREAM_SUBSAMPLE, STREAM_BATCH, CONFIGS, rng_for, radii_linspace,
    radii_nonuniform, throughput, psf_cube, ring_scene, planets, add_planets,
    random_ring_params, scene_batch, config_inputs, DISK_TRUE, DISK_START, noisy_counts,
    MIXED_SIZES, MIXED_WAVELENGTHS, mixed_workload,
)
