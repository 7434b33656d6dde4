"""Seeded synthetic workloads (velocity, reflectivity, acquisition geometry,
noise and test vectors) shared by the oracle tests, the GPU tests and the
benchmark.

This package describes inputs only. It contains none of the method's
arithmetic (no wavelet, stencil, sponge, propagation or solver); both the GPU
library and the CPU oracle implement those themselves.
"""
from .configs import (  # noqa: F401
    Workload,
    Shot,
    SsfShot,
    SsfWorkload,
    ssf_small,
    ssf2d_256x1024,
    layers2d_64x64,
    faulted2d_512x1024,
    layered3d_256x320x320,
    model_at,
    noise_like,
    stream2d_512x1024,
    streaming,
    tiny2d,
    tiny3d,
    rng,
    gaussian,
)
