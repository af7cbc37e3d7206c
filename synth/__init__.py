"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package produces inputs only: antenna layouts, Earth-rotation (u,v,w)
tracks, point-source skies and the visibilities they give, and model images.
It holds none of the imaging method's arithmetic (no kernels, no gridding,
no FFTs, no corrections), so the FP64 oracle and the GPU path can both consume
its output without sharing any code.
"""

from .workloads import (  # noqa: F401
    Workload,
    area_uniform_disk,
    array_tracks,
    point_source_vis,
    support_ramp,
    kernel_image_size_rule,
    cfg1,
    cfg1w,
    cfg2,
    cfg3,
    cfg4,
    cfg5_model_image,
    cfg5,
    small_tracks,
)
