"""MI355X (gfx950) w-projection imaging: Python binding of libwproj.so.

The compute path is the HIP library built from csrc/ (see include/wproj.h for
the C ABI); this package only marshals torch tensors into it.
"""

from .wproj import (  # noqa: F401
    ALGO_PLAIN,
    ALGO_TILED,
    F32,
    F32_F16TABLE,
    F64,
    GRID_TO_IMAGE,
    GRID_TO_IMAGE_RAW,
    IMAGE_TO_GRID,
    Kernels,
    Plan,
    WprojError,
    autotune,
    check_weights,
    chi2,
    degrid,
    footprints,
    gather_rows,
    grid,
    grid_noalloc,
    image,
    last_error,
    make_kernels,
    measure_lds,
    measure_vmem,
    noalloc_scratch_bytes,
    regroup_channels,
    regroup_rows,
    version,
)
