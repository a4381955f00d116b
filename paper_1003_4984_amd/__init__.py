"""MI355X-native FLINTS: kriging interpolation of spin-0 and spin-2 HEALPix maps.

The compute path is the HIP library libflints.so (C ABI in include/flints.h);
this package only marshals arguments to it.  Importing the package does not load
the library; the first call does, and raises if it has not been built.
"""
from .flints import (  # noqa: F401
    Plan, Batch, FlintsError, load_library, interpolate, interpolate_tqu, supersample, pixel_centres, tqu_shared,
    stencil, table_eval, BATCH_AUTOTUNE, synthesize, lensed_directions, lens_tqu, alm_mmajor,
    FP64, FP32_IR, S2_FULL, S2_PAPER, NUG_ALWAYS, NUG_ON_FAILURE, VAR_PAPER, VAR_MSE,
    STENCIL_NEAREST, STENCIL_PIXEL, MAP_F64, MAP_F32,
)
