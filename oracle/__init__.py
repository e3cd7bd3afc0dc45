"""CPU oracle of the two-layer terrain ray cast -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library:
  core.py        ctypes front end of oracle.c (exact flat cell walk, fp64 depth)
                 and march.c (the sampled march of Section 3.1 in fp32)
                 and shade.c (palette, gradient normal, shadow ray, fog)
  edits.py       SET / CRATER edit semantics on numpy planes
  pyramid.py     the min/max pyramid, the occupancy masks, the window
                 levels and the voxel occupancy pyramid, written as their
                 definitions
  bruteforce.py  every box of every cell in exact rationals (tiny maps)
"""
from .core import (render, cast_rays, cast_rays_exact, cast_pixels, decode,
                   march, march_rays, march_pixels, shade, shade_pixels, MISS,
                   VIEW_DT, lib)
from .edits import apply_edits, valid_columns, EDIT_SET, EDIT_CRATER
from .pyramid import (pyramid_level, pyramid_level_fast, occupancy_level, window_level,
                      window_level_fast, voxel_dims, voxel_levels, voxel_level_direct)
from . import bruteforce

__all__ = ["render", "cast_rays", "cast_rays_exact", "cast_pixels", "decode",
           "march", "march_rays", "march_pixels", "shade", "shade_pixels",
           "MISS", "VIEW_DT", "lib", "apply_edits", "valid_columns",
           "EDIT_SET", "EDIT_CRATER", "pyramid_level", "pyramid_level_fast",
           "occupancy_level", "window_level", "window_level_fast", "voxel_dims",
           "voxel_levels", "voxel_level_direct",
           "bruteforce"]
