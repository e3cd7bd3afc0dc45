"""MI355X-native ray casting of editable two-layer height-column terrain.

The product is libtc.so (HIP kernels for gfx950 behind the C ABI of
include/tc.h); this package holds its sources (csrc/), its build step
(build.py) and a thin ctypes binding (_tc.py) with the same names.
"""
from ._tc import (Context, Frame, Server, TCError, tc_create, tc_view, tc_edit, render,
                  split_hits, view_total_rays, view_struct, views_struct, edits_struct, load_library, LIB_PATH,
                  SIGNATURES, TC_OK, TC_INVALID_ARG, TC_OUT_OF_MEMORY,
                  TC_NO_MAP, TC_DEVICE_ERROR, TC_OVER_BUDGET, TC_TIMEOUT,
                  TC_SERVER_AUTO_RELEASE, TC_MISS, TC_S, TC_MAX_DIM, TC_MAX_CELLS,
                  TC_MAX_DIR, TC_FACE_TOP, TC_FACE_UNDER, TC_FACE_WMX, TC_FACE_WPX,
                  TC_FACE_WMY, TC_FACE_WPY, TC_FACE_INSIDE,
                  TC_EDIT_SET, TC_EDIT_CRATER, TC_OPT_RENDER_MODE,
                  TC_OPT_START_LEVEL, TC_OPT_MAX_LEVEL, TC_OPT_XCD_REMAP,
                  TC_OPT_PERSIST_WAVES, TC_OPT_REFILL_MIN,
                  TC_OPT_REFILL_ITERS, TC_OPT_COUNT_READS,
                  TC_OPT_TILE_ORDER, TC_OPT_PRIORITY_BOOST, TC_OPT_SPLIT_BUDGET,
                  TC_OPT_SPLIT_QUEUE, TC_OPT_KERNEL_TIMING,
                  TC_OPT_MARCH_STEPS, TC_OPT_MARCH_BISECT, TC_OPT_MARCH_FAR,
                  TC_OPT_BEAM_PASSES, TC_OPT_SPLIT_WAVES, TC_INFO_ALLOCATIONS,
                  TC_OPT_PACKET_WIDTH, TC_OPT_VOXEL_SHAPE, TC_OPT_INLINE_TABLES,
                  TC_FACE_SAMPLED)
