"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package draws random numbers and lays out inputs (maps, camera views as
integer ray parameters, edit lists, request arrival times). It contains none
of the ray-casting arithmetic: neither the per-pixel ray generation, nor the
traversal, nor the edit semantics. Both the CPU oracle and the HIP library
consume exactly the integers produced here.

The paper measures on the 2048x16384 "Fostral" level of Vangers (Section 2),
which is not available here; the seeded maps below stand in for it with the
same shape, the same two-interval column encoding and a comparable share of
double-level cells.
"""
from .configs import CONFIGS, SEEDS, config
from .maps import make_map, make_map_from_config, pack_columns_check, cave_map
from .views import (S, MAX_DIR, VIEW_DTYPE, perspective_view, ortho_view,
                    shadow_view, views_array, config_views, view_rays,
                    batched_views, request_view, eye_above_floor, pitch_views)
from .edits import crater_list, random_set_patches, EDIT_CRATER, EDIT_SET
from .arrivals import poisson_arrivals
from .palette import default_palette, rgba

__all__ = [
    "CONFIGS", "SEEDS", "config", "make_map", "make_map_from_config", "cave_map",
    "pack_columns_check", "S", "MAX_DIR", "VIEW_DTYPE", "perspective_view",
    "ortho_view", "shadow_view", "views_array", "config_views", "view_rays",
    "batched_views", "request_view", "eye_above_floor", "pitch_views",
    "crater_list", "random_set_patches", "EDIT_CRATER", "EDIT_SET",
    "poisson_arrivals", "default_palette", "rgba",
]
