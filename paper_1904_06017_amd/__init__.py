"""MI355X (gfx950) road-stereo library: HIP kernels behind a C ABI, with a
thin Python binding.  See include/stereo.h for the ABI."""
from . import _lib
from .api import (Plan, bilateral_aggregate, cost_volume, lr_check, make_params, match,
                  params_from_workload, road_transform, warp, wta_subpixel)

__all__ = ["Plan", "make_params", "params_from_workload", "warp", "cost_volume",
           "bilateral_aggregate", "wta_subpixel", "lr_check", "match", "road_transform",
           "_lib"]
