"""Seeded synthetic road-scene stereo pairs and the named workloads.

This package generates inputs only.  It holds none of the stereo method's
arithmetic (no warp, cost, aggregation, selection or road fit), so both the
FP64 oracle and the GPU path can draw their inputs from it without sharing
any computation.
"""
from .presets import (Workload, WORKLOADS, workload, batch_workloads,
                      crop_workload)
from .scenes import (Scene, make_scene, make_workload_pair, road_sequence, skew_matrix,
                     skewed_pair)

__all__ = ["skew_matrix", "skewed_pair", "road_sequence", "Workload", "WORKLOADS", "workload", "batch_workloads",
           "crop_workload", "Scene", "make_scene", "make_workload_pair"]
