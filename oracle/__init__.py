"""FP64 CPU oracle for the road-stereo hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded numpy implementation of what the method
computes, written step by step from the paper's equations.  It exists to
check the GPU path; it is never part of it.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it.  It imports nothing
from the GPU package and shares no code with it.

Modules:
  stereo   perspective warp, NCC costs, bilateral aggregation, WTA, sub-pixel,
           left-right check, shift back (Sec. 3.1-3.2, Eqs. 4, 8-13)
  road     roll angle / disparity projection fit and the disparity
           transformation (Sec. 3.3, Eqs. 14-29)
  soft     soft-argmin disparity head, photometric L1 loss and their
           analytic FP64 adjoint (the differentiable form)
  metrics  e_p, e_r (Eqs. 33-35), Mde/s (Eq. 36), sigma_d (Eq. 37)
"""
import os as _os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    _os.environ.setdefault(_v, "1")

from . import stereo, road, metrics  # noqa: E402

__all__ = ["stereo", "road", "metrics"]
