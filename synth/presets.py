"""Named workloads: image size, disparity search range, road plane, window
radii and filter sigmas, plus the scene recipe (pothole / crack counts, seed).

Notation follows the paper:
  * ``num_disp`` (D) residual disparity levels d' in [0, D) searched after the
    perspective transformation (Sec. 3.1); ``delta_p`` is the paper's delta_p,
    so the residual disparity is d' - delta_p.
  * ``plane`` = (c0, c1, c2): road disparity d_road(u, v) = c0 + c1*u + c2*v.
    With c1 = 0 this is the row-linear road disparity of Eq. (4); c1 != 0
    models a non-zero roll angle (Sec. 3.3): c = (a0, -a1 sin psi, a1 cos psi).
  * ``ncc_radius`` r: the NCC block is (2r+1)^2 pixels (Eq. 8, N+_p).
  * ``bil_radius`` R, ``sigma_s``, ``sigma_r``: the bilateral window is
    (2R+1)^2 and the weight is exp(-|p-q|^2/sigma_s^2 - dI^2/sigma_r^2), i.e.
    sigma_0 and sigma_1 of Eq. (10).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    dtype: str                 # "u8" or "f32" image pixels
    num_disp: int              # D
    delta_p: float             # level offset: residual = d' - delta_p
    perspective: bool          # warp the target by the road plane first
    plane: Tuple[float, float, float]   # method's road plane (c0, c1, c2)
    ncc_radius: int            # r
    bil_radius: int            # R
    sigma_s: float             # sigma_0 of Eq. (10)
    sigma_r: float             # sigma_1 of Eq. (10)
    n_potholes: int
    n_cracks: int
    seed: int
    scene_plane: Tuple[float, float, float] = None   # true plane (default: plane)
    lr_delta: float = 1.0      # delta_r of Eq. (12)
    lr_check: bool = True
    softargmin_T: float = 0.1
    # full Eq. (3) warp in place of the plane's row shift: 9 entries, row-major
    homography: Tuple[float, ...] = None

    @property
    def true_plane(self):
        return self.scene_plane if self.scene_plane is not None else self.plane

    @property
    def elements(self) -> int:
        """W*H*D: the pixel-disparity evaluations one pass performs."""
        return self.width * self.height * self.num_disp


_C1 = Workload("road320x240_d32", 320, 240, "u8", 32, 16.0, True,
               (8.0, 0.0, 0.1), 2, 4, 3.0, 10.0, 6, 0, 1)
_C2 = Workload("road640x480_d48", 640, 480, "u8", 48, 24.0, True,
               (16.0, 0.0, 0.1), 3, 5, 4.0, 12.0, 10, 2, 2)
_C3A = Workload("road1280x720_d64_persp", 1280, 720, "u8", 64, 32.0, True,
                (24.0, 0.0, 0.1), 3, 7, 5.0, 12.0, 10, 2, 3)
# Same pair as 3a, searched over the full range 0..127 without the
# perspective transformation (the range-reduction comparison).
_C3B = replace(_C3A, name="road1280x720_d128_raw", num_disp=128, delta_p=0.0,
               perspective=False, scene_plane=_C3A.plane)
_C5 = Workload("road1280x720_f32_d48_soft", 1280, 720, "f32", 48, 24.0, True,
               (24.0, 0.0, 0.1), 3, 5, 4.0, 12.0, 10, 2, 5)
# The paper's own parameter set: 640x360 input, 11x11 windows
# ("120-connected", Sec. 4.4.1), sigma_0 = 1.5, sigma_1 = 5.5, and the
# disparity count implied by its Mde/s figure (30).
_PAPER = Workload("paper640x360_d30", 640, 360, "u8", 30, 15.0, True,
                  (12.0, 0.0, 0.1), 5, 5, 1.5, 5.5, 6, 1, 7)

WORKLOADS = {w.name: w for w in (_C1, _C2, _C3A, _C3B, _C5, _PAPER)}
ALIASES = {"c1": _C1.name, "c2": _C2.name, "c3a": _C3A.name,
           "c3b": _C3B.name, "c5": _C5.name, "paper": _PAPER.name}


def workload(name: str) -> Workload:
    return WORKLOADS[ALIASES.get(name, name)]


def crop_workload(w: Workload, width: int, height: int, **kw) -> Workload:
    """A smaller scene with the same method parameters (test sizes)."""
    return replace(w, name=f"{w.name}_crop{width}x{height}", width=width,
                   height=height, **kw)


# Mixed batch: 16 x 320x240, 24 x 640x480, 16 x 1280x720, 8 x 1920x1080.
# Window radii / sigmas follow the per-size classes of the single-pair
# workloads; the largest class uses the 1280x720 parameters.
_BATCH_CLASSES = [
    (16, 320, 240, 2, 4, 3.0, 10.0, 6, 0),
    (24, 640, 480, 3, 5, 4.0, 12.0, 10, 2),
    (16, 1280, 720, 3, 7, 5.0, 12.0, 10, 2),
    (8, 1920, 1080, 3, 7, 5.0, 12.0, 10, 2),
]


def batch_workloads(seed: int = 4, scale: float = 1.0) -> List[Workload]:
    """64 pairs of uneven size, disparity range and roll.

    Per pair: D ~ U{32..96}, delta_p = floor(D/2), road slope a1 ~ U[0.05, 0.2]
    px/row, roll psi ~ U[-10, 10] degrees, plane c = (a0, -a1 sin psi,
    a1 cos psi) with a0 chosen so the smallest road disparity is 4 px.
    ``scale`` < 1 shrinks every image (for CPU-sized tests).
    """
    children = np.random.SeedSequence(seed).spawn(64)
    out = []
    k = 0
    for count, w, h, r, R, ss, sr, npot, ncr in _BATCH_CLASSES:
        for _ in range(count):
            rng = np.random.Generator(np.random.PCG64(children[k]))
            D = int(rng.integers(32, 97))
            a1 = float(rng.uniform(0.05, 0.2))
            psi = float(rng.uniform(-10.0, 10.0)) * math.pi / 180.0
            ww = max(16, int(round(w * scale)))
            hh = max(16, int(round(h * scale)))
            c1 = -a1 * math.sin(psi)
            c2 = a1 * math.cos(psi)
            a0 = 4.0 - min(0.0, c1 * (ww - 1))
            scene_seed = int(rng.integers(0, 2**31 - 1))
            out.append(Workload(f"batch{k:02d}_{ww}x{hh}_d{D}", ww, hh, "u8", D,
                                float(D // 2), True, (a0, c1, c2), r, R, ss,
                                sr, npot, ncr, scene_seed))
            k += 1
    return out
