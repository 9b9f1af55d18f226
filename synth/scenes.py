"""Seeded synthetic road scenes with ground-truth disparity.

Recipe (stands in for the paper's UAV / KITTI / EISATS data, none of which is
available): a blurred uniform-noise texture painted on a road plane with
elliptical potholes and thin cracks, seen by a rectified stereo pair.

  * texture N ~ U(-20*sqrt(3), 20*sqrt(3)) (std 20) on the reference grid plus
    a right margin; crack pixels darkened by 40 before blurring;
    T = 128 + GaussianBlur(N, sigma = 1, truncate 4 sigma, reflect);
  * ground truth d_gt(u, v) = d_road(u, v) - sum_k depth_k max(0, 1 - rho_k^2)
    - 2 [within 1 px of a crack polyline] (a depression is farther away, so
    its disparity is smaller);
  * ref(u, v) = T(u, v); tar(x, v) = T(u*, v) with u* - d_gt(u*, v) = x, found
    by fixed-point iteration and read by linear interpolation along the row;
  * u8 images are rounded and clipped to [0, 255]; f32 images are not.

Only numpy / scipy.ndimage are used; nothing here is part of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage

from .presets import Workload


@dataclass
class Scene:
    ref: np.ndarray        # [H][W] uint8 or float32
    tar: np.ndarray        # [H][W] uint8 or float32
    d_gt: np.ndarray       # [H][W] float64 ground-truth disparity (ref view)
    road_mask: np.ndarray  # [H][W] bool: plain road (no pothole / crack)
    visible: np.ndarray    # [H][W] bool: ref pixel visible in the target
    damage_mask: np.ndarray  # [H][W] bool: pothole or crack


class _Geometry:
    def __init__(self, width, height, plane, n_potholes, n_cracks, rng):
        self.W, self.H = width, height
        self.c0, self.c1, self.c2 = (float(x) for x in plane)
        W, H = width, height
        self.pot = []
        for _ in range(n_potholes):
            depth = rng.uniform(1.0, 4.0)
            lo = max(W / 40.0, 3.0 * depth)
            hi = max(W / 16.0, lo + 1.0)
            a = rng.uniform(lo, hi)
            b = rng.uniform(lo, hi)
            cu = rng.uniform(0.1 * W, 0.9 * W)
            cv = rng.uniform(0.1 * H, 0.9 * H)
            ang = rng.uniform(0.0, math.pi)
            self.pot.append((cu, cv, a, b, math.cos(ang), math.sin(ang), depth))
        self.cracks = []
        for _ in range(n_cracks):
            pts = [(rng.uniform(0.1 * W, 0.9 * W), rng.uniform(0.1 * H, 0.9 * H))]
            heading = rng.uniform(0.0, 2.0 * math.pi)
            for _ in range(3):
                seg = rng.uniform(0.1 * W, 0.25 * W)
                heading += rng.uniform(-math.pi / 6.0, math.pi / 6.0)
                x, y = pts[-1]
                pts.append((x + seg * math.cos(heading), y + seg * math.sin(heading)))
            self.cracks.append(pts)

    def road(self, u, v):
        return self.c0 + self.c1 * u + self.c2 * v

    def pothole_drop(self, u, v):
        out = np.zeros(np.broadcast(u, v).shape)
        for cu, cv, a, b, ca, sa, depth in self.pot:
            du, dv = u - cu, v - cv
            x = du * ca + dv * sa
            y = -du * sa + dv * ca
            rho2 = (x / a) ** 2 + (y / b) ** 2
            out += depth * np.maximum(0.0, 1.0 - rho2)
        return out

    def crack(self, u, v):
        u, v = np.broadcast_arrays(np.asarray(u, float), np.asarray(v, float))
        hit = np.zeros(u.shape, dtype=bool)
        for pts in self.cracks:
            for (x0, y0), (x1, y1) in zip(pts[:-1], pts[1:]):
                # only points inside the segment's bounding box (+1 px) can hit
                box = ((u >= min(x0, x1) - 1.0) & (u <= max(x0, x1) + 1.0) &
                       (v >= min(y0, y1) - 1.0) & (v <= max(y0, y1) + 1.0))
                if not box.any():
                    continue
                ub, vb = u[box], v[box]
                ex, ey = x1 - x0, y1 - y0
                L2 = ex * ex + ey * ey
                t = np.clip(((ub - x0) * ex + (vb - y0) * ey) / L2, 0.0, 1.0)
                dx = ub - (x0 + t * ex)
                dy = vb - (y0 + t * ey)
                hit[box] |= (dx * dx + dy * dy) <= 1.0
        return hit

    def d_gt(self, u, v):
        return self.road(u, v) - self.pothole_drop(u, v) - 2.0 * self.crack(u, v)

    def inverse(self, x, v, iters=30):
        """u* with u* - d_gt(u*, v) = x (the ref column seen at tar column x)."""
        x, v = np.broadcast_arrays(np.asarray(x, float), np.asarray(v, float))
        # exact for the plane alone, then fixed-point for the local damage;
        # only points that have not settled keep iterating
        u = ((x + self.c0 + self.c2 * v) / (1.0 - self.c1)).ravel().copy()
        xf, vf = x.ravel(), v.ravel()
        act = np.arange(u.size)
        for _ in range(iters):
            un = xf[act] + self.d_gt(u[act], vf[act])
            moved = np.abs(un - u[act]) >= 1e-10
            u[act] = un
            act = act[moved]
            if act.size == 0:
                break
        return u.reshape(x.shape)


def _row_lerp(T, u, v_idx):
    """Linear interpolation of T along each row at real columns u."""
    Wt = T.shape[1]
    uc = np.clip(u, 0.0, Wt - 1.0)
    i0 = np.floor(uc).astype(np.int64)
    i1 = np.minimum(i0 + 1, Wt - 1)
    f = uc - i0
    return (1.0 - f) * T[v_idx, i0] + f * T[v_idx, i1]


def make_scene(width, height, plane, n_potholes, n_cracks, seed,
               float_images=False) -> Scene:
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _Geometry(width, height, plane, n_potholes, n_cracks, rng)
    W, H = width, height
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    dmax = float(np.max(g.road(np.array([0.0, W - 1.0, 0.0, W - 1.0]),
                               np.array([0.0, 0.0, H - 1.0, H - 1.0]))))
    margin = int(math.ceil(max(dmax, 0.0))) + 8
    Wt = W + margin
    tv, tu = np.mgrid[0:H, 0:Wt].astype(np.float64)
    N = rng.uniform(-20.0 * math.sqrt(3.0), 20.0 * math.sqrt(3.0), size=(H, Wt))
    N[g.crack(tu, tv)] -= 40.0
    T = 128.0 + ndimage.gaussian_filter(N, 1.0, mode="reflect", truncate=4.0)

    d_gt = g.d_gt(uu, vv)
    ustar = g.inverse(uu, vv)               # tar column x = uu
    vi = vv.astype(np.int64)
    ref_f = T[:, :W].copy()
    tar_f = _row_lerp(T, ustar, vi)
    if float_images:
        ref = ref_f.astype(np.float32)
        tar = tar_f.astype(np.float32)
    else:
        ref = np.clip(np.rint(ref_f), 0, 255).astype(np.uint8)
        tar = np.clip(np.rint(tar_f), 0, 255).astype(np.uint8)
    xt = uu - d_gt
    back = g.inverse(xt, vv)
    visible = (np.abs(back - uu) <= 0.5) & (xt >= 0.0)
    damage = (g.pothole_drop(uu, vv) > 0.0) | g.crack(uu, vv)
    return Scene(ref=ref, tar=tar, d_gt=d_gt, road_mask=~damage,
                 visible=visible, damage_mask=damage)


def make_workload_pair(w: Workload) -> Scene:
    return make_scene(w.width, w.height, w.true_plane, w.n_potholes,
                      w.n_cracks, w.seed, float_images=(w.dtype == "f32"))


def road_sequence(width, height, n_frames, seed, n_potholes=4, n_cracks=1, slope=0.1,
                  psi0_deg=2.0, dpsi_deg=0.4, da0=0.25, dslope=0.01, float_images=False):
    """Frames of a road whose plane drifts slowly (a vehicle moving on it):
    slope a1_t = slope (1 + dslope t) px/row, roll psi_t = psi0 + dpsi t
    degrees, offset a0_t = a0 + da0 t px with a0 chosen so that the smallest
    road disparity of frame 0 is 4 px; plane c_t = (a0_t, -a1_t sin psi_t,
    a1_t cos psi_t).  Each frame has its own damage and texture, seeded from
    SeedSequence(seed).  Returns [(plane, psi_rad, Scene)] per frame."""
    kids = np.random.SeedSequence(seed).spawn(n_frames)
    psi0 = math.radians(psi0_deg)
    ys = [v * math.cos(psi0) - u * math.sin(psi0)
          for u in (0.0, width - 1.0) for v in (0.0, height - 1.0)]
    a0 = 4.0 - slope * min(ys)
    out = []
    for t in range(n_frames):
        psi = math.radians(psi0_deg + dpsi_deg * t)
        a1 = slope * (1.0 + dslope * t)
        c = (a0 + da0 * t, -a1 * math.sin(psi), a1 * math.cos(psi))
        s = int(kids[t].generate_state(1)[0])
        out.append((c, psi, make_scene(width, height, c, n_potholes, n_cracks, s,
                                       float_images=float_images)))
    return out


def skew_matrix(width, height, angle_deg=0.3, dy=0.8):
    """A small in-plane rotation of the target camera about the image centre
    plus a vertical offset: a rig outside the rectified hypotheses."""
    a = math.radians(angle_deg)
    cx, cy = (width - 1) / 2.0, (height - 1) / 2.0
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, cx - c * cx + s * cy],
                     [s, c, cy - s * cx - c * cy + dy],
                     [0.0, 0.0, 1.0]])


def skewed_pair(w: Workload, angle_deg=0.3, dy=0.8):
    """The workload's pair with the target re-imaged by skew_matrix G:
    tar2(p) = tar(G^-1 p) (bilinear, clamped; rounded for uint8).  Returns
    (scene, tar2, G, H, disp_true) where H = G . (row shift of the true plane)
    maps reference pixels of the road plane into tar2, and disp_true(u, v) is
    u minus the column of the true correspondence in tar2."""
    sc = make_workload_pair(w)
    H_, W_ = sc.tar.shape
    G = skew_matrix(W_, H_, angle_deg, dy)
    Gi = np.linalg.inv(G)
    vv, uu = np.mgrid[0:H_, 0:W_].astype(np.float64)
    den = Gi[2, 0] * uu + Gi[2, 1] * vv + Gi[2, 2]
    X = (Gi[0, 0] * uu + Gi[0, 1] * vv + Gi[0, 2]) / den
    Y = (Gi[1, 0] * uu + Gi[1, 1] * vv + Gi[1, 2]) / den
    t = sc.tar.astype(np.float64)
    Xc, Yc = np.clip(X, 0, W_ - 1.0), np.clip(Y, 0, H_ - 1.0)
    i0, j0 = np.floor(Xc).astype(np.int64), np.floor(Yc).astype(np.int64)
    i1, j1 = np.minimum(i0 + 1, W_ - 1), np.minimum(j0 + 1, H_ - 1)
    fx, fy = Xc - i0, Yc - j0
    t2 = ((1 - fy) * ((1 - fx) * t[j0, i0] + fx * t[j0, i1]) +
          fy * ((1 - fx) * t[j1, i0] + fx * t[j1, i1]))
    tar2 = (t2.astype(np.float32) if w.dtype == "f32"
            else np.clip(np.rint(t2), 0, 255).astype(np.uint8))
    c0, c1, c2 = w.true_plane
    Hrow = np.array([[1.0 - c1, -c2, -c0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    H = G @ Hrow
    xt = uu - sc.d_gt                      # true correspondence in the rectified target
    xs = (G[0, 0] * xt + G[0, 1] * vv + G[0, 2]) / (G[2, 0] * xt + G[2, 1] * vv + G[2, 2])
    return sc, tar2, G, H, uu - xs
