"""FP64 oracle of the dense road stereo path -- test infrastructure only.

Steps, each written from the paper (citations name the section / equation):

  warp            perspective transformation, Sec. 3.1, Eq. (4): every row v
                  of the target is shifted right by (Delta u - delta_p)
  ncc_volumes     matching cost c(p, d) of Eq. (8) for the reference- and the
                  target-anchored cost volumes (Sec. 3.2.1)
  bilateral       normalised bilateral aggregation, Eqs. (10)-(11)
  wta             winner-take-all, Sec. 3.2.2
  subpixel        parabola vertex, Eq. (13)
  lr_check        left-right occlusion test, Eq. (12)
  shift_back      add the road disparity back, Sec. 3.2.2

Readings where the paper is silent (each also listed in the design notes):
  * block reads replicate the border (clamp each coordinate independently);
  * mu / sigma of a block are population values (divide by n), which makes
    Eq. (8) identical to 1 - Pearson correlation;
  * a block whose variance is below 1e-6 (gray^2) has no defined NCC: its
    cost is 1 ("no information");
  * the bilateral window is truncated to the image and renormalised;
  * the target volume is anchored at target pixels, and its bilateral weights
    are guided by the warped target image (the mirror of Eq. (10));
  * d_road is evaluated at the reference coordinate x + delta_p, so that a
    road pixel lands exactly on level delta_p also when c1 != 0;
  * the left-right check compares integer WTA levels in the warped domain,
    and a match that falls outside the target image is invalid;
  * the sub-pixel step uses the aggregated cost E that WTA minimised, and is
    skipped at the ends of the range or where the parabola is not convex;
  * WTA ties go to the smallest level.
"""
from __future__ import annotations

import numpy as np

FLAT_VAR = 1e-6        # gray^2: below this a block carries no texture
F64 = np.float64


def d_road(plane, u, v):
    """Road disparity of the plane c = (c0, c1, c2) at (u, v)."""
    c0, c1, c2 = (float(c) for c in plane)
    return c0 + c1 * np.asarray(u, F64) + c2 * np.asarray(v, F64)


def lerp_row(img, v, X):
    """Linear interpolation along row v at real column X, X clamped to the row."""
    W = img.shape[1]
    Xc = np.clip(np.asarray(X, F64), 0.0, W - 1.0)
    i0 = np.floor(Xc).astype(np.int64)
    f = Xc - i0
    i1 = np.minimum(i0 + 1, W - 1)
    return (1.0 - f) * img[v, i0] + f * img[v, i1]


def warp(tar, plane, delta_p, perspective=True):
    """Sec. 3.1: shift each target row right by (Delta u - delta_p).

    tar_w(x, v) = tar(X, v) with X = x + delta_p - d_road(x + delta_p, v),
    read by linear interpolation (v is integral, so bilinear reduces to a
    1-D lerp) and clamped to the row.  Without the perspective step the
    target is used as it is.
    """
    t = np.asarray(tar, F64)
    if not perspective:
        return t.copy()
    H, W = t.shape
    v, x = np.mgrid[0:H, 0:W]
    X = x + delta_p - d_road(plane, x + delta_p, v)
    return lerp_row(t, v, X)


def plane_homography(plane):
    """The row shift of the plane as a homography (Eq. 3 under the
    hypotheses of Sec. 3.1): H (u, v, 1) = (u - d_road(u, v), v, 1)."""
    c0, c1, c2 = (float(c) for c in plane)
    return np.array([[1.0 - c1, -c2, -c0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def homography_map(Hm, u, v):
    """Eq. (3): the target point (X, Y) of the reference point (u, v)."""
    Hm = np.asarray(Hm, F64).reshape(3, 3)
    u = np.asarray(u, F64)
    v = np.asarray(v, F64)
    x = Hm[0, 0] * u + Hm[0, 1] * v + Hm[0, 2]
    y = Hm[1, 0] * u + Hm[1, 1] * v + Hm[1, 2]
    z = Hm[2, 0] * u + Hm[2, 1] * v + Hm[2, 2]
    return x / z, y / z


def bilerp(img, X, Y):
    """Bilinear interpolation at real (X, Y), each clamped to the image."""
    H, W = img.shape
    Xc = np.clip(np.asarray(X, F64), 0.0, W - 1.0)
    Yc = np.clip(np.asarray(Y, F64), 0.0, H - 1.0)
    i0 = np.floor(Xc).astype(np.int64)
    j0 = np.floor(Yc).astype(np.int64)
    fx = Xc - i0
    fy = Yc - j0
    i1 = np.minimum(i0 + 1, W - 1)
    j1 = np.minimum(j0 + 1, H - 1)
    top = (1.0 - fx) * img[j0, i0] + fx * img[j0, i1]
    bot = (1.0 - fx) * img[j1, i0] + fx * img[j1, i1]
    return (1.0 - fy) * top + fy * bot


def warp_homography(tar, Hm, delta_p):
    """Sec. 3.1 with the general homography of Eq. (3): the warped target at
    (x, v) is the target at H (x + delta_p, v, 1)^T, read bilinearly with
    clamped coordinates, so that a point of the road plane lands at level
    delta_p.  For H = plane_homography(plane) this is warp()."""
    t = np.asarray(tar, F64)
    H, W = t.shape
    v, x = np.mgrid[0:H, 0:W]
    X, Y = homography_map(Hm, x + delta_p, v)
    return bilerp(t, X, Y)


def shift_back_homography(ell, valid, Hm, delta_p):
    """Disparity along the row of the general warp: u - X where (X, Y) =
    H (u - l + delta_p, v); the plane case gives shift_back().  NaN if invalid."""
    H, W = ell.shape
    v, u = np.mgrid[0:H, 0:W]
    X, _ = homography_map(Hm, u - ell + delta_p, v)
    return np.where(valid, u - X, np.nan)


# --------------------------------------------------------------------------
# Matching cost, Eq. (8)
# --------------------------------------------------------------------------

def eq8_cost(mu_r, sd_r, mu_t, sd_t, cross, n):
    """Eq. (8): c = (s_r s_t + mu_r mu_t)/(s_r s_t) - cross/(n s_r s_t).

    ``cross`` is sum_q i_ref(q) i_tar(q - [d, 0]) over the block.  Blocks with
    (near) zero variance get cost 1.
    """
    ss = sd_r * sd_t
    flat = (sd_r * sd_r < FLAT_VAR) | (sd_t * sd_t < FLAT_VAR)
    ss_safe = np.where(flat, 1.0, ss)
    c = (ss_safe + mu_r * mu_t) / ss_safe - cross / (n * ss_safe)
    return np.where(flat, 1.0, c)


def _block_mean_std(P, r, H, ncols):
    """Population mean / std of every (2r+1)^2 block of the padded array P.

    Block k covers P[v:v+2r+1, k:k+2r+1]; the result is [H][ncols].
    """
    k = 2 * r + 1
    n = k * k
    s = np.zeros((H, ncols))
    for i in range(k):
        for j in range(k):
            s += P[i:i + H, j:j + ncols]
    mu = s / n
    q = np.zeros((H, ncols))
    for i in range(k):
        for j in range(k):
            e = P[i:i + H, j:j + ncols] - mu
            q += e * e
    return mu, np.sqrt(q / n)


def ncc_volumes(ref, tar_w, D, r, want_target=True):
    """Both cost volumes of Sec. 3.2.1 as [D][H][W] float64 arrays.

    C_R(u, v, d) compares the ref block at (u, v) with the warped-target
    block at (u - d, v); C_T(x, v, d) compares the ref block at (x + d, v)
    with the warped-target block at (x, v).  Reads are clamped.
    """
    X = np.asarray(ref, F64)
    Y = np.asarray(tar_w, F64)
    H, W = X.shape
    k = 2 * r + 1
    n = k * k
    # X block centred at column c in [0, W + D - 1) is Xp[:, c : c + k]
    Xp = np.pad(X, ((r, r), (r, r + D - 1)), mode="edge")
    # Y block centred at column x in [-(D-1), W) is Yp[:, x + D - 1 : ... + k]
    Yp = np.pad(Y, ((r, r), (r + D - 1, r)), mode="edge")
    muX, sdX = _block_mean_std(Xp, r, H, W + D - 1)
    muY, sdY = _block_mean_std(Yp, r, H, W + D - 1)
    CR = np.empty((D, H, W))
    CT = np.empty((D, H, W)) if want_target else None
    for d in range(D):
        s = np.zeros((H, W))
        for i in range(k):
            for j in range(k):
                s += Xp[i:i + H, j:j + W] * Yp[i:i + H, j + D - 1 - d:j + D - 1 - d + W]
        CR[d] = eq8_cost(muX[:, :W], sdX[:, :W],
                         muY[:, D - 1 - d:D - 1 - d + W], sdY[:, D - 1 - d:D - 1 - d + W],
                         s, n)
        if want_target:
            s = np.zeros((H, W))
            for i in range(k):
                for j in range(k):
                    s += Xp[i:i + H, j + d:j + d + W] * Yp[i:i + H, j + D - 1:j + D - 1 + W]
            CT[d] = eq8_cost(muX[:, d:d + W], sdX[:, d:d + W],
                             muY[:, D - 1:D - 1 + W], sdY[:, D - 1:D - 1 + W], s, n)
    return CR, CT


# --------------------------------------------------------------------------
# Bilateral aggregation, Eqs. (10)-(11)
# --------------------------------------------------------------------------

def bilateral(C, guide, R, sigma_s, sigma_r):
    """Eq. (11): E(p, d) = sum_q w(p, q) C(q, d) / sum_q w(p, q).

    q runs over the (2R+1)^2 window around p, truncated to the image;
    w(p, q) = exp(-|p - q|^2 / sigma_s^2 - (G(p) - G(q))^2 / sigma_r^2),
    Eq. (10), with the guide image G.
    """
    C = np.asarray(C, F64)
    G = np.asarray(guide, F64)
    D, H, W = C.shape
    num = np.zeros((D, H, W))
    den = np.zeros((H, W))
    for dy in range(-R, R + 1):
        py = slice(max(0, -dy), min(H, H - dy))
        qy = slice(max(0, dy), min(H, H + dy))
        for dx in range(-R, R + 1):
            px = slice(max(0, -dx), min(W, W - dx))
            qx = slice(max(0, dx), min(W, W + dx))
            g = G[py, px] - G[qy, qx]
            w = np.exp(-(dx * dx + dy * dy) / sigma_s ** 2 - g * g / sigma_r ** 2)
            num[:, py, px] += w[None] * C[:, qy, qx]
            den[py, px] += w
    return num / den[None]


# --------------------------------------------------------------------------
# Disparity optimisation and refinement, Sec. 3.2.2
# --------------------------------------------------------------------------

def wta(E):
    """Winner-take-all: the first level of minimum aggregated cost."""
    return np.argmin(E, axis=0).astype(np.int64)


def subpixel(E, dint):
    """Eq. (13) on the aggregated cost: l = d + (E- - E+)/(2E- + 2E+ - 4E).

    Applied where d has both neighbours and the parabola is convex
    (denominator > 0); elsewhere l = d.
    """
    D = E.shape[0]
    dm = np.clip(dint - 1, 0, D - 1)
    dp = np.clip(dint + 1, 0, D - 1)
    e0 = np.take_along_axis(E, dint[None], 0)[0]
    em = np.take_along_axis(E, dm[None], 0)[0]
    ep = np.take_along_axis(E, dp[None], 0)[0]
    den = 2.0 * em + 2.0 * ep - 4.0 * e0
    ok = (dint > 0) & (dint < D - 1) & (den > 0)
    off = np.where(ok, (em - ep) / np.where(ok, den, 1.0), 0.0)
    return dint + off


def lr_check(dint_R, dint_T, delta_r=1.0):
    """Eq. (12): p is occluded iff (l_ref(p) - l_tar(p - [l_ref(p), 0]))^2 > delta_r."""
    H, W = dint_R.shape
    v, u = np.mgrid[0:H, 0:W]
    x = u - dint_R
    inside = x >= 0
    lt = dint_T[v, np.clip(x, 0, W - 1)]
    diff = (dint_R - lt).astype(F64)
    return inside & (diff * diff <= delta_r)


def shift_back(ell, valid, plane, delta_p, perspective=True):
    """Full-domain disparity: l - delta_p + d_road(u - l + delta_p, v); NaN if invalid."""
    H, W = ell.shape
    v, u = np.mgrid[0:H, 0:W]
    if perspective:
        disp = ell - delta_p + d_road(plane, u - ell + delta_p, v)
    else:
        disp = np.asarray(ell, F64).copy()
    return np.where(valid, disp, np.nan)


def match(ref, tar, p, keep_volumes=False):
    """The whole plain forward path for one pair.

    ``p`` carries num_disp, delta_p, perspective, plane, ncc_radius,
    bil_radius, sigma_s, sigma_r, lr_delta (e.g. a synth.Workload).
    """
    delta_p = p.delta_p if p.perspective else 0.0
    Hm = getattr(p, "homography", None) if p.perspective else None
    tar_w = warp(tar, p.plane, delta_p, p.perspective) if Hm is None \
        else warp_homography(tar, Hm, delta_p)
    CR, CT = ncc_volumes(ref, tar_w, p.num_disp, p.ncc_radius)
    ER = bilateral(CR, ref, p.bil_radius, p.sigma_s, p.sigma_r)
    ET = bilateral(CT, tar_w, p.bil_radius, p.sigma_s, p.sigma_r)
    dR = wta(ER)
    dT = wta(ET)
    ell = subpixel(ER, dR)
    valid = lr_check(dR, dT, p.lr_delta)
    disp = shift_back(ell, valid, p.plane, delta_p, p.perspective) if Hm is None \
        else shift_back_homography(ell, valid, Hm, delta_p)
    out = dict(tar_w=tar_w, dint_R=dR, dint_T=dT, ell=ell, valid=valid,
               disp=disp)
    if keep_volumes:
        out.update(C_R=CR, C_T=CT, E_R=ER, E_T=ET)
    return out


# --------------------------------------------------------------------------
# Point-wise evaluation (for sampled checks at full image size)
# --------------------------------------------------------------------------

def _clamped_blocks(img, uc, vc, r):
    """Blocks centred at (uc, vc) (int arrays, shape S) -> [S..., (2r+1)^2]."""
    H, W = img.shape
    o = np.arange(-r, r + 1)
    ii = np.clip(vc[..., None, None] + o[:, None], 0, H - 1)
    jj = np.clip(uc[..., None, None] + o[None, :], 0, W - 1)
    return img[ii, jj].reshape(uc.shape + ((2 * r + 1) ** 2,))


def ncc_cost_at(ref, tar_w, u_ref, u_tar, v, r):
    """Eq. (8) for ref blocks at (u_ref, v) and target blocks at (u_tar, v)."""
    X = _clamped_blocks(np.asarray(ref, F64), u_ref, v, r)
    Y = _clamped_blocks(np.asarray(tar_w, F64), u_tar, v, r)
    n = X.shape[-1]
    mx, my = X.mean(-1), Y.mean(-1)
    sx = np.sqrt(((X - mx[..., None]) ** 2).mean(-1))
    sy = np.sqrt(((Y - my[..., None]) ** 2).mean(-1))
    return eq8_cost(mx, sx, my, sy, (X * Y).sum(-1), n)


def aggregated_at(ref, tar_w, u, v, p, volume="R"):
    """E_R or E_T at pixel (u, v) for all levels -> (D,) array."""
    H, W = np.shape(ref)
    D, r, R = p.num_disp, p.ncc_radius, p.bil_radius
    G = np.asarray(ref if volume == "R" else tar_w, F64)
    dy, dx = np.mgrid[-R:R + 1, -R:R + 1]
    qv, qu = v + dy.ravel(), u + dx.ravel()
    inside = (qv >= 0) & (qv < H) & (qu >= 0) & (qu < W)
    qv, qu = qv[inside], qu[inside]
    ddx, ddy = dx.ravel()[inside], dy.ravel()[inside]
    g = G[v, u] - G[qv, qu]
    w = np.exp(-(ddx * ddx + ddy * ddy) / p.sigma_s ** 2 - g * g / p.sigma_r ** 2)
    d = np.arange(D)
    QU = np.broadcast_to(qu[:, None], (qu.size, D))
    QV = np.broadcast_to(qv[:, None], (qv.size, D))
    DD = np.broadcast_to(d[None, :], (qu.size, D))
    if volume == "R":
        C = ncc_cost_at(ref, tar_w, QU, QU - DD, QV, r)
    else:
        C = ncc_cost_at(ref, tar_w, QU + DD, QU, QV, r)
    return (w[:, None] * C).sum(0) / w.sum()


def match_at(ref, tar, p, pixels, tar_w=None):
    """Plain-path outputs at a list of (u, v) pixels (sampled full-size checks)."""
    delta_p = p.delta_p if p.perspective else 0.0
    Hm = getattr(p, "homography", None) if p.perspective else None
    if tar_w is None:
        tar_w = warp(tar, p.plane, delta_p, p.perspective) if Hm is None \
            else warp_homography(tar, Hm, delta_p)
    H, W = np.shape(ref)
    D = p.num_disp
    out = []
    for (u, v) in pixels:
        ER = aggregated_at(ref, tar_w, u, v, p, "R")
        dR = int(np.argmin(ER))
        srt = np.sort(ER)
        ell = float(subpixel(ER[:, None, None], np.array([[dR]]))[0, 0])
        x = u - dR
        if x >= 0:
            ET = aggregated_at(ref, tar_w, x, v, p, "T")
            dT = int(np.argmin(ET))
            srtT = np.sort(ET)
            gapT = float(srtT[1] - srtT[0])
            valid = (dR - dT) ** 2 <= p.lr_delta
        else:
            dT, gapT, valid = -1, np.inf, False
        if Hm is not None:
            disp = u - float(homography_map(Hm, u - ell + delta_p, v)[0])
        elif p.perspective:
            disp = ell - delta_p + float(d_road(p.plane, u - ell + delta_p, v))
        else:
            disp = ell
        out.append(dict(u=u, v=v, E_R=ER, dint_R=dR, gap=float(srt[1] - srt[0]),
                        ell=ell, dint_T=dT, gap_T=gapT, valid=bool(valid),
                        disp=disp if valid else np.nan))
    return out
