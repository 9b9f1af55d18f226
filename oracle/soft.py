"""FP64 oracle of the differentiable form -- test infrastructure only.

Forward (reference volume only):
  tar_w = warp(tar, c)                       Sec. 3.1, Eq. (4)
  C(p, d) = Eq. (8) cost                     Sec. 3.2.1
  E(p, d) = Eq. (11) with Eq. (10) weights guided by ref
  P(p, .) = softmax_d(-E(p, .) / T)          soft-argmin head
  dh(p)  = sum_d d P(p, d)                   residual level (soft WTA)
  D(p)   = dh - delta_p + d_road(u - dh + delta_p, v)   (shift back)
  L      = mean_p | ref(p) - lerp(tar, v, u - D(p)) |   photometric L1

Backward: the analytic adjoint of every step, by the chain rule:
  * soft-argmin: dE(p,d) = g'(p) (-1/T) P(p,d) (d - dh(p)),
    g' = dL/dD (1 - c1); dD/dc = (1, u - dh + delta_p, v);
  * aggregation: dC(q,d) = sum_p w_pq / W_p dE(p,d);
    dw_pq = sum_d dE(p,d) (C(q,d) - E(p,d)) / W_p;
    dG(p) -= H, dG(q) += H with H = dw_pq w_pq 2 (G(p) - G(q)) / sigma_r^2;
  * NCC (rho = 1 - C, population statistics):
    drho/dX_i = ((Y_i - muY) / (sX sY) - rho (X_i - muX) / sX^2) / n and
    symmetrically for Y; flat blocks (constant cost) have zero gradient;
    clamped reads send their gradient to the clamped pixel;
  * warp: tar_w = (1-f) tar(i0) + f tar(i1), X = x + delta_p - d_road(x +
    delta_p, v): dtar(i0) += (1-f) g, dtar(i1) += f g, and
    dX = g (tar(i1) - tar(i0)) inside the row, dc = -dX (1, x + delta_p, v);
  * L1: d|a - s| = sign(a - s), with ds/dX = tar(i1) - tar(i0) inside the row.
"""
from __future__ import annotations

import numpy as np

from . import stereo as S

F64 = np.float64


def _grid(H, W):
    v, u = np.mgrid[0:H, 0:W]
    return u.astype(F64), v.astype(F64)


def soft_forward(ref, tar, plane, p, T=None):
    """Everything the backward needs, as FP64 arrays."""
    T = p.softargmin_T if T is None else T
    D, r, R = p.num_disp, p.ncc_radius, p.bil_radius
    X = np.asarray(ref, F64)
    tar_w = S.warp(tar, plane, p.delta_p, True)
    C, _ = S.ncc_volumes(X, tar_w, D, r, want_target=False)
    E = S.bilateral(C, X, R, p.sigma_s, p.sigma_r)
    z = -E / T
    m = z.max(axis=0)
    ez = np.exp(z - m[None])
    Z = ez.sum(axis=0)
    P = ez / Z[None]
    d = np.arange(D, dtype=F64)
    dh = np.tensordot(d, P, axes=(0, 0))
    H, W = X.shape
    u, v = _grid(H, W)
    c0, c1, c2 = (float(c) for c in plane)
    dfull = dh - p.delta_p + c0 + c1 * (u - dh + p.delta_p) + c2 * v
    return dict(tar_w=tar_w, C=C, E=E, P=P, dh=dh, disp=dfull, m=m, logZ=np.log(Z))


def photometric_l1(ref, tar, disp):
    X = np.asarray(ref, F64)
    H, W = X.shape
    u, v = _grid(H, W)
    s = S.lerp_row(np.asarray(tar, F64), v.astype(np.int64), u - disp)
    return float(np.mean(np.abs(X - s)))


def _lerp_parts(img, v, X):
    W = img.shape[1]
    Xc = np.clip(X, 0.0, W - 1.0)
    i0 = np.floor(Xc).astype(np.int64)
    f = Xc - i0
    i1 = np.minimum(i0 + 1, W - 1)
    inside = (X > 0.0) & (X < W - 1.0)
    return i0, i1, f, inside


def photometric_l1_backward(ref, tar, disp, g_loss=1.0):
    """(g_ref, g_tar, g_disp) of L = mean |ref - lerp(tar, v, u - disp)|."""
    X = np.asarray(ref, F64)
    Tt = np.asarray(tar, F64)
    H, W = X.shape
    u, v = _grid(H, W)
    vi = v.astype(np.int64)
    Xs = u - disp
    i0, i1, f, inside = _lerp_parts(Tt, vi, Xs)
    s = (1.0 - f) * Tt[vi, i0] + f * Tt[vi, i1]
    sg = np.sign(X - s) * (g_loss / X.size)
    g_ref = sg
    g_s = -sg
    g_tar = np.zeros_like(Tt)
    np.add.at(g_tar, (vi, i0), (1.0 - f) * g_s)
    np.add.at(g_tar, (vi, i1), f * g_s)
    slope = np.where(inside, Tt[vi, i1] - Tt[vi, i0], 0.0)
    g_disp = -g_s * slope
    return g_ref, g_tar, g_disp


def _fold_pad(gp, top, bottom, left, right):
    """Adjoint of edge padding: padded rows / columns return to the edge."""
    g = gp.copy()
    if top:
        g[top] += g[:top].sum(axis=0)
    if bottom:
        g[-bottom - 1] += g[-bottom:].sum(axis=0)
    g = g[top:g.shape[0] - bottom]
    if left:
        g[:, left] += g[:, :left].sum(axis=1)
    if right:
        g[:, -right - 1] += g[:, -right:].sum(axis=1)
    return g[:, left:g.shape[1] - right]


def soft_backward(ref, tar, plane, p, fwd, g_disp, T=None):
    """Vector-Jacobian product of D(p) (the soft disparity) with g_disp.

    Returns (g_ref, g_tar, g_plane[3]).
    """
    T = p.softargmin_T if T is None else T
    D, r, R = p.num_disp, p.ncc_radius, p.bil_radius
    X = np.asarray(ref, F64)
    Tt = np.asarray(tar, F64)
    H, W = X.shape
    u, v = _grid(H, W)
    c0, c1, c2 = (float(c) for c in plane)
    g_disp = np.asarray(g_disp, F64)
    dh, P, E, C, Y = fwd["dh"], fwd["P"], fwd["E"], fwd["C"], fwd["tar_w"]

    # --- shift back and soft-argmin
    g_plane = np.array([g_disp.sum(), (g_disp * (u - dh + p.delta_p)).sum(), (g_disp * v).sum()])
    gdh = g_disp * (1.0 - c1)
    d = np.arange(D, dtype=F64)[:, None, None]
    gE = gdh[None] * (-1.0 / T) * P * (d - dh[None])

    # --- bilateral aggregation (guide = ref)
    gC = np.zeros_like(C)
    gG = np.zeros_like(X)
    Wp = np.zeros_like(X)
    taps = []
    for dy in range(-R, R + 1):
        py = slice(max(0, -dy), min(H, H - dy))
        qy = slice(max(0, dy), min(H, H + dy))
        for dx in range(-R, R + 1):
            px = slice(max(0, -dx), min(W, W - dx))
            qx = slice(max(0, dx), min(W, W + dx))
            g = X[py, px] - X[qy, qx]
            w = np.exp(-(dx * dx + dy * dy) / p.sigma_s ** 2 - g * g / p.sigma_r ** 2)
            Wp[py, px] += w
            taps.append((py, px, qy, qx, g, w))
    for py, px, qy, qx, g, w in taps:
        a = w / Wp[py, px]
        gC[:, qy, qx] += a[None] * gE[:, py, px]
        gw = (gE[:, py, px] * (C[:, qy, qx] - E[:, py, px])).sum(axis=0) / Wp[py, px]
        Hh = gw * w * 2.0 * g / p.sigma_r ** 2
        gG[py, px] -= Hh
        gG[qy, qx] += Hh

    # --- NCC adjoint (reference volume), padded arrays then folded back
    k = 2 * r + 1
    n = k * k
    Xp = np.pad(X, r, mode="edge")
    Yp = np.pad(Y, ((r, r), (r + D - 1, r)), mode="edge")
    muX, sdX = S._block_mean_std(Xp, r, H, W)
    muYall, sdYall = S._block_mean_std(Yp, r, H, W + D - 1)
    gXp = np.zeros_like(Xp)
    gYp = np.zeros_like(Yp)
    for dd in range(D):
        off = D - 1 - dd
        muY = muYall[:, off:off + W]
        sdY = sdYall[:, off:off + W]
        flat = (sdX * sdX < S.FLAT_VAR) | (sdY * sdY < S.FLAT_VAR)
        ss = np.where(flat, 1.0, sdX * sdY)
        rho = 1.0 - C[dd]
        A = np.where(flat, 0.0, -gC[dd] / n)
        cxy = A / ss
        cxx = np.where(flat, 0.0, -A * rho / np.where(flat, 1.0, sdX * sdX))
        cyy = np.where(flat, 0.0, -A * rho / np.where(flat, 1.0, sdY * sdY))
        for i in range(k):
            for j in range(k):
                xs = Xp[i:i + H, j:j + W]
                ys = Yp[i:i + H, j + off:j + off + W]
                gXp[i:i + H, j:j + W] += cxy * (ys - muY) + cxx * (xs - muX)
                gYp[i:i + H, j + off:j + off + W] += cxy * (xs - muX) + cyy * (ys - muY)
    g_ref = _fold_pad(gXp, r, r, r, r) + gG
    g_tarw = _fold_pad(gYp, r, r, r + D - 1, r)

    # --- warp adjoint
    vi = v.astype(np.int64)
    Xw = u + p.delta_p - (c0 + c1 * (u + p.delta_p) + c2 * v)
    i0, i1, f, inside = _lerp_parts(Tt, vi, Xw)
    g_tar = np.zeros_like(Tt)
    np.add.at(g_tar, (vi, i0), (1.0 - f) * g_tarw)
    np.add.at(g_tar, (vi, i1), f * g_tarw)
    gX = np.where(inside, g_tarw * (Tt[vi, i1] - Tt[vi, i0]), 0.0)
    g_plane -= np.array([gX.sum(), (gX * (u + p.delta_p)).sum(), (gX * v).sum()])
    return g_ref, g_tar, g_plane
