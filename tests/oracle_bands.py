"""Full-frame oracle results in row bands, one band per worker process.

Test infrastructure: the FP64 oracle on a 1280x720 frame takes about a minute
of one core per volume pass, so the full-frame parity tests split the output
rows into bands and run the oracle functions, unchanged, on a row crop per
band.  A crop holds the band plus the rows its outputs read: bilateral window
(R rows) and NCC block (r rows) on each side, cut at the image edges, so that
every output row of the band sees exactly the values, clamps and window
truncations it sees in the whole frame.  Rows of the crop outside the band
are computed and discarded.  Only the row coordinate of the plane (or of the
homography) is re-expressed in crop coordinates.

The same construction gives the soft-argmin gradient: the loss restricted to
a band's rows depends on the crop only, its vector-Jacobian product is taken
on the crop by the oracle's adjoint, and the gradients of the bands add up to
the full one (the upstream gradient is split by rows).

`tests/test_oracle_bands.py` pins both decompositions to the whole-frame
oracle on small frames.  Workers are started with the "spawn" method: they
never inherit a process that has initialised a GPU, and they import numpy and
the oracle only.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

import oracle.soft as SO
import oracle.stereo as OS


def worker_count():
    return max(1, min(16, os.cpu_count() or 1))


def process_pool(n=None):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
    os.environ.setdefault("MKL_NUM_THREADS", "1")
    return cf.ProcessPoolExecutor(n or worker_count(), mp_context=mp.get_context("spawn"))


def bands(H, n):
    """n contiguous row bands [v0, v1) covering [0, H)."""
    n = max(1, min(n, H))
    edges = np.linspace(0, H, n + 1).round().astype(int)
    return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def _translate_rows(Hm, v0):
    """Homography acting on (u, v_local + v0, 1)."""
    T = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, float(v0)], [0.0, 0.0, 1.0]])
    return (np.asarray(Hm, np.float64).reshape(3, 3) @ T).ravel()


def _match_band(args):
    ref_c, tarw_c, p, a, v0, v1, H = args
    D, r, R = p.num_disp, p.ncc_radius, p.bil_radius
    CR, CT = OS.ncc_volumes(ref_c, tarw_c, D, r)
    c0, c1 = max(0, v0 - R), min(H, v1 + R)           # cost rows the band's windows read
    g_ref = np.asarray(ref_c, np.float64)[c0 - a:c1 - a]
    g_tar = np.asarray(tarw_c, np.float64)[c0 - a:c1 - a]
    ER = OS.bilateral(CR[:, c0 - a:c1 - a], g_ref, R, p.sigma_s, p.sigma_r)[:, v0 - c0:v1 - c0]
    ET = OS.bilateral(CT[:, c0 - a:c1 - a], g_tar, R, p.sigma_s, p.sigma_r)[:, v0 - c0:v1 - c0]
    dR, dT = OS.wta(ER), OS.wta(ET)
    ell = OS.subpixel(ER, dR)
    valid = OS.lr_check(dR, dT, p.lr_delta)
    delta_p = p.delta_p if p.perspective else 0.0
    Hm = getattr(p, "homography", None) if p.perspective else None
    if Hm is not None:
        disp = OS.shift_back_homography(ell, valid, _translate_rows(Hm, v0), delta_p)
    else:
        c = p.plane
        plane_b = (c[0] + c[2] * v0, c[1], c[2])
        disp = OS.shift_back(ell, valid, plane_b, delta_p, p.perspective)
    sR, sT = np.sort(ER, axis=0), np.sort(ET, axis=0)
    Dn = ER.shape[0]
    e0 = np.take_along_axis(ER, dR[None], 0)[0]
    em = np.take_along_axis(ER, np.clip(dR - 1, 0, Dn - 1)[None], 0)[0]
    ep = np.take_along_axis(ER, np.clip(dR + 1, 0, Dn - 1)[None], 0)[0]
    return dict(v0=v0, v1=v1, dint_R=dR, dint_T=dT, ell=ell, valid=valid, disp=disp,
                gapR=sR[1] - sR[0], gapT=sT[1] - sT[0], curv=(em - e0) + (ep - e0))


def match_full(ref, tar, p, pool, n_bands=None):
    """OS.match outputs for the whole frame, plus the two smallest-cost gaps of
    both volumes (gapR, gapT) and the parabola curvature a + b at the chosen
    level (curv), assembled from row bands."""
    H, W = np.shape(ref)
    delta_p = p.delta_p if p.perspective else 0.0
    Hm = getattr(p, "homography", None) if p.perspective else None
    tar_w = OS.warp(tar, p.plane, delta_p, p.perspective) if Hm is None \
        else OS.warp_homography(tar, Hm, delta_p)
    halo = p.bil_radius + p.ncc_radius
    jobs = []
    for v0, v1 in bands(H, n_bands or 2 * worker_count()):
        a, b = max(0, v0 - halo), min(H, v1 + halo)
        jobs.append((np.ascontiguousarray(ref[a:b]), np.ascontiguousarray(tar_w[a:b]), p, a, v0, v1, H))
    out = {k: np.empty((H, W), dt) for k, dt in
           (("dint_R", np.int64), ("dint_T", np.int64), ("ell", np.float64), ("valid", bool),
            ("disp", np.float64), ("gapR", np.float64), ("gapT", np.float64),
            ("curv", np.float64))}
    for res in pool.map(_match_band, jobs):
        for k in out:
            out[k][res["v0"]:res["v1"]] = res[k]
    out["tar_w"] = tar_w
    return out


def _soft_band(args):
    ref_c, tar_c, plane_c, p, g_c, a = args
    fwd = SO.soft_forward(ref_c, tar_c, plane_c, p)
    g_ref, g_tar, g_plane = SO.soft_backward(ref_c, tar_c, plane_c, p, fwd, g_c)
    return a, g_ref, g_tar, g_plane


def soft_grad_full(ref, tar, plane, p, g_disp, pool, n_bands=None):
    """(g_ref, g_tar, g_plane) of SO.soft_backward for the whole frame,
    assembled from row bands (upstream gradient split by rows)."""
    H, W = np.shape(ref)
    halo = p.bil_radius + p.ncc_radius
    c0, c1, c2 = (float(c) for c in plane)
    jobs = []
    for v0, v1 in bands(H, n_bands or 2 * worker_count()):
        a, b = max(0, v0 - halo), min(H, v1 + halo)
        g = np.zeros((b - a, W))
        g[v0 - a:v1 - a] = np.asarray(g_disp, np.float64)[v0:v1]
        jobs.append((np.ascontiguousarray(ref[a:b]), np.ascontiguousarray(tar[a:b]),
                     (c0 + c2 * a, c1, c2), p, g, a))
    g_ref = np.zeros((H, W))
    g_tar = np.zeros((H, W))
    g_plane = np.zeros(3)
    for a, gr, gt, gp in pool.map(_soft_band, jobs):
        g_ref[a:a + gr.shape[0]] += gr
        g_tar[a:a + gt.shape[0]] += gt
        # crop plane (c0 + c2 a, c1, c2): chain rule back to (c0, c1, c2)
        g_plane += np.array([gp[0], gp[1], gp[2] + a * gp[0]])
    return g_ref, g_tar, g_plane
