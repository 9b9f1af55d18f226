"""Pins of the FP64 road-fit oracle (Sec. 3.3) against closed forms:
ordinary least squares, the literal matrix form of Eqs. (26)-(27), finite
differences, and the rotated-map protocol of Sec. 4.4.2 (CPU only)."""
import math

import numpy as np
import pytest

import oracle.road as RD
import oracle.stereo as OS
from oracle import metrics
from synth import make_scene, workload

OR, OM = RD, metrics


def _rolled_points(rng, W=640, H=480, step=5, noise=0.3, psi=None, a1=None):
    psi = rng.uniform(-10, 10) * math.pi / 180 if psi is None else psi
    a1 = rng.uniform(0.05, 0.2) if a1 is None else a1
    a0 = rng.uniform(5, 30)
    v, u = np.mgrid[0:H:step, 0:W:step].astype(float)
    d = a0 + a1 * (v * math.cos(psi) - u * math.sin(psi))
    d = d + rng.normal(0, noise, d.shape) if noise else d
    return u.ravel(), v.ravel(), d.ravel(), psi, a0, a1


def _lstsq_plane(u, v, d):
    A = np.stack([np.ones_like(u), u, v], 1)
    c, res, *_ = np.linalg.lstsq(A, d, rcond=None)
    return c, float(np.sum((A @ c - d) ** 2))


@pytest.mark.parametrize("seed", range(6))
def test_roll_equals_least_squares_plane(seed):
    """min over psi of Eq. (23) is the 3-parameter plane fit; so psi must be
    atan(-c1/c2) of numpy's lstsq plane, and alpha, E_min follow."""
    rng = np.random.default_rng(200 + seed)
    u, v, d, *_ = _rolled_points(rng)
    fit = RD.fit_roll(u, v, d, 640, 480)
    c, resid = _lstsq_plane(u, v, d)
    psi_ls = math.atan(-c[1] / c[2])
    assert fit.converged
    assert abs(fit.psi - psi_ls) < 10 * RD.DELTA_PSI
    assert abs(fit.alpha0 - c[0]) < 1e-4 * abs(c[0])
    assert abs(fit.alpha1 - c[2] / math.cos(psi_ls)) < 1e-4 * abs(fit.alpha1)
    assert abs(fit.e_min - resid) < 1e-6 * resid


def test_energy_eq23_is_the_least_squares_residual():
    rng = np.random.default_rng(210)
    u, v, d, *_ = _rolled_points(rng)
    for psi in (-0.3, 0.0, 0.05, 1.2):
        Y = np.stack([np.ones_like(u), v * math.cos(psi) - u * math.sin(psi)], 1)
        a, *_ = np.linalg.lstsq(Y, d, rcond=None)
        assert abs(RD.energy(u, v, d, psi) - np.sum((Y @ a - d) ** 2)) < 1e-8 * np.sum(d * d)


def test_gradient_equals_literal_matrix_form():
    """Eqs. (26)-(27) with the n x n matrices W = (I - Y J) dY J, on 50 points."""
    rng = np.random.default_rng(211)
    u, v = rng.uniform(0, 100, 50), rng.uniform(0, 80, 50)
    d = 10 + 0.1 * v - 0.02 * u + rng.normal(0, 0.5, 50)
    for psi in (-0.4, -0.05, 0.0, 0.2, 1.0):
        Y = np.stack([np.ones(50), v * math.cos(psi) - u * math.sin(psi)], 1)
        dY = np.stack([np.zeros(50), -v * math.sin(psi) - u * math.cos(psi)], 1)
        J = np.linalg.inv(Y.T @ Y) @ Y.T
        Wm = (np.eye(50) - Y @ J) @ dY @ J
        lit = -2.0 * d @ Wm @ d
        assert abs(RD.gradient(u, v, d, psi) - lit) < 1e-9 * max(1.0, abs(lit))


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(212)
    u, v, d, *_ = _rolled_points(rng, step=8)
    for psi in (-0.2, 0.01, 0.15):
        h = 1e-6
        fd = (RD.energy(u, v, d, psi + h) - RD.energy(u, v, d, psi - h)) / (2 * h)
        g = RD.gradient(u, v, d, psi)
        assert abs(g - fd) < 1e-5 * max(1.0, abs(fd))


@pytest.mark.parametrize("psi_true", [-0.17, -0.05, 0.0, 0.03, 0.12, 0.17])
def test_rotated_map_protocol(psi_true):
    """Sec. 4.4.2: rotate a zero-roll disparity map by a known angle and
    recover it.  Noise-free, the estimate is exact to the stopping tolerance."""
    rng = np.random.default_rng(213)
    u, v, d, *_ = _rolled_points(rng, psi=psi_true, a1=0.12, noise=0.0)
    fit = RD.fit_roll(u, v, d, 640, 480)
    assert abs(fit.psi - psi_true) < 10 * RD.DELTA_PSI
    assert fit.iters <= 10


def test_warm_start_from_previous_psi():
    rng = np.random.default_rng(214)
    u, v, d, psi, *_ = _rolled_points(rng, psi=0.1, noise=0.2)
    cold = RD.fit_roll(u, v, d, 640, 480)
    warm = RD.fit_roll(u, v, d, 640, 480, psi0=cold.psi + 1e-4)
    assert abs(warm.psi - cold.psi) < 10 * RD.DELTA_PSI
    assert warm.iters <= cold.iters


def test_roll_removal_lowers_sigma_d():
    """Sec. 4.4.3's direction: removing the roll leaves a flatter map than a
    fit forced to psi = 0."""
    rng = np.random.default_rng(215)
    H, W = 120, 160
    v, u = np.mgrid[0:H, 0:W].astype(float)
    d = 12 + 0.1 * (v * math.cos(0.12) - u * math.sin(0.12)) + rng.normal(0, 0.2, (H, W))
    fit, dt = RD.road_transform(d)
    uu, vv, dd = RD.road_points(d)
    a = RD.alpha(uu, vv, dd, 0.0)
    fit0 = RD.RoadFit(0.0, a[0], a[1], 0.0, 0, True, False)
    assert metrics.sigma_d(dt) < metrics.sigma_d(RD.transform(d, fit0))
    assert metrics.sigma_d(dt) < 0.25


def test_transform_subtracts_the_fitted_plane():
    fit = RD.RoadFit(0.1, 5.0, 0.2, 0.0, 3, True, False)
    d = np.random.default_rng(216).uniform(0, 40, (6, 9))
    v, u = np.mgrid[0:6, 0:9]
    c0, c1, c2 = fit.plane
    assert np.allclose(RD.transform(d, fit, 3.0), d - (c0 + c1 * u + c2 * v) + 3.0,
                       atol=1e-12)


def test_flat_map_returns_psi0():
    d = np.full((20, 30), 7.0)
    fit, dt = RD.road_transform(d, psi0=0.02)
    assert fit.flat and fit.psi == 0.02
    assert np.allclose(dt, 0.0, atol=1e-9)


def test_iteration_cap_reports_not_converged():
    rng = np.random.default_rng(217)
    u, v, d, *_ = _rolled_points(rng, psi=0.15)
    fit = RD.fit_roll(u, v, d, 640, 480, max_iter=1)
    assert not fit.converged and fit.iters == 1


def test_wrap_into_half_open_interval():
    for x in (-math.pi / 2, math.pi / 2, 0.3, 2.0, -2.0, 3 * math.pi / 2):
        w = RD._wrap(x)
        assert -math.pi / 2 < w <= math.pi / 2
        assert abs(math.sin(2 * (w - x))) < 1e-12


def test_damage_mask_threshold_rule():
    """Hand-built FP32 values around the level delta_t - tau (Sec. 4.4.3)."""
    dt = np.array([[0.0, -0.49, -0.5, -0.51, np.nan],
                   [-np.inf, np.inf, 1.0, -3.0, np.float32(-0.5) - np.float32(1e-7)]],
                  np.float32)
    m = OR.damage_mask(dt, 0.0, 0.5)
    assert m.tolist() == [[False, False, False, True, False],
                          [False, False, False, True, True]]
    # delta_t shifts the level; the comparison is strict
    assert OR.damage_mask(np.float32([[2.5]]), 3.0, 0.5).tolist() == [[False]]
    assert OR.damage_mask(np.float32([[2.49]]), 3.0, 0.5).tolist() == [[True]]


def test_iou_small_cases():
    a = np.array([[1, 1, 0], [0, 0, 0]], bool)
    b = np.array([[0, 1, 1], [0, 0, 0]], bool)
    assert OM.iou(a, b) == pytest.approx(1.0 / 3.0)
    assert OM.iou(a, a) == 1.0
    assert OM.iou(a, ~a) == 0.0
    assert OM.iou(np.zeros((2, 2), bool), np.zeros((2, 2), bool)) == 1.0
    sel = np.array([[1, 1, 0], [1, 1, 1]], bool)      # drops the disagreeing pixel
    assert OM.iou(a, b, sel) == pytest.approx(0.5)


@pytest.mark.parametrize("seed,npot,ncr", [(11, 6, 2), (12, 4, 1), (13, 0, 0)])
def test_damage_segmentation_on_synthetic_roads(seed, npot, ncr):
    """Sanity bounds against the generator's ground truth, not parity: on
    interior visible pixels the damage found at tau = 0.5 overlaps the
    region deeper than tau with IoU >= 0.75, and plain road is almost never
    flagged; a scene without damage gives an empty mask."""
    w = workload("c1")
    sc = make_scene(w.width, w.height, w.plane, npot, ncr, seed)
    o = OS.match(sc.ref, sc.tar, w)
    fit, dt = OR.road_transform(o["disp"], o["valid"])
    vv, uu = np.mgrid[0:w.height, 0:w.width]
    depth = w.plane[0] + w.plane[1] * uu + w.plane[2] * vv - sc.d_gt
    r = w.ncc_radius + w.bil_radius
    sel = np.zeros(sc.visible.shape, bool)
    sel[r:-r, w.num_disp + r:-r] = True
    sel &= sc.visible
    m = OR.damage_mask(dt, 0.0, 0.5)
    assert OM.iou(m, depth >= 0.5, sel) >= 0.75
    assert np.mean(m[sel & sc.road_mask]) <= 0.005
    if npot == 0 and ncr == 0:
        assert not m[sel].any()


def test_plane_from_fit_closed_form():
    """An exact rolled planar disparity map: the fit's plane is the map's."""
    c = (7.5, -0.012, 0.094)
    vv, uu = np.mgrid[0:120, 0:160].astype(float)
    d = c[0] + c[1] * uu + c[2] * vv
    fit, _ = RD.road_transform(d)
    # the descent stops within its step tolerance delta_psi of the roll
    assert abs(fit.psi - math.atan(-c[1] / c[2])) <= 10 * RD.DELTA_PSI
    p = RD.plane_from_fit(fit)
    err = (p[0] - c[0]) + (p[1] - c[1]) * uu + (p[2] - c[2]) * vv
    assert np.max(np.abs(err)) <= 1e-4


def test_closed_loop_tracks_a_drifting_road():
    """Frame t matched with the plane fitted on frame t-1 (bootstrap: a
    full-range pass without the perspective transformation on frame 0)
    follows a slowly drifting plane and keeps road pixels accurate
    (sanity bounds against ground truth)."""
    from dataclasses import replace
    from synth import road_sequence
    w = workload("c1")
    seq = road_sequence(w.width, w.height, 4, seed=21)
    wr = replace(w, perspective=False, delta_p=0.0, num_disp=48)
    _, _, sc0 = seq[0]
    o = OS.match(sc0.ref, sc0.tar, wr)
    fit, _ = RD.road_transform(o["disp"], o["valid"])
    plane, psi = RD.plane_from_fit(fit), fit.psi
    vv, uu = np.mgrid[0:w.height, 0:w.width]
    r = w.ncc_radius + w.bil_radius
    for c, psi_true, sc in seq[1:]:
        o = OS.match(sc.ref, sc.tar, replace(w, plane=tuple(plane)))
        sel = np.zeros(sc.visible.shape, bool)
        sel[r:-r, w.num_disp + r:-r] = True
        sel &= sc.visible & sc.road_mask & np.isfinite(o["disp"])
        assert metrics.error_pixel_percent(o["disp"], sc.d_gt, 1.0, sel) <= 1.0
        fit, _ = RD.road_transform(o["disp"], o["valid"], psi0=psi)
        plane, psi = RD.plane_from_fit(fit), fit.psi
        err = (plane[0] - c[0]) + (plane[1] - c[1]) * uu + (plane[2] - c[2]) * vv
        assert np.max(np.abs(err)) <= 0.3
        assert abs(psi - psi_true) <= math.radians(0.5)
