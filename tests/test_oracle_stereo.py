"""Pins of the FP64 oracle's stereo steps against things other than itself:
brute force on tiny inputs, textbook routines the method reduces to, closed
forms and invariants (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle.stereo as S

OS = S
from oracle import metrics
from synth import crop_workload, make_scene, workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class P:  # minimal parameter bag
    def __init__(self, **kw):
        self.__dict__.update(dict(delta_p=0.0, perspective=False, plane=(0, 0, 0),
                                  lr_delta=1.0), **kw)


def _rand_img(rng, H, W):
    return rng.integers(0, 256, size=(H, W)).astype(np.float64)


def _pearson_cost(xb, yb):
    """1 - Pearson correlation (textbook definition, numpy's corrcoef)."""
    if np.var(xb) < S.FLAT_VAR or np.var(yb) < S.FLAT_VAR:
        return 1.0
    return 1.0 - np.corrcoef(xb, yb)[0, 1]


def _block(img, u, v, r):
    H, W = img.shape
    return np.array([img[min(max(v + i, 0), H - 1), min(max(u + j, 0), W - 1)]
                     for i in range(-r, r + 1) for j in range(-r, r + 1)])


def test_ncc_equals_one_minus_pearson_bruteforce():
    """Eq. (8) with population statistics is 1 - Pearson correlation; checked
    with explicit loops over every pixel, level and clamped block."""
    rng = np.random.default_rng(100)
    H, W, D, r = 7, 9, 4, 1
    X, Y = _rand_img(rng, H, W), _rand_img(rng, H, W)
    CR, CT = S.ncc_volumes(X, Y, D, r)
    for d in range(D):
        for v in range(H):
            for u in range(W):
                cr = _pearson_cost(_block(X, u, v, r), _block(Y, u - d, v, r))
                ct = _pearson_cost(_block(X, u + d, v, r), _block(Y, u, v, r))
                assert abs(CR[d, v, u] - cr) < 1e-12
                assert abs(CT[d, v, u] - ct) < 1e-12


@pytest.mark.parametrize("a,b,expect", [(1.7, -30.0, 0.0), (0.5, 12.0, 0.0),
                                        (-1.3, 200.0, 2.0)])
def test_ncc_affine_copy(a, b, expect):
    """An affine-intensity copy has NCC = +1 (cost 0) for a > 0 and -1
    (cost 2) for a < 0, at level 0, for every pixel."""
    rng = np.random.default_rng(101)
    X = _rand_img(rng, 12, 15)
    CR, CT = S.ncc_volumes(X, a * X + b, 3, 2)
    assert np.max(np.abs(CR[0] - expect)) < 1e-12
    assert np.max(np.abs(CT[0] - expect)) < 1e-12


def test_ncc_flat_block_cost_is_one():
    X = np.full((6, 8), 77.0)
    rng = np.random.default_rng(102)
    CR, _ = S.ncc_volumes(X, _rand_img(rng, 6, 8), 3, 1)
    assert np.all(CR == 1.0)


def test_identical_images_give_zero_disparity():
    rng = np.random.default_rng(103)
    img = ndimage.gaussian_filter(rng.uniform(0, 255, (30, 40)), 1.0)
    p = P(num_disp=8, ncc_radius=2, bil_radius=2, sigma_s=2.0, sigma_r=10.0)
    out = S.match(img, img, p)
    assert np.all(out["dint_R"] == 0)
    assert np.all(out["dint_T"] == 0)
    assert np.all(out["valid"])
    assert np.all(out["disp"] == 0.0)


def test_warp_integer_shift_is_exact():
    """c1 = c2 = 0 and integral c0, delta_p: every row moves by c0 - delta_p."""
    rng = np.random.default_rng(104)
    tar = _rand_img(rng, 5, 20)
    tw = S.warp(tar, (7.0, 0.0, 0.0), 3.0)
    x = np.arange(20)
    src = np.clip(x + 3 - 7, 0, 19)
    assert np.array_equal(tw, tar[:, src])


def test_warp_fractional_shift_is_linear_interpolation():
    tar = np.tile(np.arange(10, dtype=np.float64) ** 2, (3, 1))
    tw = S.warp(tar, (0.25, 0.0, 0.0), 0.0)
    X = np.clip(np.arange(10) - 0.25, 0, 9)
    assert np.allclose(tw[0], np.interp(X, np.arange(10), tar[0]), atol=1e-12)


def test_planar_scene_lands_on_level_delta_p():
    """With the road plane known, every interior road pixel of a scene with no
    damage matches at residual 0, i.e. at level delta_p (Sec. 3.1)."""
    w = crop_workload(workload("c1"), 160, 96, n_potholes=0, n_cracks=0)
    sc = make_scene(w.width, w.height, w.plane, 0, 0, 11)
    out = S.match(sc.ref, sc.tar, w)
    inner = out["dint_R"][8:-8, 40:-8]
    assert np.mean(inner == int(w.delta_p)) > 0.99


def _sep_gaussian_normalised(C, R, sigma_s):
    k = np.arange(-R, R + 1)
    g = np.exp(-(k * k) / sigma_s ** 2)

    def filt(a):
        a = ndimage.correlate1d(a, g, axis=-1, mode="constant", cval=0.0)
        return ndimage.correlate1d(a, g, axis=-2, mode="constant", cval=0.0)

    return filt(C) / filt(np.ones(C.shape[-2:]))[None]


def test_bilateral_infinite_range_sigma_is_gaussian():
    """sigma_r -> infinity: Eq. (11) is a normalised separable Gaussian on the
    image-truncated window (zero padding, divided by the filtered ones)."""
    rng = np.random.default_rng(105)
    C = rng.uniform(0, 2, (3, 17, 23))
    G = _rand_img(rng, 17, 23)
    E = S.bilateral(C, G, 4, 2.5, 1e30)
    assert np.max(np.abs(E - _sep_gaussian_normalised(C, 4, 2.5))) < 1e-12


def test_bilateral_constant_slice_stays_constant():
    rng = np.random.default_rng(106)
    C = np.broadcast_to(np.array([0.3, 1.1, 1.9])[:, None, None], (3, 9, 11)).copy()
    E = S.bilateral(C, _rand_img(rng, 9, 11), 3, 1.5, 5.5)
    assert np.max(np.abs(E - C)) < 1e-14


def test_bilateral_bruteforce_four_loops():
    rng = np.random.default_rng(107)
    D, H, W, R, ss, sr = 2, 5, 6, 2, 1.7, 9.0
    C = rng.uniform(0, 2, (D, H, W))
    G = _rand_img(rng, H, W)
    E = S.bilateral(C, G, R, ss, sr)
    for d in range(D):
        for v in range(H):
            for u in range(W):
                num = den = 0.0
                for qv in range(v - R, v + R + 1):
                    for qu in range(u - R, u + R + 1):
                        if 0 <= qv < H and 0 <= qu < W:
                            w = math.exp(-((qu - u) ** 2 + (qv - v) ** 2) / ss ** 2
                                         - (G[v, u] - G[qv, qu]) ** 2 / sr ** 2)
                            num += w * C[d, qv, qu]
                            den += w
                assert abs(E[d, v, u] - num / den) < 1e-13


def test_wta_subpixel_recovers_parabola_vertex():
    D = 16
    d = np.arange(D, dtype=np.float64)
    for d0 in [1.0, 3.25, 7.5, 10.9, 14.0]:
        E = ((d - d0) ** 2)[:, None, None] + 0.4
        dint = S.wta(E)
        ell = S.subpixel(E, dint)
        assert abs(ell[0, 0] - d0) < 1e-12


def test_subpixel_offset_is_bounded_by_half():
    rng = np.random.default_rng(108)
    E = rng.uniform(0, 2, (9, 40, 40))
    dint = S.wta(E)
    off = S.subpixel(E, dint) - dint
    assert np.all(np.abs(off) <= 0.5 + 1e-15)


def test_subpixel_skips_range_ends():
    E = np.array([0.1, 0.5, 0.9, 1.0, 0.95])[:, None, None]
    assert S.subpixel(E, S.wta(E))[0, 0] == 0.0
    E = E[::-1].copy()
    assert S.subpixel(E, S.wta(E))[0, 0] == 4.0


def test_wta_first_minimum_on_ties():
    E = np.array([0.5, 0.2, 0.2, 0.7])[:, None, None]
    assert S.wta(E)[0, 0] == 1


def test_lr_check_handbuilt():
    dR = np.array([[0, 1, 2, 2, 4, 1]])
    dT = np.array([[0, 1, 0, 5, 0, 0]])
    # u=0: x=0, dT=0 -> ok; u=1: x=0, |1-0|^2=1 -> ok; u=2: x=0, 4 > 1 -> bad
    # u=3: x=1, |2-1|=1 -> ok; u=4: x=0, 16 -> bad; u=5: x=4, |1-0|=1 -> ok
    assert S.lr_check(dR, dT, 1.0).tolist() == [[True, True, False, True, False, True]]
    dR2 = np.array([[3, 0]])
    assert S.lr_check(dR2, np.zeros((1, 2), int), 1.0).tolist() == [[False, True]]


def test_shift_back_inverts_the_warp_with_roll():
    """A level-delta_p match maps back to d_road at the same pixel for c1 != 0."""
    plane = (10.0, -0.03, 0.08)
    ell = np.full((4, 50), 20.0)
    disp = S.shift_back(ell, np.ones((4, 50), bool), plane, 20.0)
    v, u = np.mgrid[0:4, 0:50]
    assert np.allclose(disp, S.d_road(plane, u, v), atol=1e-12)


def test_end_to_end_planar_road_accuracy():
    """Ground-truth sanity bounds on a damage-free road (not parity)."""
    w = crop_workload(workload("c1"), 160, 120, n_potholes=0, n_cracks=0)
    sc = make_scene(w.width, w.height, w.plane, 0, 0, 12)
    out = S.match(sc.ref, sc.tar, w)
    sel = np.zeros_like(sc.visible)
    sel[6:-6, 30:-6] = True
    sel &= sc.visible & out["valid"]
    err = out["disp"][sel] - sc.d_gt[sel]
    assert metrics.error_pixel_percent(out["disp"][sel], sc.d_gt[sel], 1.0) <= 2.0
    assert abs(np.median(err)) <= 0.25


def test_perspective_transform_not_less_accurate():
    """Sec. 5: the perspective transformation improves accuracy; with it, the
    damage-scene error is no larger than a plain full-range search."""
    w = crop_workload(workload("c1"), 160, 120, n_potholes=3, n_cracks=0)
    sc = make_scene(w.width, w.height, w.plane, 3, 0, 13)
    on = S.match(sc.ref, sc.tar, w)
    from dataclasses import replace
    off = S.match(sc.ref, sc.tar, replace(w, num_disp=28, delta_p=0.0, perspective=False))
    sel = np.zeros_like(sc.visible)
    sel[6:-6, 30:-6] = True
    sel &= sc.visible
    both = sel & on["valid"] & off["valid"]
    e_on = metrics.rms_error(on["disp"][both], sc.d_gt[both])
    e_off = metrics.rms_error(off["disp"][both], sc.d_gt[both])
    assert both.sum() > 0.8 * sel.sum()
    assert e_on <= e_off


def test_pointwise_matches_full_volume():
    w = crop_workload(workload("c1"), 64, 40)
    sc = make_scene(w.width, w.height, w.plane, 2, 0, 14)
    full = S.match(sc.ref, sc.tar, w, keep_volumes=True)
    pts = [(0, 0), (63, 39), (17, 3), (40, 20), (5, 39)]
    for q in S.match_at(sc.ref, sc.tar, w, pts, tar_w=full["tar_w"]):
        u, v = q["u"], q["v"]
        assert np.max(np.abs(q["E_R"] - full["E_R"][:, v, u])) < 1e-12
        assert q["dint_R"] == full["dint_R"][v, u]
        assert q["valid"] == full["valid"][v, u]


def test_mde_metric_reproduces_paper_figure():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["speed_example"]
    m = metrics.mde_per_s(g["u_max"], g["v_max"], g["d_max_implied"], g["t_seconds"])
    assert abs(m - g["mde_per_s"]) < 5e-4


def test_error_metrics_small_cases():
    gt = np.array([0.0, 1.0, 2.0, 3.0])
    ell = np.array([0.0, 1.5, 4.5, 3.0])
    assert metrics.error_pixel_percent(ell, gt, 2.0) == 25.0
    assert metrics.error_pixel_percent(ell, gt, 0.4) == 50.0
    assert abs(metrics.rms_error(ell, gt) - math.sqrt((0.25 + 6.25) / 4)) < 1e-15
    assert abs(metrics.sigma_d([1.0, 3.0]) - 1.0) < 1e-15


@pytest.mark.parametrize("plane", [(8.0, 0.0, 0.1), (9.5, -0.031, 0.087), (3.2, 0.02, 0.05)])
def test_homography_warp_reduces_to_the_row_shift(plane):
    """Eq. (3) with the plane's homography is the row shift of Sec. 3.1."""
    rng = np.random.default_rng(61)
    tar = rng.uniform(0, 255, (40, 90))
    Hm = OS.plane_homography(plane)
    assert np.allclose(OS.warp_homography(tar, Hm, 12.0), OS.warp(tar, plane, 12.0), atol=1e-9)
    ell = rng.uniform(0, 30, (40, 90))
    valid = rng.uniform(size=(40, 90)) < 0.8
    a = OS.shift_back_homography(ell, valid, Hm, 12.0)
    b = OS.shift_back(ell, valid, plane, 12.0)
    assert np.allclose(a, b, atol=1e-9, equal_nan=True)


def test_homography_identity_and_translation():
    rng = np.random.default_rng(62)
    tar = rng.uniform(0, 255, (30, 50))
    assert np.array_equal(OS.warp_homography(tar, np.eye(3), 0.0), tar)
    T = np.array([[1.0, 0.0, 3.0], [0.0, 1.0, 2.0], [0.0, 0.0, 1.0]])
    tw = OS.warp_homography(tar, T, 0.0)
    assert np.allclose(tw[:-2, :-3], tar[2:, 3:], atol=1e-12)
    # a projective H: the map of Eq. (3) divides by the third row
    P = np.array([[1.0, 0.1, 2.0], [0.0, 1.2, -1.0], [1e-3, 2e-3, 1.0]])
    X, Y = OS.homography_map(P, np.array([10.0]), np.array([5.0]))
    z = 1e-3 * 10 + 2e-3 * 5 + 1.0
    assert X[0] == pytest.approx((10 + 0.5 + 2) / z) and Y[0] == pytest.approx((6 - 1) / z)


def test_homography_map_composes():
    rng = np.random.default_rng(63)
    A = np.eye(3) + rng.normal(0, 0.01, (3, 3))
    B = np.eye(3) + rng.normal(0, 0.01, (3, 3))
    u, v = rng.uniform(0, 100, 20), rng.uniform(0, 80, 20)
    X1, Y1 = OS.homography_map(A @ B, u, v)
    X2, Y2 = OS.homography_map(A, *OS.homography_map(B, u, v))
    assert np.allclose(X1, X2, atol=1e-9) and np.allclose(Y1, Y2, atol=1e-9)


def test_skewed_rig_needs_the_general_homography():
    """A target camera rotated 0.3 degrees and shifted 0.8 rows: matched
    through Eq. (3) the disparities stay accurate (sanity bound against the
    generator's ground truth); the row shift alone is measurably worse."""
    from dataclasses import replace
    from synth import skewed_pair
    w = workload("c1")
    sc, tar2, _, Hm, dtrue = skewed_pair(w)
    r = w.ncc_radius + w.bil_radius
    sel = np.zeros(sc.visible.shape, bool)
    sel[r:-r, w.num_disp + r:-r] = True
    sel &= sc.visible
    o = OS.match(sc.ref, tar2, replace(w, homography=tuple(Hm.ravel())))
    fin = sel & np.isfinite(o["disp"])
    e_h = metrics.error_pixel_percent(o["disp"], dtrue, 1.0, fin)
    o1 = OS.match(sc.ref, tar2, w)
    fin1 = sel & np.isfinite(o1["disp"])
    e_row = metrics.error_pixel_percent(o1["disp"], dtrue, 1.0, fin1)
    assert e_h <= 0.5 and metrics.rms_error(o["disp"], dtrue, fin) <= 0.2
    assert e_row > 2.0 * max(e_h, 0.5)
