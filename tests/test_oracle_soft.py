"""Pins of the differentiable-form oracle: central finite differences in FP64
of its forward pass, and the soft-argmin's hard limit (CPU only).

Finite differences cannot cross a kink without error, so the test plane puts
every warp sample at least 0.05 px from a lerp knot: with delta_p = 24 and
c = (24.05, 0, 0.1), X = x - 0.05 - 0.1 v has fractional parts 0.05..0.95.
Steps: h = 1e-3 for images, c0 and c2 (|dX| <= 0.047), h = 5e-4 for c1
(|dX| <= 5e-4 (x + 24) < 0.05 on a 64-wide crop).  The L1 loss is checked
where |ref - s| > 1e-2 (away from its kink).
"""
from dataclasses import replace

import numpy as np
import pytest
from scipy import ndimage

import oracle.soft as SO
import oracle.stereo as OS
from synth import crop_workload, make_scene, workload

PLANE = (24.05, 0.0, 0.1)


@pytest.fixture(scope="module")
def setup():
    w = crop_workload(workload("c5"), 64, 48, num_disp=16, delta_p=24.0, bil_radius=3,
                      sigma_s=2.5, plane=PLANE)
    sc = make_scene(64, 48, (24.0, 0.0, 0.1), 1, 0, 41, float_images=True)
    ref = sc.ref.astype(np.float64)
    tar = sc.tar.astype(np.float64)
    rng = np.random.default_rng(400)
    g = ndimage.gaussian_filter(rng.normal(size=(48, 64)), 2.0)
    fwd = SO.soft_forward(ref, tar, PLANE, w)
    g_ref, g_tar, g_plane = SO.soft_backward(ref, tar, PLANE, w, fwd, g)
    return w, ref, tar, g, g_ref, g_tar, g_plane


def _Lg(w, ref, tar, plane, g):
    return float(np.sum(g * SO.soft_forward(ref, tar, plane, w)["disp"]))


def _rel(a, b, scale):
    return abs(a - b) / max(abs(b), 1e-8 * scale)


def test_plane_gradient_matches_fd(setup):
    w, ref, tar, g, g_ref, g_tar, g_plane = setup
    for k, h in ((0, 1e-3), (1, 5e-4), (2, 1e-3)):
        cp = list(PLANE); cm = list(PLANE)
        cp[k] += h; cm[k] -= h
        fd = (_Lg(w, ref, tar, cp, g) - _Lg(w, ref, tar, cm, g)) / (2 * h)
        assert _rel(g_plane[k], fd, np.abs(g_plane).max()) < 1e-3, (k, g_plane[k], fd)


@pytest.mark.parametrize("which", ["ref", "tar"])
def test_image_gradients_match_fd(setup, which):
    w, ref, tar, g, g_ref, g_tar, g_plane = setup
    grad = g_ref if which == "ref" else g_tar
    rng = np.random.default_rng(401 if which == "ref" else 402)
    h = 1e-3
    idx = list(zip(rng.integers(0, 48, 24), rng.integers(0, 64, 24)))
    idx += [(0, 0), (47, 63), (0, 63), (20, 0), (47, 30)]      # clamped borders
    scale = np.abs(grad).max()
    for (y, x) in idx:
        a = ref.copy() if which == "ref" else tar.copy()
        b = a.copy()
        a[y, x] += h
        b[y, x] -= h
        if which == "ref":
            fd = (_Lg(w, a, tar, PLANE, g) - _Lg(w, b, tar, PLANE, g)) / (2 * h)
        else:
            fd = (_Lg(w, ref, a, PLANE, g) - _Lg(w, ref, b, PLANE, g)) / (2 * h)
        assert _rel(grad[y, x], fd, scale) < 1e-3, (which, y, x, grad[y, x], fd)


def test_directional_derivatives_match_fd(setup):
    w, ref, tar, g, g_ref, g_tar, g_plane = setup
    rng = np.random.default_rng(403)
    h = 1e-3
    for _ in range(4):
        dr = rng.normal(size=ref.shape)
        dt = rng.normal(size=tar.shape)
        an = float(np.sum(g_ref * dr) + np.sum(g_tar * dt))
        fd = (_Lg(w, ref + h * dr, tar + h * dt, PLANE, g)
              - _Lg(w, ref - h * dr, tar - h * dt, PLANE, g)) / (2 * h)
        assert _rel(an, fd, abs(fd)) < 1e-3, (an, fd)


def test_l1_backward_matches_fd():
    rng = np.random.default_rng(404)
    sc = make_scene(40, 24, (6.0, 0.0, 0.1), 0, 0, 42, float_images=True)
    ref, tar = sc.ref.astype(np.float64), sc.tar.astype(np.float64)
    disp = 6.0 + 0.1 * np.arange(24)[:, None] + rng.uniform(-0.4, 0.4, (24, 40)) + 0.013
    g_ref, g_tar, g_disp = SO.photometric_l1_backward(ref, tar, disp, 1.0)
    v, u = np.mgrid[0:24, 0:40]
    s = OS.lerp_row(tar, v, u - disp)
    ok = np.abs(ref - s) > 1e-2
    frac = np.abs((u - disp) - np.rint(u - disp)) > 2e-3
    h = 1e-4
    for (y, x) in zip(rng.integers(0, 24, 30), rng.integers(10, 40, 30)):
        if not (ok[y, x] and frac[y, x]):
            continue
        dp, dm = disp.copy(), disp.copy()
        dp[y, x] += h
        dm[y, x] -= h
        fd = (SO.photometric_l1(ref, tar, dp) - SO.photometric_l1(ref, tar, dm)) / (2 * h)
        assert abs(g_disp[y, x] - fd) < 1e-6 * max(1.0, abs(fd)) + 1e-9
        rp, rm = ref.copy(), ref.copy()
        rp[y, x] += h
        rm[y, x] -= h
        fd = (SO.photometric_l1(rp, tar, disp) - SO.photometric_l1(rm, tar, disp)) / (2 * h)
        assert abs(g_ref[y, x] - fd) < 1e-9
    dt = rng.normal(size=tar.shape)
    fd = (SO.photometric_l1(ref, tar + 1e-5 * dt, disp)
          - SO.photometric_l1(ref, tar - 1e-5 * dt, disp)) / 2e-5
    assert abs(np.sum(g_tar * dt) - fd) < 1e-6 * abs(fd)


def test_soft_argmin_hard_limit_is_wta():
    """T -> 0: the soft level equals the WTA level wherever the minimum is clear."""
    w = crop_workload(workload("c5"), 48, 32, num_disp=12, delta_p=6.0, bil_radius=2)
    sc = make_scene(48, 32, (6.0, 0.0, 0.1), 1, 0, 43, float_images=True)
    fwd = SO.soft_forward(sc.ref, sc.tar, w.plane, w, T=1e-4)
    dint = OS.wta(fwd["E"])
    s = np.sort(fwd["E"], axis=0)
    clear = (s[1] - s[0]) > 1e-2
    assert clear[:, 20:].mean() > 0.5
    assert np.max(np.abs(fwd["dh"][clear] - dint[clear])) < 1e-9
    assert fwd["dh"].min() >= 0.0 and fwd["dh"].max() <= w.num_disp - 1


def test_soft_forward_reuses_the_plain_pipeline():
    """The soft head's E is the plain path's aggregated reference volume."""
    w = crop_workload(workload("c5"), 40, 30, num_disp=10, delta_p=5.0, bil_radius=2,
                      plane=(5.0, 0.0, 0.1))
    sc = make_scene(40, 30, w.plane, 1, 0, 44, float_images=True)
    fwd = SO.soft_forward(sc.ref, sc.tar, w.plane, w)
    plain = OS.match(sc.ref, sc.tar, w, keep_volumes=True)
    assert np.array_equal(fwd["E"], plain["E_R"])
    assert np.allclose(fwd["P"].sum(0), 1.0)


def test_softmax_state_closed_form_on_uniform_costs():
    """A uniform reference has zero-variance blocks everywhere, so every cost
    is 1 (Eq. 8 undefined, read as 1) and so is every aggregated cost: the
    soft-argmin is then uniform over the D levels, with max_d(-E/T) = -1/T,
    log Z = ln D (Z = sum_d exp(-E/T - max)) and soft level (D - 1) / 2."""
    w = crop_workload(workload("c5"), 37, 23, num_disp=11, delta_p=5.0, bil_radius=2,
                      ncc_radius=1, plane=(5.3, 0.0, 0.1))
    sc = make_scene(37, 23, (5.3, 0.0, 0.1), 0, 0, 71, float_images=True)
    ref = np.full((23, 37), 97.25)
    f = SO.soft_forward(ref, sc.tar, w.plane, w, T=0.25)
    assert np.all(f["C"] == 1.0)
    assert np.allclose(f["E"], 1.0, rtol=0, atol=1e-14)
    assert np.allclose(f["m"], -1.0 / 0.25, rtol=0, atol=1e-12)
    assert np.allclose(f["logZ"], np.log(11.0), rtol=0, atol=1e-12)
    assert np.allclose(f["P"], 1.0 / 11.0, rtol=0, atol=1e-14)
    assert np.allclose(f["dh"], 5.0, rtol=0, atol=1e-12)


def test_softmax_state_is_the_log_partition_function():
    """On a textured pair: m is the maximum of -E/T over levels and m + log Z
    is log sum_d exp(-E/T), computed by scipy's logsumexp (its own
    max-shifted evaluation); P sums to one; the soft level lies in [0, D-1]."""
    from scipy.special import logsumexp
    w = crop_workload(workload("c5"), 41, 29, num_disp=13, delta_p=6.0, bil_radius=2,
                      ncc_radius=1, plane=(6.2, 0.0, 0.1))
    sc = make_scene(41, 29, (6.2, 0.0, 0.1), 1, 0, 72, float_images=True)
    T = 0.1
    f = SO.soft_forward(sc.ref, sc.tar, w.plane, w, T=T)
    z = -f["E"] / T
    assert np.array_equal(f["m"], z.max(axis=0))
    assert np.allclose(f["m"] + f["logZ"], logsumexp(z, axis=0), rtol=0, atol=1e-12)
    assert np.allclose(f["P"].sum(axis=0), 1.0, rtol=0, atol=1e-13)
    assert np.all((f["dh"] >= 0) & (f["dh"] <= 12))
    # a two-level closed form: P(d=1) = 1 / (1 + exp((E1 - E0) / T))
    two = crop_workload(w, 41, 29, num_disp=2, delta_p=1.0)
    f2 = SO.soft_forward(sc.ref, sc.tar, w.plane, two, T=T)
    p1 = 1.0 / (1.0 + np.exp((f2["E"][1] - f2["E"][0]) / T))
    assert np.allclose(f2["dh"], p1, rtol=0, atol=1e-13)
    assert np.allclose(f2["logZ"], np.log1p(np.exp(-np.abs(f2["E"][1] - f2["E"][0]) / T)),
                       rtol=0, atol=1e-13)
