"""The row-band decomposition used by the full-frame parity tests equals the
whole-frame oracle: plain outputs (levels, validity, sub-pixel levels and
disparities, the tie gaps and the parabola curvature) and the soft-argmin
gradient, on small frames with a rolled plane and a general homography."""
from dataclasses import replace

import numpy as np
import pytest

import oracle.soft as SO
import oracle.stereo as OS
from synth import crop_workload, make_scene, skewed_pair, workload
from tests import oracle_bands as OB


@pytest.fixture(scope="module")
def pool():
    with OB.process_pool(3) as p:
        yield p


def _cases():
    w1 = crop_workload(workload("c1"), 61, 37, num_disp=9, delta_p=4.0, ncc_radius=2,
                       bil_radius=3, plane=(6.2, -0.03, 0.08))
    s1 = make_scene(w1.width, w1.height, w1.plane, 1, 1, 131)
    w2 = crop_workload(workload("c1"), 52, 33, num_disp=8, delta_p=4.0, ncc_radius=1,
                       bil_radius=2)
    sc, tar2, _, Hm, _ = skewed_pair(w2, angle_deg=0.5, dy=0.6)
    w2 = replace(w2, homography=tuple(Hm.ravel()))
    w3 = crop_workload(workload("c3b"), 47, 29, num_disp=10, ncc_radius=1, bil_radius=2)
    s3 = make_scene(w3.width, w3.height, (5.0, 0.0, 0.1), 1, 0, 133)
    return {"rolled": (w1, s1.ref, s1.tar), "homography": (w2, sc.ref, tar2),
            "raw": (w3, s3.ref, s3.tar)}


@pytest.mark.parametrize("name", ["rolled", "homography", "raw"])
def test_match_bands_equal_whole_frame(pool, name):
    w, ref, tar = _cases()[name]
    full = OS.match(ref, tar, w, keep_volumes=True)
    got = OB.match_full(ref, tar, w, pool, n_bands=5)
    for k in ("dint_R", "dint_T", "valid"):
        assert np.array_equal(got[k], full[k]), k
    assert np.allclose(got["ell"], full["ell"], rtol=0, atol=1e-12)
    assert np.array_equal(np.isnan(got["disp"]), np.isnan(full["disp"]))
    fin = ~np.isnan(full["disp"])
    assert np.allclose(got["disp"][fin], full["disp"][fin], rtol=0, atol=1e-9)
    for k, E in (("gapR", full["E_R"]), ("gapT", full["E_T"])):
        s = np.sort(E, axis=0)
        assert np.allclose(got[k], s[1] - s[0], rtol=0, atol=1e-13), k
    D = w.num_disp
    d = full["dint_R"]
    e = lambda k: np.take_along_axis(full["E_R"], np.clip(k, 0, D - 1)[None], 0)[0]
    assert np.allclose(got["curv"], e(d - 1) + e(d + 1) - 2 * e(d), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n_bands", [4, 8, 13])
def test_soft_gradient_bands_equal_whole_frame(pool, n_bands):
    """The plane (5.05, 0, 0.1) keeps every warp sample 0.05 px or more from
    a lerp knot (X = x - 2.05 - 0.1 v): at a knot the warp's derivative in
    the plane is one-sided, and which side a sample takes would depend on
    the rounding of the plane's row term in crop coordinates."""
    w = crop_workload(workload("c5"), 46, 61, num_disp=7, delta_p=3.0, bil_radius=2,
                      ncc_radius=1, plane=(5.05, 0.0, 0.1))
    sc = make_scene(w.width, w.height, w.plane, 1, 0, 134, float_images=True)
    g = np.random.default_rng(135).normal(size=(w.height, w.width))
    fwd = SO.soft_forward(sc.ref, sc.tar, w.plane, w)
    full = SO.soft_backward(sc.ref, sc.tar, w.plane, w, fwd, g)
    got = OB.soft_grad_full(sc.ref, sc.tar, w.plane, w, g, pool, n_bands=n_bands)
    for a, b in zip(got[:2], full[:2]):
        assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(b)
    assert np.allclose(got[2], full[2], rtol=1e-11, atol=0)
