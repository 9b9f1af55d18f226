"""Differentiable form on the GPU vs the FP64 oracle (through the C ABI).

Bars: soft disparity and softmax state within 1e-4 * max(|x|, 1); every
gradient tensor within a relative L2 error of 1e-3, the three plane
components each within 1e-3 relative.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle.soft as SO
import oracle.stereo as OS
from synth import crop_workload, make_scene, make_workload_pair, workload

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1904_06017_amd.api")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _rel_l2(g, o):
    return float(np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30))


CASES = {
    # ragged sizes: several 32x32 / 16x16 tiles plus tails; D not a multiple of 16
    "c5_crop": dict(w=(150, 77), D=45, dp=22.0, plane=(24.0, 0.0, 0.1), R=5, r=3, seed=51),
    "rolled": dict(w=(130, 70), D=28, dp=14.0, plane=(14.3, -0.02, 0.09), R=4, r=2, seed=52),
    # the compiled maximum radii
    "max_radii": dict(w=(80, 40), D=20, dp=10.0, plane=(14.0, 0.01, 0.09), R=8, r=8, seed=55),
    # an exactly uniform reference patch (zero-variance blocks: cost 1, no
    # NCC gradient) and a uniform target strip along the bottom border
    "flat": dict(w=(120, 64), D=24, dp=12.0, plane=(14.3, 0.0, 0.1), R=4, r=2, seed=56,
                 flat_ref=(14, 44, 40, 80), flat_tar=(54, 64, 0, 120)),
}
FLAT_VALUE = 131.0
_cache = {}


def case(name):
    if name not in _cache:
        c = CASES[name]
        W, H = c["w"]
        w = crop_workload(workload("c5"), W, H, num_disp=c["D"], delta_p=c["dp"],
                          plane=c["plane"], bil_radius=c["R"], ncc_radius=c["r"])
        sc = make_scene(W, H, c["plane"], 2, 1, c["seed"], float_images=True)
        if "flat_ref" in c:
            ref, tar = sc.ref.copy(), sc.tar.copy()
            y0, y1, x0, x1 = c["flat_ref"]
            ref[y0:y1, x0:x1] = FLAT_VALUE
            y0, y1, x0, x1 = c["flat_tar"]
            tar[y0:y1, x0:x1] = FLAT_VALUE
            sc = replace(sc, ref=ref, tar=tar)
        rng = np.random.default_rng(c["seed"])
        g = ndimage.gaussian_filter(rng.normal(size=(H, W)), 2.0).astype(np.float32)
        print(f"[grad] case {name}: {W}x{H} D={c['D']} R={c['R']} r={c['r']}", flush=True)
        fwd = SO.soft_forward(sc.ref, sc.tar, c["plane"], w)
        bwd = SO.soft_backward(sc.ref, sc.tar, c["plane"], w, fwd, g.astype(np.float64))
        _cache[name] = (w, sc, g, fwd, bwd)
    return _cache[name]


@pytest.mark.parametrize("engine", [2, 1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_soft_forward(name, engine):
    """Every aggregation engine (2: matrix cores with split-FP16 operands, 1:
    matrix cores with FP32 operands, 0: vector ALU)."""
    w, sc, g, fwd, bwd = case(name)
    plan = api.Plan.from_workload(w)
    plan.set_tuning("agg_engine", engine)
    disp, saved = api.soft_forward(plan, _dev(sc.ref), _dev(sc.tar), w.plane)
    disp, saved = _host(disp), _host(saved)
    assert np.max(np.abs(disp - fwd["disp"]) / np.maximum(np.abs(fwd["disp"]), 1)) < 1e-4
    assert np.max(np.abs(saved[2] - fwd["dh"]) / np.maximum(np.abs(fwd["dh"]), 1)) < 1e-4
    assert np.max(np.abs(saved[0] - fwd["m"]) / np.maximum(np.abs(fwd["m"]), 1)) < 1e-4
    assert np.max(np.abs(saved[1] - fwd["logZ"]) / np.maximum(np.abs(fwd["logZ"]), 1)) < 1e-4


@pytest.mark.parametrize("engine", [2, 0], ids=["mfma16", "valu"])
@pytest.mark.parametrize("name", list(CASES))
def test_backward_matches_fp64_adjoint(name, engine):
    """engine 2: the aggregation passes on the split-FP16 matrix cores (R <= 5;
    the R = 8 case takes the vector ALU on both); engine 0: the vector ALU."""
    w, sc, g, fwd, bwd = case(name)
    plan = api.Plan.from_workload(w)
    plan.set_tuning("agg_engine", engine)
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    disp, saved = api.soft_forward(plan, ref, tar, w.plane)
    g_ref, g_tar, g_plane = api.backward(plan, ref, tar, w.plane, saved, _dev(g))
    o_ref, o_tar, o_plane = bwd
    assert _rel_l2(_host(g_ref), o_ref) < 1e-3
    assert _rel_l2(_host(g_tar), o_tar) < 1e-3
    gp = _host(g_plane)
    for k in range(3):
        assert abs(gp[k] - o_plane[k]) <= 1e-3 * max(abs(o_plane[k]), 1e-6 * np.abs(o_plane).max()), (k, gp, o_plane)


@pytest.mark.parametrize("engine", [2, 0], ids=["mfma16", "valu"])
def test_flat_patch_has_no_ncc_gradient(engine):
    """Inside an exactly uniform reference patch, deeper than 2r (every block
    reading the pixel is uniform: cost 1, no NCC gradient) and deeper than R
    (every guide difference is zero: no range-weight gradient), the
    reference gradient is exactly zero, on the GPU as in the oracle."""
    w, sc, g, fwd, bwd = case("flat")
    c = CASES["flat"]
    plan = api.Plan.from_workload(w)
    plan.set_tuning("agg_engine", engine)
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    disp, saved = api.soft_forward(plan, ref, tar, w.plane)
    g_ref, _, _ = api.backward(plan, ref, tar, w.plane, saved, _dev(g))
    y0, y1, x0, x1 = c["flat_ref"]
    m = max(c["R"], 2 * c["r"]) + 1
    inner = (slice(y0 + m, y1 - m), slice(x0 + m, x1 - m))
    assert np.all(bwd[0][inner] == 0.0)
    assert np.all(_host(g_ref)[inner] == 0.0)
    assert np.any(bwd[0][y0:y1, x0:x1] != 0.0)     # the patch rim still has gradient


def test_backward_is_deterministic_and_tile_invariant():
    w, sc, g, fwd, bwd = case("c5_crop")
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    res = []
    for lv in (16, 16, 8, None):
        plan = api.Plan.from_workload(w)
        if lv is None:
            # the default: every level (45, rounded up to 48) in one tile
            assert plan.get_tuning("grad_levels") == 48
        else:
            plan.set_tuning("grad_levels", lv)
        disp, saved = api.soft_forward(plan, ref, tar, w.plane)
        res.append([_host(x) for x in api.backward(plan, ref, tar, w.plane, saved, _dev(g))])
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)          # same tiling: bitwise
    for other in (res[2], res[3]):
        for a, b in zip(res[0], other):
            assert _rel_l2(a, b) < 1e-5      # another tiling: rounding only


@pytest.mark.parametrize("name", list(CASES))
def test_photometric_l1(name):
    w, sc, g, fwd, bwd = case(name)
    plan = api.Plan.from_workload(w)
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    disp = _dev(fwd["disp"])
    loss = float(_host(api.photometric_l1(plan, ref, tar, disp)))
    o_loss = SO.photometric_l1(sc.ref.astype(np.float64), sc.tar.astype(np.float64),
                               fwd["disp"].astype(np.float32).astype(np.float64))
    assert abs(loss - o_loss) <= 1e-5 * abs(o_loss)
    g_ref, g_tar, g_disp = api.photometric_l1_bwd(plan, ref, tar, disp, 2.5)
    o = SO.photometric_l1_backward(sc.ref.astype(np.float64), sc.tar.astype(np.float64),
                                   fwd["disp"].astype(np.float32).astype(np.float64), 2.5)
    for gg, oo in zip((g_ref, g_tar, g_disp), o):
        assert _rel_l2(_host(gg), oo) < 1e-3


def test_autograd_functions_chain():
    from paper_1904_06017_amd.autograd import PhotometricL1, SoftDisparity
    w, sc, g, fwd, bwd = case("rolled")
    plan = api.Plan.from_workload(w)
    ref = _dev(sc.ref).requires_grad_(True)
    tar = _dev(sc.tar).requires_grad_(True)
    plane = torch.tensor(w.plane, dtype=torch.float64, requires_grad=True)
    disp = SoftDisparity.apply(ref, tar, plane, plan)
    loss = PhotometricL1.apply(ref, tar, disp, plan)
    loss.backward()
    # the same chain assembled from the oracle pieces
    d64 = _host(disp)
    l_ref, l_tar, l_disp = SO.photometric_l1_backward(sc.ref.astype(np.float64),
                                                      sc.tar.astype(np.float64), d64, 1.0)
    s_ref, s_tar, s_plane = SO.soft_backward(sc.ref, sc.tar, w.plane, w, fwd, l_disp)
    assert _rel_l2(_host(ref.grad), l_ref + s_ref) < 1e-3
    assert _rel_l2(_host(tar.grad), l_tar + s_tar) < 1e-3
    assert np.allclose(plane.grad.numpy(), s_plane, rtol=1e-3, atol=1e-6 * np.abs(s_plane).max())


def test_full_size_soft_forward_sampled():
    """1280x720 F32 pair, 48 levels, 11x11 aggregation: the bench's launch
    configuration; soft levels checked at sampled pixels against the oracle."""
    w = workload("c5")
    sc = make_workload_pair(w)
    plan = api.Plan.from_workload(w)
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    disp, saved = api.soft_forward(plan, ref, tar, w.plane)
    dh = _host(saved)[2]
    tw = OS.warp(sc.tar, w.plane, w.delta_p, True)
    rng = np.random.default_rng(53)
    pts = [(0, 0), (w.width - 1, w.height - 1), (640, 360)] + \
          [(int(rng.integers(0, w.width)), int(rng.integers(0, w.height))) for _ in range(20)]
    for (u, v) in pts:
        E = OS.aggregated_at(sc.ref, tw, u, v, w, "R")
        z = -E / w.softargmin_T
        P = np.exp(z - z.max())
        P /= P.sum()
        ref_dh = float(np.sum(np.arange(w.num_disp) * P))
        assert abs(dh[v, u] - ref_dh) <= 1e-4 * max(abs(ref_dh), 1), (u, v, dh[v, u], ref_dh)
    # full-size backward runs and agrees with a central difference of the GPU loss in c0
    g_ref, g_tar, g_plane = api.backward(plan, ref, tar, w.plane, saved,
                                         torch.ones_like(disp) / disp.numel())
    gp = _host(g_plane)
    assert np.all(np.isfinite(gp)) and np.all(np.isfinite(_host(g_ref)))
    h = 0.02
    f = []
    for s in (+1, -1):
        pl = (w.plane[0] + s * h, w.plane[1], w.plane[2])
        d, _ = api.soft_forward(plan, ref, tar, pl)
        f.append(float(_host(d).mean()))
    fd = (f[0] - f[1]) / (2 * h)
    assert abs(gp[0] - fd) < 2e-2 * max(abs(fd), 1e-3), (gp[0], fd)


@pytest.mark.parametrize("engine", [2, 1])
def test_soft_engines_agree_at_full_size(engine):
    """1280x720 F32 pair, 48 levels, 11x11 aggregation: each matrix-core
    engine and the vector-ALU engine sum in different orders; their soft
    levels and softmax state agree to FP32 rounding at every pixel."""
    w = workload("c5")
    sc = make_workload_pair(w)
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    out = []
    for engine in (engine, 0):
        plan = api.Plan.from_workload(w)
        plan.set_tuning("agg_engine", engine)
        disp, saved = api.soft_forward(plan, ref, tar, w.plane)
        out.append((_host(disp), _host(saved)))
    (d1, s1), (d0, s0) = out
    assert np.max(np.abs(d1 - d0) / np.maximum(np.abs(d0), 1)) < 2e-4
    for k in range(3):
        assert np.max(np.abs(s1[k] - s0[k]) / np.maximum(np.abs(s0[k]), 1)) < 2e-4, k
