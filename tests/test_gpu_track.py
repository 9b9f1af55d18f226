"""Closed-loop plane tracking on the GPU (through the C ABI).

The device-state path must equal the host-plane path bitwise; the state
update must follow the fit; the GPU loop over a drifting road must follow
the oracle loop's planes.
"""
import math
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle.road as RD
import oracle.stereo as OS
from synth import road_sequence, workload

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1904_06017_amd.api")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def seq():
    w = workload("c1")
    print("[track] sequence 320x240 x 4 frames", flush=True)
    return w, road_sequence(w.width, w.height, 4, seed=21)


def test_tracked_match_equals_plan_plane(seq):
    w, frames = seq
    c, _, sc = frames[2]
    plane = (c[0] + 0.3, c[1], c[2] * 1.01)           # any plane: both paths take it
    ref, tar = _dev(sc.ref), _dev(sc.tar)
    host = api.match(api.Plan.from_workload(replace(w, plane=plane)), ref, tar,
                     want_target=True)
    tr = api.PlaneTracker(api.Plan.from_workload(w))
    tr.set(plane, psi=0.0)
    dev = tr.step(ref, tar, want_target=True)
    for k in ("dint_R", "dint_T", "dsub", "valid", "disp"):
        assert np.array_equal(_host(host[k]), _host(dev[k]), equal_nan=True), k


def test_tracked_fit_updates_state(seq):
    w, frames = seq
    c, psi_true, sc = frames[1]
    plan = api.Plan.from_workload(w)
    tr = api.PlaneTracker(plan)
    tr.set(c, psi=0.01, frames=5)
    out = tr.step(_dev(sc.ref), _dev(sc.tar))
    st = tr.read()
    fit = api.road_fit_from_bytes(tr.fit_buf)
    assert st["frames"] == 6 and st["psi"] == fit["psi"] and st["plane"] == fit["plane"]
    # a flat fit (no valid pixel) leaves the state alone
    nan = torch.full((w.height, w.width), float("nan"), device="cuda")
    zero = torch.zeros((w.height, w.width), dtype=torch.uint8, device="cuda")
    lib = api._lib.load()
    ws = plan.workspace(nan.device)
    api.check(lib.stereo_road_transform_tracked(
        plan.handle, api._p(nan), api._p(zero), 10.0, math.pi / 1.8e6, 100, 0.0,
        api._p(tr.state), api._p(tr.fit_buf), api._p(out["disp_t"]), api._p(ws),
        plan.workspace_bytes, api._stream()))
    assert tr.read() == st
    assert api.road_fit_from_bytes(tr.fit_buf)["flat"]


def test_closed_loop_follows_the_oracle(seq):
    """Bootstrap (full-range pass without the warp on frame 0), then each
    frame with the previous frame's plane: per-frame planes within 2e-3 px of
    road disparity over the image and 1e-4 rad of roll of the oracle loop's."""
    w, frames = seq
    wr = replace(w, perspective=False, delta_p=0.0, num_disp=48)
    _, _, sc0 = frames[0]
    # oracle loop
    o = OS.match(sc0.ref, sc0.tar, wr)
    fit, _ = RD.road_transform(o["disp"], o["valid"])
    o_planes = [(RD.plane_from_fit(fit), fit.psi)]
    for c, _, sc in frames[1:]:
        o = OS.match(sc.ref, sc.tar, replace(w, plane=tuple(o_planes[-1][0])))
        fit, _ = RD.road_transform(o["disp"], o["valid"], psi0=o_planes[-1][1])
        o_planes.append((RD.plane_from_fit(fit), fit.psi))
    # GPU loop
    raw = api.Plan.from_workload(wr)
    m = api.match(raw, _dev(sc0.ref), _dev(sc0.tar))
    gfit, _ = api.road_transform(raw, m["disp"], m["valid"])
    tr = api.PlaneTracker(api.Plan.from_workload(w))
    tr.init_from_fit(gfit)
    g_planes = [(gfit["plane"], gfit["psi"])]
    for _, _, sc in frames[1:]:
        tr.step(_dev(sc.ref), _dev(sc.tar))
        st = tr.read()
        g_planes.append((st["plane"], st["psi"]))
    vv, uu = np.mgrid[0:w.height, 0:w.width]
    for (pg, sg), (po, so) in zip(g_planes, o_planes):
        err = (pg[0] - po[0]) + (pg[1] - po[1]) * uu + (pg[2] - po[2]) * vv
        assert np.max(np.abs(err)) <= 2e-3, (pg, po)
        assert abs(sg - so) <= 1e-4
