"""Full-frame parity at the measured workloads, element by element, in the
launch configuration the benchmark times:

  * the plain path (both volumes, WTA, sub-pixel, LR check, shift back) at
    640x480 (D = 48), 1280x720 with the perspective transformation (D = 64)
    and 1280x720 without it (D = 128), on both aggregation engines;
  * the soft-argmin adjoint at 1280x720 FP32 (D = 48, 11x11 aggregation):
    gradients of both images and the three plane parameters.

The FP64 oracle runs once per workload on the host, in row bands over worker
processes (tests/oracle_bands.py; the band decomposition is pinned to the
whole-frame oracle by tests/test_oracle_bands.py).
"""
import time
from dataclasses import replace

import numpy as np
import pytest
import torch
from scipy import ndimage

from synth import make_workload_pair, workload
from tests import oracle_bands as OB
from tests import parity_rules as PR

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1904_06017_amd.api")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def pool():
    with OB.process_pool() as p:
        yield p


_oracle = {}


def _plain(name, pool):
    if name not in _oracle:
        w = workload(name)
        sc = make_workload_pair(w)
        t = time.time()
        ora = OB.match_full(sc.ref, sc.tar, w, pool)
        print(f"[full-frame] oracle {w.name}: {time.time() - t:.1f} s on "
              f"{OB.worker_count()} workers", flush=True)
        _oracle[name] = (w, sc, ora)
    return _oracle[name]


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("engine", [2, 1, 0], ids=["mfma16", "mfma", "valu"])
@pytest.mark.parametrize("name", ["c2", "c3a", "c3b"])
def test_full_frame_match(pool, name, engine):
    w, sc, ora = _plain(name, pool)
    plan = api.Plan.from_workload(w)
    plan.set_tuning("agg_engine", engine)
    print(f"[full-frame] {w.name} engine {engine}", flush=True)
    out = api.match(plan, torch.from_numpy(sc.ref).cuda(), torch.from_numpy(sc.tar).cuda(),
                    want_target=True)
    counts = PR.check_selection(w, ora, _host(out["dint_R"]), _host(out["dint_T"]),
                                _host(out["dsub"]), _host(out["valid"]), _host(out["disp"]))
    print(f"[full-frame] {w.name} engine {engine}: {counts}", flush=True)
    assert PR.flat_share_ok(counts, w), counts
    # near ties stay an exception away from the left band
    band = w.num_disp + w.bil_radius + w.ncc_radius
    assert np.mean(ora["gapR"][:, band:] < PR.TIE_GAP) < 1e-3


def _rel_l2(g, o):
    return float(np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-30))


@pytest.mark.timeout(900)
def test_full_frame_soft_gradient(pool):
    """stereo_backward at 1280x720, D = 48, against the FP64 adjoint of the
    whole frame: relative L2 error below 1e-3 for each image gradient and for
    each plane component, with a seeded smooth upstream gradient.

    The plane is the workload's (24, 0, 0.1) moved by 0.05 px in c0: with
    c0 = 24 every tenth row samples the target exactly at lerp knots
    (X = x - 0.1 v), where the warp's derivative in the plane is one-sided
    and each side's rounding picks a different slope; at c0 = 24.05 every
    sample is 0.05 px or more from a knot (X = x - 0.05 - 0.1 v)."""
    w = workload("c5")
    w = replace(w, plane=(w.plane[0] + 0.05, w.plane[1], w.plane[2]), scene_plane=w.true_plane)
    sc = make_workload_pair(w)
    rng = np.random.default_rng(505)
    g = ndimage.gaussian_filter(rng.normal(size=(w.height, w.width)), 3.0)
    g = (g / np.abs(g).max()).astype(np.float32)
    plan = api.Plan.from_workload(w)
    ref = torch.from_numpy(sc.ref).cuda()
    tar = torch.from_numpy(sc.tar).cuda()
    print(f"[full-frame] soft gradient {w.name}", flush=True)
    disp, saved = api.soft_forward(plan, ref, tar, w.plane)
    g_ref, g_tar, g_plane = api.backward(plan, ref, tar, w.plane, saved,
                                         torch.from_numpy(g).cuda())
    g_ref, g_tar = _host(g_ref).astype(np.float64), _host(g_tar).astype(np.float64)
    gp = _host(g_plane).astype(np.float64)
    t = time.time()
    o_ref, o_tar, o_plane = OB.soft_grad_full(sc.ref, sc.tar, w.plane, w,
                                              g.astype(np.float64), pool)
    print(f"[full-frame] oracle adjoint: {time.time() - t:.1f} s", flush=True)
    e_ref, e_tar = _rel_l2(g_ref, o_ref), _rel_l2(g_tar, o_tar)
    e_plane = [abs(gp[k] - o_plane[k]) / max(abs(o_plane[k]), 1e-6 * np.abs(o_plane).max())
               for k in range(3)]
    print(f"[full-frame] rel L2 ref {e_ref:.2e} tar {e_tar:.2e} plane "
          f"{['%.2e' % e for e in e_plane]} (gpu {gp.tolist()}, oracle {o_plane.tolist()})",
          flush=True)
    assert e_ref < 1e-3 and e_tar < 1e-3
    assert max(e_plane) < 1e-3
