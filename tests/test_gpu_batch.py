"""Batched form and autotuner on the GPU (through the C ABI).

Each pair of a batch must be bitwise the plain per-pair path with the same
plan; a captured graph must reproduce the eager batch on every replay, with
eager work and synchronisations between the replays; the autotuner's choice
must not change any result.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle.stereo as OS
from synth import batch_workloads, make_workload_pair
from tests import parity_rules as PR

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1904_06017_amd.api")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def small_batch():
    """12 pairs across all four size classes of the 64-pair recipe, shrunk."""
    ws = batch_workloads(scale=0.2)
    pick = [0, 1, 2, 16, 17, 18, 40, 41, 42, 56, 57, 63]
    pairs = []
    for i in pick:
        w = ws[i]
        sc = make_workload_pair(w)
        pairs.append((w, sc))
    print(f"[batch] {len(pairs)} pairs, sizes {[ (w.width, w.height, w.num_disp) for w, _ in pairs]}",
          flush=True)
    return pairs


def _make(pairs):
    items = []
    for w, sc in pairs:
        plan = api.Plan.from_workload(w)
        items.append((plan, torch.from_numpy(sc.ref).cuda(), torch.from_numpy(sc.tar).cuda()))
    return items


@pytest.mark.timeout(900)
def test_full_batch_equals_plain_path():
    """The whole 64-pair batch (16 x 320x240, 24 x 640x480, 16 x 1280x720,
    8 x 1920x1080; 32-96 levels per pair) in the benchmark's launch
    configuration: every pair bitwise equal to its plain per-pair match."""
    import time

    from synth import make_workload_pair as gen
    from tests import oracle_bands as OB
    ws = batch_workloads()
    t = time.time()
    with OB.process_pool() as pool:
        scenes = list(pool.map(gen, ws))
    print(f"[batch] generated {len(ws)} pairs in {time.time() - t:.1f} s", flush=True)
    items = [(api.Plan.from_workload(w), torch.from_numpy(sc.ref).cuda(),
              torch.from_numpy(sc.tar).cuda()) for w, sc in zip(ws, scenes)]
    b = api.Batch(items)
    outs = b.submit()
    torch.cuda.synchronize()
    for i, ((plan, ref, tar), o) in enumerate(zip(items, outs)):
        m = api.match(plan, ref, tar)
        for k in ("dint_R", "valid", "disp"):
            assert np.array_equal(_host(m[k]), _host(o[k]), equal_nan=True), (i, k, ws[i].name)
        plan._ws = None                      # release the per-pair workspace
        del m
    print(f"[batch] {len(items)} pairs bitwise equal to the plain path", flush=True)


@pytest.mark.parametrize("engine", [2, 1, 0], ids=["mfma16", "mfma", "valu"])
def test_batch_equals_plain_path(small_batch, engine):
    items = _make(small_batch)
    b = api.Batch(items)
    b.set_tuning("agg_engine", engine)
    outs = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    for (plan, ref, tar), o in zip(items, outs):
        plan.set_tuning("agg_engine", engine)
        m = api.match(plan, ref, tar)
        assert np.array_equal(_host(m["dint_R"]), o["dint_R"])
        assert np.array_equal(_host(m["valid"]), o["valid"])
        assert np.array_equal(_host(m["disp"]), o["disp"], equal_nan=True)


def test_batch_graph_replays(small_batch):
    items = _make(small_batch)
    b = api.Batch(items)
    eager = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    b.instantiate()
    for rep in range(3):
        for o in b.outputs:              # eager work between replays
            o["dint_R"].fill_(-1)
            o["disp"].zero_()
        torch.cuda.synchronize()
        outs = b.launch()
        got = [{k: _host(v) for k, v in o.items()} for o in outs]
        for e, g in zip(eager, got):
            for k in e:
                assert np.array_equal(e[k], g[k], equal_nan=True), (rep, k)


def test_batch_tuning_does_not_change_results(small_batch):
    items = _make(small_batch)
    b = api.Batch(items)
    ref = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    for wg, lv, band, nl, ov in ((1, 16, 1, 16, 0), (4, 8, 32, 64, 1), (2, 8, 2, 32, 0)):
        b.set_tuning("wg_per_cu", wg)
        b.set_tuning("agg_levels_u8", lv)
        b.set_tuning("agg_levels_f32", lv)
        b.set_tuning("tile_band", band)      # the matrix-core engine's tile order
        b.set_tuning("ncc_levels", nl)       # the NCC level block of the job lists
        b.set_tuning("group_overlap", ov)    # the two-branch schedule
        assert b.get_tuning("tile_band") == band
        assert b.get_tuning("ncc_levels") == nl
        assert b.get_tuning("group_overlap") == ov
        got = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
        for e, g in zip(ref, got):
            for k in e:
                assert np.array_equal(e[k], g[k], equal_nan=True), (wg, lv, band, nl, ov, k)


def test_batch_pairs_match_the_oracle(small_batch):
    items = _make(small_batch[:3])
    b = api.Batch(items)
    outs = b.submit()
    for (w, sc), o in zip(small_batch[:3], outs):
        ora = OS.match(sc.ref, sc.tar, w, keep_volumes=True)
        tie = PR.top2_gap(ora["E_R"]) < PR.TIE_GAP
        dR = _host(o["dint_R"])
        assert not np.any((dR != ora["dint_R"]) & ~tie)


def test_plan_autotune_and_cache(small_batch, tmp_path):
    w, sc = small_batch[-1]
    plan = api.Plan.from_workload(w)
    ref, tar = torch.from_numpy(sc.ref).cuda(), torch.from_numpy(sc.tar).cuda()
    before = {k: _host(v) for k, v in api.match(plan, ref, tar).items()}
    cache = str(tmp_path / "tune.json")
    ms = api.autotune(plan, ref, tar, cache, reps=2)
    assert ms > 0 and os.path.exists(cache)
    entries = json.load(open(cache))
    assert len(entries) == 1
    key = next(iter(entries))
    assert "gfx" in key and f"W={w.width}" in key
    knobs = ("agg_levels_u8", "agg_levels_f32", "ncc_levels")
    chosen = tuple(plan.get_tuning(k) for k in knobs)
    assert chosen == tuple(int(entries[key][k]) for k in knobs)
    assert chosen[2] in (16, 32, 64)
    plan2 = api.Plan.from_workload(w)
    api.autotune(plan2, ref, tar, cache, reps=2)        # cached: applied without timing
    assert tuple(plan2.get_tuning(k) for k in knobs) == chosen
    after = {k: _host(v) for k, v in api.match(plan, ref, tar).items()}
    for k in before:
        assert np.array_equal(before[k], after[k], equal_nan=True)


def test_batch_autotune(small_batch, tmp_path):
    items = _make(small_batch[:6])
    b = api.Batch(items)
    ref = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    cache = str(tmp_path / "btune.json")
    ms = b.autotune(cache, reps=1)
    assert ms > 0
    entries = json.load(open(cache))
    key = next(iter(entries))
    assert "batch" in key
    # the default engine's knob was swept and the choice applied
    assert int(entries[key]["tile_band"]) in (2, 4, 8, 16)
    assert b.get_tuning("tile_band") == int(entries[key]["tile_band"])
    assert int(entries[key]["ncc_levels"]) in (16, 32, 64)
    assert b.get_tuning("ncc_levels") == int(entries[key]["ncc_levels"])
    assert int(entries[key]["group_overlap"]) in (0, 1)
    assert b.get_tuning("group_overlap") == int(entries[key]["group_overlap"])
    got = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    for e, g in zip(ref, got):
        for k in e:
            assert np.array_equal(e[k], g[k], equal_nan=True)


def test_batch_with_homography_pair(small_batch):
    """A pair warped by a general homography (Eq. 3) next to plane pairs:
    every pair is bitwise its per-pair result."""
    from dataclasses import replace
    from synth import crop_workload, skewed_pair, workload
    w = crop_workload(workload("c1"), 170, 90, num_disp=36, delta_p=18.0)
    sc, tar2, _, Hm, _ = skewed_pair(w, angle_deg=0.4, dy=0.7)
    wh = replace(w, homography=tuple(Hm.ravel()))
    items = _make(small_batch[:2])
    items.insert(1, (api.Plan.from_workload(wh), torch.from_numpy(sc.ref).cuda(),
                     torch.from_numpy(tar2).cuda()))
    b = api.Batch(items)
    outs = [{k: _host(v) for k, v in o.items()} for o in b.submit()]
    for (plan, ref, tar), o in zip(items, outs):
        m = api.match(plan, ref, tar)
        for k in ("dint_R", "valid", "disp"):
            assert np.array_equal(_host(m[k]), o[k], equal_nan=True), k
