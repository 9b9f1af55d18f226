#!/usr/bin/env python3
"""Benchmark of the road-stereo hot path on one MI355X.

One step = the whole plain path on one 1280x720 uint8 pair (perspective
transformation, NCC cost volume, bilateral aggregation + WTA of both
volumes, sub-pixel, left-right check, shift back) plus the road fit and
disparity transformation, inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_HBM_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: the FP32 vector
# rate of plain v_fma_f32.  Packed FP32 (v_pk_fma_f32) would double it to the
# published 157.3 TFLOP/s; the library is compiled without packed FP32.
MI355X_FP32_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
MI355X_FP32_PACKED_TFLOPS = 157.3
# dense FP32 matrix-core rate: v_mfma_f32_16x16x4f32 is 16*16*4 FMAs per SIMD
# every 32 cycles, 256 CUs x 4 SIMDs x 2.4 GHz
MI355X_FP32_MFMA_TFLOPS = 157.3
# dense FP16 matrix-core rate (v_mfma_f32_16x16x32_f16), published
MI355X_FP16_MFMA_TFLOPS = 2500.0


def mfma16_k(R):
    """Union positions one pixel-level of the split-FP16 aggregation multiplies:
    a 4x4 pixel block's (4 + 2R)-row window union, cut in 2-row x 4-column
    patches (columns rounded up to whole quads), four patches per product."""
    n_patch = (R + 2) * (((4 + 2 * R + 3) & ~3) // 4)
    return ((n_patch + 3) // 4) * 32


def host_cpu():
    """Logical CPUs visible to this process and the CPU model name."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return n, model


def _sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _traffic(kernel_src, launches_bytes_key,
             name="traffic_bilateral_road1280x720_d64_persp.json"):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only
    if the kernel source is unchanged since they were taken."""
    f = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    if d.get("source_sha") != _sha(kernel_src):
        return None
    return d.get(launches_bytes_key)


def cpu_baseline(w, sc, rows):
    from dataclasses import replace

    from threadpoolctl import threadpool_limits

    import oracle.stereo as OS
    ws = replace(w, height=rows)
    with threadpool_limits(limits=1):        # the oracle as written: one core
        t0 = time.perf_counter()
        OS.match(sc.ref[:rows], sc.tar[:rows], ws)
        dt = time.perf_counter() - t0
    nproc, model = host_cpu()
    return dict(value=w.width * rows * w.num_disp / dt / 1e9, unit="G pixel·disparities/s",
                cores=1, kind="oracle", seconds=round(dt, 2), host_nproc=nproc, host_cpu=model,
                sample=f"rows 0..{rows - 1} of the {w.width}x{w.height} pair, D={w.num_disp}, "
                       f"full plain path (FP64 numpy, single thread)")


def _gen(w):
    from synth import make_workload_pair
    sc = make_workload_pair(w)
    return sc.ref, sc.tar


def batch_scenes(serial=False):
    """The 64 seeded pairs of the mixed batch, the tracking sequence and the
    skewed rig, generated on host cores: by a pool of fresh ("spawn") worker
    processes that import numpy and the generator only, closed and joined
    when done, or in this process (serial=True, for runs under a profiler,
    which would follow every worker)."""
    import multiprocessing as mp
    from synth import batch_workloads
    ws = batch_workloads()
    if serial:
        imgs = []
        for i, w in enumerate(ws):
            imgs.append(_gen(w))
            if i % 16 == 15:
                print(f"[bench] generated {i + 1}/{len(ws)} batch pairs", file=sys.stderr,
                      flush=True)
        return (ws, imgs), (sequence_frames(), skewed_frames())
    pool = mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1))
    try:
        seq = pool.apply_async(sequence_frames)
        sk = pool.apply_async(skewed_frames)
        imgs = pool.map(_gen, ws)
        seq = seq.get()
        sk = sk.get()
    finally:
        pool.close()
        pool.join()
    return (ws, imgs), (seq, sk)


def sequence_frames():
    """4 frames of a 1280x720 road whose plane drifts (slope, roll, offset)."""
    from synth import road_sequence, workload
    w = workload("c3a")
    return w, road_sequence(w.width, w.height, 4, seed=31, n_potholes=w.n_potholes,
                            n_cracks=w.n_cracks)


def skewed_frames():
    """The 1280x720 pair re-imaged by a target camera rotated 0.3 degrees and
    shifted 0.8 rows (a rig outside the rectified hypotheses)."""
    from synth import skewed_pair, workload
    w = workload("c3a")
    sc, tar2, _, Hm, dtrue = skewed_pair(w)
    return w, sc, tar2, Hm, dtrue


def skewed_rig(args, sk):
    """Matching the skewed pair through the general homography (Eq. 3) vs the
    row shift of the plane: time per match and error pixels (> 1 px) against
    the generator's ground truth on interior visible pixels."""
    from dataclasses import replace

    import numpy as np
    import torch

    from paper_1904_06017_amd import api
    w, sc, tar2, Hm, dtrue = sk
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(sc.ref).to(dev)
    tar = torch.from_numpy(tar2).to(dev)
    r = w.ncc_radius + w.bil_radius
    sel = np.zeros(sc.visible.shape, bool)
    sel[r:-r, w.num_disp + r:-r] = True
    sel &= sc.visible
    res = {}
    for name, wk in (("homography", replace(w, homography=tuple(Hm.ravel()))), ("row_shift", w)):
        plan = api.Plan.from_workload(wk)
        o = None
        for _ in range(3):
            o = api.match(plan, ref, tar, out=o)
        torch.cuda.synchronize()
        n = max(10, args.steps // 2)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            api.match(plan, ref, tar, out=o)
        b.record()
        torch.cuda.synchronize()
        disp = o["disp"].cpu().numpy()
        fin = sel & np.isfinite(disp)
        err = np.abs(disp[fin] - dtrue[fin])
        res[name] = dict(match_ms=round(a.elapsed_time(b) / n, 4),
                         error_pixels_pct=round(float(np.mean(err > 1.0) * 100), 3),
                         rms_px=round(float(np.sqrt(np.mean(err ** 2))), 4),
                         valid_fraction=round(float(fin.sum() / sel.sum()), 4))
    return dict(workload=w.name, rotation_deg=0.3, row_offset=0.8, **res)


def closed_loop(args, seq):
    """Plane tracking over a frame sequence: bootstrap with a full-range pass
    (128 levels, no warp) on frame 0, then each frame matched with the plane
    fitted on the previous one (device-resident state, no host sync)."""
    from dataclasses import replace

    import numpy as np
    import torch

    from paper_1904_06017_amd import api
    w, frames = seq
    dev = torch.device("cuda:0")
    imgs = [(torch.from_numpy(sc.ref).to(dev), torch.from_numpy(sc.tar).to(dev))
            for _, _, sc in frames]
    raw = api.Plan.from_workload(replace(w, perspective=False, delta_p=0.0, num_disp=128))
    m = api.match(raw, *imgs[0])
    fit0, _ = api.road_transform(raw, m["disp"], m["valid"])
    tr = api.PlaneTracker(api.Plan.from_workload(w))
    out = None
    for _ in range(2):                               # warm-up passes over the sequence
        tr.init_from_fit(fit0)
        for ref, tar in imgs[1:]:
            out = tr.step(ref, tar, out=out)
    reps = max(3, args.steps // 10)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t = 0.0
    errs = []
    vv, uu = np.mgrid[0:w.height, 0:w.width]
    for rep in range(reps):
        tr.init_from_fit(fit0)
        torch.cuda.synchronize()
        ev[0].record()
        for ref, tar in imgs[1:]:
            out = tr.step(ref, tar, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        t += ev[0].elapsed_time(ev[1])
    # plane error of the last pass, frame by frame (re-run with reads)
    tr.init_from_fit(fit0)
    for (c, _, _), (ref, tar) in zip(frames[1:], imgs[1:]):
        tr.step(ref, tar, out=out)
        p = tr.read()["plane"]
        errs.append(float(np.max(np.abs((p[0] - c[0]) + (p[1] - c[1]) * uu + (p[2] - c[2]) * vv))))
    n = len(imgs) - 1
    return dict(frames=n, workload=w.name, bootstrap_levels=128,
                ms_per_tracked_frame=round(t / reps / n, 4),
                max_road_disparity_error_px=[round(e, 4) for e in errs])


def settle(fn, seconds):
    """Untimed calls of fn until `seconds` of back-to-back GPU work have run:
    the first tenths of a second after the GPU idles run at a lower clock
    (measured: 0.733 against 0.692 ms per match step at 1280x720, D = 64,
    with the same buffers)."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def batched(args, scenes):
    """64 pairs of mixed size / range / roll: one captured graph (persistent
    aggregation over all pairs' tiles) vs the plain per-pair path."""
    import torch

    from paper_1904_06017_amd import api
    ws, imgs = scenes
    dev = torch.device("cuda:0")
    items = []
    for w, (ref, tar) in zip(ws, imgs):
        items.append((api.Plan.from_workload(w), torch.from_numpy(ref).to(dev),
                      torch.from_numpy(tar).to(dev)))
    el = sum(w.width * w.height * w.num_disp for w in ws)
    b = api.Batch(items)
    b.submit()
    tuned_ms = b.autotune(None, reps=2)
    b.instantiate()
    b.launch()
    torch.cuda.synchronize()
    n = max(3, args.steps // 10)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(n):
        b.launch()
    e[1].record()
    torch.cuda.synchronize()
    t_b = e[0].elapsed_time(e[1]) / n
    outs = [dict(dint_R=torch.empty_like(o["dint_R"]), dsub=torch.empty_like(o["disp"]),
                 valid=torch.empty_like(o["valid"]), disp=torch.empty_like(o["disp"]))
            for o in b.outputs]
    for (plan, ref, tar), o in zip(items, outs):     # warm the per-pair path
        api.match(plan, ref, tar, out=o)
    torch.cuda.synchronize()
    e[2].record()
    for _ in range(n):
        for (plan, ref, tar), o in zip(items, outs):
            api.match(plan, ref, tar, out=o)
    e[3].record()
    torch.cuda.synchronize()
    t_p = e[2].elapsed_time(e[3]) / n
    same = all(torch.equal(o["dint_R"], p["dint_R"]) for o, p in zip(b.outputs, outs))
    # the persistent aggregation launches (every group), timed live around a
    # plain submission of the same batch
    import ctypes
    lib = api._lib.load()
    agg = []
    for _ in range(n):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for x in ev:
            x.record()                   # materialise the underlying event objects
        evp = (ctypes.c_void_p * 2)(*[x.cuda_event for x in ev])
        api.check(lib.stereo_submit_batch_profiled(b._h, api._p(b.ws), b.workspace_bytes, evp,
                                                   api._stream()))
        agg.append(ev)
    torch.cuda.synchronize()
    agg_ms = sum(e[0].elapsed_time(e[1]) for e in agg) / n
    flops = sum(2 * 2.0 * (2 * w.bil_radius + 1) ** 2 * w.width * w.height * w.num_disp for w in ws)
    achieved = flops / (agg_ms / 1e3) / 1e12
    engine = b.get_tuning("agg_engine")
    if engine == 2:
        issued = sum(2 * 3 * 2.0 * mfma16_k(w.bil_radius) * w.width * w.height * w.num_disp
                     for w in ws)
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_mfma16.h")
        roof = dict(kernel="agg_mfma16_kernel, queued (all groups of the batch)", bound="mfma",
                    achieved=round(achieved, 2), peak=MI355X_FP16_MFMA_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / MI355X_FP16_MFMA_TFLOPS, 4),
                    issued_frac=round(issued / (agg_ms / 1e3) / 1e12 / MI355X_FP16_MFMA_TFLOPS, 4),
                    frac_vs_fp32_peak=round(achieved / MI355X_FP32_MFMA_TFLOPS, 4),
                    flops_per_batch=flops, issued_flops_per_batch=issued,
                    aggregation_ms=round(agg_ms, 3),
                    traffic=_traffic(src, "hbm_bytes_per_batch",
                                     "traffic_batch_mixed64.json"))
    else:
        roof = dict(kernel="queued aggregation (all groups of the batch)",
                    bound="mfma" if engine == 1 else "alu", achieved=round(achieved, 2),
                    peak=MI355X_FP32_MFMA_TFLOPS if engine == 1 else round(MI355X_FP32_VALU_TFLOPS, 1),
                    unit="TFLOP/s", aggregation_ms=round(agg_ms, 3), flops_per_batch=flops,
                    traffic=None)
        roof["frac"] = round(achieved / roof["peak"], 4)
    return dict(pairs=len(ws), elements=el, batch_ms=round(t_b, 3),
                batch_gpd_s=round(el / (t_b / 1e3) / 1e9, 3), per_pair_ms=round(t_p, 3),
                per_pair_gpd_s=round(el / (t_p / 1e3) / 1e9, 3),
                speedup_vs_per_pair=round(t_p / t_b, 3), equal_to_per_pair=bool(same),
                tuning={k: b.get_tuning(k) for k in ("agg_engine", "tile_band", "ncc_levels",
                                                     "group_overlap", "wg_per_cu", "agg_levels_u8",
                                                     "agg_levels_f32")},
                autotune_best_ms=round(tuned_ms, 3), roofline=roof)


def run(args):
    scenes, (seq, sk) = batch_scenes(args.serial_inputs) if args.extra else (None, (None, None))
    import torch

    from paper_1904_06017_amd import api
    from synth import make_workload_pair, workload

    dev = torch.device("cuda:0")
    w = workload("c3a")
    sc = make_workload_pair(w)
    plan = api.Plan.from_workload(w)
    for kv in args.tune:
        k, v = kv.split("=")
        plan.set_tuning(k, int(v))
    ref = torch.from_numpy(sc.ref).to(dev)
    tar = torch.from_numpy(sc.tar).to(dev)
    H, W = w.height, w.width
    out = dict(dint_R=torch.empty((H, W), dtype=torch.int16, device=dev),
               dint_T=torch.empty((H, W), dtype=torch.int16, device=dev),
               dsub=torch.empty((H, W), dtype=torch.float32, device=dev),
               valid=torch.empty((H, W), dtype=torch.uint8, device=dev),
               disp=torch.empty((H, W), dtype=torch.float32, device=dev))
    fit_buf = torch.empty(80, dtype=torch.uint8, device=dev)
    disp_t = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    lib = api._lib.load()
    import ctypes

    def step(ev=None):
        evp = None
        if ev is not None:
            arr = (ctypes.c_void_p * 7)(*[e.cuda_event for e in ev])
            evp = arr
        api.check(lib.stereo_match_profiled(
            plan.handle, api._p(ref), api._p(tar), api._p(out["dint_R"]), api._p(out["dint_T"]),
            api._p(out["dsub"]), api._p(out["valid"]), api._p(out["disp"]), api._p(ws),
            plan.workspace_bytes, evp, api._stream()))
        api.road_transform(plan, out["disp"], None, fit_buf=fit_buf, out=disp_t, read_fit=False)

    settle(step, args.settle_s)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(K)]
    for e in evs:
        for x in e:
            x.record()   # materialise the underlying event objects
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(K):
        step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms = total_ms / K
    stage = lambda i, j: sum(evs[k][i].elapsed_time(evs[k][j]) for k in range(K)) / K
    st = dict(warp_ms=stage(0, 1), stats_ms=stage(1, 2), ncc_ms=stage(2, 3),
              aggregate_wta_ref_ms=stage(3, 4), aggregate_wta_tar_ms=stage(4, 5),
              lr_check_ms=stage(5, 6), match_ms=stage(0, 6))
    st["road_ms"] = ms - st["match_ms"]

    elements = W * H * w.num_disp
    taps = (2 * w.bil_radius + 1) ** 2
    flops_per_launch = 2.0 * taps * elements          # multiply-adds of Eq. (11)
    agg_s = (st["aggregate_wta_ref_ms"] + st["aggregate_wta_tar_ms"]) / 2.0 / 1e3
    achieved = flops_per_launch / agg_s / 1e12
    engine = plan.get_tuning("agg_engine")
    if engine == 2:
        # matrix cores with split-FP16 operands: each 4x4 pixel block multiplies
        # over its patch-padded window union (mfma16_k positions per
        # pixel-level) and every product is three FP16 MFMAs (hi.hi, hi.lo,
        # lo.hi), so the issued FP16 flops are 3 x 2 x mfma16_k per element
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_mfma16.h")
        issued = 3 * 2.0 * mfma16_k(w.bil_radius) * elements
        roof = dict(kernel="agg_mfma16_kernel (aggregation + fused WTA, both volumes)",
                    bound="mfma", achieved=round(achieved, 2), peak=MI355X_FP16_MFMA_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / MI355X_FP16_MFMA_TFLOPS, 4),
                    issued_tflops=round(issued / agg_s / 1e12, 1),
                    issued_frac=round(issued / agg_s / 1e12 / MI355X_FP16_MFMA_TFLOPS, 4),
                    frac_vs_fp32_peak=round(achieved / MI355X_FP32_MFMA_TFLOPS, 4),
                    flops_per_launch=flops_per_launch, issued_flops_per_launch=issued,
                    avg_launch_ms=round(agg_s * 1e3, 4),
                    traffic=_traffic(src, "hbm_bytes_per_launch"))
    elif engine == 1:
        # matrix cores: each 4x4 pixel block multiplies over its (2R + 4)^2
        # window union, (2R + 4)^2 / (2R + 1)^2 of the algorithmic products
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_mfma.h")
        union = (2 * w.bil_radius + 4) ** 2
        roof = dict(kernel="agg_wta_mfma_kernel (aggregation + fused WTA, both volumes)",
                    bound="mfma", achieved=round(achieved, 2), peak=MI355X_FP32_MFMA_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / MI355X_FP32_MFMA_TFLOPS, 4),
                    issued_frac=round(achieved * union / taps / MI355X_FP32_MFMA_TFLOPS, 4),
                    flops_per_launch=flops_per_launch, avg_launch_ms=round(agg_s * 1e3, 4),
                    traffic=_traffic(src, "hbm_bytes_per_launch"))
    else:
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_impl.h")
        roof = dict(kernel="bilateral_kernel (aggregation + fused WTA, both volumes)",
                    bound="alu", achieved=round(achieved, 2), peak=round(MI355X_FP32_VALU_TFLOPS, 1),
                    unit="TFLOP/s", frac=round(achieved / MI355X_FP32_VALU_TFLOPS, 4),
                    frac_of_packed_peak=round(achieved / MI355X_FP32_PACKED_TFLOPS, 4),
                    flops_per_launch=flops_per_launch, avg_launch_ms=round(agg_s * 1e3, 4),
                    traffic=_traffic(src, "hbm_bytes_per_launch"))
    # NCC stage: HBM-bound when the volume is materialised.  Engines 0 and 1
    # write one FP32 reference-anchored volume over the extended columns
    # (the target volume is its re-indexing); engine 2 writes the two
    # anchored volumes, each element as two FP16 halves.
    if engine == 2:
        ncc_bytes = 2 * 4.0 * w.num_disp * H * W
        ncc_kernel = "ncc_kernel (split-FP16 output, both anchors)"
    else:
        ncc_bytes = 4.0 * w.num_disp * H * (W + w.num_disp - 1)
        ncc_kernel = "ncc_kernel (FP32 quad output)"
    ncc_gbs = ncc_bytes / (st["ncc_ms"] / 1e3) / 1e9
    hbm = achievable_hbm(int(ncc_bytes))
    ncc = dict(kernel=ncc_kernel, bound="hbm", achieved=round(ncc_gbs, 1),
               peak=MI355X_HBM_GBS, unit="GB/s",
               frac=round(ncc_gbs / MI355X_HBM_GBS, 4),
               bytes_per_launch=ncc_bytes,
               # the volume write dominates the kernel's bytes: also against a
               # plain device fill of the same size measured in this run
               achievable=hbm, frac_of_achievable_write=round(ncc_gbs / hbm["fill_gbs"], 4))

    # cost + filter together (NCC + both aggregations), read as a roofline of
    # the method: its FP32 work (8 flops per element for the NCC, 2 (2R+1)^2
    # + 1 per element and volume for the aggregation) at the published FP32
    # rate, against the HBM time of the bytes this engine materialises (the
    # volumes written once and read once); the larger of the two binds
    t_meas = st["ncc_ms"] + st["aggregate_wta_ref_ms"] + st["aggregate_wta_tar_ms"]
    model_flops = (8.0 + 2 * (2.0 * taps + 1)) * elements
    cf_bytes = 2 * ncc_bytes if engine == 2 else ncc_bytes + 2 * 4.0 * elements
    t_comp = model_flops / (MI355X_FP32_MFMA_TFLOPS * 1e12) * 1e3
    t_hbm = cf_bytes / (MI355X_HBM_GBS * 1e9) * 1e3
    cost_filter = dict(stages="ncc + aggregation of both volumes", measured_ms=round(t_meas, 4),
                       compute_bound_ms=round(t_comp, 4), hbm_bound_ms=round(t_hbm, 4),
                       model_flops=model_flops, materialised_bytes=cf_bytes,
                       binding="fp32 compute" if t_comp >= t_hbm else "hbm",
                       frac=round(max(t_comp, t_hbm) / t_meas, 4))

    value = elements / (ms / 1e3) / 1e9
    res = {
        "metric": "G pixel·disparities/s (fwd, fwd+bwd) and fps at 1280×720, vs plain per-pair",
        "value": round(value, 3),
        "unit": "G pixel·disparities/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "warmup_settle_s": args.settle_s,
        "ms_per_step": round(ms, 4),
        "fps": round(1e3 / ms, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "width": W, "height": H, "num_disp": w.num_disp,
                   "ncc": f"{2 * w.ncc_radius + 1}x{2 * w.ncc_radius + 1}",
                   "bilateral": f"{2 * w.bil_radius + 1}x{2 * w.bil_radius + 1}",
                   "sigma_s": w.sigma_s, "sigma_r": w.sigma_r, "perspective": True,
                   "input": "uint8", "step": "plain path + road fit/transform"},
        "stages_ms": {k: round(v, 4) for k, v in st.items()},
        "tuning": {k: plan.get_tuning(k) for k in ("agg_engine", "agg_levels_u8", "agg_levels_f32",
                                                   "ncc_levels")},
        "roofline": roof,
        "roofline_ncc": ncc,
        "roofline_cost_filter": cost_filter,
    }
    if args.extra:
        res["damage_segmentation"] = damage_segmentation(args, plan, w, sc, disp_t)
        res["range_reduction"] = range_reduction(args, sc, ms)
        res["fwd_bwd"] = fwd_bwd(args)
        res["paper_preset"] = paper_preset(args)
        res["closed_loop"] = closed_loop(args, seq)
        res["skewed_rig"] = skewed_rig(args, sk)
        res["batched"] = batched(args, scenes)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, sc, args.cpu_rows)
    return res


def range_reduction(args, sc, ms_3a):
    """Same pair searched over the full 0..127 range without the warp."""
    import torch

    from paper_1904_06017_amd import api
    from synth import workload
    w = workload("c3b")
    plan = api.Plan.from_workload(w)
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(sc.ref).to(dev)
    tar = torch.from_numpy(sc.tar).to(dev)
    o = None
    for _ in range(3):
        o = api.match(plan, ref, tar, out=o)
    torch.cuda.synchronize()
    n = max(5, args.steps // 4)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        api.match(plan, ref, tar, out=o)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / n
    return dict(workload=w.name, num_disp=w.num_disp, match_ms=round(ms, 4),
                gpd_s=round(w.width * w.height * w.num_disp / (ms / 1e3) / 1e9, 3),
                speedup_of_perspective=round(ms / ms_3a, 3))


def damage_segmentation(args, plan, w, sc, disp_t, tau=0.5):
    """Damage below the flattened road on the step's transformed map
    (threshold tau px), its time, and its overlap with the generator's
    ground truth (region deeper than tau) on interior visible pixels."""
    import numpy as np
    import torch

    from paper_1904_06017_amd import api
    m = api.damage_mask(plan, disp_t, 0.0, tau)
    torch.cuda.synchronize()
    n = max(20, args.steps)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        api.damage_mask(plan, disp_t, 0.0, tau, out=m)
    b.record()
    torch.cuda.synchronize()
    mask = m.cpu().numpy().astype(bool)
    vv, uu = np.mgrid[0:w.height, 0:w.width]
    depth = w.plane[0] + w.plane[1] * uu + w.plane[2] * vv - sc.d_gt
    r = w.ncc_radius + w.bil_radius
    sel = np.zeros(sc.visible.shape, bool)
    sel[r:-r, w.num_disp + r:-r] = True
    sel &= sc.visible
    p, t = mask[sel], (depth >= tau)[sel]
    inter, union = np.count_nonzero(p & t), np.count_nonzero(p | t)
    return dict(tau_px=tau, mask_ms=round(a.elapsed_time(b) / n, 4),
                iou_vs_ground_truth=round(inter / max(union, 1), 4),
                false_positive_rate_on_road=round(float(np.mean(mask[sel & sc.road_mask])), 5),
                damaged_fraction=round(float(np.mean(t)), 4))


def paper_preset(args):
    """The paper's own parameter set (640x360, 11x11 NCC and aggregation
    windows, sigma 1.5 / 5.5, 30 levels) on a synthetic pair of that size:
    a frame rate beside the 152.889 ms the paper reports on its embedded GPU
    (different hardware and data: context, not a target)."""
    import torch

    from paper_1904_06017_amd import api
    from synth import make_workload_pair, workload
    w = workload("paper")
    sc = make_workload_pair(w)
    plan = api.Plan.from_workload(w)
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(sc.ref).to(dev)
    tar = torch.from_numpy(sc.tar).to(dev)
    o = None
    for _ in range(3):
        o = api.match(plan, ref, tar, out=o)
    torch.cuda.synchronize()
    n = max(10, args.steps)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        api.match(plan, ref, tar, out=o)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / n
    return dict(workload=w.name, width=w.width, height=w.height, num_disp=w.num_disp,
                ncc="11x11", bilateral="11x11", match_ms=round(ms, 4), fps=round(1e3 / ms, 1),
                gpd_s=round(w.width * w.height * w.num_disp / (ms / 1e3) / 1e9, 3),
                paper_ms_other_hardware=152.889)


def achievable_hbm(nbytes):
    """HBM rates a plain device fill (write only) and copy (read + write) of
    nbytes reach on this GPU, timed with events like the path's stages."""
    import torch
    n = max(nbytes // 4, 1 << 20)
    a = torch.empty(n, device="cuda")
    b = torch.empty(n, device="cuda")
    out = {}
    for name, f, moved in (("fill_gbs", lambda: a.fill_(1.0), 4 * n),
                           ("copy_gbs", lambda: b.copy_(a), 8 * n)):
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            f()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(moved / (e0.elapsed_time(e1) / 20 / 1e3) / 1e9, 1)
    del a, b
    return out


def copy_calibration(mib):
    """A plain device copy of known size, for scaling HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 3}), flush=True)


def fwd_bwd(args):
    """Differentiable form at 1280x720 FP32, 48 levels: soft-argmin forward,
    photometric L1, its backward and the backward of the soft head.  The
    backward's two aggregation passes are timed live with events on the
    stream they run on (the dominant kernels: roofline)."""
    import ctypes

    import torch

    from paper_1904_06017_amd import api
    from synth import make_workload_pair, workload
    w = workload("c5")
    sc = make_workload_pair(w)
    plan = api.Plan.from_workload(w)
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(sc.ref).to(dev)
    tar = torch.from_numpy(sc.tar).to(dev)
    H, W = w.height, w.width
    lib = api._lib.load()
    g_ref = torch.empty((H, W), dtype=torch.float32, device=dev)
    g_tar = torch.empty_like(g_ref)
    g_plane = torch.empty(3, dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)

    def step(ev=None):
        disp, saved = api.soft_forward(plan, ref, tar, w.plane)
        loss = api.photometric_l1(plan, ref, tar, disp)
        _, _, g_disp = api.photometric_l1_bwd(plan, ref, tar, disp, 1.0)
        evp = None if ev is None else (ctypes.c_void_p * 6)(*[e.cuda_event for e in ev])
        api.check(lib.stereo_backward_profiled(
            plan.handle, api._p(ref), api._p(tar), api._plane3(w.plane), api._p(saved),
            api._p(g_disp), api._p(g_ref), api._p(g_tar), api._p(g_plane), api._p(ws),
            plan.workspace_bytes, evp, api._stream()))
        return loss

    settle(step, args.settle_s)
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    n = max(3, args.steps // 10)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(n)]
    for e in evs:
        for x in e:
            x.record()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    c = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        api.soft_forward(plan, ref, tar, w.plane)
    b.record()
    for k in range(n):
        step(evs[k])
    c.record()
    torch.cuda.synchronize()
    f_ms = a.elapsed_time(b) / n
    fb_ms = b.elapsed_time(c) / n
    st = lambda i, j: sum(evs[k][i].elapsed_time(evs[k][j]) for k in range(n)) / n
    p1, p2, bwd = st(1, 2), st(3, 4), st(0, 5)
    el = w.width * w.height * w.num_disp
    engine = plan.get_tuning("agg_engine")
    R = w.bil_radius
    taps = (2 * R + 1) ** 2
    # each pass: two weighted window sums per pixel-level (the weights, and the
    # weights times the guide difference), 2 (2R+1)^2 flops each
    flops = 2 * 2.0 * taps * el
    dom_ms = max(p1, p2)
    achieved = flops / (dom_ms / 1e3) / 1e12
    if engine == 2 and R <= 5:
        issued = 2 * 3 * 2.0 * mfma16_k(R) * el
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_mfma16_bwd.h")
        roof = dict(kernel="agg_mfma16_bwd_kernel (slower of the two passes)", bound="mfma",
                    achieved=round(achieved, 2), peak=MI355X_FP16_MFMA_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / MI355X_FP16_MFMA_TFLOPS, 4),
                    issued_tflops=round(issued / (dom_ms / 1e3) / 1e12, 1),
                    issued_frac=round(issued / (dom_ms / 1e3) / 1e12 / MI355X_FP16_MFMA_TFLOPS, 4),
                    frac_vs_fp32_peak=round(achieved / MI355X_FP32_MFMA_TFLOPS, 4),
                    flops_per_launch=flops, issued_flops_per_launch=issued,
                    avg_launch_ms=round(dom_ms, 4),
                    traffic=_traffic(src, "pass1_bytes" if p1 >= p2 else "pass2_bytes",
                                     "traffic_bwd_road1280x720_f32_d48_soft.json"))
    else:
        src = os.path.join(ROOT, "paper_1904_06017_amd", "csrc", "bilateral_impl.h")
        roof = dict(kernel="bilateral_kernel modes 5/6 (slower of the two passes)", bound="alu",
                    achieved=round(achieved, 2), peak=round(MI355X_FP32_VALU_TFLOPS, 1),
                    unit="TFLOP/s", frac=round(achieved / MI355X_FP32_VALU_TFLOPS, 4),
                    flops_per_launch=flops, avg_launch_ms=round(dom_ms, 4), traffic=None)
    return dict(workload=w.name, num_disp=w.num_disp, fwd_ms=round(f_ms, 4),
                fwd_gpd_s=round(el / (f_ms / 1e3) / 1e9, 3), fwd_bwd_ms=round(fb_ms, 4),
                fwd_bwd_gpd_s=round(el / (fb_ms / 1e3) / 1e9, 3),
                bwd_ms=round(bwd, 4), bwd_pass1_ms=round(p1, 4), bwd_pass2_ms=round(p2, 4),
                grad_levels=plan.get_tuning("grad_levels"), agg_engine=engine, roofline=roof)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--settle-s", type=float, default=0.3,
                    help="untimed back-to-back steps for this many seconds before the "
                         "warm-up steps (GPU clock ramp after idle)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=240)
    ap.add_argument("--no-extra", dest="extra", action="store_false")
    ap.add_argument("--only", choices=("fwd_bwd", "batched"), default=None,
                    help="run one extra section alone and print its JSON (profiling runs)")
    ap.add_argument("--serial-inputs", action="store_true",
                    help="generate the batch inputs in this process (runs under a profiler)")
    ap.add_argument("--tune", action="append", default=[],
                    help="plan tuning key=value (e.g. agg_levels_f32=16)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs on one GPU (the multi-GPU split is a "
                                   "design only); --gpus must be 1"}))
        sys.exit(2)
    if args.only == "fwd_bwd":
        print(json.dumps({"fwd_bwd": fwd_bwd(args)}), flush=True)
        return
    if args.only == "batched":
        scenes, _ = batch_scenes(args.serial_inputs)
        print(json.dumps({"batched": batched(args, scenes)}), flush=True)
        return
    res = run(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
