"""Python binding of the C ABI (argument marshalling only).

Torch tensors provide device memory and the current HIP stream; every step
runs in the library's HIP kernels.  Function names follow include/stereo.h.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from . import _lib
from ._lib import PlaneState, RoadFit, StereoParams, check

DELTA_PSI = math.pi / 1.8e6
LAMBDA0 = 10.0


def make_params(width, height, num_disp, *, dtype="u8", delta_p=0.0, perspective=True,
                plane=(0.0, 0.0, 0.0), ncc_radius=3, bil_radius=5, sigma_s=4.0,
                sigma_r=12.0, lr_delta=1.0, lr_check=True, softargmin_T=0.1,
                pitch_ref=None, pitch_tar=None) -> StereoParams:
    p = StereoParams()
    p.width, p.height = int(width), int(height)
    p.pitch_ref = int(pitch_ref if pitch_ref is not None else width)
    p.pitch_tar = int(pitch_tar if pitch_tar is not None else width)
    p.dtype = _lib.U8 if dtype in ("u8", "uint8", torch.uint8) else _lib.F32
    p.num_disp = int(num_disp)
    p.delta_p = float(delta_p if perspective else 0.0)
    p.perspective = 1 if perspective else 0
    for i in range(3):
        p.plane[i] = float(plane[i])
    p.ncc_radius, p.bil_radius = int(ncc_radius), int(bil_radius)
    p.sigma_s, p.sigma_r = float(sigma_s), float(sigma_r)
    p.lr_delta = float(lr_delta)
    p.lr_check = 1 if lr_check else 0
    p.softargmin_T = float(softargmin_T)
    return p


def params_from_workload(w, **override) -> StereoParams:
    kw = dict(dtype=w.dtype, delta_p=w.delta_p, perspective=w.perspective, plane=w.plane,
              ncc_radius=w.ncc_radius, bil_radius=w.bil_radius, sigma_s=w.sigma_s,
              sigma_r=w.sigma_r, lr_delta=w.lr_delta, lr_check=w.lr_check,
              softargmin_T=w.softargmin_T)
    kw.update(override)
    return make_params(w.width, w.height, w.num_disp, **kw)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """An immutable host plan plus a device workspace owned by this object."""

    def __init__(self, params: StereoParams):
        lib = _lib.load()
        h = ctypes.c_void_p()
        check(lib.stereo_plan_create(ctypes.byref(params), ctypes.byref(h)))
        self._h = h
        self.params = params
        self.homography = None
        n = ctypes.c_size_t()
        check(lib.stereo_plan_workspace_bytes(h, ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self._ws = None

    @classmethod
    def from_workload(cls, w, **override):
        plan = cls(params_from_workload(w, **override))
        if getattr(w, "homography", None) is not None and plan.params.perspective:
            plan.set_homography(w.homography)
        return plan

    @property
    def handle(self):
        return self._h

    @property
    def W(self):
        return self.params.width

    @property
    def H(self):
        return self.params.height

    @property
    def D(self):
        return self.params.num_disp

    @property
    def img_dtype(self):
        return torch.uint8 if self.params.dtype == _lib.U8 else torch.float32

    def set_homography(self, H):
        """Full Eq. (3) warp by the 3x3 homography H (None: the plane's row shift)."""
        if H is None:
            check(_lib.load().stereo_plan_set_homography(self.handle, None))
            self.homography = None
            return
        vals = [float(x) for x in (H.ravel().tolist() if hasattr(H, "ravel") else list(H))]
        if len(vals) != 9:
            raise ValueError("H must have 9 entries")
        arr = (ctypes.c_double * 9)(*vals)
        check(_lib.load().stereo_plan_set_homography(self.handle, ctypes.cast(arr, ctypes.c_void_p)))
        self.homography = tuple(vals)

    def set_tuning(self, key: str, value: int):
        lib = _lib.load()
        check(lib.stereo_plan_set_tuning(self._h, key.encode(), int(value)))
        n = ctypes.c_size_t()
        check(lib.stereo_plan_workspace_bytes(self._h, ctypes.byref(n)))
        if int(n.value) != self.workspace_bytes:
            self.workspace_bytes = int(n.value)
            self._ws = None

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_int32()
        check(_lib.load().stereo_plan_get_tuning(self._h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def workspace(self, device="cuda"):
        if self._ws is None or self._ws.device != torch.device(device):
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        return self._ws

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                _lib.load().stereo_plan_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass


def warp(plan: Plan, tar):
    _need(tar, plan.img_dtype, (plan.H, plan.W), "tar")
    out = torch.empty((plan.H, plan.W), dtype=torch.float32, device=tar.device)
    check(_lib.load().stereo_warp(plan.handle, _p(tar), _p(out), _stream()))
    return out


def cost_volume(plan: Plan, ref, tar_w, want_target=True):
    _need(ref, plan.img_dtype, (plan.H, plan.W), "ref")
    _need(tar_w, torch.float32, (plan.H, plan.W), "tar_w")
    shape = (plan.D, plan.H, plan.W)
    cR = torch.empty(shape, dtype=torch.float32, device=ref.device)
    cT = torch.empty(shape, dtype=torch.float32, device=ref.device) if want_target else None
    ws = plan.workspace(ref.device)
    check(_lib.load().stereo_cost_volume(plan.handle, _p(ref), _p(tar_w), _p(cR), _p(cT),
                                         _p(ws), plan.workspace_bytes, _stream()))
    return cR, cT


def bilateral_aggregate(plan: Plan, guide, cost):
    if guide.dtype not in (torch.uint8, torch.float32):
        raise ValueError("guide must be uint8 or float32")
    _need(guide, guide.dtype, (plan.H, plan.W), "guide")
    _need(cost, torch.float32, (plan.D, plan.H, plan.W), "cost")
    out = torch.empty_like(cost)
    gdt = _lib.U8 if guide.dtype == torch.uint8 else _lib.F32
    check(_lib.load().stereo_bilateral_aggregate(plan.handle, _p(guide), gdt, plan.W,
                                                 _p(cost), _p(out), _stream()))
    return out


def wta_subpixel(plan: Plan, agg):
    _need(agg, torch.float32, (plan.D, plan.H, plan.W), "agg")
    dint = torch.empty((plan.H, plan.W), dtype=torch.int16, device=agg.device)
    dsub = torch.empty((plan.H, plan.W), dtype=torch.float32, device=agg.device)
    check(_lib.load().stereo_wta_subpixel(plan.handle, _p(agg), _p(dint), _p(dsub), _stream()))
    return dint, dsub


def lr_check(plan: Plan, dint_R, dint_T, dsub_R):
    _need(dint_R, torch.int16, (plan.H, plan.W), "dint_R")
    if dint_T is not None:
        _need(dint_T, torch.int16, (plan.H, plan.W), "dint_T")
    if dsub_R is not None:
        _need(dsub_R, torch.float32, (plan.H, plan.W), "dsub_R")
    valid = torch.empty((plan.H, plan.W), dtype=torch.uint8, device=dint_R.device)
    disp = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dint_R.device)
    check(_lib.load().stereo_lr_check(plan.handle, _p(dint_R), _p(dint_T), _p(dsub_R),
                                      _p(valid), _p(disp), _stream()))
    return valid, disp


def match(plan: Plan, ref, tar, want_target=False, out=None):
    """Whole plain forward; returns dint_R, dsub, valid, disp (and dint_T)."""
    _need(ref, plan.img_dtype, (plan.H, plan.W), "ref")
    _need(tar, plan.img_dtype, (plan.H, plan.W), "tar")
    dev = ref.device
    if out is None:
        out = dict(
            dint_R=torch.empty((plan.H, plan.W), dtype=torch.int16, device=dev),
            dsub=torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev),
            valid=torch.empty((plan.H, plan.W), dtype=torch.uint8, device=dev),
            disp=torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev))
        if want_target:
            out["dint_T"] = torch.empty((plan.H, plan.W), dtype=torch.int16, device=dev)
    ws = plan.workspace(dev)
    check(_lib.load().stereo_match(plan.handle, _p(ref), _p(tar), _p(out["dint_R"]),
                                   _p(out.get("dint_T")), _p(out["dsub"]), _p(out["valid"]),
                                   _p(out["disp"]), _p(ws), plan.workspace_bytes, _stream()))
    return out


def road_fit_from_bytes(buf: torch.Tensor) -> dict:
    raw = bytes(buf.cpu().numpy().tobytes())
    f = RoadFit.from_buffer_copy(raw)
    return dict(psi=f.psi, alpha0=f.alpha0, alpha1=f.alpha1, e_min=f.e_min,
                plane=tuple(f.plane), n_points=f.n_points, iters=f.iters,
                converged=bool(f.converged), flat=bool(f.flat))


def road_transform(plan: Plan, disp, mask=None, psi_init=0.0, lambda0=LAMBDA0,
                   delta_psi=DELTA_PSI, max_iter=100, delta_t=0.0, fit_buf=None,
                   out=None, read_fit=True):
    """Roll fit + disparity transformation; returns (fit dict or buffer, disp_t)."""
    _need(disp, torch.float32, (plan.H, plan.W), "disp")
    if mask is not None:
        _need(mask, torch.uint8, (plan.H, plan.W), "mask")
    dev = disp.device
    if fit_buf is None:
        fit_buf = torch.empty(ctypes.sizeof(RoadFit), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty_like(disp)
    ws = plan.workspace(dev)
    check(_lib.load().stereo_road_transform(
        plan.handle, _p(disp), _p(mask), float(psi_init), float(lambda0), float(delta_psi),
        int(max_iter), float(delta_t), _p(fit_buf), _p(out), _p(ws), plan.workspace_bytes,
        _stream()))
    return (road_fit_from_bytes(fit_buf) if read_fit else fit_buf), out


def road_transform_noalloc(plan: Plan, disp, mask=None, psi_init=0.0, lambda0=LAMBDA0,
                           delta_psi=DELTA_PSI, max_iter=100, delta_t=0.0, fit_buf=None,
                           out=None, read_fit=True):
    """road_transform through the entry point that uses the library's fixed
    device buffer instead of the plan's workspace (allocates nothing on the
    device when fit_buf and out are given)."""
    _need(disp, torch.float32, (plan.H, plan.W), "disp")
    if mask is not None:
        _need(mask, torch.uint8, (plan.H, plan.W), "mask")
    dev = disp.device
    if fit_buf is None:
        fit_buf = torch.empty(ctypes.sizeof(RoadFit), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty_like(disp)
    check(_lib.load().stereo_road_transform_noalloc(
        plan.handle, _p(disp), _p(mask), float(psi_init), float(lambda0), float(delta_psi),
        int(max_iter), float(delta_t), _p(fit_buf), _p(out), _stream()))
    return (road_fit_from_bytes(fit_buf) if read_fit else fit_buf), out


class PlaneTracker:
    """Closed-loop plane estimation over a frame sequence: each frame is
    matched with the plane fitted on the previous one (state in device
    memory, no host synchronisation per frame).  Initialise with set() or
    init_from_fit() (e.g. the fit of a full-range pass without the warp)."""

    def __init__(self, plan: Plan, device="cuda"):
        if not plan.params.perspective:
            raise ValueError("tracking needs a plan with perspective = 1")
        self.plan = plan
        self.state = torch.zeros(ctypes.sizeof(PlaneState), dtype=torch.uint8, device=device)
        self.fit_buf = torch.zeros(ctypes.sizeof(RoadFit), dtype=torch.uint8, device=device)

    def set(self, plane, psi=0.0, frames=0):
        st = PlaneState()
        for k in range(3):
            st.plane[k] = float(plane[k])
        st.psi = float(psi)
        st.frames = int(frames)
        host = torch.frombuffer(bytearray(bytes(st)), dtype=torch.uint8)
        self.state.copy_(host)

    def init_from_fit(self, fit: dict):
        self.set(fit["plane"], fit["psi"], 0)

    def read(self) -> dict:
        st = PlaneState.from_buffer_copy(bytes(self.state.cpu().numpy().tobytes()))
        return dict(plane=tuple(st.plane), psi=st.psi, frames=st.frames)

    def step(self, ref, tar, out=None, disp_t=None, delta_t=0.0, lambda0=LAMBDA0,
             delta_psi=DELTA_PSI, max_iter=100, want_target=False):
        """Match with the current plane, then fit and fold the new plane in.
        Returns the match outputs plus disp_t (transformed map)."""
        plan = self.plan
        _need(ref, plan.img_dtype, (plan.H, plan.W), "ref")
        _need(tar, plan.img_dtype, (plan.H, plan.W), "tar")
        dev = ref.device
        if out is None:
            out = dict(
                dint_R=torch.empty((plan.H, plan.W), dtype=torch.int16, device=dev),
                dsub=torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev),
                valid=torch.empty((plan.H, plan.W), dtype=torch.uint8, device=dev),
                disp=torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev))
            if want_target:
                out["dint_T"] = torch.empty((plan.H, plan.W), dtype=torch.int16, device=dev)
        if disp_t is None:
            disp_t = out.get("disp_t")
            if disp_t is None:
                disp_t = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
        ws = plan.workspace(dev)
        lib = _lib.load()
        check(lib.stereo_match_tracked(plan.handle, _p(ref), _p(tar), _p(self.state),
                                       _p(out["dint_R"]), _p(out.get("dint_T")),
                                       _p(out["dsub"]), _p(out["valid"]), _p(out["disp"]),
                                       _p(ws), plan.workspace_bytes, _stream()))
        check(lib.stereo_road_transform_tracked(plan.handle, _p(out["disp"]), _p(out["valid"]),
                                                float(lambda0), float(delta_psi), int(max_iter),
                                                float(delta_t), _p(self.state),
                                                _p(self.fit_buf), _p(disp_t), _p(ws),
                                                plan.workspace_bytes, _stream()))
        out["disp_t"] = disp_t
        return out


def damage_mask(plan: Plan, disp_t, delta_t=0.0, tau=0.5, out=None):
    """uint8 [H][W]: 1 where the transformed disparity lies more than tau
    below the flattened road level delta_t (Sec. 4.4.3)."""
    _need(disp_t, torch.float32, (plan.H, plan.W), "disp_t")
    if out is None:
        out = torch.empty((plan.H, plan.W), dtype=torch.uint8, device=disp_t.device)
    check(_lib.load().stereo_damage_mask(plan.handle, _p(disp_t), float(delta_t), float(tau),
                                         _p(out), _stream()))
    return out


# ---- differentiable form ----------------------------------------------------
def _plane3(plane):
    vals = [float(x) for x in (plane.detach().cpu().tolist() if isinstance(plane, torch.Tensor)
                               else plane)]
    if len(vals) != 3:
        raise ValueError("plane must have 3 entries")
    return (ctypes.c_double * 3)(*vals)


def soft_forward(plan: Plan, ref, tar, plane):
    """Soft-argmin disparity; returns (disp_soft [H][W], saved [3][H][W])."""
    _need(ref, torch.float32, (plan.H, plan.W), "ref")
    _need(tar, torch.float32, (plan.H, plan.W), "tar")
    disp = torch.empty((plan.H, plan.W), dtype=torch.float32, device=ref.device)
    saved = torch.empty((3, plan.H, plan.W), dtype=torch.float32, device=ref.device)
    ws = plan.workspace(ref.device)
    check(_lib.load().stereo_soft_forward(plan.handle, _p(ref), _p(tar), _plane3(plane), _p(disp),
                                          _p(saved), _p(ws), plan.workspace_bytes, _stream()))
    return disp, saved


def backward(plan: Plan, ref, tar, plane, saved, grad_disp):
    """VJP of soft_forward: returns (grad_ref, grad_tar, grad_plane[3] float64)."""
    _need(saved, torch.float32, (3, plan.H, plan.W), "saved")
    _need(grad_disp, torch.float32, (plan.H, plan.W), "grad_disp")
    dev = ref.device
    g_ref = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
    g_tar = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
    g_plane = torch.empty(3, dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)
    check(_lib.load().stereo_backward(plan.handle, _p(ref), _p(tar), _plane3(plane), _p(saved),
                                      _p(grad_disp), _p(g_ref), _p(g_tar), _p(g_plane), _p(ws),
                                      plan.workspace_bytes, _stream()))
    return g_ref, g_tar, g_plane


def photometric_l1(plan: Plan, ref, tar, disp):
    _need(disp, torch.float32, (plan.H, plan.W), "disp")
    loss = torch.empty((), dtype=torch.float64, device=ref.device)
    ws = plan.workspace(ref.device)
    check(_lib.load().stereo_photometric_l1(plan.handle, _p(ref), _p(tar), _p(disp), _p(loss),
                                            _p(ws), plan.workspace_bytes, _stream()))
    return loss


def photometric_l1_bwd(plan: Plan, ref, tar, disp, grad_loss=1.0):
    dev = ref.device
    g_ref = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
    g_tar = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
    g_disp = torch.empty((plan.H, plan.W), dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    check(_lib.load().stereo_photometric_l1_bwd(plan.handle, _p(ref), _p(tar), _p(disp),
                                                float(grad_loss), _p(g_ref), _p(g_tar),
                                                _p(g_disp), _p(ws), plan.workspace_bytes,
                                                _stream()))
    return g_ref, g_tar, g_disp


# ---- autotuner and batched form --------------------------------------------
def autotune(plan: Plan, ref, tar, cache_path: Optional[str] = None, reps: int = 3) -> float:
    """Time the plan's launch-shape variants on (ref, tar) and keep the fastest;
    returns its time in ms.  Synchronous; results never depend on the choice."""
    best = ctypes.c_double()
    ws = plan.workspace(ref.device)
    check(_lib.load().stereo_plan_autotune(plan.handle, _p(ref), _p(tar), _p(ws),
                                           plan.workspace_bytes, _stream(),
                                           cache_path.encode() if cache_path else None,
                                           int(reps), ctypes.byref(best)))
    return float(best.value)


class Batch:
    """Many pairs (each with its own plan) enqueued together; see stereo.h.

    pairs: list of (plan, ref, tar).  Outputs per pair: dint_R, valid, disp.
    """

    def __init__(self, pairs, device="cuda"):
        lib = _lib.load()
        self.plans = [p for p, _, _ in pairs]
        self.inputs = [(r, t) for _, r, t in pairs]
        self.outputs = []
        items = (_lib.BatchItem * len(pairs))()
        for i, (plan, ref, tar) in enumerate(pairs):
            _need(ref, plan.img_dtype, (plan.H, plan.W), f"ref[{i}]")
            _need(tar, plan.img_dtype, (plan.H, plan.W), f"tar[{i}]")
            o = dict(dint_R=torch.empty((plan.H, plan.W), dtype=torch.int16, device=device),
                     valid=torch.empty((plan.H, plan.W), dtype=torch.uint8, device=device),
                     disp=torch.empty((plan.H, plan.W), dtype=torch.float32, device=device))
            self.outputs.append(o)
            items[i].plan = plan.handle.value
            items[i].ref = ref.data_ptr()
            items[i].tar = tar.data_ptr()
            items[i].dint_R = o["dint_R"].data_ptr()
            items[i].valid = o["valid"].data_ptr()
            items[i].disp = o["disp"].data_ptr()
        h = ctypes.c_void_p()
        check(lib.stereo_batch_create(items, len(pairs), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_size_t()
        check(lib.stereo_batch_workspace_bytes(h, ctypes.byref(n)))
        self.workspace_bytes = int(n.value)
        self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def set_tuning(self, key, value):
        check(_lib.load().stereo_batch_set_tuning(self._h, key.encode(), int(value)))

    def get_tuning(self, key):
        v = ctypes.c_int32()
        check(_lib.load().stereo_batch_get_tuning(self._h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def submit(self):
        check(_lib.load().stereo_submit_batch(self._h, _p(self.ws), self.workspace_bytes,
                                              _stream()))
        return self.outputs

    def instantiate(self):
        check(_lib.load().stereo_batch_instantiate(self._h, _p(self.ws), self.workspace_bytes,
                                                   _stream()))

    def launch(self):
        check(_lib.load().stereo_batch_launch(self._h, _stream()))
        return self.outputs

    def autotune(self, cache_path=None, reps=3):
        best = ctypes.c_double()
        check(_lib.load().stereo_batch_autotune(self._h, _p(self.ws), self.workspace_bytes,
                                                _stream(),
                                                cache_path.encode() if cache_path else None,
                                                int(reps), ctypes.byref(best)))
        return float(best.value)

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                _lib.load().stereo_batch_destroy(self._h)
                self._h = ctypes.c_void_p()
        except Exception:
            pass
