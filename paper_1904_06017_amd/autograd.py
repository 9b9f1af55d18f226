"""torch.autograd.Function wrappers of the differentiable form.

    disp = SoftDisparity.apply(ref, tar, plane, plan)       # [H][W]
    loss = PhotometricL1.apply(ref, tar, disp, plan)        # scalar (float64)
    loss.backward()                                          # grads of ref, tar, plane

ref and tar are [H][W] float32 CUDA tensors; plane is a 3-vector (a CPU
float64 tensor avoids a device sync when its values are read).  The plan must
be an F32 plan with the perspective step.  Forward and backward run in the
library's HIP kernels; nothing falls back to PyTorch ops.
"""
from __future__ import annotations

import torch

from . import api


class SoftDisparity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ref, tar, plane, plan):
        ref = ref.contiguous()
        tar = tar.contiguous()
        disp, saved = api.soft_forward(plan, ref, tar, plane)
        ctx.plan = plan
        ctx.plane_values = [float(x) for x in plane.detach().cpu().tolist()]
        ctx.plane_meta = (plane.dtype, plane.device)
        ctx.save_for_backward(ref, tar, saved)
        return disp

    @staticmethod
    def backward(ctx, grad_disp):
        ref, tar, saved = ctx.saved_tensors
        g_ref, g_tar, g_plane = api.backward(ctx.plan, ref, tar, ctx.plane_values, saved,
                                             grad_disp.contiguous().float())
        dtype, device = ctx.plane_meta
        return g_ref, g_tar, g_plane.to(device=device, dtype=dtype), None


class PhotometricL1(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ref, tar, disp, plan):
        ref, tar, disp = ref.contiguous(), tar.contiguous(), disp.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(ref, tar, disp)
        return api.photometric_l1(plan, ref, tar, disp)

    @staticmethod
    def backward(ctx, grad_loss):
        ref, tar, disp = ctx.saved_tensors
        g_ref, g_tar, g_disp = api.photometric_l1_bwd(ctx.plan, ref, tar, disp,
                                                      float(grad_loss))
        return g_ref, g_tar, g_disp, None
