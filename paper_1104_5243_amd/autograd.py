"""torch.autograd wrappers of the backprojector / forward-projector pair.

The backprojection B (fdk_backproject) and the matched forward projection
F = B^T (fdk_forward_project) are linear and each is the other's adjoint,
so the gradient of one is the other applied to the incoming gradient.
Both run in the library's HIP kernels; these classes only allocate the
outputs and call through the C ABI on the current stream.  A leading batch
dimension is processed one item at a time (all calls are asynchronous).
"""
from __future__ import annotations

import numpy as np
import torch

from . import backproject, forward_project


def _geometry(P, voxel_size, origin):
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 3, 4))
    o = tuple(float(v) for v in np.asarray(origin, dtype=np.float64).reshape(3))
    return P, float(voxel_size), o


def _bp(proj, P, N, vs, o):
    """(..., V, H, W) -> (..., N, N, N)."""
    lead = proj.shape[:-3]
    p = proj.reshape(-1, *proj.shape[-3:])
    out = torch.zeros(p.shape[0], N, N, N, device=proj.device, dtype=torch.float32)
    for b in range(p.shape[0]):
        backproject(out[b], p[b].contiguous(), P, vs, o)
    return out.reshape(*lead, N, N, N)


def _fp(vol, P, H, W, vs, o):
    """(..., N, N, N) -> (..., V, H, W)."""
    lead = vol.shape[:-3]
    v = vol.reshape(-1, *vol.shape[-3:])
    out = torch.zeros(v.shape[0], P.shape[0], H, W, device=vol.device, dtype=torch.float32)
    for b in range(v.shape[0]):
        forward_project(out[b], v[b].contiguous(), P, vs, o)
    return out.reshape(*lead, P.shape[0], H, W)


class BackProject(torch.autograd.Function):
    """volume = B(proj); backward: grad_proj = F(grad_volume)."""

    @staticmethod
    def forward(ctx, proj, P, N, voxel_size, origin):
        if proj.dtype != torch.float32:
            raise TypeError("BackProject takes float32 projections")
        P, vs, o = _geometry(P, voxel_size, origin)
        ctx.geom = (P, vs, o, proj.shape[-2], proj.shape[-1])
        return _bp(proj.contiguous(), P, int(N), vs, o)

    @staticmethod
    def backward(ctx, grad_vol):
        P, vs, o, H, W = ctx.geom
        grad = _fp(grad_vol.contiguous().float(), P, H, W, vs, o) if ctx.needs_input_grad[0] else None
        return grad, None, None, None, None


class ForwardProject(torch.autograd.Function):
    """proj = F(volume) = B^T volume; backward: grad_volume = B(grad_proj)."""

    @staticmethod
    def forward(ctx, vol, P, H, W, voxel_size, origin):
        if vol.dtype != torch.float32:
            raise TypeError("ForwardProject takes a float32 volume")
        P, vs, o = _geometry(P, voxel_size, origin)
        ctx.geom = (P, vs, o, vol.shape[-1])
        return _fp(vol.contiguous(), P, int(H), int(W), vs, o)

    @staticmethod
    def backward(ctx, grad_proj):
        P, vs, o, N = ctx.geom
        grad = _bp(grad_proj.contiguous().float(), P, N, vs, o) if ctx.needs_input_grad[0] else None
        return grad, None, None, None, None, None


def backproject_op(proj, P, N, voxel_size, origin):
    return BackProject.apply(proj, P, N, voxel_size, origin)


def forward_project_op(vol, P, H, W, voxel_size, origin):
    return ForwardProject.apply(vol, P, H, W, voxel_size, origin)
