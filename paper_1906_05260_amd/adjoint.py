"""Gradients of the rod solver with respect to rest radii and activations.

``RodFrames`` is a ``torch.autograd.Function`` around the C-ABI adjoint
(include/viper.h: viper_step_checkpointed / viper_step_backward): its forward
builds a scene from the given rest radii r (Sec. 3) and activations a (Sec. 8),
advances it ``frames`` frames from rest with a checkpoint of the state at every
substep start, and returns the final pill positions; its backward replays the
substeps in reverse on the GPU and returns dL/dr and dL/da.  Only argument
marshalling happens here.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import viper


class RodFrames(torch.autograd.Function):
    """x_end(rbar, act): pill positions after ``frames`` frames from rest."""

    @staticmethod
    def forward(ctx, rbar, act, desc, dt, substeps, iterations, frames, precision, device):
        d = dataclasses.replace(desc, rest_radius=rbar.detach().double().cpu().numpy().copy(),
                                activation=act.detach().double().cpu().numpy().copy(), collisions=False)
        sc = viper.Scene(d, precision, device=device)
        ckpt = sc.step_checkpointed(dt, frames, substeps, iterations)
        x = sc.get("x").double()
        ctx.scene, ctx.ckpt = sc, ckpt
        ctx.args = (float(dt), int(frames), int(substeps), int(iterations))
        ctx.like = (rbar.dtype, rbar.device, act.dtype, act.device)
        return x

    @staticmethod
    def backward(ctx, gx):
        sc = ctx.scene
        dt, frames, substeps, iterations = ctx.args
        drbar, dact = sc.backward(dt, frames, substeps, iterations, ctx.ckpt, gx)
        rd, rdev, ad, adev = ctx.like
        return (drbar.to(device=rdev, dtype=rd), dact.to(device=adev, dtype=ad),
                None, None, None, None, None, None, None)


def rod_frames(rbar, act, desc, dt, substeps, iterations, frames=1, precision="f32", device="cuda:0"):
    """Final pill positions [P, 3] (float64, world frame) after ``frames`` frames from rest,
    differentiable with respect to ``rbar`` [P] and ``act`` [R]."""
    return RodFrames.apply(rbar, act, desc, dt, substeps, iterations, frames, precision, device)


def end_loss(x, desc, targets):
    """L = sum over rods of |x(last pill) - target|^2."""
    last = torch.as_tensor(np.asarray(desc.rod_offsets[1:]) - 1, device=x.device, dtype=torch.long)
    t = torch.as_tensor(np.asarray(targets).reshape(-1, 3), device=x.device, dtype=x.dtype)
    return ((x[last] - t) ** 2).sum()
