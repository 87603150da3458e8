"""Differentiation of the mechanical step through torch.autograd.

* :class:`MechStep`  one step: (x, y, z, d, kappa, gamma) -> displacement,
  backward through ``ms_mech_step_backward``.
* :func:`rollout`    T steps p_{t+1} = p_t + Delta(p_t) with the grid rebuilt
  every step (Section IV-A).  Only every K-th position is stored; backward
  recomputes each K-step segment from its checkpoint and walks it in reverse
  with ``ms_mech_step_backward_accumulate``, which forms
  pbar_t = pbar_{t+1} + J_Delta(p_t)^T pbar_{t+1} and adds the gradients of
  the diameters and of kappa, gamma on the device (this module only
  allocates, copies and calls).  Every kernel sums in a fixed order, so the
  recomputed trajectory and the gradients do not depend on K.

kappa and gamma may be Python floats or 0-d CPU float64 tensors (the
parameters are passed to the kernels by value, so a device tensor would force
a synchronisation anyway).
"""
from __future__ import annotations

import torch

from . import (grid_build, integrate, mech_step, mech_step_backward,
               mech_step_backward_accumulate, Workspace)


def _f(v) -> float:
    return float(v.item()) if isinstance(v, torch.Tensor) else float(v)


def _params(kappa, gamma, rest):
    return dict(kappa=_f(kappa), gamma=_f(gamma), dt=float(rest["dt"]),
                max_disp=float(rest["max_disp"]), adherence=float(rest.get("adherence", 0.0)))


def _grad_like(g, ref):
    if not isinstance(ref, torch.Tensor):
        return None
    return g.to(device=ref.device, dtype=ref.dtype).reshape(ref.shape)


class MechStep(torch.autograd.Function):
    """Displacements of one step, differentiable wrt positions, diameters,
    kappa and gamma."""

    @staticmethod
    def forward(ctx, x, y, z, d, kappa, gamma, ws: Workspace, rest: dict, edge: float = 0.0):
        p = _params(kappa, gamma, rest)
        grid_build(ws, x, y, z, d, edge)
        ws.keep_forces = True
        D = mech_step(ws, p)
        ctx.save_for_backward(x, y, z, d)
        ctx.ws, ctx.p, ctx.edge, ctx.builds = ws, p, edge, ws.builds
        ctx.kg_ref = (kappa, gamma)
        return D

    @staticmethod
    def backward(ctx, gdx, gdy, gdz):
        x, y, z, d = ctx.saved_tensors
        ws = ctx.ws
        if ws.builds != ctx.builds:                 # the workspace was reused: rebuild
            grid_build(ws, x, y, z, d, ctx.edge)
        g = [(t if t is not None else torch.zeros(ws.n_agents, device=ws.device))
             .to(ws.out_dtype).contiguous() for t in (gdx, gdy, gdz)]
        gx, gy, gz, gd, gkg = mech_step_backward(ws, ctx.p, *g)
        kappa, gamma = ctx.kg_ref
        return (gx.to(x.dtype), gy.to(y.dtype), gz.to(z.dtype), gd.to(d.dtype),
                _grad_like(gkg[0], kappa), _grad_like(gkg[1], gamma), None, None, None)


def mech_step_fn(x, y, z, d, kappa, gamma, ws: Workspace, rest: dict, edge: float = 0.0):
    return MechStep.apply(x, y, z, d, kappa, gamma, ws, rest, edge)


class _Rollout(torch.autograd.Function):

    @staticmethod
    def forward(ctx, x, y, z, d, kappa, gamma, ws: Workspace, rest: dict, steps: int,
                ckpt_every: int, edge: float):
        p = _params(kappa, gamma, rest)
        pos = [x.detach().clone(), y.detach().clone(), z.detach().clone()]
        ckpts = {}
        for t in range(steps):
            if t % ckpt_every == 0:
                ckpts[t] = [a.clone() for a in pos]
            grid_build(ws, *pos, d, edge)
            D = mech_step(ws, p)
            integrate(*pos, *D)
        ctx.save_for_backward(d)
        ctx.ckpts, ctx.ws, ctx.p, ctx.steps, ctx.K, ctx.edge = ckpts, ws, p, steps, ckpt_every, edge
        ctx.kg_ref = (kappa, gamma)
        return pos[0], pos[1], pos[2]

    @staticmethod
    def backward(ctx, gx, gy, gz):
        (d,) = ctx.saved_tensors
        ws, p, steps, K, edge = ctx.ws, ctx.p, ctx.steps, ctx.K, ctx.edge
        ref = ctx.ckpts[0][0]
        pbar = [(g if g is not None else torch.zeros_like(ref)).to(ref.dtype).contiguous().clone()
                for g in (gx, gy, gz)]
        dbar = torch.zeros(d.numel(), dtype=ref.dtype, device=d.device)
        kg = torch.zeros(2, dtype=torch.float64, device=d.device)
        for s0 in sorted(ctx.ckpts, reverse=True):
            s1 = min(s0 + K, steps)
            traj = []
            pos = [a.clone() for a in ctx.ckpts[s0]]
            for t in range(s0, s1):
                traj.append([a.clone() for a in pos])
                if t < s1 - 1:
                    grid_build(ws, *pos, d, edge)
                    D = mech_step(ws, p)
                    integrate(*pos, *D)
            for t in range(s1 - 1, s0 - 1, -1):
                grid_build(ws, *traj[t - s0], d, edge)
                mech_step_backward_accumulate(ws, p, pbar, dbar, kg)
        kappa, gamma = ctx.kg_ref
        return (pbar[0], pbar[1], pbar[2], dbar.to(d.dtype), _grad_like(kg[0], kappa),
                _grad_like(kg[1], gamma), None, None, None, None, None)


def rollout(x, y, z, d, kappa, gamma, ws: Workspace, rest: dict, steps: int, ckpt_every: int = 10,
            edge: float = 0.0):
    """Positions after ``steps`` steps; differentiable with K-step checkpoints."""
    if steps < 1 or ckpt_every < 1:
        raise ValueError("steps and ckpt_every must be >= 1")
    return _Rollout.apply(x, y, z, d, kappa, gamma, ws, rest, int(steps), int(ckpt_every), float(edge))
