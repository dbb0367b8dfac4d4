"""torch.autograd binding of the forward modelling and its adjoint.

``FDTraces.apply(v, grid, shots, ckpt_every[, group])`` returns the traces of every
shot (``[nshots, nt, nrec]``, FP32) for the velocity model ``v`` (FP32, one
entry per cell).  Its backward pass calls ``fd_adjoint_gradient_shots`` on
groups of shots: each checkpoint segment is recomputed from the states the forward pass
saved every ``ckpt_every`` steps, the adjoint field is stepped backward in
time with the incoming trace gradient injected at the receivers, and the
velocity gradient is summed over time and shots in FP64 on the device.
Every step runs in the library's HIP kernels; this module only allocates
buffers and orders the calls.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import Grid, Model, Shot, _alloc

# Shots are independent: a call processes them in groups of up to
# GROUP shots with the library's multi-shot entry points (fd_run_shots,
# fd_adjoint_gradient_shots, fd_rtm_image_shots), which in 2D advance every
# shot of a group with one kernel launch per time step.  Each shot of a
# group holds its own state, checkpoints and work buffer.
GROUP = 16


def _groups(n: int, group: int):
    group = max(1, int(group))
    return [list(range(i, min(n, i + group))) for i in range(0, n, group)]


class FDTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v: torch.Tensor, grid: Grid, shots: Sequence[Shot], ckpt_every: int,
                group: int = GROUP):
        if v.dtype != torch.float32:
            raise ValueError("velocity must be FP32")
        nt = shots[0].nt
        nrec = shots[0].nrec
        for s in shots:
            if s.nt != nt or s.nrec != nrec:
                raise ValueError("all shots of one call share nt and the receiver count")
        model = Model(grid, v.detach().reshape(-1))
        traces = torch.empty((len(shots), nt, nrec), dtype=torch.float32, device=v.device)
        ckpts = [model.checkpoint_buffer(nt, ckpt_every) for _ in shots]
        for idx in _groups(len(shots), group):
            states = [model.new_state() for _ in idx]
            model.run_shots(states, [shots[i] for i in idx], traces[idx[0]:idx[-1] + 1],
                            [ckpts[i] for i in idx], ckpt_every)
        ctx.model = model
        ctx.shots = list(shots)
        ctx.ckpts = ckpts
        ctx.every = ckpt_every
        ctx.vshape = v.shape
        ctx.group = group
        return traces

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        model: Model = ctx.model
        shots = ctx.shots
        g = torch.zeros(model.grid.ncells, dtype=torch.float64, device=grad_traces.device)
        adj = grad_traces.to(torch.float32).contiguous()
        need = model.sizes_for(shots[0].nt, ctx.every).adjoint_work
        for idx in _groups(len(shots), ctx.group):
            works = [_alloc(need, model.device) for _ in idx]
            model.adjoint_gradient_shots([shots[i] for i in idx], [adj[i] for i in idx],
                                         [ctx.ckpts[i] for i in idx], ctx.every, g, works=works)
        ctx.ckpts = None
        return g.reshape(ctx.vshape).to(torch.float32), None, None, None, None


def modelled_traces(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                    ckpt_every: int = 50, group: int = GROUP) -> torch.Tensor:
    """Differentiable traces of `shots` in the velocity model `v`."""
    return FDTraces.apply(v, grid, shots, ckpt_every, group)


def l2_misfit_gradient(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                       observed: torch.Tensor, ckpt_every: int = 50, group: int = GROUP):
    """J = 1/2 ||d(v) - d_obs||^2 and dJ/dv (FP64), without autograd
    bookkeeping: the adjoint source of each shot is its residual.  The FP64
    gradient is summed shot after shot in the order of `shots`."""
    model = Model(grid, v.detach().reshape(-1).to(torch.float32))
    nt = shots[0].nt
    for s in shots:
        if s.nt != nt:
            raise ValueError("all shots of one call share nt")
    g = torch.zeros(grid.ncells, dtype=torch.float64, device=v.device)
    J = torch.zeros((), dtype=torch.float64, device=v.device)
    need = model.sizes_for(nt, ckpt_every).adjoint_work
    for idx in _groups(len(shots), group):
        sh = [shots[i] for i in idx]
        states = [model.new_state() for _ in idx]
        ckpts = [model.checkpoint_buffer(nt, ckpt_every) for _ in idx]
        tr = model.run_shots(states, sh, None, ckpts, ckpt_every)
        res = (tr - observed[idx[0]:idx[-1] + 1]).contiguous()
        J += 0.5 * (res.double() ** 2).sum()
        works = [_alloc(need, model.device) for _ in idx]
        model.adjoint_gradient_shots(sh, [res[k] for k in range(len(idx))], ckpts, ckpt_every, g,
                                     works=works)
    return float(J), g


def rtm_image(v: torch.Tensor, grid: Grid, shots: Sequence[Shot], data: torch.Tensor,
              ckpt_every: int = 50, group: int = GROUP) -> torch.Tensor:
    """Sum over shots of the reverse-time-migration image (fd_rtm_image) of
    the recorded `data` ([nshots, nt, nrec]) in the model `v`: each shot's
    source field is modelled with checkpoints, then correlated with its
    back-propagated data.  FP64, one entry per cell."""
    model = Model(grid, v.detach().reshape(-1).to(torch.float32))
    nt = shots[0].nt
    img = torch.zeros(grid.ncells, dtype=torch.float64, device=v.device)
    need = model.sizes_for(nt, ckpt_every).adjoint_work
    d = data.to(torch.float32).contiguous()
    for idx in _groups(len(shots), group):
        sh = [shots[i] for i in idx]
        states = [model.new_state() for _ in idx]
        ckpts = [model.checkpoint_buffer(nt, ckpt_every) for _ in idx]
        model.run_shots(states, sh, None, ckpts, ckpt_every)
        works = [_alloc(need, model.device) for _ in idx]
        model.rtm_image_shots(sh, [d[i] for i in idx], ckpts, ckpt_every, img, works=works)
    return img
