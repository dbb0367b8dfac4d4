"""torch.autograd binding of the forward modelling and its adjoint.

``FDTraces.apply(v, grid, shots, ckpt_every)`` returns the traces of every
shot (``[nshots, nt, nrec]``, FP32) for the velocity model ``v`` (FP32, one
entry per cell).  Its backward pass calls ``fd_adjoint_gradient`` once per
shot: each checkpoint segment is recomputed from the states the forward pass
saved every ``ckpt_every`` steps, the adjoint field is stepped backward in
time with the incoming trace gradient injected at the receivers, and the
velocity gradient is summed over time and shots in FP64 on the device.
Every step runs in the library's HIP kernels; this module only allocates
buffers and orders the calls.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import Grid, Model, Shot


class FDTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v: torch.Tensor, grid: Grid, shots: Sequence[Shot], ckpt_every: int):
        if v.dtype != torch.float32:
            raise ValueError("velocity must be FP32")
        nt = shots[0].nt
        nrec = shots[0].nrec
        for s in shots:
            if s.nt != nt or s.nrec != nrec:
                raise ValueError("all shots of one call share nt and the receiver count")
        model = Model(grid, v.detach().reshape(-1))
        state = model.new_state()
        traces = torch.empty((len(shots), nt, nrec), dtype=torch.float32, device=v.device)
        ckpts = []
        for i, s in enumerate(shots):
            ck = model.checkpoint_buffer(nt, ckpt_every)
            model.run_shot(state, s, traces[i], ckpt=ck, ckpt_every=ckpt_every)
            ckpts.append(ck)
        ctx.model = model
        ctx.shots = list(shots)
        ctx.ckpts = ckpts
        ctx.every = ckpt_every
        ctx.vshape = v.shape
        return traces

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        model: Model = ctx.model
        g = torch.zeros(model.grid.ncells, dtype=torch.float64, device=grad_traces.device)
        work = None
        for i, s in enumerate(ctx.shots):
            adj = grad_traces[i].to(torch.float32).contiguous()
            if work is None:
                from . import _alloc
                work = _alloc(model.sizes_for(s.nt, ctx.every).adjoint_work, model.device)
            model.adjoint_gradient(s, adj, ctx.ckpts[i], ctx.every, g, work=work)
        ctx.ckpts = None
        return g.reshape(ctx.vshape).to(torch.float32), None, None, None


def modelled_traces(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                    ckpt_every: int = 50) -> torch.Tensor:
    """Differentiable traces of `shots` in the velocity model `v`."""
    return FDTraces.apply(v, grid, shots, ckpt_every)


def l2_misfit_gradient(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                       observed: torch.Tensor, ckpt_every: int = 50):
    """J = 1/2 ||d(v) - d_obs||^2 and dJ/dv (FP64), without autograd
    bookkeeping: the adjoint source of each shot is its residual."""
    model = Model(grid, v.detach().reshape(-1).to(torch.float32))
    state = model.new_state()
    g = torch.zeros(grid.ncells, dtype=torch.float64, device=v.device)
    J = 0.0
    work = None
    for i, s in enumerate(shots):
        ck = model.checkpoint_buffer(s.nt, ckpt_every)
        tr = model.run_shot(state, s, ckpt=ck, ckpt_every=ckpt_every)
        res = (tr - observed[i]).contiguous()
        J += 0.5 * float((res.double() ** 2).sum())
        if work is None:
            from . import _alloc
            work = _alloc(model.sizes_for(s.nt, ckpt_every).adjoint_work, model.device)
        model.adjoint_gradient(s, res, ck, ckpt_every, g, work=work)
    return J, g
