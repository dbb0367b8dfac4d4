"""torch.autograd binding of the forward modelling and its adjoint.

``FDTraces.apply(v, grid, shots, ckpt_every[, lanes])`` returns the traces of every
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

from typing import List, Sequence

import torch

from . import Grid, Model, Shot, _alloc

# Shots are independent: they run on a few streams at once ("lanes"), each
# with its own state, checkpoints, work buffer and FP64 accumulator, so the
# small per-step launches of different shots overlap on the device.
DEFAULT_LANES = 4


def _lanes(model: Model, nshots: int, nt: int, ckpt_every: int, lanes: int,
           accumulate: bool) -> List[dict]:
    main = torch.cuda.current_stream(model.device)
    out = []
    for _ in range(max(1, min(lanes, nshots))):
        st = torch.cuda.Stream(device=model.device)
        st.wait_stream(main)
        with torch.cuda.stream(st):
            lane = dict(stream=st, state=model.new_state(),
                        ck=model.checkpoint_buffer(nt, ckpt_every) if ckpt_every else None)
            if accumulate:
                lane["work"] = _alloc(model.sizes_for(nt, ckpt_every).adjoint_work, model.device)
                lane["acc"] = torch.zeros(model.grid.ncells, dtype=torch.float64, device=model.device)
        out.append(lane)
    return out


def _join(lanes: List[dict]) -> None:
    """The current stream waits for every lane; the lane results it reads
    are recorded on it, so the allocator keeps them until it has."""
    main = torch.cuda.current_stream()
    for lane in lanes:
        main.wait_stream(lane["stream"])
        for key in ("acc", "J"):
            if key in lane:
                lane[key].record_stream(main)


class FDTraces(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v: torch.Tensor, grid: Grid, shots: Sequence[Shot], ckpt_every: int,
                lanes: int = DEFAULT_LANES):
        if v.dtype != torch.float32:
            raise ValueError("velocity must be FP32")
        nt = shots[0].nt
        nrec = shots[0].nrec
        for s in shots:
            if s.nt != nt or s.nrec != nrec:
                raise ValueError("all shots of one call share nt and the receiver count")
        model = Model(grid, v.detach().reshape(-1))
        traces = torch.empty((len(shots), nt, nrec), dtype=torch.float32, device=v.device)
        ln = _lanes(model, len(shots), nt, 0, lanes, accumulate=False)
        ckpts = []
        for i, s in enumerate(shots):
            lane = ln[i % len(ln)]
            with torch.cuda.stream(lane["stream"]):
                ck = model.checkpoint_buffer(nt, ckpt_every)
                model.run_shot(lane["state"], s, traces[i], ckpt=ck, ckpt_every=ckpt_every)
            ckpts.append(ck)
        _join(ln)
        ctx.model = model
        ctx.shots = list(shots)
        ctx.ckpts = ckpts
        ctx.every = ckpt_every
        ctx.vshape = v.shape
        ctx.lanes = lanes
        return traces

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        model: Model = ctx.model
        shots = ctx.shots
        ln = _lanes(model, len(shots), shots[0].nt, ctx.every, ctx.lanes, accumulate=True)
        for i, s in enumerate(shots):
            lane = ln[i % len(ln)]
            # the checkpoints were allocated on a forward lane's stream
            ctx.ckpts[i].record_stream(lane["stream"])
            with torch.cuda.stream(lane["stream"]):
                adj = grad_traces[i].to(torch.float32).contiguous()
                model.adjoint_gradient(s, adj, ctx.ckpts[i], ctx.every, lane["acc"],
                                       work=lane["work"])
        _join(ln)
        g = ln[0]["acc"]
        for lane in ln[1:]:
            g = g + lane["acc"]
        ctx.ckpts = None
        return g.reshape(ctx.vshape).to(torch.float32), None, None, None, None


def modelled_traces(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                    ckpt_every: int = 50, lanes: int = DEFAULT_LANES) -> torch.Tensor:
    """Differentiable traces of `shots` in the velocity model `v`."""
    return FDTraces.apply(v, grid, shots, ckpt_every, lanes)


def l2_misfit_gradient(v: torch.Tensor, grid: Grid, shots: Sequence[Shot],
                       observed: torch.Tensor, ckpt_every: int = 50, lanes: int = DEFAULT_LANES):
    """J = 1/2 ||d(v) - d_obs||^2 and dJ/dv (FP64), without autograd
    bookkeeping: the adjoint source of each shot is its residual.  Shots run
    on `lanes` streams at once; the FP64 gradient is summed per lane, then
    over the lanes."""
    model = Model(grid, v.detach().reshape(-1).to(torch.float32))
    ln = _lanes(model, len(shots), shots[0].nt, ckpt_every, lanes, accumulate=True)
    for lane in ln:
        lane["J"] = torch.zeros((), dtype=torch.float64, device=v.device)
    for i, s in enumerate(shots):
        lane = ln[i % len(ln)]
        if s.nt != shots[0].nt:
            raise ValueError("all shots of one call share nt")
        with torch.cuda.stream(lane["stream"]):
            tr = model.run_shot(lane["state"], s, ckpt=lane["ck"], ckpt_every=ckpt_every)
            res = (tr - observed[i]).contiguous()
            lane["J"] += 0.5 * (res.double() ** 2).sum()
            model.adjoint_gradient(s, res, lane["ck"], ckpt_every, lane["acc"], work=lane["work"])
    _join(ln)
    g = ln[0]["acc"]
    J = ln[0]["J"]
    for lane in ln[1:]:
        g = g + lane["acc"]
        J = J + lane["J"]
    return float(J), g


def rtm_image(v: torch.Tensor, grid: Grid, shots: Sequence[Shot], data: torch.Tensor,
              ckpt_every: int = 50, lanes: int = DEFAULT_LANES) -> torch.Tensor:
    """Sum over shots of the reverse-time-migration image (fd_rtm_image) of
    the recorded `data` ([nshots, nt, nrec]) in the model `v`: each shot's
    source field is modelled with checkpoints, then correlated with its
    back-propagated data.  FP64, one entry per cell."""
    model = Model(grid, v.detach().reshape(-1).to(torch.float32))
    ln = _lanes(model, len(shots), shots[0].nt, ckpt_every, lanes, accumulate=True)
    for i, s in enumerate(shots):
        lane = ln[i % len(ln)]
        if s.nt != shots[0].nt:
            raise ValueError("all shots of one call share nt")
        with torch.cuda.stream(lane["stream"]):
            model.run_shot(lane["state"], s, ckpt=lane["ck"], ckpt_every=ckpt_every)
            model.rtm_image(s, data[i].to(torch.float32).contiguous(), lane["ck"], ckpt_every,
                            lane["acc"], work=lane["work"])
    _join(ln)
    img = ln[0]["acc"]
    for lane in ln[1:]:
        img = img + lane["acc"]
    return img
