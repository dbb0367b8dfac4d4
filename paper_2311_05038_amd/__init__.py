"""MI355X (gfx950) finite-difference acoustic wave engine.

The wave equation of arXiv 2311.05038 (Section 7, Eq. 1), stepped with the
fused form of Listing 3's routine sequence by hand-written HIP kernels behind
the C ABI of include/fd.h.  This module is a thin layer over that ABI: torch
supplies device memory and streams; every step of the computation runs in
libfd.so.  There is no CPU fallback: importing fails if the library is not
built.

    m = Model(grid_kwargs, velocity_tensor)      # fd_create_model
    s = m.new_state()                            # fd_create_state
    traces = m.run_shot(s, shot)                 # fd_run_shot
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _abi
from ._abi import (FDError, FD_BF16, FD_C_F32, FD_C_FIXED16, FD_F16, FD_F32, FD_BATCH_MAX,
                   fd_batch_item, fd_grid, fd_receivers, fd_shot, fd_sizes)

__all__ = ["Grid", "Receivers", "Shot", "Model", "State", "ShotGraph", "FDError", "FD_F32", "FD_F16",
           "FD_BF16", "FD_C_F32", "FD_C_FIXED16", "step_batch", "slab_exchange", "ensure_built"]

FACES_NO_TOP = 0x3E


def ensure_built() -> None:
    _abi.lib()


def _stream_handle(stream: Optional[torch.cuda.Stream] = None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _buf(t: torch.Tensor, what: str, dtype, numel: int) -> int:
    """Address of a caller's device tensor after checking that it can hold
    what the library reads or writes there (the C calls take raw pointers
    and cannot): a contiguous CUDA tensor of `dtype` with at least `numel`
    elements."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous {dtype}")
    if t.numel() < numel:
        raise ValueError(f"{what} holds {t.numel()} elements, {numel} are needed")
    return t.data_ptr()


def _same_len(shots, **lists) -> None:
    """The multi-shot calls read one entry of each array per shot."""
    for name, v in lists.items():
        if v is not None and len(v) != len(shots):
            raise ValueError(f"{name} has {len(v)} entries for {len(shots)} shots")


def _nbytes(t: torch.Tensor) -> int:
    """Size in bytes of a caller's device buffer (any element type)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("buffers must be contiguous device tensors")
    return t.numel() * t.element_size()


def _alloc(nbytes: int, device) -> torch.Tensor:
    """A 256-byte aligned device byte buffer (torch's caching allocator
    returns at least 512-byte aligned blocks)."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


@dataclass
class Grid:
    """Grid and discretisation (fd_grid)."""
    ndim: int
    nz: int
    ny: int
    nx: int
    dh: float
    dt: float
    sponge_width: int = 0
    sponge_alpha: float = 0.0
    sponge_faces: int = FACES_NO_TOP
    storage: int = FD_F32
    c_storage: int = FD_C_F32
    radius: int = 4
    bc: int = 0
    # z-slab [slab_z0, slab_z0 + nz) of a grid of slab_nz_global planes
    # (0: an ordinary grid); see `slabs` and `slab_exchange`
    slab_z0: int = 0
    slab_nz_global: int = 0

    def c(self) -> fd_grid:
        return fd_grid(ndim=self.ndim, radius=self.radius, bc=self.bc,
                       sponge_width=self.sponge_width, nz=self.nz, ny=self.ny, nx=self.nx,
                       dh=self.dh, dt=self.dt, sponge_alpha=self.sponge_alpha,
                       sponge_faces=self.sponge_faces, storage=self.storage,
                       c_storage=self.c_storage, slab_z0=self.slab_z0,
                       slab_nz_global=self.slab_nz_global)

    def slabs(self, counts: Sequence[int]) -> list:
        """This grid cut along z into consecutive slabs of `counts` planes
        (summing to nz), each a Grid of its own."""
        if sum(counts) != self.nz:
            raise ValueError(f"slab planes sum to {sum(counts)}, the grid has {self.nz}")
        out, z0 = [], 0
        for k in counts:
            out.append(Grid(**{**self.__dict__, "nz": int(k), "slab_z0": z0,
                               "slab_nz_global": self.nz}))
            z0 += int(k)
        return out

    @property
    def shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nz * self.ny * self.nx


@dataclass
class Receivers:
    z0: int = 0
    y0: int = 0
    x0: int = 0
    nz: int = 0
    ny: int = 0
    nx: int = 0
    dz: int = 1
    dy: int = 1
    dx: int = 1

    @property
    def count(self) -> int:
        return self.nz * self.ny * self.nx

    def c(self) -> fd_receivers:
        return fd_receivers(z0=self.z0, y0=self.y0, x0=self.x0, nz=self.nz, ny=self.ny,
                            nx=self.nx, dz=self.dz, dy=self.dy, dx=self.dx)


class Shot:
    """A point source with its wavelet (device FP32 tensor) and receivers."""

    def __init__(self, src, wavelet: torch.Tensor, receivers: Receivers):
        if wavelet.dtype != torch.float32 or not wavelet.is_cuda or not wavelet.is_contiguous():
            raise ValueError("wavelet must be a contiguous FP32 device tensor")
        self.src = tuple(int(v) for v in src)
        self.wavelet = wavelet
        self.receivers = receivers
        self.nt = int(wavelet.numel())
        self._c = fd_shot(src_z=self.src[0], src_y=self.src[1], src_x=self.src[2],
                          wavelet=wavelet.data_ptr(), nt=self.nt, rec=receivers.c())

    @property
    def nrec(self) -> int:
        return self.receivers.count


class Model:
    """fd_create_model over torch-owned device memory."""

    def __init__(self, grid: Grid, velocity: torch.Tensor, stream=None):
        if velocity.dtype != torch.float32 or not velocity.is_cuda:
            raise ValueError("velocity must be an FP32 device tensor")
        if velocity.numel() != grid.ncells:
            raise ValueError(f"velocity has {velocity.numel()} cells, grid has {grid.ncells}")
        velocity = velocity.contiguous()
        self.grid = grid
        self.device = velocity.device
        self._g = grid.c()
        self.sizes: fd_sizes = _abi.fd_query_bytes(self._g)
        self.buf = _alloc(self.sizes.model, self.device)
        self.handle = _abi.fd_create_model(self._g, velocity.data_ptr(), self.buf.data_ptr(),
                                           self.sizes.model, _stream_handle(stream))

    def sizes_for(self, nt: int, ckpt_every: int) -> fd_sizes:
        return _abi.fd_query_bytes(self._g, nt, ckpt_every)

    def new_state(self) -> "State":
        return State(self)

    def run_shot(self, state: "State", shot: Shot, traces: Optional[torch.Tensor] = None,
                 ckpt: Optional[torch.Tensor] = None, ckpt_every: int = 0,
                 stream=None) -> torch.Tensor:
        if traces is None:
            traces = torch.empty((shot.nt, shot.nrec), dtype=torch.float32,
                                 device=self.device)
        tp = _buf(traces, "traces", torch.float32, shot.nt * shot.nrec) if shot.nrec > 0 else None
        _abi.fd_run_shot(self.handle, state.handle, shot._c, tp,
                         ckpt.data_ptr() if ckpt is not None else None,
                         _nbytes(ckpt) if ckpt is not None else 0, ckpt_every,
                         _stream_handle(stream))
        state.next = shot.nt
        return traces

    def checkpoint_buffer(self, nt: int, ckpt_every: int) -> torch.Tensor:
        return _alloc(self.sizes_for(nt, ckpt_every).checkpoints, self.device)

    def adjoint_gradient(self, shot: Shot, adj: torch.Tensor, ckpt: torch.Tensor,
                         ckpt_every: int, grad_v: torch.Tensor,
                         work: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        ap = _buf(adj, "adj", torch.float32, shot.nt * shot.nrec)
        if grad_v.dtype != torch.float64 or grad_v.numel() != self.grid.ncells:
            raise ValueError("grad_v must be an FP64 tensor of the grid's size")
        gp = _buf(grad_v, "grad_v", torch.float64, self.grid.ncells)
        need = self.sizes_for(shot.nt, ckpt_every).adjoint_work
        if work is None:
            work = _alloc(need, self.device)
        _abi.fd_adjoint_gradient(self.handle, shot._c, ap, ckpt.data_ptr(),
                                 _nbytes(ckpt), ckpt_every, work.data_ptr(), _nbytes(work),
                                 gp, _stream_handle(stream))
        return grad_v

    def rtm_image(self, shot: Shot, data: torch.Tensor, ckpt: torch.Tensor, ckpt_every: int,
                  image: torch.Tensor, work: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        """fd_rtm_image: image += sum_k z^k w^{k-1} for the receiver field
        back-propagated from `data` ([nt][nrec] FP32) and the source field
        recomputed from `ckpt` (saved by run_shot with the same ckpt_every)."""
        dp = _buf(data, "data", torch.float32, shot.nt * shot.nrec)
        if image.dtype != torch.float64 or image.numel() != self.grid.ncells:
            raise ValueError("image must be an FP64 tensor of the grid's size")
        ip = _buf(image, "image", torch.float64, self.grid.ncells)
        need = self.sizes_for(shot.nt, ckpt_every).adjoint_work
        if work is None:
            work = _alloc(need, self.device)
        _abi.fd_rtm_image(self.handle, shot._c, dp, ckpt.data_ptr(), _nbytes(ckpt),
                          ckpt_every, work.data_ptr(), _nbytes(work), ip,
                          _stream_handle(stream))
        return image

    # ---- several shots at once (fd_run_shots / fd_*_shots) ----------------
    def run_shots(self, states: Sequence["State"], shots: Sequence[Shot],
                  traces: Optional[torch.Tensor] = None,
                  ckpts: Optional[Sequence[torch.Tensor]] = None, ckpt_every: int = 0,
                  stream=None) -> torch.Tensor:
        """fd_run_shots: every shot of `shots` with its own state (and
        checkpoint buffer); traces [nshots, nt, nrec]."""
        nt = shots[0].nt
        nrec = shots[0].nrec
        if any(s.nt != nt or s.nrec != nrec for s in shots):
            raise ValueError("the shots must share nt and the receiver count")
        _same_len(shots, states=states, ckpts=ckpts)
        if traces is None:
            traces = torch.empty((len(shots), nt, nrec), dtype=torch.float32, device=self.device)
        base = _buf(traces, "traces", torch.float32, len(shots) * nt * nrec) if nrec > 0 else 0
        _abi.fd_run_shots(self.handle, [st.handle for st in states], [s._c for s in shots],
                          [base + 4 * i * nt * nrec if s.nrec > 0 else None for i, s in enumerate(shots)],
                          [c.data_ptr() for c in ckpts] if ckpts is not None else None,
                          min(_nbytes(c) for c in ckpts) if ckpts is not None else 0, ckpt_every,
                          _stream_handle(stream))
        for st in states:
            st.next = nt
        return traces

    def _backward_shots(self, fn, shots, srcs, ckpts, ckpt_every, out, works, stream):
        _same_len(shots, sources=srcs, ckpts=ckpts, works=works)
        ptrs = [_buf(t, "adjoint source", torch.float32, sh.nt * sh.nrec) for t, sh in zip(srcs, shots)]
        if out.dtype != torch.float64 or out.numel() != self.grid.ncells:
            raise ValueError("the output must be an FP64 tensor of the grid's size")
        op = _buf(out, "the output", torch.float64, self.grid.ncells)
        need = self.sizes_for(shots[0].nt, ckpt_every).adjoint_work
        if works is None:
            works = [_alloc(need, self.device) for _ in shots]
        fn(self.handle, [s._c for s in shots], ptrs,
           [c.data_ptr() for c in ckpts], min(_nbytes(c) for c in ckpts), ckpt_every,
           [w.data_ptr() for w in works], min(_nbytes(w) for w in works), op, _stream_handle(stream))
        return out

    def adjoint_gradient_shots(self, shots: Sequence[Shot], adj: Sequence[torch.Tensor],
                               ckpts: Sequence[torch.Tensor], ckpt_every: int,
                               grad_v: torch.Tensor,
                               works: Optional[Sequence[torch.Tensor]] = None,
                               stream=None) -> torch.Tensor:
        """fd_adjoint_gradient_shots: grad_v += the gradient of every shot."""
        return self._backward_shots(_abi.fd_adjoint_gradient_shots, shots, adj, ckpts, ckpt_every,
                                    grad_v, works, stream)

    def rtm_image_shots(self, shots: Sequence[Shot], data: Sequence[torch.Tensor],
                        ckpts: Sequence[torch.Tensor], ckpt_every: int, image: torch.Tensor,
                        works: Optional[Sequence[torch.Tensor]] = None,
                        stream=None) -> torch.Tensor:
        """fd_rtm_image_shots: image += the image of every shot."""
        return self._backward_shots(_abi.fd_rtm_image_shots, shots, data, ckpts, ckpt_every,
                                    image, works, stream)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _abi.fd_destroy_model(h)
            except Exception:
                pass
            self.handle = None


class State:
    """fd_create_state: the two time levels of one shot in flight."""

    def __init__(self, model: Model):
        self.model = model
        self.buf = _alloc(model.sizes.state, model.device)
        self.handle = _abi.fd_create_state(model.handle, self.buf.data_ptr(), model.sizes.state)
        self.next = -1

    @staticmethod
    def _row(trace_row: Optional[torch.Tensor], shot: Shot):
        """Address of one step's trace row (nrec FP32 values), or None."""
        if trace_row is None or shot.nrec == 0:
            return None
        return _buf(trace_row, "trace_row", torch.float32, shot.nrec)

    def begin(self, shot: Shot, stream=None) -> None:
        _abi.fd_begin_shot(self.model.handle, self.handle, shot._c, _stream_handle(stream))
        self.next = 0

    def step(self, shot: Shot, n: int, trace_row: Optional[torch.Tensor] = None,
             stream=None) -> None:
        _abi.fd_step(self.model.handle, self.handle, shot._c, n, self._row(trace_row, shot),
                     _stream_handle(stream))
        self.next = n + 1

    def step_routines(self, shot: Shot, n: int, work: torch.Tensor,
                      trace_row: Optional[torch.Tensor] = None, stream=None) -> None:
        """Step n as one kernel per routine (fd_step_routines); `work` is a
        device byte buffer of at least Model.sizes.routines_work bytes."""
        _abi.fd_step_routines(self.model.handle, self.handle, shot._c, n, self._row(trace_row, shot),
                              work.data_ptr(), _nbytes(work), _stream_handle(stream))
        self.next = n + 1

    def step_routines_noalloc(self, shot: Shot, n: int, trace_row: Optional[torch.Tensor] = None,
                              stream=None) -> None:
        """Step n as one kernel per routine with the library's static work
        area (fd_step_routines_noalloc): no buffer is allocated or passed;
        grids whose routine work exceeds the area raise FDError."""
        _abi.fd_step_routines_noalloc(self.model.handle, self.handle, shot._c, n,
                                      self._row(trace_row, shot), _stream_handle(stream))
        self.next = n + 1

    def check_finite(self, flags: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Enqueues fd_check_finite: returns a device int32 tensor of one
        element whose bit 0 (P) and bit 1 (Pold) are set when that level
        holds a NaN or an infinity (0: the shot is healthy).  Pass `flags`
        to reuse a buffer."""
        if flags is None:
            flags = torch.empty(1, dtype=torch.int32, device=self.model.device)
        _abi.fd_check_finite(self.handle, _buf(flags, "flags", torch.int32, 1), _stream_handle(stream))
        return flags

    def is_finite(self, stream=None) -> bool:
        """True when both stored levels are finite (waits for the check)."""
        return int(self.check_finite(stream=stream).item()) == 0

    def wavefield(self, which: int = 0, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.model.grid.shape, dtype=torch.float32,
                              device=self.model.device)
        _abi.fd_get_wavefield(self.handle, which, _buf(out, "out", torch.float32, self.model.grid.ncells),
                              _stream_handle(stream))
        return out

    def set_wavefield(self, which: int, values: torch.Tensor, stream=None) -> None:
        if values.dtype != torch.float32 or values.numel() != self.model.grid.ncells:
            raise ValueError("values must be FP32 with one entry per cell")
        values = values.contiguous()
        _abi.fd_set_wavefield(self.handle, which,
                              _buf(values, "values", torch.float32, self.model.grid.ncells),
                              _stream_handle(stream))
        if self.next < 0:
            self.next = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _abi.fd_destroy_state(h)
            except Exception:
                pass
            self.handle = None


class ShotGraph:
    """fd_shot_graph_create: the launches of Model.run_shot(state, shot,
    traces) recorded once into a HIP graph; launch() replays them (one graph
    launch instead of one kernel launch per step).  The graph keeps the
    addresses of the model, state, wavelet and traces, which this object
    keeps alive; replays read their contents as they are then."""

    def __init__(self, model: "Model", state: "State", shot: Shot,
                 traces: Optional[torch.Tensor] = None):
        if traces is None:
            traces = torch.empty((shot.nt, shot.nrec), dtype=torch.float32, device=model.device)
        tp = _buf(traces, "traces", torch.float32, shot.nt * shot.nrec) if shot.nrec > 0 else None
        self.model, self.state, self.shot, self.traces = model, state, shot, traces
        self.handle = _abi.fd_shot_graph_create(model.handle, state.handle, shot._c, tp)

    def launch(self, stream=None) -> torch.Tensor:
        _abi.fd_shot_graph_launch(self.handle, _stream_handle(stream))
        self.state.next = self.shot.nt
        return self.traces

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                _abi.fd_shot_graph_destroy(h)
            except Exception:
                pass
            self.handle = None


def slab_exchange(upper: "State", lower: "State", stream=None) -> None:
    """fd_slab_exchange: refresh the ghost planes between two neighbouring
    z-slabs (upper's planes end where lower's begin)."""
    _abi.fd_slab_exchange(upper.handle, lower.handle, _stream_handle(stream))


def step_batch(entries: Sequence[tuple], nsteps: int, stream=None) -> list:
    """fd_step_batch over (model, state, shot, traces) entries, each at its
    state's next step.  Returns the next step of every entry."""
    if len(entries) > FD_BATCH_MAX:
        raise ValueError(f"at most {FD_BATCH_MAX} entries")
    arr = (fd_batch_item * max(len(entries), 1))()
    keep = []
    for i, (model, state, shot, traces) in enumerate(entries):
        arr[i].model = model.handle
        arr[i].state = state.handle
        arr[i].shot = ctypes.pointer(shot._c)
        keep.append(arr[i].shot)
        arr[i].n = state.next
        arr[i].traces = (_buf(traces, "traces", torch.float32, shot.nt * shot.nrec)
                         if traces is not None and shot.nrec > 0 else None)
    if entries:
        _abi.check(_abi.lib().fd_step_batch(arr, len(entries), nsteps, _stream_handle(stream)))
    out = []
    for i, (_, state, _, _) in enumerate(entries):
        state.next = int(arr[i].n)
        out.append(state.next)
    return out
