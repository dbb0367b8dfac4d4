"""Glue between the seeded workload descriptions (fd_inputs) and the GPU
library, for the tests and the benchmark."""
from __future__ import annotations

import numpy as np
import torch

import fd_inputs as fi


def grid_of(p: fi.Problem, storage: int = 0, c_storage: int = 0):
    import paper_2311_05038_amd as fd
    return fd.Grid(ndim=p.ndim, nz=p.nz, ny=p.ny, nx=p.nx, dh=p.dh, dt=p.dt,
                   sponge_width=p.sponge_width, sponge_alpha=p.sponge_alpha,
                   sponge_faces=p.sponge_faces, storage=storage, c_storage=c_storage)


def receivers_of(p: fi.Problem):
    import paper_2311_05038_amd as fd
    r = p.receivers
    return fd.Receivers(r.z0, r.y0, r.x0, r.nz, r.ny, r.nx, r.dz, r.dy, r.dx)


def setup(p: fi.Problem, v: np.ndarray = None, storage: int = 0, device="cuda", c_storage: int = 0):
    """(model, state, shot) on the GPU for a workload."""
    import paper_2311_05038_amd as fd
    if v is None:
        v = p.velocity()
    vt = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32).reshape(-1)).to(device)
    model = fd.Model(grid_of(p, storage, c_storage), vt)
    wav = torch.from_numpy(p.wavelet()).to(device)
    shot = fd.Shot(p.src, wav, receivers_of(p))
    return model, model.new_state(), shot


def run(p: fi.Problem, v: np.ndarray = None, storage: int = 0, c_storage: int = 0):
    """Whole shot on the GPU; returns (traces, final field) as numpy."""
    model, state, shot = setup(p, v, storage, c_storage=c_storage)
    tr = model.run_shot(state, shot)
    cur = state.wavefield(0)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), cur.cpu().numpy()


def rel_l2(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))
