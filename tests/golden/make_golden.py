"""Writes oracle-computed expected values for the full-size parity tests.

Calls only the FP64 oracle (oracle/) on the seeded inputs of fd_inputs; no
value here comes from the GPU path.  Full-size runs take the oracle tens of
minutes (512^3) to hours (768x768x512), so the stored files hold samples:

  traces_idx / traces      : every 32nd receiver in y and x (64 receivers),
                             all time steps, float64
  cells_idx / cells        : 8192 seeded random cells of the final field
  blocks                   : sums of the final field over 16^3 blocks
  trace_norm / field_norm  : L2 norms of the whole traces and final field

For adjoint2d_1024 (the 1024^2 / 2000-step gradient model, shot 0, start
model v0, a seeded N(0,1) adjoint source r stored as FP32 in the file) the
FP64 velocity gradient is stored the same way (cells, 16^2 block sums, norm).

For serving2d_2048x4096 (one shot of the serving stream's largest grid,
1000 steps) the traces of every 16th receiver, 8192 final cells, 16^2 block
sums and the norms are stored.

Usage:  python tests/golden/make_golden.py layered3d_512 [precision3d_768] [adjoint2d_1024]
        [serving2d_2048x4096]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fd_inputs as fi  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_plan(p: fi.Problem):
    rec = p.receivers
    ry = np.arange(0, rec.ny, 32)
    rx = np.arange(0, rec.nx, 32)
    traces_idx = (ry[:, None] * rec.nx + rx[None, :]).ravel().astype(np.int64)
    rng = np.random.default_rng(1234)
    cells_idx = rng.integers(0, p.ncells, 8192).astype(np.int64)
    return traces_idx, cells_idx


def block_sums(field: np.ndarray, b: int = 16) -> np.ndarray:
    nz, ny, nx = field.shape
    f = field[: nz // b * b, : ny // b * b, : nx // b * b]
    return f.reshape(nz // b, b, ny // b, b, nx // b, b).sum(axis=(1, 3, 5))


def adjoint_residual(p: fi.Problem) -> np.ndarray:
    return np.random.default_rng(777).standard_normal((p.nt, p.receivers.count)).astype(np.float32)


def make_adjoint(name: str) -> str:
    t0 = time.time()
    shots, _, v0 = fi.adjoint2d()
    p = shots[0]
    r = adjoint_residual(p)
    gv, _ = oracle.adjoint(oracle.grid_of(p), v0.reshape(p.nz, 1, p.nx), p.wavelet(), p.nt,
                           p.src, p.rec_index(), r.astype(np.float64))
    g = gv.reshape(p.nz, p.nx)
    rng = np.random.default_rng(4321)
    cells_idx = rng.integers(0, p.ncells, 8192).astype(np.int64)
    b = 16
    blocks = g.reshape(p.nz // b, b, p.nx // b, b).sum(axis=(1, 3))
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, cells_idx=cells_idx, cells=g.ravel()[cells_idx], blocks=blocks,
                        grad_norm=np.linalg.norm(g), seconds=time.time() - t0)
    print(name, "written in %.0f s" % (time.time() - t0), flush=True)
    return path


def serving_shot() -> fi.Problem:
    """The largest grid of the serving stream's range (2048 x 4096, 1000
    steps, random-field velocity): one shot, as the batched kernel runs it."""
    return fi.surface2d(2048, 4096, 1000, seed=5050, name="serving2d_2048x4096")


def make_serving(name: str) -> str:
    t0 = time.time()
    p = serving_shot()
    v = p.velocity()
    out = oracle.forward(oracle.grid_of(p), v.reshape(p.nz, 1, p.nx), p.wavelet(), p.nt, p.src,
                         p.rec_index())
    cur = out["cur"].reshape(p.nz, p.nx)
    traces_idx = np.arange(0, p.receivers.count, 16).astype(np.int64)
    rng = np.random.default_rng(1234)
    cells_idx = rng.integers(0, p.ncells, 8192).astype(np.int64)
    b = 16
    blocks = cur.reshape(p.nz // b, b, p.nx // b, b).sum(axis=(1, 3))
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, traces_idx=traces_idx, traces=out["traces"][:, traces_idx],
                        cells_idx=cells_idx, cells=cur.ravel()[cells_idx], blocks=blocks,
                        trace_norm=np.linalg.norm(out["traces"]), field_norm=np.linalg.norm(cur),
                        seconds=time.time() - t0)
    print(name, "written in %.0f s" % (time.time() - t0), flush=True)
    return path


def make(name: str) -> str:
    if name == "adjoint2d_1024":
        return make_adjoint(name)
    if name == "serving2d_2048x4096":
        return make_serving(name)
    p = {"layered3d_512": fi.layered3d(), "precision3d_768": fi.precision3d()}[name]
    t0 = time.time()
    v = p.velocity()
    g = oracle.grid_of(p)
    w = p.wavelet()
    rec = p.rec_index()
    traces = np.empty((p.nt, rec.size))
    prev = cur = None
    chunk = 50
    # Continuing from the previous chunk's (prev, cur) with the wavelet slice
    # of the next steps is the same arithmetic as one long run.
    for n0 in range(0, p.nt, chunk):
        k = min(chunk, p.nt - n0)
        out = oracle.forward(g, v, w[n0:n0 + k], k, p.src, rec, init_prev=prev, init_cur=cur)
        traces[n0:n0 + k] = out["traces"]
        prev, cur = out["prev"], out["cur"]
        print(f"{name}: step {n0 + k}/{p.nt} after {time.time() - t0:.0f} s", flush=True)
    out = dict(traces=traces)
    traces_idx, cells_idx = sample_plan(p)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(
        path, traces_idx=traces_idx, traces=out["traces"][:, traces_idx],
        cells_idx=cells_idx, cells=cur.ravel()[cells_idx], blocks=block_sums(cur),
        trace_norm=np.linalg.norm(out["traces"]), field_norm=np.linalg.norm(cur),
        seconds=time.time() - t0)
    print(name, "written in %.0f s" % (time.time() - t0), flush=True)
    return path


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)
