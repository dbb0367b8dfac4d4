"""Writes oracle-computed expected values for the full-size parity tests.

Calls only the FP64 oracle (oracle/) on the seeded inputs of fd_inputs; no
value here comes from the GPU path.  Full-size runs take the oracle tens of
minutes (512^3) to hours (768x768x512), so the stored files hold samples:

  traces_idx / traces      : every 32nd receiver in y and x (64 receivers),
                             all time steps, float64
  cells_idx / cells        : 8192 seeded random cells of the final field
  blocks                   : sums of the final field over 16^3 blocks
  trace_norm / field_norm  : L2 norms of the whole traces and final field

Usage:  python tests/golden/make_golden.py layered3d_512 [precision3d_768]
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


def make(name: str) -> str:
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
