"""Benchmark of the fused finite-difference step on one MI355X.

Workload (the headline case): 3D acoustic, 512^3 cells, dh = 10 m, dt = 1 ms,
1000 steps, seeded layered velocity (1500-4500 m/s), 32-cell sponge on every
face but the top, 12 Hz Ricker source at (4, 256, 256), 256 x 256 receiver
block at depth index 2, FP32 fields.  One benchmark step = one whole shot
(fd_run_shot: 1000 fused time steps, traces written), inputs resident in HBM.

Prints ONE JSON line with Mcell-updates/s, the roofline of the dominant
kernel (the 3D step kernel: 16 algorithmic bytes per cell-update in FP32 -
read P, Pold and c, write Pnew) and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def headline(steps: int, warmup: int):
    import torch
    import fd_inputs as fi
    from helpers import setup

    p = fi.layered3d()
    log(f"[bench] building inputs {p.name}")
    model, state, shot = setup(p)
    traces = torch.empty((p.nt, p.receivers.count), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        model.run_shot(state, shot, traces)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i} done")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        model.run_shot(state, shot, traces)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    cells = p.ncells * p.nt
    mcell = cells * steps / (ms * 1e-3) / 1e6
    per_launch_s = ms * 1e-3 / (steps * p.nt)
    alg_bytes = 16.0 * p.ncells
    achieved = alg_bytes / per_launch_s / 1e9
    log(f"[bench] {steps} shots in {ms:.1f} ms (wall {wall:.2f} s): {mcell:.0f} Mcell/s, "
        f"{achieved:.0f} GB/s algorithmic")
    return dict(p=p, ms=ms, mcell=mcell, achieved=achieved, per_launch_us=per_launch_s * 1e6)


def copy_probe(nbytes: int = 1 << 30, reps: int = 20):
    """A plain streaming kernel of known size (elementwise negation: 4 B read
    and 4 B written per element, 1 GiB each way): the practical HBM roof (the
    role BabelStream plays in the paper's roofline) and the calibration
    kernel for the rocprofv3 byte counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return dict(bytes_per_copy=2 * nbytes, gbs=2 * nbytes * reps / (ms * 1e-3) / 1e9)


def cpu_baseline(nsteps: int = 4):
    """The FP64 oracle on the same 512^3 model for a few steps."""
    import oracle
    import fd_inputs as fi
    p = fi.layered3d(nt=nsteps)
    v = p.velocity()
    g = oracle.grid_of(p)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(threads)
    t = time.perf_counter()
    oracle.forward(g, v, p.wavelet(), p.nt, p.src, p.rec_index())
    dt = time.perf_counter() - t
    return dict(value=p.ncells * nsteps / dt / 1e6, unit="Mcell-updates/s", cores=threads,
                kind="oracle",
                sample=f"512^3 layered model, {nsteps} time steps (incl. set-up), FP64, "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-only", action="store_true",
                    help="only the 1 GiB copy probe (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_2311_05038_amd as fd
    fd.ensure_built()

    probe = copy_probe()
    log(f"[bench] copy probe: {probe['gbs']:.0f} GB/s")
    if args.probe_only:
        print(json.dumps({"copy_probe": probe}), flush=True)
        return
    h = headline(args.steps, args.warmup)
    cpu = None if args.no_cpu else cpu_baseline()
    out = {
        "metric": "Mcell-updates/s",
        "value": round(h["mcell"], 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered3d 512x512x512, nt=1000, 32-cell sponge, 256x256 receivers",
                   "cells": h["p"].ncells, "nt": h["p"].nt, "step": "one shot (fd_run_shot)"},
        "hbm_frac": round(h["achieved"] / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(h["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_step3d<f32>",
                     "bytes_per_cell": 16, "avg_launch_us": round(h["per_launch_us"], 2)},
        "cpu_baseline": cpu,
        "copy_roof_gbs": round(probe["gbs"], 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
