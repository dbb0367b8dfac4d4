"""Benchmark of the fused finite-difference step on one MI355X.

Workload (the headline case): 3D acoustic, 512^3 cells, dh = 10 m, dt = 1 ms,
1000 steps, seeded layered velocity (1500-4500 m/s), 32-cell sponge on every
face but the top, 12 Hz Ricker source at (4, 256, 256), 256 x 256 receiver
block at depth index 2, FP32 fields.  One benchmark step = one whole shot
(fd_run_shot: 1000 fused time steps, traces written), inputs resident in HBM.

Prints ONE JSON line with Mcell-updates/s, the roofline of the dominant
kernel (the 3D step kernel: 16 algorithmic bytes per cell-update in FP32 -
read P, Pold and c, write Pnew) and the FP64 CPU oracle timed on a bounded
sample of the same workload.  Further legs (each against the plain FP32 path
on the same GPU) add keys to the same line:
  half     16-bit field storage on the 768x768x512 precision grid, 2000 steps
  adjoint  the 8-shot velocity gradient on the 1024^2 model, 2000 steps
  serve    a Poisson stream of 2D shots, continuous batching vs sequential
  routines the step as one kernel per routine vs the fused step
  slab     one eighth of the headline grid as a z-slab with ghost planes (the
           share of one device when the model is cut along z), with the
           ghost exchange timed beside it
  small2d  single small 2D shots (the 256^2 case, a 1024^2 shot) against 16
           of them batched in one launch per step
  cpu      the host back-end (libfd_cpu.so: the same ABI, OpenMP + AVX) on
           the headline model for a few steps and on the 2D 256^2 case,
           against a host stream probe of the step's access pattern
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
    # one event per shot boundary as well: the spread of the single shots
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    marks[0].record(stream)
    for i in range(steps):
        model.run_shot(state, shot, traces)
        marks[i + 1].record(stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    shot_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(steps))
    cells = p.ncells * p.nt
    mcell = cells * steps / (ms * 1e-3) / 1e6
    per_launch_s = ms * 1e-3 / (steps * p.nt)
    alg_bytes = 16.0 * p.ncells
    achieved = alg_bytes / per_launch_s / 1e9
    log(f"[bench] {steps} shots in {ms:.1f} ms (wall {wall:.2f} s): {mcell:.0f} Mcell/s, "
        f"{achieved:.0f} GB/s algorithmic; single shots {shot_ms[0]:.1f} .. {shot_ms[-1]:.1f} ms")
    med = shot_ms[steps // 2] if steps % 2 else 0.5 * (shot_ms[steps // 2 - 1] + shot_ms[steps // 2])
    stats = dict(median=round(med, 3), min=round(shot_ms[0], 3), max=round(shot_ms[-1], 3), n=steps)
    return dict(p=p, ms=ms, mcell=mcell, achieved=achieved, per_launch_us=per_launch_s * 1e6, shot_ms=stats)


def _timed_probe(kind: int, arrays, n: int, reps: int) -> float:
    """Median microseconds of one fd_stream_probe launch (HIP events on the
    stream it runs on)."""
    import statistics
    import torch
    from paper_2311_05038_amd import _abi
    s = torch.cuda.current_stream()
    a, b, out = arrays
    bp = b.data_ptr() if b is not None else None
    for _ in range(3):
        _abi.fd_stream_probe(kind, a.data_ptr(), bp, out.data_ptr(), n, s.cuda_stream)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        _abi.fd_stream_probe(kind, a.data_ptr(), bp, out.data_ptr(), n, s.cuda_stream)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return statistics.median(ts)


def copy_probe(nbytes: int = 1 << 30, reps: int = 20):
    """The library's copy probe (fd_stream_probe kind 0: 1 GiB read and 1 GiB
    written, non-temporal, each XCD streaming one contiguous eighth): the
    practical HBM roof of a plain stream, and the calibration kernel for the
    rocprofv3 byte counters."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    out = torch.empty_like(a)
    us = _timed_probe(0, (a, None, out), n, reps)
    del a, out
    torch.cuda.empty_cache()
    return dict(bytes_per_copy=2 * nbytes, us=us, gbs=2 * nbytes / (us * 1e-6) / 1e9)


def stream_probe(cells: int = 512 ** 3, reps: int = 20):
    """The step's traffic without the stencil (fd_stream_probe kind 1: out =
    a + b * out over three FP32 arrays of the 512^3 size, 12 B read and 4 B
    written per element in place, the step kernel's accesses): the practical
    roof of the FP32 step on this GPU."""
    import torch
    a = torch.ones(cells, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    out = torch.zeros_like(a)
    us = _timed_probe(1, (a, b, out), cells, reps)
    del a, b, out
    torch.cuda.empty_cache()
    return dict(us=us, gbs=16 * cells / (us * 1e-6) / 1e9)


def small2d_leg(reps: int = 5):
    """Small 2D shots, where a step is too small to fill the GPU: the 256^2
    Green's-function case (500 steps) and a 1024^2 shot (2000 steps) as
    single fd_run_shot calls (one launch per step) and as recorded graphs
    (fd_shot_graph_launch: one graph launch per shot), and 16 shots of the
    256^2 case in one fd_run_shots call (one batched launch per step)."""
    import statistics
    import torch
    import fd_inputs as fi
    from helpers import setup
    out = {}
    s = torch.cuda.current_stream()

    def timed(fn, steps, cells):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        us = statistics.median(ts)
        return dict(us_per_step=round(us / steps, 2), mcell_per_s=round(cells * steps / us, 1),
                    spread_pct=round(100 * (max(ts) - min(ts)) / us, 1))

    import paper_2311_05038_amd as fd
    for name, p in (("green2d_256", fi.green2d()), ("surface2d_1024", fi.surface2d(1024, 1024, 2000, seed=5))):
        model, state, shot = setup(p)
        tr = torch.empty((p.nt, p.receivers.count), device="cuda")
        out[name] = timed(lambda: model.run_shot(state, shot, tr), p.nt, p.ncells)
        # the same shot recorded once as a graph (fd_shot_graph_*) and replayed
        g = fd.ShotGraph(model, state, shot, tr)
        out[name + "_graph"] = timed(g.launch, p.nt, p.ncells)
        del g
    p = fi.green2d()
    model, _, shot = setup(p)
    states = [model.new_state() for _ in range(16)]
    shots = [shot] * 16
    out["green2d_256_x16_batched"] = timed(lambda: model.run_shots(states, shots), p.nt, 16 * p.ncells)
    log(f"[bench] small 2D: {out}")
    return out


def half_leg(nt: int = 2000):
    """16-bit storage vs FP32 on the 768x768x512 grid (same model, source,
    receivers): Mcell-updates/s of one whole shot each, with c in FP32
    (10 B/cell) and in 16-bit fixed point (8 B/cell) for the 16-bit fields."""
    import torch
    import fd_inputs as fi
    from helpers import setup
    p = fi.precision3d(nt=nt)
    v = p.velocity()
    out = {}
    for name, st, c16 in (("f32", 0, 0), ("f16", 1, 0), ("bf16", 2, 0), ("f16_c16", 1, 1),
                          ("bf16_c16", 2, 1)):
        model, state, shot = setup(p, v, storage=st, c_storage=c16)
        traces = torch.empty((p.nt, p.receivers.count), device="cuda")
        model.run_shot(state, shot, traces)     # warm-up shot
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        model.run_shot(state, shot, traces)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        bpc = 16 if st == 0 else (8 if c16 else 10)
        out[name] = dict(mcell_per_s=round(p.ncells * p.nt / (ms * 1e-3) / 1e6, 1),
                         ms_per_shot=round(ms, 2), bytes_per_cell=bpc,
                         alg_gbs=round(bpc * p.ncells * p.nt / (ms * 1e-3) / 1e9, 1))
        log(f"[bench] half leg {name}: {out[name]}")
        del model, state, shot, traces
        torch.cuda.empty_cache()
    for name in ("f16", "bf16", "f16_c16", "bf16_c16"):
        out["speedup_" + name] = round(out[name]["mcell_per_s"] / out["f32"]["mcell_per_s"], 3)
    out["workload"] = f"precision3d 768x768x512, nt={nt}"
    return out


def adjoint_leg(nt: int = 2000, every: int = 50):
    """The 8-shot L2-misfit gradient on the 1024^2 model: forward with
    checkpoints, then recompute + adjoint per shot (FP64 time sum)."""
    import torch
    import fd_inputs as fi
    from helpers import receivers_of
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.autograd import l2_misfit_gradient
    shots_p, vtrue, v0 = fi.adjoint2d(nt=nt)
    p = shots_p[0]
    grid = fd.Grid(ndim=2, nz=p.nz, ny=1, nx=p.nx, dh=p.dh, dt=p.dt,
                   sponge_width=p.sponge_width, sponge_faces=p.sponge_faces)
    wav = torch.from_numpy(p.wavelet()).cuda()
    shots = [fd.Shot(q.src, wav, receivers_of(q)) for q in shots_p]
    vt = torch.from_numpy(vtrue.ravel()).cuda()
    mt = fd.Model(grid, vt)
    st = mt.new_state()
    obs = torch.stack([mt.run_shot(st, s).clone() for s in shots])
    v0t = torch.from_numpy(v0.ravel()).cuda()
    l2_misfit_gradient(v0t, grid, shots[:1], obs[:1], every)     # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    J, g = l2_misfit_gradient(v0t, grid, shots, obs, every)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    cells = p.ncells * p.nt * len(shots)
    # reverse-time-migration image of the 8 observed shots in the start model
    # (forward with checkpoints, then recompute + back-propagation per shot)
    from paper_2311_05038_amd.autograd import rtm_image
    rtm_image(v0t, grid, shots[:1], obs[:1], every)     # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    img = rtm_image(v0t, grid, shots, obs, every)
    torch.cuda.synchronize()
    sec_img = time.perf_counter() - t
    # the same gradient with one shot per call (one launch per shot and step)
    l2_misfit_gradient(v0t, grid, shots, obs, every, group=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    l2_misfit_gradient(v0t, grid, shots, obs, every, group=1)
    torch.cuda.synchronize()
    sec_1 = time.perf_counter() - t
    out = dict(workload="adjoint2d 1024^2, 8 shots, nt=2000, K=50", seconds_per_gradient=round(sec, 3),
               forward_equiv_mcell_per_s=round(3 * cells / sec / 1e6, 1), misfit=J,
               grad_norm=float(g.norm()), seconds_per_rtm_image=round(sec_img, 3),
               image_norm=float(img.norm()), shots_per_launch=len(shots),
               seconds_per_gradient_one_shot_per_launch=round(sec_1, 3))
    log(f"[bench] adjoint leg: {out}")
    return out


# A tiny fd_stream_probe launch (SERVE_MARK_N floats: a grid of
# SERVE_MARK_N / 4 threads that no other launch of the bench has) before and
# after the batched 50/s serving run, so that a kernel trace can be cut to
# that run (summarize_serving_trace).
SERVE_MARK_N = 4 * 768


def _serve_marker():
    import torch
    from paper_2311_05038_amd import _abi
    a = torch.zeros(SERVE_MARK_N, device="cuda")
    b = torch.zeros_like(a)
    _abi.fd_stream_probe(0, a.data_ptr(), None, b.data_ptr(), SERVE_MARK_N,
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()


def summarize_serving_trace(kt_dir: str, requests: int):
    """GPU busy time of the batched serving run from a rocprofv3 kernel trace
    (`--kernel-trace -f csv`) of `bench.py --legs serve`: the union of kernel
    intervals between the two markers, the largest kernels and the gaps.
    Writes profiles/k_step2d_batch_serving.md."""
    import collections
    import csv
    import glob
    path = sorted(glob.glob(os.path.join(kt_dir, "**", "*kernel_trace.csv"), recursive=True))[0]
    rows = list(csv.DictReader(open(path)))
    ks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"],
                 int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)) for r in rows)
    marks = [k for k in ks if "k_stream" in k[2] and k[3] == SERVE_MARK_N // 4]
    if len(marks) < 2:
        raise SystemExit("the trace holds no pair of serving markers")
    t0, t1 = marks[0][1], marks[1][0]
    win = [k for k in ks if k[0] >= t0 and k[1] <= t1 and k is not marks[1]]
    busy, cs, ce, gaps = 0, None, None, []
    for s_, e_, _, _ in win:
        if ce is None or s_ > ce:
            if ce is not None:
                busy += ce - cs
                gaps.append(s_ - ce)
            cs, ce = s_, e_
        else:
            ce = max(ce, e_)
    busy += ce - cs
    span = t1 - t0
    tot = collections.Counter()
    cnt = collections.Counter()
    for s_, e_, n, _ in win:
        tot[n.split("(")[0]] += e_ - s_
        cnt[n.split("(")[0]] += 1
    gaps.sort()
    cmd = f"python -u bench.py --steps 1 --warmup 0 --no-cpu --legs serve --serve-requests {requests}"
    lines = [f"# Batched serving ({requests} Poisson 2D shots at 50/s): GPU busy time", "",
             "Kernel trace:", "",
             "    cd /tmp && export TMPDIR=/tmp",
             f"    rocprofv3 --kernel-trace -T -f csv -d {kt_dir} -o sv -- {cmd}", "",
             "The window runs from the end of the first serving marker (a "
             f"{SERVE_MARK_N // 4}-thread fd_stream_probe launch) to the start of the second, "
             "around the batched run of the 50/s stream.", "",
             f"Window {span / 1e9:.3f} s; kernels running {busy / 1e9:.3f} s "
             f"(**{100 * busy / span:.1f}%**); {len(win)} launches; "
             f"{len(gaps)} gaps totalling {sum(gaps) / 1e9:.3f} s "
             f"(median {gaps[len(gaps) // 2] / 1e3:.1f} us, largest {gaps[-1] / 1e6:.2f} ms).", "",
             "| kernel | launches | total s | avg us |", "|---|---|---|---|"]
    for n, t in tot.most_common(8):
        lines.append(f"| {n} | {cnt[n]} | {t / 1e9:.3f} | {t / cnt[n] / 1e3:.1f} |")
    lines += ["", f"Summary written by `python bench.py --summarize-serving-trace {kt_dir} "
                  f"--serve-requests {requests}`.", ""]
    with open(os.path.join(ROOT, "profiles", "k_step2d_batch_serving.md"), "w") as fh:
        fh.write("\n".join(lines))
    print(json.dumps(dict(window_s=span / 1e9, busy_frac=busy / span, launches=len(win))))


def serve_leg(n_requests: int = 1000, seed: int = 50, n_sub: int = 500, sub_frac: float = 0.7):
    """Poisson streams of 2D shots on grids drawn from 512^2..2048x4096 (nt
    1000..4000), each shot with its own seeded random-field velocity model
    (generated on the device before any clock starts): continuous batching
    against sequential plain FP32 runs of the same arrival trace.  Two
    rates: 50 shots/s (n_requests shots; above what the device sustains, so
    the queue grows), and sub_frac of the sustained rate the batched run
    measured (the first n_sub shots on a fresh seeded trace)."""
    import numpy as np
    import torch
    import fd_inputs as fi
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.serve import Request, Scheduler, TorchDevice, summarize
    reqs_in = fi.serving_stream(n_requests, seed=seed)
    t_gen = time.perf_counter()
    vel = {}
    for r in reqs_in:
        vel[r.rid] = fi.grf_velocity_torch((r.nz, r.nx), r.seed, device="cuda").reshape(-1)
        if (r.rid + 1) % 200 == 0:
            torch.cuda.synchronize()
            log(f"[bench] serve: {r.rid + 1} models generated ({time.perf_counter() - t_gen:.1f} s)")
    torch.cuda.synchronize()
    log(f"[bench] serve: {n_requests} seeded models in {time.perf_counter() - t_gen:.1f} s")
    wav_all = torch.from_numpy(fi.ricker(10.0, 1e-3, 4000)).cuda()

    def make_inputs(req):
        p = fi.surface2d(req.nz, req.nx, req.nt, req.rid)
        g = fd.Grid(ndim=2, nz=p.nz, ny=1, nx=p.nx, dh=p.dh, dt=p.dt,
                    sponge_width=p.sponge_width, sponge_faces=p.sponge_faces)
        r = p.receivers
        shot = fd.Shot(p.src, wav_all[: p.nt], fd.Receivers(r.z0, r.y0, r.x0, r.nz, r.ny, r.nx))
        return g, vel[req.rid], shot

    cells = {r.rid: r.nz * r.nx * r.nt for r in reqs_in}
    warm = [Request(r.rid, 0.0, r.nz, r.nx, 200) for r in reqs_in[:4]]
    Scheduler(TorchDevice(make_inputs, batched=True), hbm_budget=200 << 30).run(warm)
    Scheduler(TorchDevice(make_inputs, batched=False), max_slots=1, policy="all",
              hbm_budget=200 << 30).run(warm)

    def run_pair(reqs, tag):
        out = {}
        last = [time.perf_counter()]

        def progress(done, total):
            if time.perf_counter() - last[0] > 10.0 or done == total:
                last[0] = time.perf_counter()
                log(f"[bench] serve {tag}: {done}/{total} shots done")
        # "batched": the earliest-arrived resident shot and then the shots
        # with the least remaining work advance, enough of them to give each
        # launch 20 M cells per step (fields that fit the Infinity Cache),
        # the others wait resident
        for name, batched, slots, policy in (("batched", True, 64, "srpt_oldest"),
                                             ("sequential", False, 1, "all")):
            torch.cuda.synchronize()
            sch = Scheduler(TorchDevice(make_inputs, batched=batched), max_slots=slots,
                            hbm_budget=200 << 30, chunk=25, policy=policy, launch_cells=20 << 20,
                            progress=progress)
            mark = tag == "50/s" and batched       # brackets for a kernel trace of this run
            if mark:
                _serve_marker()
            o = sch.run(reqs)
            if mark:
                torch.cuda.synchronize()
                _serve_marker()
            out[name] = {k: (round(v, 4) if isinstance(v, float) else v)
                         for k, v in summarize(o, cells.get).items()}
            out[name]["peak_slots"] = sch.peak_slots
            log(f"[bench] serve {tag} {name}: {out[name]}")
        span = reqs[-1].arrival - reqs[0].arrival
        out["offered_gcell_per_s"] = round(sum(cells[r.rid] for r in reqs) / span / 1e9, 1)
        out["rate_shots_per_s"] = round((len(reqs) - 1) / span, 2)
        out["requests"] = len(reqs)
        return out

    reqs = [Request(r.rid, r.arrival, r.nz, r.nx, r.nt) for r in reqs_in]
    res = {"rate50": run_pair(reqs, "50/s")}
    # sub-saturation: the first n_sub shots, seeded exponential gaps at
    # sub_frac of the rate the batched run sustained (by work, not count)
    n_sub = min(n_sub, n_requests)
    sustained = res["rate50"]["batched"]["gcell_per_s"] * 1e9
    mean_work = float(np.mean([cells[r.rid] for r in reqs_in[:n_sub]]))
    rate = sub_frac * sustained / mean_work
    gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, n_sub)
    arr = np.cumsum(gaps)
    sub = [Request(r.rid, float(t), r.nz, r.nx, r.nt) for r, t in zip(reqs_in[:n_sub], arr)]
    res["sub"] = run_pair(sub, f"{rate:.1f}/s")
    res["sub"]["fraction_of_sustained"] = sub_frac
    res["workload"] = (f"serving streams of 2D shots, 512^2..2048x4096, nt 1000..4000, own seeded GRF model "
                       f"each: {n_requests} Poisson arrivals at 50/s, and {n_sub} at {sub_frac:.0%} of the "
                       f"sustained rate")
    return res


def routines_leg(nsteps: int = 50):
    """The step as one kernel per routine (fd_step_routines: derivative
    fields materialised, then the time update and the source addition)
    against the fused step, on the 512^3 headline model and on a 2048x4096
    2D grid: microseconds per step and algorithmic GB/s (52 B per cell in 3D,
    40 B in 2D, against 16 B fused).  Per-kernel times are in the committed
    rocprofv3 kernel trace."""
    import torch
    import fd_inputs as fi
    from helpers import setup
    out = {}
    for name, p, bpc in (("3d", fi.layered3d(nt=nsteps + 5), 52),
                         ("2d", fi.surface2d(2048, 4096, nsteps + 5, seed=7), 40)):
        model, state, shot = setup(p)
        work = torch.empty(model.sizes.routines_work, dtype=torch.uint8, device="cuda")
        res = {}
        for form in ("routines", "fused"):
            state.begin(shot)
            step = ((lambda n: state.step_routines(shot, n, work)) if form == "routines"
                    else (lambda n: state.step(shot, n)))
            for n in range(5):
                step(n)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for n in range(5, 5 + nsteps):
                step(n)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / nsteps
            b = bpc if form == "routines" else 16
            res[form] = dict(us_per_step=round(us, 2), bytes_per_cell=b,
                             alg_gbs=round(b * p.ncells / (us * 1e-6) / 1e9, 1))
        res["fused_speedup"] = round(res["routines"]["us_per_step"] / res["fused"]["us_per_step"], 3)
        res["grid"] = "x".join(str(d) for d in p.shape)
        out[name] = res
        log(f"[bench] routines leg {name}: {res}")
        del model, state, shot, work
        torch.cuda.empty_cache()
    return out


def traffic_from_profiles(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2311_05038_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        h.update(open(os.path.join(src, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec["bytes_per_launch"]


def cpu_baseline(nsteps: int = 48, threads: int = 0):
    """The FP64 oracle on the same 512^3 model for a few steps, on all the
    host cores this process may use (threads=0) or on the given count."""
    import oracle
    import fd_inputs as fi
    p = fi.layered3d(nt=nsteps)
    v = p.velocity()
    g = oracle.grid_of(p)
    if threads <= 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    threads = oracle.set_threads(threads)
    t = time.perf_counter()
    oracle.forward(g, v, p.wavelet(), p.nt, p.src, p.rec_index())
    dt = time.perf_counter() - t
    return dict(value=p.ncells * nsteps / dt / 1e6, unit="Mcell-updates/s", cores=threads,
                kind="oracle",
                sample=f"512^3 layered model, {nsteps} time steps (incl. set-up), FP64, "
                       f"{dt:.1f} s")


def oracle_table():
    """The FP64 oracle's rate on bounded samples of every configuration, on
    one core and on all the cores this process may use: the 256^2 / 500-step
    case whole, the 512^3 and 768x768x512 layered models for a few steps
    (incl. set-up), and one shot of the 1024^2 gradient model forward and
    forward + adjoint for 200 steps (the adjoint stores every step's
    Laplacian, nt x 8 MiB); one-core samples are cut to at most 4e8
    cell-updates.  Mcell-updates/s per sample."""
    import oracle
    import fd_inputs as fi
    allc = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    rows = []
    cases = [("[0] 2D 256^2", fi.green2d(), "forward"),
             ("[1] 3D 512^3", fi.layered3d(nt=6), "forward"),
             ("[2] 3D 768x768x512", fi.precision3d(nt=4), "forward"),
             ("[4] 2D 1024^2, one shot", fi.surface2d(1024, 1024, 200, seed=5), "forward"),
             ("[4] 2D 1024^2, one shot", fi.surface2d(1024, 1024, 200, seed=5), "adjoint")]
    for name, p, kind in cases:
        v = p.velocity()
        g = oracle.grid_of(p)
        shp = (p.nz, p.ny, p.nx)
        for threads in (allc, 1):
            if threads == 1 and p.ncells * p.nt > 4e8:   # one core: about 15 s of work at most
                p = p.scaled(nt=max(1, int(4e8 // p.ncells)))
            oracle.set_threads(threads)
            t = time.perf_counter()
            if kind == "forward":
                oracle.forward(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index())
                work = p.ncells * p.nt
            else:
                import numpy as np
                r = np.ones((p.nt, p.receivers.count))
                oracle.adjoint(g, v.reshape(shp), p.wavelet(), p.nt, p.src, p.rec_index(), r)
                work = 2 * p.ncells * p.nt   # a forward and an adjoint pass
            dt = time.perf_counter() - t
            row = dict(config=name, kind=kind, cells=p.ncells, steps=p.nt, cores=threads,
                       seconds=round(dt, 2), mcell_per_s=round(work / dt / 1e6, 1))
            log(f"[bench] oracle {row}")
            rows.append(row)
    oracle.set_threads(allc)
    return rows


def slab_leg(nsteps: int = 200, ranks: int = 8):
    """One rank's share of the 512^3 headline model cut along z into `ranks`
    slabs: an interior slab (planes [192, 256), plus 4 ghost planes per side)
    stepped alone with fd_step, from a random field, against 1/ranks of the
    whole-grid step time measured here too; the same for 2, 4 and 16 slabs
    (`shares`).  Also times fd_slab_exchange between two such slabs on this
    one device (two device-to-device copies of 4 planes, 1 MiB per plane;
    between devices this would be the point-to-point link transfer, not
    measured here)."""
    import numpy as np
    import torch
    import fd_inputs as fi
    from helpers import grid_of, receivers_of, setup
    import paper_2311_05038_amd as fd
    p = fi.layered3d(nt=nsteps + 100)
    v = p.velocity().reshape(p.nz, p.ny, p.nx)
    shot = fd.Shot(p.src, torch.from_numpy(p.wavelet()).cuda(), receivers_of(p))
    gen = torch.Generator(device="cuda").manual_seed(5)

    def slab_state(nslabs, k):
        g = grid_of(p).slabs([p.nz // nslabs] * nslabs)[k]
        vt = torch.from_numpy(np.ascontiguousarray(v[g.slab_z0:g.slab_z0 + g.nz]).reshape(-1)).cuda()
        m = fd.Model(g, vt)
        st = m.new_state()
        st.begin(shot)
        for which in (1, 0):
            st.set_wavefield(which, 1e-3 * torch.randn(g.ncells, device="cuda", generator=gen))
        return g, m, st

    def timed(fn, n, warm=100):
        # a long warm-up: the first few hundred microseconds of a short
        # kernel after host work measured up to 10% slow
        for i in range(warm):
            fn(i)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for i in range(warm, warm + n):
            fn(i)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / n

    wm, wst, _ = setup(p)
    wst.begin(shot)
    whole_us = timed(lambda n: wst.step(shot, n), nsteps)
    del wm, wst
    torch.cuda.empty_cache()
    mid = ranks // 2 - 1
    g, m, st = slab_state(ranks, mid)
    _, m2, st2 = slab_state(ranks, mid + 1)
    ex_us = timed(lambda n: fd.slab_exchange(st, st2), nsteps)   # both at step 0
    del m2, st2
    us = timed(lambda n: st.step(shot, n), nsteps)
    del m, st
    cells = g.ncells
    shares = {}
    for r in (2, 4, 8, 16):
        if r == ranks:
            u = us
        else:
            _, mr, sr = slab_state(r, r // 2 - 1)
            u = timed(lambda n: sr.step(shot, n), nsteps)
            del mr, sr
        shares[str(r)] = dict(planes=p.nz // r, us_per_step=round(u, 2),
                              share_us=round(whole_us / r, 2),
                              efficiency=round(whole_us / r / u, 3))
    torch.cuda.empty_cache()
    res = dict(grid=f"{g.nz}x{p.ny}x{p.nx} (+2x4 ghost planes), planes [{g.slab_z0}, "
                    f"{g.slab_z0 + g.nz}) of {p.nz}",
               us_per_step=round(us, 2), mcell_per_s=round(cells / (us * 1e-6) / 1e6, 1),
               alg_gbs=round(16 * cells / (us * 1e-6) / 1e9, 1),
               whole_grid_us_per_step=round(whole_us, 2),
               whole_grid_share_us=round(whole_us / ranks, 2),
               exchange_us_one_device=round(ex_us, 2), shares=shares)
    log(f"[bench] slab leg: {res}")
    return res


def cpu_leg(nsteps: int = 10):
    """The host back-end on this machine's cores: Mcell-updates/s of the
    fused FP32 step on the 512^3 headline model (a few steps) and of the
    whole 256^2 / 500-step 2D shot, and the fraction of the host bandwidth
    (fd_cpu_stream_probe: three FP32 streams read, one rewritten in place,
    16 B per element, the step's own pattern) that the 3D step reaches at
    16 algorithmic bytes per cell."""
    import fd_inputs as fi
    from helpers import grid_of, receivers_of
    from paper_2311_05038_amd import cpu
    out = dict(threads=cpu.threads(), isa=cpu.isa())
    probe = cpu.stream_probe(1 << 27, 5)     # 3 x 512 MiB
    out["stream_probe_gbs"] = round(probe, 1)
    for name, p in (("layered3d_512", fi.layered3d(nt=nsteps + 2)), ("green2d_256", fi.green2d())):
        v = p.velocity()
        m = cpu.Model(grid_of(p), v)
        s = m.new_state()
        shot = cpu.Shot(p.src, p.wavelet(), receivers_of(p))
        m.run_shot(s, shot)                  # warm-up (first touch)
        best = float("inf")
        for _ in range(3):
            if p.ndim == 3:                  # steps 2.. of the shot, without the set-up
                s.begin(shot)
                s.step(shot, 0)
                s.step(shot, 1)
                t = time.perf_counter()
                for n in range(2, p.nt):
                    s.step(shot, n)
            else:                            # the whole shot (fd_run_shot)
                t = time.perf_counter()
                m.run_shot(s, shot)
            best = min(best, time.perf_counter() - t)
        steps = p.nt - 2 if p.ndim == 3 else p.nt
        mc = p.ncells * steps / best / 1e6
        out[name] = dict(steps=steps, seconds=round(best, 4), mcell_per_s=round(mc, 1),
                         alg_gbs=round(16 * mc / 1e3, 1), frac_of_probe=round(16 * mc / 1e3 / probe, 3))
        del m, s
    log(f"[bench] cpu leg: {out}")
    return out


def _csv_rows(root: str, suffix: str):
    import csv
    rows = []
    for d, _, files in os.walk(root):
        for f in files:
            if f.endswith(suffix):
                with open(os.path.join(d, f), newline="") as fh:
                    rows.extend(csv.DictReader(fh))
    return rows


def summarize_profiles(kt_dir: str, fetch_dir: str, write_dir: str, kernel: str = "k_step3d",
                       copy_kernel: str = "k_stream", cells: int = 512 ** 3, copy_bytes: int = 1 << 30):
    """Reads rocprofv3 CSV output (a --kernel-trace --stats run and two --pmc
    runs, FETCH_SIZE and WRITE_SIZE, of `bench.py --steps 1 --warmup 0
    --no-cpu --legs none`) and writes the step kernel's summary and traffic
    record under profiles/.  The byte counters are calibrated on the copy
    probe's own dispatches (fd_stream_probe kind 0: copy_bytes read and
    copy_bytes written)."""
    import hashlib
    stats = _csv_rows(kt_dir, "kernel_stats.csv")
    trace = _csv_rows(kt_dir, "kernel_trace.csv")
    # kernel names as rocprofv3 -T gives them (the function's base name); the
    # copy probe's dispatches are told from the step-pattern probe's by their
    # grid (one thread per float4 of the 1 GiB arrays)
    copy_threads = copy_bytes // 16
    step = [r for r in trace if r["Kernel_Name"].startswith(kernel)]
    durs = sorted((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in step)
    avg = sum(durs) / len(durs)

    def per_dispatch(rows, name, counter, grid=None):
        vals = {}
        for r in rows:
            if (r.get("Counter_Name") == counter and r["Kernel_Name"].startswith(name) and
                    (grid is None or int(r["Grid_Size"]) == grid)):
                vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        return list(vals.values())

    fetch_rows = _csv_rows(fetch_dir, "counter_collection.csv")
    write_rows = _csv_rows(write_dir, "counter_collection.csv")
    f_step = per_dispatch(fetch_rows, kernel, "FETCH_SIZE")
    w_step = per_dispatch(write_rows, kernel, "WRITE_SIZE")
    f_copy = per_dispatch(fetch_rows, copy_kernel, "FETCH_SIZE", copy_threads)
    w_copy = per_dispatch(write_rows, copy_kernel, "WRITE_SIZE", copy_threads)
    mean = lambda x: sum(x) / len(x)
    kib = copy_bytes / 1024
    fscale, wscale = kib / mean(f_copy), kib / mean(w_copy)
    fetch_kib, write_kib = mean(f_step), mean(w_step)
    traffic = fetch_kib * 1024 * fscale + write_kib * 1024 * wscale
    alg = 16.0 * cells
    src = os.path.join(ROOT, "paper_2311_05038_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        h.update(open(os.path.join(src, f), "rb").read())
    rec = dict(kernel="k_step3d<f32>", workload="layered3d 512^3, nt=1000", bytes_per_launch=traffic,
               fetch_kib=fetch_kib, write_kib=write_kib, fetch_scale=fscale, write_scale=wscale,
               avg_launch_us=avg, launches=len(durs), source_sha256=h.hexdigest())
    with open(os.path.join(ROOT, "profiles", "k_step3d_f32_layered3d_512_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0)))[:8]:
        nm = r["Name"]
        lines.append(f"| {nm} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    cmd = "python -u bench.py --steps 1 --warmup 0 --no-cpu --legs none"
    md = f"""# k_step3d<f32> on layered3d 512x512x512 (1 shot, 1000 steps)

Kernel trace:

    cd /tmp && export TMPDIR=/tmp
    rocprofv3 --kernel-trace --stats -T -f csv -d {kt_dir} -o kt -- {cmd}

{chr(10).join(lines)}

Average k_step3d duration {avg:.1f} us over {len(durs)} launches -> {alg / (avg * 1e-6) / 1e9:.1f} GB/s
algorithmic (16 B per cell-update x {cells:,} cells per launch = {alg / 1e9:.3f} GB),
i.e. {100 * alg / (avg * 1e-6) / 8e12:.1f}% of the 8 TB/s HBM peak.

Byte counters (one pass each):

    rocprofv3 --pmc FETCH_SIZE --kernel-include-regex "k_step3d|k_stream" -T -f csv -d {fetch_dir} -o f -- {cmd}
    rocprofv3 --pmc WRITE_SIZE --kernel-include-regex "k_step3d|k_stream" -T -f csv -d {write_dir} -o w -- {cmd}

| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | dispatches |
|---|---|---|---|
| k_step3d | {fetch_kib:.0f} | {write_kib:.0f} | {len(f_step)} |
| copy probe (fd_stream_probe kind 0, 1 GiB in + 1 GiB out) | {mean(f_copy):.0f} | {mean(w_copy):.0f} | {len(f_copy)} |

Calibration (the probe moves {kib:,.0f} KiB each way): FETCH_SIZE x {fscale:.3f},
WRITE_SIZE x {wscale:.3f}.  Scaled traffic per k_step3d launch:
{fetch_kib * fscale / 1048576:.3f} GiB read + {write_kib * wscale / 1048576:.3f} GiB written
= {traffic / 1e9:.3f} GB vs {alg / 1e9:.3f} GB algorithmic ({traffic / alg:.3f}x).
FETCH_SIZE counts L2 misses, including those the Infinity Cache serves.

Summary written by `python bench.py --summarize-profiles {kt_dir} {fetch_dir} {write_dir}`.
"""
    with open(os.path.join(ROOT, "profiles", "k_step3d_f32_layered3d_512.md"), "w") as fh:
        fh.write(md)
    print(json.dumps(rec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed shots; their median and spread are reported beside the mean")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-only", action="store_true",
                    help="only the 1 GiB copy probe (counter calibration)")
    ap.add_argument("--legs", default="half,adjoint,serve,routines,slab,small2d,cpu",
                    help="comma list of extra legs (half, adjoint, serve, routines, slab, small2d, "
                         "cpu) or 'none'")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--half-nt", type=int, default=2000,
                    help="steps per shot of the 16-bit leg (a few for counter runs)")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("KT_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 CSV output (host only)")
    ap.add_argument("--summarize-serving-trace", metavar="KT_DIR",
                    help="GPU busy time of the batched serving run from a rocprofv3 kernel trace "
                         "of --legs serve (writes profiles/k_step2d_batch_serving.md)")
    ap.add_argument("--oracle-table", action="store_true",
                    help="only the FP64 oracle's rate on samples of every configuration (host only)")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles)
        return
    if args.summarize_serving_trace:
        summarize_serving_trace(args.summarize_serving_trace, args.serve_requests)
        return
    if args.oracle_table:
        print(json.dumps({"oracle_table": oracle_table()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(a z-slab steps one device's share; the exchange between devices is not built)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_2311_05038_amd as fd
    fd.ensure_built()

    probe = copy_probe()
    log(f"[bench] copy probe (fd_stream_probe kind 0, 1 GiB each way): {probe['us']:.1f} us, {probe['gbs']:.0f} GB/s")
    sprobe = stream_probe()
    log(f"[bench] step-pattern stream probe (fd_stream_probe kind 1, 512^3): {sprobe['us']:.1f} us, "
        f"{sprobe['gbs']:.0f} GB/s")
    if args.probe_only:
        print(json.dumps({"copy_probe": probe}), flush=True)
        return
    h = headline(args.steps, args.warmup)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    extra = {}
    if "half" in legs:
        extra["half_storage"] = half_leg(args.half_nt)
    if "adjoint" in legs:
        extra["adjoint"] = adjoint_leg()
    if "serve" in legs:
        extra["serving"] = serve_leg(args.serve_requests)
    if "routines" in legs:
        extra["routines"] = routines_leg()
    if "slab" in legs:
        extra["slab"] = slab_leg()
    if "small2d" in legs:
        extra["small2d"] = small2d_leg()
    if "cpu" in legs:
        extra["cpu_backend"] = cpu_leg()
    cpu = cpu1 = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        log(f"[bench] oracle on {cpu['cores']} cores: {cpu['value']:.0f} Mcell-updates/s")
        cpu1 = cpu_baseline(2, threads=1)
        log(f"[bench] oracle on 1 core: {cpu1['value']:.1f} Mcell-updates/s")
    traffic = traffic_from_profiles("k_step3d_f32_layered3d_512")
    out = {
        "metric": "Mcell-updates/s",
        "value": round(h["mcell"], 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"] / args.steps, 3),
        "shot_ms": h["shot_ms"],
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
                     "traffic": traffic, "kernel": "k_step3d<f32>",
                     "bytes_per_cell": 16, "avg_launch_us": round(h["per_launch_us"], 2)},
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "copy_roof_gbs": round(probe["gbs"], 1),
        "stream_roof_gbs": round(sprobe["gbs"], 1),
        "frac_of_stream_roof": round(h["achieved"] / sprobe["gbs"], 4),
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
