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


def stream_probe(cells: int = 512 ** 3, reps: int = 20):
    """The stencil step's traffic without the stencil: d = a + b * c
    elementwise over three FP32 inputs and one output of the 512^3 size
    (torch.addcmul: 12 B read + 4 B written per element), i.e. the practical
    roof of a 3-read / 1-write stream on this GPU."""
    import torch
    a = torch.ones(cells, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    d = torch.empty_like(a)
    for _ in range(3):
        torch.addcmul(a, b, c, out=d)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        torch.addcmul(a, b, c, out=d)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b, c, d
    torch.cuda.empty_cache()
    return dict(us=ms * 1e3, gbs=16 * cells / (ms * 1e-3) / 1e9)


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
    out["workload"] = "precision3d 768x768x512, nt=2000"
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


def serve_leg(n_requests: int = 60, seed: int = 50):
    """A Poisson stream (50 shots/s) of 2D shots on grids drawn from
    512^2..2048x4096: continuous batching vs sequential plain FP32 runs."""
    import numpy as np
    import torch
    import fd_inputs as fi
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.serve import Request, Scheduler, TorchDevice, summarize
    reqs_in = fi.serving_stream(n_requests, seed=seed)
    K = 4
    base = [torch.from_numpy(fi.grf_velocity((2048, 4096), seed * 100 + k)).cuda() for k in range(K)]
    wav_all = torch.from_numpy(fi.ricker(10.0, 1e-3, 4000)).cuda()

    def make_inputs(req):
        p = fi.surface2d(req.nz, req.nx, req.nt, req.rid)
        g = fd.Grid(ndim=2, nz=p.nz, ny=1, nx=p.nx, dh=p.dh, dt=p.dt,
                    sponge_width=p.sponge_width, sponge_faces=p.sponge_faces)
        v = base[req.rid % K][: p.nz, : p.nx].contiguous().reshape(-1)
        r = p.receivers
        shot = fd.Shot(p.src, wav_all[: p.nt], fd.Receivers(r.z0, r.y0, r.x0, r.nz, r.ny, r.nx))
        return g, v, shot

    reqs = [Request(r.rid, r.arrival, r.nz, r.nx, r.nt) for r in reqs_in]
    cells = {r.rid: r.nz * r.nx * r.nt for r in reqs}
    res = {}
    # "batched": the earliest-arrived resident shot and then the shots with
    # the least remaining work advance, enough of them to give each launch
    # 12 M cells per step, the others wait resident; "batched_all": every
    # admitted shot advances in every launch
    warm = [Request(i, 0.0, 512 + 256 * i, 1024, 200) for i in range(4)]
    Scheduler(TorchDevice(make_inputs, batched=True), hbm_budget=200 << 30).run(warm)
    Scheduler(TorchDevice(make_inputs, batched=False), max_slots=1, policy="all",
              hbm_budget=200 << 30).run(warm)
    for name, batched, slots, policy in (("batched", True, 64, "srpt_oldest"),
                                         ("batched_all", True, 16, "all"),
                                         ("sequential", False, 1, "all")):
        torch.cuda.synchronize()
        sch = Scheduler(TorchDevice(make_inputs, batched=batched), max_slots=slots,
                        hbm_budget=200 << 30, chunk=25, policy=policy, launch_cells=12 << 20)
        out = sch.run(reqs)
        res[name] = {k: (round(v, 4) if isinstance(v, float) else v)
                     for k, v in summarize(out, cells.get).items()}
        res[name]["peak_slots"] = sch.peak_slots
        log(f"[bench] serve {name}: {res[name]}")
    offered = sum(cells.values()) / (reqs[-1].arrival - reqs[0].arrival)
    res["offered_gcell_per_s"] = round(offered / 1e9, 1)
    res["workload"] = f"serving stream: {n_requests} Poisson shots at 50/s, 512^2..2048x4096, nt 1000..4000"
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-only", action="store_true",
                    help="only the 1 GiB copy probe (counter calibration)")
    ap.add_argument("--legs", default="half,adjoint,serve,routines,slab,cpu",
                    help="comma list of extra legs (half, adjoint, serve, routines, slab, cpu) "
                         "or 'none'")
    ap.add_argument("--serve-requests", type=int, default=60)
    args = ap.parse_args()
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
    log(f"[bench] copy probe: {probe['gbs']:.0f} GB/s")
    sprobe = stream_probe()
    log(f"[bench] 3-read/1-write stream probe (512^3): {sprobe['us']:.1f} us, {sprobe['gbs']:.0f} GB/s")
    if args.probe_only:
        print(json.dumps({"copy_probe": probe}), flush=True)
        return
    h = headline(args.steps, args.warmup)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    extra = {}
    if "half" in legs:
        extra["half_storage"] = half_leg()
    if "adjoint" in legs:
        extra["adjoint"] = adjoint_leg()
    if "serve" in legs:
        extra["serving"] = serve_leg(args.serve_requests)
    if "routines" in legs:
        extra["routines"] = routines_leg()
    if "slab" in legs:
        extra["slab"] = slab_leg()
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
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
