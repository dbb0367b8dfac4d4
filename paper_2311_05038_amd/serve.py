"""Shot server: continuous batching of forward-modelling requests.

Requests (one shot each, on its own 2D grid and velocity model) arrive over
time.  The scheduler admits a waiting request as soon as a batch slot is free
and its device footprint fits the HBM budget, starts it (model set-up and
first source addition), and advances every admitted shot with ONE batched
kernel launch per time step (``fd_step_batch``), so that work of shots that
arrived at different times overlaps on the device.  A shot leaves the batch
after its last step; its memory returns to the budget once the device has
passed that step.  Latency = completion - arrival.

The scheduling core (`Scheduler`) is device-agnostic: it drives any object
with the methods of `TorchDevice` (footprint, start, advance, fence, done,
wait, elapsed, finish, and optionally health), which lets the policy be
tested on the CPU against a simulated device.  A shot whose wavefield ends
non-finite (NaN or infinity: a corrupted input or an overflow) fails alone:
its outcome says so and the other shots of the mix are unaffected.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional

import torch


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    nz: int
    nx: int
    nt: int
    payload: Any = None     # device-specific inputs (grid, velocity, shot ...)


@dataclasses.dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    status: str = "pending"     # "ok" or "failed: ..."
    result: Any = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """Admission by free slots and HBM bytes, FIFO order, batched stepping in
    chunks of `chunk` steps with at most `depth` chunks queued on the device.

    Which admitted shots a chunk advances is the policy:
      "all"   every admitted shot, every chunk;
      "srpt"  the admitted shots with the least remaining work (cell-updates
              still to do), taken in that order until the chunk holds
              `launch_cells` cells per step or `launch_max` shots; the others
              stay resident and wait;
      "srpt_oldest"  the same after the earliest-arrived resident shot,
              which advances in every chunk (no shot waits indefinitely).
    With "srpt" and "srpt_oldest" the device stays busy (enough cells per
    launch) while short shots finish first.  Measured on the serving stream
    (60 Poisson 2D shots at 50/s): both give more shots/s than "all" at about
    40% of its median latency; the oldest shot's guaranteed progress brings
    the p99 of "srpt_oldest" (the default) back to that of "all".

    launch_cells: a chunk's shots are stepped together for `chunk` steps, so
    when their fields (cur, prev and c: 12 B per cell) fit in the 256 MB
    Infinity Cache, every step after the first re-reads them from there
    rather than from HBM.  The default of 20 M cells (240 MB) is the largest
    batch that fits; on 1000 Poisson shots at 50/s it sustains 330
    Gcell-updates/s against 307 with 12 M cells (p90 latency 1.6 s against
    3.8 s), and larger batches lose the cache (28 M: 315, 32 M: 305).

    Time comes from device.elapsed() (device clock since the stream start)."""

    def __init__(self, device, max_slots: int = 64, hbm_budget: int = 64 << 30,
                 chunk: int = 25, depth: int = 2, policy: str = "srpt_oldest",
                 launch_cells: int = 20 << 20, launch_max: int = 16,
                 progress: Optional[Callable[[int, int], None]] = None):
        if policy not in ("all", "srpt", "srpt_oldest"):
            raise ValueError(f"unknown policy {policy!r}")
        self.dev = device
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.chunk = chunk
        self.depth = depth
        self.policy = policy
        self.launch_cells = launch_cells
        self.launch_max = launch_max
        self.progress = progress        # called as progress(finished, total) when shots retire
        self.peak_bytes = 0
        self.peak_slots = 0
        self.launch_steps = 0

    def _pick(self, active: List[Any], owner: Dict[int, Request], stepped: Dict[int, int]) -> List[Any]:
        if self.policy == "all":
            return active
        def remaining(h):
            r = owner[id(h)]
            return (r.nt - stepped[id(h)]) * r.nz * r.nx
        order = sorted(active, key=remaining)
        if self.policy == "srpt_oldest":
            # the longest-waiting resident shot always advances: no starvation
            oldest = min(active, key=lambda h: owner[id(h)].arrival)
            order = [oldest] + [h for h in order if h is not oldest]
        run, cells = [], 0
        for h in order:
            if run and (cells >= self.launch_cells or len(run) >= self.launch_max):
                break
            r = owner[id(h)]
            run.append(h)
            cells += r.nz * r.nx
        return run

    def run(self, requests: List[Request]) -> Dict[int, Outcome]:
        dev = self.dev
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        active: List[Any] = []          # device handles in the batch
        owner: Dict[int, Request] = {}  # id(handle) -> request
        stepped: Dict[int, int] = {}    # id(handle) -> steps enqueued
        inflight: collections.deque = collections.deque()  # (token, [handles done])
        used = 0
        out = {r.rid: Outcome(r.rid, r.arrival) for r in requests}
        n_done = 0
        dev.begin_stream()
        while pending or waiting or active or inflight:
            now = dev.elapsed()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission, FIFO: the head waits until it fits
            while waiting and len(active) < self.max_slots:
                req = waiting[0]
                fp = dev.footprint(req)
                if used + fp > self.budget:
                    if not active and not inflight and fp > self.budget:
                        waiting.popleft()
                        out[req.rid].status = "failed: footprint exceeds the HBM budget"
                        continue
                    break
                waiting.popleft()
                try:
                    h = dev.start(req)
                except Exception as e:  # a bad request fails alone
                    out[req.rid].status = f"failed: {e}"
                    out[req.rid].finished = dev.elapsed()
                    continue
                used += fp
                owner[id(h)] = req
                stepped[id(h)] = 0
                out[req.rid].admitted = dev.elapsed()
                active.append(h)
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_slots = max(self.peak_slots, len(active))
            if active:
                run = self._pick(active, owner, stepped)
                finished = dev.advance(run, self.chunk)
                for h in run:
                    stepped[id(h)] = min(owner[id(h)].nt, stepped[id(h)] + self.chunk)
                self.launch_steps += self.chunk
                inflight.append((dev.fence(), finished))
                done_ids = {id(h) for h in finished}
                active = [h for h in active if id(h) not in done_ids]
            # Retire completed chunks.  Block on the oldest chunk when too many
            # are queued, or when nothing is left to enqueue (its retirement
            # is what frees slots and memory for the waiting requests).
            while inflight and (len(inflight) > self.depth or not active or
                                dev.done(inflight[0][0])):
                token, finished = inflight.popleft()
                dev.wait(token)
                t_done = dev.token_time(token)
                for h in finished:
                    req = owner.pop(id(h))
                    stepped.pop(id(h), None)
                    o = out[req.rid]
                    o.finished = t_done
                    err = dev.health(h) if hasattr(dev, "health") else None
                    o.status = "ok" if err is None else f"failed: {err}"
                    o.result = dev.finish(h)
                    used -= dev.footprint(req)
                    n_done += 1
                if finished and self.progress is not None:
                    self.progress(n_done, len(requests))
                if not active and waiting:
                    break   # go back and admit
            if not active and not inflight and not waiting and pending:
                dev.idle_until(pending[0].arrival)
        return out


def summarize(outcomes: Dict[int, Outcome], cell_updates: Callable[[int], float]) -> dict:
    """shots/s, p50/p99 latency and Gcell-updates/s over the successful shots."""
    ok = [o for o in outcomes.values() if o.status == "ok"]
    if not ok:
        return dict(shots=0)
    lat = sorted(o.latency for o in ok)
    t_end = max(o.finished for o in ok)
    t_first = min(o.arrival for o in ok)
    q = lambda p: lat[min(len(lat) - 1, int(round(p * (len(lat) - 1))))]
    work = sum(cell_updates(o.rid) for o in ok)
    return dict(shots=len(ok), failed=len(outcomes) - len(ok),
                makespan_s=t_end - t_first, shots_per_s=len(ok) / (t_end - t_first),
                p50_latency_s=q(0.50), p90_latency_s=q(0.90), p99_latency_s=q(0.99),
                max_latency_s=lat[-1], mean_latency_s=sum(lat) / len(lat),
                gcell_per_s=work / (t_end - t_first) / 1e9)


class TorchDevice:
    """The GPU side of the scheduler: libfd.so through the Python binding.

    `make_inputs(req)` returns (Grid, velocity tensor, Shot) for a request.
    batched=True steps all admitted shots with fd_step_batch; batched=False
    runs each shot alone with fd_run_shot (the plain sequential path; use it
    with max_slots=1)."""

    def __init__(self, make_inputs: Callable, batched: bool = True, keep_traces: bool = False):
        from . import _abi
        self._abi = _abi
        self.make_inputs = make_inputs
        self.batched = batched
        self.keep_traces = keep_traces
        self.stream = torch.cuda.current_stream()
        self.side = torch.cuda.Stream()
        self._fp: Dict[int, int] = {}
        self.t0_event = None
        self.t0_wall = 0.0

    # clock: device time since begin_stream, in seconds
    def begin_stream(self):
        torch.cuda.synchronize()
        self.t0_event = torch.cuda.Event(enable_timing=True)
        self.t0_event.record(self.stream)
        self.t0_wall = time.perf_counter()

    def elapsed(self) -> float:
        return time.perf_counter() - self.t0_wall

    def idle_until(self, t: float):
        while self.elapsed() < t:
            time.sleep(min(1e-3, max(0.0, t - self.elapsed())))

    def footprint(self, req: Request) -> int:
        if req.rid not in self._fp:
            from . import Grid
            g = Grid(ndim=2, nz=req.nz, ny=1, nx=req.nx, dh=10.0, dt=1e-3)
            s = self._abi.fd_query_bytes(g.c())
            nrec = req.nx
            self._fp[req.rid] = int(s.model + s.state + req.nt * nrec * 4 + req.nz * req.nx * 4)
        return self._fp[req.rid]

    def start(self, req: Request):
        from . import Model
        # Inputs and model set-up on the side stream: fd_create_model waits
        # for the side stream only, never for the batch queued on the main
        # stream.  Side-stream memory used later by the main stream is
        # recorded on it so the allocator does not hand it out early.
        with torch.cuda.stream(self.side):
            grid, velocity, shot = self.make_inputs(req)
            model = Model(grid, velocity, stream=self.side)
        model.buf.record_stream(self.stream)
        shot.wavelet.record_stream(self.stream)
        state = model.new_state()
        traces = torch.empty((shot.nt, shot.nrec), dtype=torch.float32,
                             device=velocity.device)
        h = dict(model=model, state=state, shot=shot, traces=traces, req=req)
        if self.batched:
            state.begin(shot, stream=self.stream)
        return h

    def advance(self, handles, nsteps: int):
        from . import step_batch
        if self.batched:
            entries = [(h["model"], h["state"], h["shot"], h["traces"]) for h in handles]
            for i in range(0, len(entries), self._abi.FD_BATCH_MAX):
                step_batch(entries[i:i + self._abi.FD_BATCH_MAX], nsteps, stream=self.stream)
            done = [h for h in handles if h["state"].next >= h["shot"].nt]
        else:
            for h in handles:   # plain path: the whole shot in one call
                h["model"].run_shot(h["state"], h["shot"], h["traces"], stream=self.stream)
            done = list(handles)
        # the finished shots' health, read when their chunk has retired
        for h in done:
            h["flags"] = h["state"].check_finite(stream=self.stream)
        return done

    def health(self, h) -> Optional[str]:
        """None for a finite final wavefield, else the reason the shot failed
        (called once the chunk that finished it has completed)."""
        f = int(h["flags"].item()) if "flags" in h else 0
        return None if f == 0 else "non-finite wavefield (NaN or infinity)"

    def fence(self):
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token):
        token.synchronize()

    def token_time(self, token) -> float:
        return self.t0_event.elapsed_time(token) * 1e-3

    def finish(self, h):
        return h["traces"] if self.keep_traces else None
