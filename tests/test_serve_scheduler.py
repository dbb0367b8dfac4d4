"""The serving policy on the CPU, against a simulated device with a virtual
clock: admission by slots and HBM bytes, FIFO order, every shot stepped
exactly nt times, failures isolated, batching beats one-at-a-time service
on a launch-bound stream."""
import pytest

from paper_2311_05038_amd.serve import Request, Scheduler, summarize


class FakeDevice:
    """One queue of chunks executed in order; a chunk of k steps over the
    active shots costs k * (launch + sum(cells) * 16 B / bandwidth)."""

    def __init__(self, bw=6e12, launch=5e-6, fail=()):
        self.bw, self.launch, self.fail = bw, launch, set(fail)
        self.now = 0.0
        self.free_at = 0.0
        self.alloc = 0
        self.peak_alloc = 0
        self.steps = {}
        self.order = []

    def begin_stream(self):
        self.now = 0.0

    def elapsed(self):
        return self.now

    def idle_until(self, t):
        self.now = max(self.now, t)

    def footprint(self, req):
        return req.nz * req.nx * 4 * 3 + req.nt * req.nx * 4

    def start(self, req):
        if req.rid in self.fail:
            raise ValueError("bad velocity")
        self.alloc += self.footprint(req)
        self.peak_alloc = max(self.peak_alloc, self.alloc)
        self.order.append(req.rid)
        self.steps[req.rid] = 0
        return {"req": req, "n": 0}

    def advance(self, handles, nsteps):
        dur = 0.0
        for _ in range(nsteps):
            act = [h for h in handles if h["n"] < h["req"].nt]
            if not act:
                break
            dur += self.launch + sum(h["req"].nz * h["req"].nx for h in act) * 16 / self.bw
            for h in act:
                h["n"] += 1
                self.steps[h["req"].rid] += 1
        self.free_at = max(self.free_at, self.now) + dur
        return [h for h in handles if h["n"] >= h["req"].nt]

    def fence(self):
        return self.free_at

    def done(self, token):
        return self.now >= token

    def wait(self, token):
        self.now = max(self.now, token)

    def token_time(self, token):
        return token

    def finish(self, h):
        self.alloc -= self.footprint(h["req"])
        return None


def _stream(n=40, rate=50.0, seed=0):
    import fd_inputs as fi
    return [Request(r.rid, r.arrival, r.nz, r.nx, r.nt)
            for r in fi.serving_stream(n, seed=seed, rate=rate)]


def test_all_shots_complete_with_exact_steps_and_fifo_admission():
    reqs = _stream()
    dev = FakeDevice()
    out = Scheduler(dev, max_slots=16, hbm_budget=1 << 40, chunk=25).run(reqs)
    assert all(o.status == "ok" for o in out.values())
    for r in reqs:
        assert dev.steps[r.rid] == r.nt
        assert out[r.rid].admitted >= r.arrival - 1e-12
        assert out[r.rid].finished > out[r.rid].admitted
    assert dev.order == sorted(dev.order, key=lambda rid: out[rid].arrival)


@pytest.mark.parametrize("slots,budget_shots", [(1, 8), (4, 2), (16, 3)])
def test_slots_and_memory_budget_respected(slots, budget_shots):
    reqs = _stream(30)
    dev = FakeDevice()
    budget = budget_shots * max(dev.footprint(r) for r in reqs)
    sch = Scheduler(dev, max_slots=slots, hbm_budget=budget, chunk=10)
    out = sch.run(reqs)
    assert all(o.status == "ok" for o in out.values())
    assert dev.peak_alloc <= budget
    assert sch.peak_bytes <= budget
    assert sch.peak_slots <= slots
    assert dev.alloc == 0


def test_failures_are_isolated():
    reqs = _stream(20)
    dev = FakeDevice(fail={3, 7})
    out = Scheduler(dev, max_slots=8, hbm_budget=1 << 40).run(reqs)
    assert out[3].status.startswith("failed") and out[7].status.startswith("failed")
    assert all(o.status == "ok" for k, o in out.items() if k not in (3, 7))
    assert dev.steps.get(3) is None


def test_request_larger_than_budget_fails_alone():
    reqs = _stream(10)
    dev = FakeDevice()
    big = max(reqs, key=lambda r: dev.footprint(r))
    budget = sorted(dev.footprint(r) for r in reqs)[-2]   # everything but the biggest fits
    out = Scheduler(dev, max_slots=4, hbm_budget=budget).run(reqs)
    assert out[big.rid].status.startswith("failed")
    assert sum(o.status == "ok" for o in out.values()) == len(reqs) - 1


def test_batching_beats_sequential_on_a_launch_bound_stream():
    # small grids: per-step launch cost dominates one shot alone
    reqs = [Request(i, i * 0.002, 256, 256, 400) for i in range(40)]   # offered > 1 shot alone
    cells = {r.rid: r.nz * r.nx * r.nt for r in reqs}
    seq = summarize(Scheduler(FakeDevice(launch=20e-6), max_slots=1, chunk=400).run(reqs),
                    cells.get)
    bat = summarize(Scheduler(FakeDevice(launch=20e-6), max_slots=16, chunk=25).run(reqs),
                    cells.get)
    assert bat["shots"] == seq["shots"] == 40
    assert bat["p99_latency_s"] < seq["p99_latency_s"]
    assert bat["shots_per_s"] > seq["shots_per_s"]


class RecordingDevice(FakeDevice):
    """FakeDevice that records which shots each chunk advanced."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.calls = []

    def advance(self, handles, nsteps):
        self.calls.append([h["req"].rid for h in handles])
        return super().advance(handles, nsteps)


def test_srpt_policy_completes_every_shot_and_keeps_launches_full():
    reqs = _stream(40)
    dev = RecordingDevice()
    cap = 4 << 20
    out = Scheduler(dev, max_slots=64, hbm_budget=1 << 40, chunk=25, policy="srpt",
                    launch_cells=cap, launch_max=16).run(reqs)
    assert all(o.status == "ok" for o in out.values())
    for r in reqs:
        assert dev.steps[r.rid] == r.nt
    size = {r.rid: r.nz * r.nx for r in reqs}
    for call in dev.calls:
        assert 1 <= len(call) <= 16
        # shots are added until the launch holds `cap` cells: dropping the
        # last one leaves it below the cap
        assert sum(size[i] for i in call[:-1]) < cap


def test_srpt_serves_short_shots_first():
    # one long shot already running, then short ones: under "srpt" the short
    # shots run alone (the long one waits), under "all" they share launches
    reqs = [Request(0, 0.0, 2048, 2048, 4000)] + [Request(i, 0.01 + 0.001 * i, 512, 512, 1000)
                                                  for i in range(1, 9)]
    res = {}
    for policy in ("all", "srpt"):
        dev = RecordingDevice()
        out = Scheduler(dev, max_slots=16, hbm_budget=1 << 40, chunk=25, policy=policy,
                        launch_cells=1 << 20).run(reqs)
        assert all(o.status == "ok" for o in out.values())
        res[policy] = out
    short_all = max(res["all"][i].latency for i in range(1, 9))
    short_srpt = max(res["srpt"][i].latency for i in range(1, 9))
    assert short_srpt < 0.7 * short_all
    assert res["srpt"][0].latency >= res["all"][0].latency - 1e-9


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Scheduler(FakeDevice(), policy="lifo")


def test_srpt_oldest_always_advances_the_earliest_shot():
    reqs = _stream(30)
    dev = RecordingDevice()
    out = Scheduler(dev, max_slots=64, hbm_budget=1 << 40, chunk=25, policy="srpt_oldest",
                    launch_cells=1 << 20, launch_max=16).run(reqs)
    assert all(o.status == "ok" for o in out.values())
    for r in reqs:
        assert dev.steps[r.rid] == r.nt
    arrival = {r.rid: r.arrival for r in reqs}
    # every chunk leads with the earliest-arrived shot still resident
    for call in dev.calls:
        assert call[0] == min(call, key=lambda i: arrival[i])
