"""Recorded shots (fd_shot_graph_create / fd_shot_graph_launch) through the C
ABI: every replay gives the bits of the eager fd_run_shot (traces and both
levels) for 2D and 3D grids and 16-bit storage, with the caller's own eager
work and synchronisations between replays; the recording itself runs
nothing and leaves the state's step counter alone; replays read the current
contents of the wavelet (doubling the wavelet doubles the traces); the state keeps working eagerly after replays."""
import pytest
import torch

import fd_inputs as fi
from helpers import rel_l2, setup

pytestmark = pytest.mark.gpu


def _cases():
    return [("green2d", fi.green2d().scaled(nt=300), 0),
            ("layered3d", fi.layered3d(nx=96, ny=40, nz=50, nt=60), 0),
            ("surface2d_bf16", fi.surface2d(96, 200, 120, seed=31), 2),
            ("layered3d_f16", fi.layered3d(nx=72, ny=36, nz=30, nt=40), 1)]


@pytest.mark.parametrize("case", range(4))
def test_replays_equal_eager_shot(case):
    import paper_2311_05038_amd as fd
    name, p, storage = _cases()[case]
    print(f"case {name} shape={p.shape} nt={p.nt} storage={storage}", flush=True)
    model, state, shot = setup(p, storage=storage)
    ref_tr = model.run_shot(state, shot).clone()
    ref_cur, ref_prev = state.wavefield(0).clone(), state.wavefield(1).clone()
    torch.cuda.synchronize()

    st2 = model.new_state()
    traces = torch.full((p.nt, p.receivers.count), -1.0, device="cuda")
    g = fd.ShotGraph(model, st2, shot, traces)
    torch.cuda.synchronize()
    assert st2.next == -1                        # recording ran nothing
    assert torch.all(traces == -1.0)
    other = model.new_state()
    for r in range(3):
        traces.fill_(float("nan"))
        model.run_shot(other, shot)              # the caller's own eager work
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(traces, ref_tr), r
        assert torch.equal(st2.wavefield(0), ref_cur), r
        assert torch.equal(st2.wavefield(1), ref_prev), r
    assert st2.next == p.nt
    # the state still steps eagerly after replays
    st2.begin(shot)
    tr = torch.zeros_like(ref_tr)
    for n in range(p.nt):
        st2.step(shot, n, tr[n])
    torch.cuda.synchronize()
    assert torch.equal(tr, ref_tr)


def test_replay_on_side_stream_reads_current_wavelet():
    import paper_2311_05038_amd as fd
    p = fi.surface2d(80, 150, 90, seed=32)
    model, state, shot = setup(p)
    ref = model.run_shot(model.new_state(), shot).clone()
    g = fd.ShotGraph(model, state, shot)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out = g.launch(stream=side)
    side.synchronize()
    assert torch.equal(out, ref)
    shot.wavelet.mul_(2.0)                       # same buffer, new contents
    torch.cuda.synchronize()
    out = g.launch()
    torch.cuda.synchronize()
    # the scheme is linear in the source: twice the wavelet gives twice the
    # traces (to FP32 rounding, which subnormal intermediates break exactly);
    # a replay that read the old wavelet would be off by one half
    assert rel_l2(out.cpu().numpy(), 2.0 * ref.cpu().numpy()) <= 1e-6
    assert float(ref.abs().max()) > 0


def test_recording_a_slab_is_refused():
    import paper_2311_05038_amd as fd
    p = fi.layered3d(nx=64, ny=32, nz=48, nt=10)
    g0 = fd.Grid(ndim=3, nz=48, ny=32, nx=64, dh=p.dh, dt=p.dt).slabs([24, 24])[0]
    v = torch.full((g0.ncells,), 2000.0, device="cuda")
    m = fd.Model(g0, v)
    wav = torch.from_numpy(p.wavelet()).cuda()
    with pytest.raises(fd.FDError) as e:
        fd.ShotGraph(m, m.new_state(), fd.Shot(p.src, wav, fd.Receivers(0, 0, 0, 1, 1, 4)))
    assert e.value.status == fd._abi.FD_ERR_UNSUPPORTED


def test_recording_before_any_eager_step_in_a_fresh_process():
    """A process whose first 3D step is a recording: the step's launch plan
    (an occupancy query, cached per process) is settled before the capture."""
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    code = f"""
import sys
sys.path.insert(0, {os.path.dirname(here)!r}); sys.path.insert(0, {here!r})
import torch
import fd_inputs as fi
import paper_2311_05038_amd as fd
from helpers import setup
p = fi.layered3d(nx=72, ny=40, nz=44, nt=30)
model, state, shot = setup(p)
g = fd.ShotGraph(model, state, shot)
out = g.launch().clone()
ref = model.run_shot(model.new_state(), shot)
torch.cuda.synchronize()
assert torch.equal(out, ref)
print("recorded-first ok", flush=True)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "recorded-first ok" in r.stdout


def test_noalloc_routine_step_first_used_under_capture():
    """A process that first calls fd_step_routines_noalloc inside a stream
    capture (torch.cuda.graph): the static area's address was settled when
    the model was created, so the capture holds plain kernel launches, and
    every replay gives the bits of the same steps run eagerly."""
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    code = f"""
import sys
sys.path.insert(0, {os.path.dirname(here)!r}); sys.path.insert(0, {here!r})
import torch
import fd_inputs as fi
from helpers import setup
p = fi.surface2d(64, 130, 12, seed=53)
model, state, shot = setup(p)
tr = torch.zeros((p.nt, p.receivers.count), device="cuda")
g = torch.cuda.CUDAGraph()
gs = torch.cuda.Stream()
gs.wait_stream(torch.cuda.current_stream())
with torch.cuda.stream(gs):
    with torch.cuda.graph(g, stream=gs):
        state.begin(shot, stream=gs)
        for n in range(p.nt):
            state.step_routines_noalloc(shot, n, tr[n], stream=gs)
torch.cuda.synchronize()
ref_state = model.new_state()
ref_tr = torch.zeros_like(tr)
ref_state.begin(shot)
for n in range(p.nt):
    ref_state.step_routines_noalloc(shot, n, ref_tr[n])
ref_f = ref_state.wavefield(0)
torch.cuda.synchronize()
for r in range(3):
    tr.zero_()
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(tr, ref_tr), r
    assert torch.equal(state.wavefield(0), ref_f), r
print("noalloc under capture ok", flush=True)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "noalloc under capture ok" in r.stdout
