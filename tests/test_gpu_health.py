"""fd_check_finite on the GPU: a healthy shot reports 0; a NaN or an infinity
planted in P through fd_set_wavefield is reported at once (bit 0 for the
level, bit 2 for the non-finite input) and, after more steps, in both levels
(bits 0 and 1) with every storage kind, where non-finite values persist
(16-bit codes decode exactly, non-finite ones included); 2D and 3D, and a z-slab; a
non-finite wavelet sample sets bit 2 at fd_begin_shot; in the shot server, a
shot whose wavelet carries a NaN fails alone while the other shots of the mix
finish with the bits they have alone.  Nothing here makes a kernel fault: the
values are planted from the host side through the library's own calls."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import grid_of, receivers_of, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_planted_nonfinite_is_reported(storage, ndim, bad):
    p = fi.surface2d(70, 150, 30, seed=3) if ndim == 2 else fi.layered3d(nx=72, ny=40, nz=36, nt=30)
    print(f"case {p.name} storage={storage} bad={bad}", flush=True)
    model, state, shot = setup(p, storage=storage)
    model.run_shot(state, shot)
    assert int(state.check_finite().item()) == 0
    assert state.is_finite()
    st = model.new_state()
    st.begin(shot)
    for n in range(6):
        st.step(shot, n)
    f = st.wavefield(0).clone().reshape(-1)
    f[f.numel() // 3] = bad
    st.set_wavefield(0, f.reshape(st.wavefield(0).shape))
    assert int(st.check_finite().item()) == 5
    for n in range(6, 12):
        st.step(shot, n)
    flags = int(st.check_finite().item())
    assert flags == 7
    assert not st.is_finite()
    # a fresh shot clears the flags; a non-finite wavelet sample sets bit 2
    st.begin(shot)
    assert int(st.check_finite().item()) == 0
    w = shot.wavelet.clone()
    w[p.nt // 2] = bad
    import paper_2311_05038_amd as fd
    bad_shot = fd.Shot(p.src, w, receivers_of(p))
    st.begin(bad_shot)
    assert int(st.check_finite().item()) == 4


def test_slab_reports_only_its_own_planes():
    import paper_2311_05038_amd as fd
    p = fi.layered3d(nx=64, ny=40, nz=48, nt=20)
    v = p.velocity()
    wav = torch.from_numpy(p.wavelet()).cuda()
    states, models, z0 = [], [], 0
    for g in grid_of(p).slabs([24, 24]):
        m = fd.Model(g, torch.from_numpy(np.ascontiguousarray(v[z0:z0 + g.nz]).ravel()).cuda())
        models.append(m)
        states.append(m.new_state())
        z0 += g.nz
    shot = fd.Shot(p.src, wav, receivers_of(p))
    for s in states:
        s.begin(shot)
    f = states[1].wavefield(0).clone()
    f[5, 7, 9] = float("nan")
    states[1].set_wavefield(0, f)
    assert int(states[0].check_finite().item()) == 0
    assert int(states[1].check_finite().item()) == 5


def test_serving_isolates_a_nonfinite_shot():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.serve import Request, Scheduler, TorchDevice
    reqs_in = fi.serving_stream(8, seed=11, rate=400.0, nz_range=(64, 160), nx_range=(64, 240),
                                nt_range=(40, 120))
    poisoned = reqs_in[3].rid

    def make_inputs(req):
        p = fi.surface2d(req.nz, req.nx, req.nt, req.rid)
        v = torch.from_numpy(fi.grf_velocity((req.nz, req.nx), req.rid, corr_cells=6.0).ravel()).cuda()
        w = p.wavelet().copy()
        if req.rid == poisoned:
            w[10] = np.nan
        shot = fd.Shot(p.src, torch.from_numpy(w).cuda(), receivers_of(p))
        return grid_of(p), v, shot

    reqs = [Request(r.rid, r.arrival, r.nz, r.nx, r.nt) for r in reqs_in]
    sch = Scheduler(TorchDevice(make_inputs, batched=True, keep_traces=True), max_slots=4,
                    hbm_budget=1 << 34, chunk=9)
    out = sch.run(reqs)
    for r in reqs:
        o = out[r.rid]
        if r.rid == poisoned:
            assert o.status.startswith("failed") and "non-finite" in o.status, o.status
            continue
        assert o.status == "ok", (r.rid, o.status)
        g, v, shot = make_inputs(r)
        m = fd.Model(g, v)
        alone = m.run_shot(m.new_state(), shot)
        torch.cuda.synchronize()
        assert torch.equal(o.result, alone), r.rid
