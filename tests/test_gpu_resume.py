"""Stopping a shot and resuming it elsewhere (through the C ABI): both
levels read back with fd_get_wavefield and copied to the host after k steps,
a fresh state (of a fresh model) given them with fd_set_wavefield, and the
rest of the shot run with a shot whose wavelet starts at sample k.  With
FP32 storage the resumed traces and final levels equal the uninterrupted
shot's bit for bit, in 2D and 3D, for k anywhere in the shot."""
import pytest
import torch

import fd_inputs as fi
from helpers import receivers_of, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case,k", [("2d", 1), ("2d", 37), ("3d", 20), ("3d", 59)])
def test_resume_from_host_snapshot_is_bitwise(case, k):
    import paper_2311_05038_amd as fd
    p = fi.surface2d(90, 170, 120, seed=51) if case == "2d" else fi.layered3d(nx=80, ny=44, nz=52, nt=60)
    print(f"case {p.name} shape={p.shape} nt={p.nt} stop after {k}", flush=True)
    model, state, shot = setup(p)
    ref_tr = model.run_shot(state, shot).clone()
    ref_cur, ref_prev = state.wavefield(0).clone(), state.wavefield(1).clone()

    st = model.new_state()
    st.begin(shot)
    tr = torch.zeros_like(ref_tr)
    for n in range(k):
        st.step(shot, n, tr[n])
    snap = (st.wavefield(0).cpu(), st.wavefield(1).cpu(), tr[:k].cpu())
    torch.cuda.synchronize()
    del st

    model2, st2, _ = setup(p)
    st2.set_wavefield(0, snap[0].cuda())
    st2.set_wavefield(1, snap[1].cuda())
    rest = fd.Shot(p.src, shot.wavelet[k:].contiguous(), receivers_of(p))
    tr2 = torch.zeros((p.nt - k, p.receivers.count), device="cuda")
    for n in range(p.nt - k):
        st2.step(rest, n, tr2[n])
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([snap[2].cuda(), tr2]), ref_tr)
    assert torch.equal(st2.wavefield(0), ref_cur)
    assert torch.equal(st2.wavefield(1), ref_prev)
