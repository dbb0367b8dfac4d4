"""z-slabs of one grid (fd_grid.slab_z0 / slab_nz_global, fd_slab_exchange):
the model cut along z into consecutive slabs, each with 4 ghost planes per
side, stepped slab by slab with a ghost exchange after every step, as one
device per slab would run it, against the whole grid on one device.

Every cell's update reads the same values in the same order whichever slab
holds it, and the damping factors are the whole grid's, so the stitched
traces and wavefields must equal the whole-grid results bit for bit; they
are also held to the FP32 parity bar (relative L2 <= 1e-4) against the FP64
oracle.  Cases: uneven slabs with damping on all six faces, slabs of the
minimum 4 planes (a ghost block is then a whole neighbour), the source on a
slab's first or last plane, receiver rows on every slab, ragged x and y."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import grid_of, receivers_of, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _slabs(p, v, counts):
    import paper_2311_05038_amd as fd
    vz = np.ascontiguousarray(v, dtype=np.float32).reshape(p.nz, p.ny, p.nx)
    shot = fd.Shot(p.src, torch.from_numpy(p.wavelet()).cuda(), receivers_of(p))
    models, states, z0 = [], [], 0
    for g in grid_of(p).slabs(counts):
        vt = torch.from_numpy(np.ascontiguousarray(vz[z0:z0 + g.nz]).reshape(-1)).cuda()
        models.append(fd.Model(g, vt))
        states.append(models[-1].new_state())
        z0 += g.nz
    return models, states, shot


def _run_slabs(p, v, counts):
    import paper_2311_05038_amd as fd
    models, states, shot = _slabs(p, v, counts)

    def exchange():
        for up, low in zip(states[:-1], states[1:]):
            fd.slab_exchange(up, low)

    for st in states:
        st.begin(shot)
    exchange()
    # NaN marks any trace entry that no slab writes
    tr = torch.full((p.nt, max(p.receivers.count, 1)), float("nan"), device="cuda")
    for n in range(p.nt):
        for st in states:
            st.step(shot, n, tr[n])
        exchange()
    cur = torch.cat([st.wavefield(0) for st in states], 0)
    old = torch.cat([st.wavefield(1) for st in states], 0)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), cur.cpu().numpy(), old.cpu().numpy()


def _whole(p, v):
    from helpers import setup
    model, state, shot = setup(p, v)
    tr = model.run_shot(state, shot)
    cur, old = state.wavefield(0), state.wavefield(1)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), cur.cpu().numpy(), old.cpu().numpy()


def _check(p, v, counts):
    print(f"case {p.name} shape={p.shape} nt={p.nt} slabs={counts} src={p.src}", flush=True)
    tr_s, cur_s, old_s = _run_slabs(p, v, counts)
    tr_w, cur_w, old_w = _whole(p, v)
    assert not np.isnan(tr_s).any()
    assert np.array_equal(tr_s, tr_w)
    assert np.array_equal(cur_s, cur_w)
    assert np.array_equal(old_s, old_w)
    ref = oracle.forward(oracle.grid_of(p), v.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt,
                         p.src, p.rec_index())
    e_tr = rel_l2(tr_s, ref["traces"])
    e_f = rel_l2(cur_s, ref["cur"].reshape(cur_s.shape))
    print(f"{p.name} vs FP64: traces {e_tr:.3e} field {e_f:.3e}", flush=True)
    assert e_tr <= TOL and e_f <= TOL


def test_uneven_slabs_all_faces_damped():
    p = fi.Problem(name="slab3d", ndim=3, nz=45, ny=41, nx=72, dh=10.0, dt=1e-3, nt=70,
                   src=(15, 20, 35), receivers=fi.Receivers(2, 1, 3, 9, 5, 17, 5, 8, 4),
                   f0=20.0, sponge_width=6, sponge_faces=fi.FACES_ALL)
    v = fi.random_velocity(p.shape, 91, 1500, 4000)
    _check(p, v, [15, 14, 16])


def test_minimum_slabs_source_on_last_plane():
    p = fi.Problem(name="slab4", ndim=3, nz=20, ny=24, nx=70, dh=10.0, dt=1e-3, nt=50,
                   src=(11, 12, 30), receivers=fi.Receivers(0, 0, 5, 7, 3, 12, 3, 10, 5),
                   f0=25.0, sponge_width=4, sponge_faces=fi.FACES_NO_TOP)
    v = fi.random_velocity(p.shape, 92, 1500, 4000)
    _check(p, v, [4, 4, 4, 8])


def test_slab_call_errors():
    import paper_2311_05038_amd as fd
    p = fi.layered3d(nx=40, ny=20, nz=24, nt=10)
    v = p.velocity()
    models, states, shot = _slabs(p, v, [12, 12])
    with pytest.raises(fd.FDError) as e:
        fd.slab_exchange(states[0], states[1])          # no shot begun
    assert e.value.status == fd._abi.FD_ERR_INVALID_ARG
    for st in states:
        st.begin(shot)
    with pytest.raises(fd.FDError) as e:
        fd.slab_exchange(states[1], states[0])          # not upper then lower
    assert e.value.status == fd._abi.FD_ERR_INVALID_ARG
    states[0].step(shot, 0)
    with pytest.raises(fd.FDError) as e:
        fd.slab_exchange(states[0], states[1])          # different steps
    assert e.value.status == fd._abi.FD_ERR_INVALID_ARG
    with pytest.raises(fd.FDError) as e:
        models[1].run_shot(states[1], shot)             # whole-shot calls: unsupported
    assert e.value.status == fd._abi.FD_ERR_UNSUPPORTED
    torch.cuda.synchronize()


def test_512_cube_in_8_slabs_equals_whole_grid():
    """The headline grid (512^3, layered, 32-cell sponge, 256x256 receivers)
    cut into the 8 slabs of 64 planes the bench times one of, 60 steps: the
    whole traces and both levels, compared on the device, bit for bit."""
    import paper_2311_05038_amd as fd
    p = fi.layered3d(nt=60)
    v = p.velocity()
    print(f"case {p.name} nt={p.nt} slabs=8x64", flush=True)
    models, states, shot = _slabs(p, v, [64] * 8)

    def exchange():
        for up, low in zip(states[:-1], states[1:]):
            fd.slab_exchange(up, low)

    for st in states:
        st.begin(shot)
    exchange()
    tr = torch.full((p.nt, p.receivers.count), float("nan"), device="cuda")
    for n in range(p.nt):
        for st in states:
            st.step(shot, n, tr[n])
        exchange()
    cur = torch.cat([st.wavefield(0) for st in states], 0)
    old = torch.cat([st.wavefield(1) for st in states], 0)
    del states, models
    from helpers import setup
    model, state, wshot = setup(p, v)
    tw = model.run_shot(state, wshot)
    assert torch.equal(tr, tw)
    assert torch.equal(cur, state.wavefield(0))
    assert torch.equal(old, state.wavefield(1))
    assert float(cur.abs().max()) > 0
    torch.cuda.synchronize()
