"""GPU parity of the fused FP32 step against the FP64 oracle, through the C ABI.

Bar: relative L2 error <= 1e-4 on traces and final wavefield (FP32
arithmetic against FP64; the scheme itself is identical, so the difference is
rounding only).  Grids cover several tiles and ragged tails in every axis,
strided receiver arrays, a receiver on the source cell, the 1-cell grid, and
shots without receivers."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import rel_l2, run, setup

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _oracle(p, v=None):
    v = p.velocity() if v is None else v
    return oracle.forward(oracle.grid_of(p), v.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt,
                          p.src, p.rec_index())


def _check(p, v=None, tol=TOL):
    print(f"case {p.name} shape={p.shape} nt={p.nt}", flush=True)
    tr, cur = run(p, v)
    ref = _oracle(p, v)
    e_tr = rel_l2(tr[:, : p.receivers.count], ref["traces"]) if p.receivers.count else 0.0
    e_f = rel_l2(cur, ref["cur"].reshape(cur.shape))
    assert e_tr <= tol and e_f <= tol, (p.name, e_tr, e_f)
    return tr, cur


def test_green2d_full_size_parity():
    tr, cur = _check(fi.green2d())
    assert np.abs(cur).max() > 0


def test_green2d_d4_symmetry():
    p = fi.green2d()
    _, cur = run(p)
    c = cur[128 - 100:128 + 101, 128 - 100:128 + 101]
    scale = np.abs(c).max()
    for t in (c[::-1, :], c[:, ::-1], c.T, c[::-1, ::-1].T):
        assert np.abs(c - t).max() <= 1e-6 * scale


def test_2d_ragged_tiles_sponge_strided_receivers():
    p = fi.Problem(name="ragged2d", ndim=2, nz=70, ny=1, nx=133, dh=10.0, dt=1e-3, nt=160,
                   src=(31, 0, 67), receivers=fi.Receivers(3, 0, 1, 4, 1, 40, 5, 1, 3), f0=18.0,
                   sponge_width=9, sponge_faces=fi.FACES_ALL)
    _check(p, fi.random_velocity(p.shape, 3, 1500, 4000))


def test_2d_receiver_on_source_and_edges():
    p = fi.Problem(name="edge2d", ndim=2, nz=33, ny=1, nx=65, dh=10.0, dt=1e-3, nt=90,
                   src=(0, 0, 64), receivers=fi.Receivers(0, 0, 0, 1, 1, 65), f0=20.0)
    tr, _ = _check(p, fi.random_velocity(p.shape, 4, 1500, 3000))


def test_2d_no_receivers():
    p = fi.Problem(name="norec2d", ndim=2, nz=40, ny=1, nx=50, dh=10.0, dt=1e-3, nt=50,
                   src=(20, 0, 25), receivers=fi.Receivers(0, 0, 0, 0, 0, 0), f0=20.0)
    _check(p)


def test_3d_layered_small():
    _check(fi.layered3d(nx=64, ny=64, nz=64, nt=80))


def test_3d_ragged_all_axes():
    p = fi.Problem(name="ragged3d", ndim=3, nz=37, ny=29, nx=71, dh=10.0, dt=1e-3, nt=60,
                   src=(18, 14, 35), receivers=fi.Receivers(2, 3, 5, 2, 6, 20, 7, 4, 3),
                   f0=20.0, sponge_width=5, sponge_faces=fi.FACES_ALL)
    _check(p, fi.random_velocity(p.shape, 5, 1500, 3500))


def test_3d_tile_multiples_and_deep_chunks():
    # 2 x-tiles, 3 y-tiles, z longer than one z-chunk with a ragged tail.
    p = fi.layered3d(nx=128, ny=48, nz=150, nt=40)
    _check(p)


def test_3d_short_column_in_short_chunks():
    # 18 planes under 18 column tiles: the plan cuts each column into chunks
    # of 5, 5, 5 and a ragged 3 (chunks down to 4 planes keep short columns
    # filling the device)
    p = fi.Problem(name="short3d", ndim=3, nz=18, ny=70, nx=300, dh=10.0, dt=1e-3, nt=40,
                   src=(9, 35, 150), receivers=fi.Receivers(1, 2, 3, 4, 7, 30, 5, 10, 10),
                   f0=25.0, sponge_width=3, sponge_faces=fi.FACES_ALL)
    _check(p, fi.random_velocity(p.shape, 6, 1500, 3500))


def test_single_cell_grids():
    for ndim in (2, 3):
        p = fi.Problem(name=f"one{ndim}", ndim=ndim, nz=1, ny=1, nx=1, dh=10.0, dt=1e-3, nt=20,
                       src=(0, 0, 0), receivers=fi.Receivers(0, 0, 0, 1, 1, 1), f0=25.0)
        _check(p, np.full(p.shape, 2000.0, np.float32))


def test_step_by_step_equals_run_shot_bitwise():
    for p in (fi.green2d().scaled(nt=60), fi.layered3d(nx=64, ny=32, nz=70, nt=30)):
        model, state, shot = setup(p)
        tr_run = model.run_shot(state, shot).clone()
        cur_run = state.wavefield(0).clone()
        state.begin(shot)
        tr_step = torch.empty_like(tr_run)
        for n in range(p.nt):
            state.step(shot, n, tr_step[n])
        cur_step = state.wavefield(0)
        torch.cuda.synchronize()
        assert torch.equal(tr_run, tr_step)
        assert torch.equal(cur_run, cur_step)


def test_runs_are_deterministic():
    p = fi.layered3d(nx=64, ny=64, nz=64, nt=40)
    a = run(p)
    b = run(p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_pold_level_matches_oracle():
    p = fi.surface2d(64, 96, 70, seed=2)
    model, state, shot = setup(p)
    model.run_shot(state, shot)
    prev = state.wavefield(1).cpu().numpy()
    ref = _oracle(p)
    assert rel_l2(prev, ref["prev"].reshape(prev.shape)) <= TOL


def _energy(g, prev, cur, c):
    Lp = oracle.laplacian(g, prev.astype(np.float64))
    return float(np.sum((cur.astype(np.float64) - prev) ** 2 / c) - np.sum(cur * Lp))


def test_discrete_energy_conserved_3d():
    """No damping, no source, zero edges: the leapfrog energy
    sum (u^{n+1}-u^n)^2/c - sum u^{n+1} L u^n is constant; in FP32 it drifts
    only by rounding."""
    import paper_2311_05038_amd as fd
    n = 96
    p = fi.Problem(name="energy3d", ndim=3, nz=n, ny=n, nx=n, dh=10.0, dt=1e-3, nt=400,
                   src=(0, 0, 0), receivers=fi.Receivers(0, 0, 0, 0, 0, 0), f0=10.0,
                   sponge_width=0)
    v = fi.random_velocity(p.shape, 14, 1500, 4500)
    model, state, _ = setup(p, v)
    zc = np.arange(n) - n / 2
    Z, Y, X = np.meshgrid(zc, zc, zc, indexing="ij")
    u0 = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / 25.0).astype(np.float32)
    state.set_wavefield(0, torch.from_numpy(u0.ravel()).cuda())
    state.set_wavefield(1, torch.from_numpy(u0.ravel()).cuda())
    shot = fd.Shot((0, 0, 0), torch.zeros(p.nt, device="cuda"), fd.Receivers())
    g = oracle.grid_of(p)
    c, _ = oracle.setup(g, v)
    Es = []
    for n_ in range(p.nt):
        state.step(shot, n_)
        if n_ % 100 == 99:
            cur = state.wavefield(0).cpu().numpy()
            prev = state.wavefield(1).cpu().numpy()
            Es.append(_energy(g, prev, cur, c))
    Es = np.array(Es)
    print("energy", Es, flush=True)
    assert np.all(Es > 0)
    assert np.abs(Es - Es[0]).max() <= 1e-4 * Es[0]


def test_layered3d_512_full_size_against_stored_oracle():
    """The 512^3 / 1000-step workload in the launch configuration the
    benchmark times, against FP64 oracle values stored by
    tests/golden/make_golden.py: sampled receivers over all steps, sampled
    final-field cells, and 16^3 block sums of the final field."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "layered3d_512.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    gold = np.load(path)
    p = fi.layered3d()
    tr, cur = run(p)
    e_tr = rel_l2(tr[:, gold["traces_idx"]], gold["traces"])
    e_cells = rel_l2(cur.ravel()[gold["cells_idx"]], gold["cells"])
    b = 16
    blocks = cur.reshape(p.nz // b, b, p.ny // b, b, p.nx // b, b).astype(np.float64).sum(axis=(1, 3, 5))
    e_blocks = rel_l2(blocks, gold["blocks"])
    e_norm_f = abs(np.linalg.norm(cur.astype(np.float64)) / float(gold["field_norm"]) - 1)
    e_norm_t = abs(np.linalg.norm(tr.astype(np.float64)) / float(gold["trace_norm"]) - 1)
    print("512^3 errors", e_tr, e_cells, e_blocks, e_norm_f, e_norm_t, flush=True)
    assert max(e_tr, e_cells, e_blocks, e_norm_f, e_norm_t) <= TOL
