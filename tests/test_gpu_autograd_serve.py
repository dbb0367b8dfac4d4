"""torch.autograd binding of the adjoint, and the shot server on the GPU.

* FDTraces: backward of sum(w * traces) equals the oracle's exact discrete
  adjoint gradient (relL2 <= 1e-3), and a central finite difference of the
  GPU forward map along a random direction agrees with <grad, dv>.
* Serving: each shot's traces and final field are the same in the batched
  mix as when run alone (bitwise: same kernel body, no cross-shot data), and
  the server never exceeds its slots."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import grid_of, receivers_of, rel_l2

pytestmark = pytest.mark.gpu


def _shots(ps):
    import paper_2311_05038_amd as fd
    return [fd.Shot(p.src, torch.from_numpy(p.wavelet()).cuda(), receivers_of(p)) for p in ps]


def test_autograd_backward_matches_oracle_adjoint():
    from paper_2311_05038_amd.autograd import FDTraces
    ps = [fi.surface2d(60, 80, 140, seed=41, src_x=x) for x in (20, 60)]
    p = ps[0]
    v = fi.random_velocity(p.shape, 42, 2000, 3000)
    vt = torch.from_numpy(v.ravel()).cuda().requires_grad_(True)
    w = torch.from_numpy(np.random.default_rng(1).standard_normal(
        (2, p.nt, p.receivers.count)).astype(np.float32)).cuda()
    tr = FDTraces.apply(vt, grid_of(p), _shots(ps), 13)
    (tr * w).sum().backward()
    g = vt.grad.detach().cpu().numpy().astype(np.float64)
    ref = np.zeros(p.ncells)
    for i, q in enumerate(ps):
        gv, _ = oracle.adjoint(oracle.grid_of(q), v.reshape(q.nz, 1, q.nx), q.wavelet(), q.nt,
                               q.src, q.rec_index(), w[i].cpu().numpy().astype(np.float64))
        ref += gv.ravel()
    err = rel_l2(g, ref)
    print("autograd gradient relL2", err, flush=True)
    assert err <= 1e-3


def test_gradient_against_finite_differences_of_gpu_forward():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.autograd import l2_misfit_gradient
    p = fi.surface2d(64, 96, 200, seed=43)
    vtrue = fi.grf_velocity(p.shape, 44, corr_cells=8.0)
    v0 = fi.gradient_velocity(p.shape)
    grid = grid_of(p)
    shots = _shots([p])
    m = fd.Model(grid, torch.from_numpy(vtrue.ravel()).cuda())
    obs = m.run_shot(m.new_state(), shots[0]).clone()[None]
    v0t = torch.from_numpy(v0.ravel()).cuda()
    J0, g = l2_misfit_gradient(v0t, grid, shots, obs, 20)
    dv = torch.from_numpy(fi.perturbation(p.shape, 45, 5.0).ravel().astype(np.float32)).cuda()
    an = float((g * dv.double()).sum())
    h = 1.0
    Jp, _ = l2_misfit_gradient(v0t + h * dv, grid, shots, obs, 20)
    Jm, _ = l2_misfit_gradient(v0t - h * dv, grid, shots, obs, 20)
    fdv = (Jp - Jm) / (2 * h)
    print("directional derivative: adjoint", an, "central FD", fdv, flush=True)
    assert abs(fdv - an) <= 1e-2 * abs(an)


def test_shot_groups_equal_single_shot_calls():
    """The multi-shot calls (one launch per step for a group of shots) give
    each shot the bits of the single-shot calls: traces, checkpoints, and
    gradient/image sums taken shot after shot in the same order."""
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.autograd import l2_misfit_gradient, rtm_image
    ps = [fi.surface2d(60, 80, 120, seed=47, src_x=x) for x in (10, 30, 50, 70, 40)]
    p = ps[0]
    grid = grid_of(p)
    vtrue = fi.grf_velocity(p.shape, 48, corr_cells=8.0)
    v0 = torch.from_numpy(fi.gradient_velocity(p.shape).ravel()).cuda()
    shots = _shots(ps)
    m = fd.Model(grid, torch.from_numpy(vtrue.ravel()).cuda())
    st = m.new_state()
    obs = torch.stack([m.run_shot(st, s).clone() for s in shots])
    # forward: grouped vs one by one, with checkpoints
    m0 = fd.Model(grid, v0)
    states = [m0.new_state() for _ in shots]
    ck_a = [m0.checkpoint_buffer(p.nt, 16) for _ in shots]
    tr_a = m0.run_shots(states, shots, None, ck_a, 16)
    s1 = m0.new_state()
    for i, s in enumerate(shots):
        ck = m0.checkpoint_buffer(p.nt, 16)
        tr = m0.run_shot(s1, s, ckpt=ck, ckpt_every=16)
        torch.cuda.synchronize()
        assert torch.equal(tr, tr_a[i]), i
        assert torch.equal(ck, ck_a[i]), i
        assert torch.equal(s1.wavefield(0), states[i].wavefield(0)), i
    # gradient and image: groups of 3 (and a group of 2) vs one shot per call
    J1, g1 = l2_misfit_gradient(v0, grid, shots, obs, 16, group=1)
    J3, g3 = l2_misfit_gradient(v0, grid, shots, obs, 16, group=3)
    torch.cuda.synchronize()
    assert torch.equal(g3, g1)
    assert abs(J3 - J1) <= 1e-13 * abs(J1)
    i1 = rtm_image(v0, grid, shots, obs, 16, group=1)
    i3 = rtm_image(v0, grid, shots, obs, 16, group=3)
    torch.cuda.synchronize()
    assert torch.equal(i3, i1)


@pytest.mark.parametrize("policy,launch_cells", [("all", 1 << 24), ("srpt", 1 << 14),
                                                 ("srpt_oldest", 1 << 14)])
def test_serving_mix_equals_alone_bitwise(policy, launch_cells):
    # "srpt" with a small cell budget pauses and resumes shots between chunks
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd.serve import Request, Scheduler, TorchDevice
    reqs_in = fi.serving_stream(10, seed=7, rate=400.0, nz_range=(64, 200), nx_range=(64, 300),
                                nt_range=(60, 200))
    base = {r.rid: fi.grf_velocity((r.nz, r.nx), r.seed, corr_cells=6.0) for r in reqs_in}

    def make_inputs(req):
        p = fi.surface2d(req.nz, req.nx, req.nt, req.rid)
        v = torch.from_numpy(base[req.rid].ravel()).cuda()
        return grid_of(p), v, _shots([p])[0]

    reqs = [Request(r.rid, r.arrival, r.nz, r.nx, r.nt) for r in reqs_in]
    sch = Scheduler(TorchDevice(make_inputs, batched=True, keep_traces=True), max_slots=4,
                    hbm_budget=1 << 34, chunk=7, policy=policy, launch_cells=launch_cells)
    out = sch.run(reqs)
    assert sch.peak_slots <= 4
    for r in reqs:
        o = out[r.rid]
        assert o.status == "ok", o.status
        g, v, shot = make_inputs(r)
        m = fd.Model(g, v)
        alone = m.run_shot(m.new_state(), shot)
        torch.cuda.synchronize()
        assert torch.equal(o.result, alone), r.rid


def test_more_shots_than_one_launch_holds():
    """18 shots in one multi-shot call (two launches per step: 16 + 2) give
    every shot the bits of its own single-shot call: traces, checkpoints,
    the gradient and the image summed shot after shot."""
    import paper_2311_05038_amd as fd
    ps = [fi.surface2d(24, 40, 40, seed=60, src_x=2 + 2 * i) for i in range(18)]
    p = ps[0]
    grid = grid_of(p)
    v = torch.from_numpy(fi.random_velocity(p.shape, 61, 2000, 3000).ravel()).cuda()
    m = fd.Model(grid, v)
    shots = _shots(ps)
    every = 7
    states = [m.new_state() for _ in shots]
    cks = [m.checkpoint_buffer(p.nt, every) for _ in shots]
    tr = m.run_shots(states, shots, None, cks, every)
    rng = np.random.default_rng(62)
    adj = [torch.from_numpy(rng.standard_normal((p.nt, p.receivers.count)).astype(np.float32)).cuda()
           for _ in shots]
    g_all = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    m.adjoint_gradient_shots(shots, adj, cks, every, g_all)
    i_all = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    m.rtm_image_shots(shots, adj, cks, every, i_all)
    g_one = torch.zeros_like(g_all)
    i_one = torch.zeros_like(i_all)
    st = m.new_state()
    for k, s in enumerate(shots):
        ck = m.checkpoint_buffer(p.nt, every)
        t = m.run_shot(st, s, ckpt=ck, ckpt_every=every)
        torch.cuda.synchronize()
        assert torch.equal(t, tr[k]), k
        assert torch.equal(ck, cks[k]), k
        m.adjoint_gradient(s, adj[k], ck, every, g_one)
        m.rtm_image(s, adj[k], ck, every, i_one)
    torch.cuda.synchronize()
    assert torch.equal(g_all, g_one)
    assert torch.equal(i_all, i_one)
