"""GPU velocity gradient (checkpointed discrete adjoint) against the oracle.

The oracle's gradient is the exact discrete adjoint in FP64 (pinned by the
dot-product and finite-difference tests); the GPU runs FP32 fields with an
FP64 time sum, so the bound is FP32 rounding accumulated over the steps:
relative L2 <= 1e-3.  Checkpointed and single-segment gradients run the same
kernels on the same states and must agree bit for bit."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import rel_l2, setup

pytestmark = pytest.mark.gpu


def _grad_gpu(p, v, resid, every):
    model, state, shot = setup(p, v)
    ck = model.checkpoint_buffer(p.nt, every)
    model.run_shot(state, shot, ckpt=ck, ckpt_every=every)
    g = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    adj = torch.from_numpy(resid.astype(np.float32)).cuda()
    model.adjoint_gradient(shot, adj, ck, every, g)
    torch.cuda.synchronize()
    return g.cpu().numpy().reshape(p.shape)


@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_matches_oracle(ndim):
    if ndim == 2:
        p = fi.surface2d(70, 90, 160, seed=21)
    else:
        p = fi.layered3d(nx=40, ny=36, nz=30, nt=60)
    v = fi.random_velocity(p.shape, 22, 2000, 3000)
    resid = np.random.default_rng(3).standard_normal((p.nt, p.receivers.count)).astype(np.float32)
    g = _grad_gpu(p, v, resid, 16)
    gv, _ = oracle.adjoint(oracle.grid_of(p), v.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt,
                           p.src, p.rec_index(), resid.astype(np.float64))
    err = rel_l2(g, gv.reshape(g.shape))
    print("gradient relL2", err, flush=True)
    assert err <= 1e-3


@pytest.mark.parametrize("every", [5, 7, 8])
def test_checkpointed_equals_single_segment_bitwise(every):
    # adjoint steps update the FP64 sum in groups of three inside a segment;
    # segments of 5, 7 and 8 steps end in groups of two, one and two steps,
    # the single 90-step segment in a group of three: the sum is the same
    # sequence of FP64 operations whatever the grouping
    p = fi.surface2d(48, 70, 90, seed=23)
    v = fi.random_velocity(p.shape, 24, 2000, 3000)
    resid = np.random.default_rng(4).standard_normal((p.nt, p.receivers.count)).astype(np.float32)
    a = _grad_gpu(p, v, resid, every)
    b = _grad_gpu(p, v, resid, p.nt)
    assert np.array_equal(a, b)


def test_gradient_accumulates():
    p = fi.surface2d(40, 48, 50, seed=25)
    v = fi.random_velocity(p.shape, 26, 2000, 3000)
    resid = np.random.default_rng(5).standard_normal((p.nt, p.receivers.count)).astype(np.float32)
    model, state, shot = setup(p, v)
    ck = model.checkpoint_buffer(p.nt, 10)
    model.run_shot(state, shot, ckpt=ck, ckpt_every=10)
    g = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    adj = torch.from_numpy(resid).cuda()
    model.adjoint_gradient(shot, adj, ck, 10, g)
    g1 = g.clone()
    model.adjoint_gradient(shot, adj, ck, 10, g)
    torch.cuda.synchronize()
    assert torch.allclose(g, 2 * g1, rtol=1e-12, atol=0)


def test_full_size_gradient_against_stored_oracle():
    """The 1024^2 / 2000-step gradient model (shot 0, start model, K = 50 as
    in the benchmark) against the FP64 oracle gradient stored by
    tests/golden/make_golden.py for the same seeded adjoint source."""
    import os
    import sys
    path = os.path.join(os.path.dirname(__file__), "golden", "adjoint2d_1024.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle gradient not generated")
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import adjoint_residual
    gold = np.load(path)
    shots, _, v0 = fi.adjoint2d()
    p = shots[0]
    g = _grad_gpu(p, v0, adjoint_residual(p), 50)
    e_cells = rel_l2(g.ravel()[gold["cells_idx"]], gold["cells"])
    b = 16
    blocks = g.reshape(p.nz // b, b, p.nx // b, b).sum(axis=(1, 3))
    e_blocks = rel_l2(blocks, gold["blocks"])
    e_norm = abs(np.linalg.norm(g) / float(gold["grad_norm"]) - 1)
    print("1024^2 gradient errors", e_cells, e_blocks, e_norm, flush=True)
    assert max(e_cells, e_blocks, e_norm) <= 1e-3
