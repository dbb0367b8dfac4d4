"""GPU reverse-time-migration image (fd_rtm_image) against the oracle.

The oracle's image (pinned by the scatterer dot-product test and central
differences) is the exact FP64 zero-lag correlation; the GPU recomputes the
source field in FP32 from checkpoints and sums in FP64, so the bound is FP32
rounding over the steps: relative L2 <= 1e-3.  Checkpointed and
single-segment images run the same kernels on the same states and must agree
bit for bit; the image is linear in the data and accumulates exactly.""" 
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import rel_l2, setup

pytestmark = pytest.mark.gpu


def _image_gpu(p, v, data, every):
    model, state, shot = setup(p, v)
    ck = model.checkpoint_buffer(p.nt, every)
    model.run_shot(state, shot, ckpt=ck, ckpt_every=every)
    img = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    d = torch.from_numpy(data.astype(np.float32)).cuda()
    model.rtm_image(shot, d, ck, every, img)
    torch.cuda.synchronize()
    return img.cpu().numpy().reshape(p.shape)


@pytest.mark.parametrize("ndim", [2, 3])
def test_image_matches_oracle(ndim):
    if ndim == 2:
        p = fi.surface2d(70, 90, 160, seed=81)
    else:
        p = fi.layered3d(nx=40, ny=36, nz=30, nt=60)
    v = fi.random_velocity(p.shape, 82, 2000, 3000)
    # data: the traces of a model with a reflector, as a shot record would be
    vr = v.copy()
    vr.reshape(p.nz, -1)[p.nz // 2:] *= 1.3
    obs = oracle.forward(oracle.grid_of(p), vr.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt,
                         p.src, p.rec_index())["traces"]
    img = _image_gpu(p, v, obs, 16)
    ref = oracle.image(oracle.grid_of(p), v.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt, p.src,
                       p.rec_index(), obs.astype(np.float32).astype(np.float64))
    err = rel_l2(img, ref.reshape(img.shape))
    print(f"{p.name} image relL2 {err:.3e}", flush=True)
    assert err <= 1e-3


def test_image_checkpointed_equals_single_segment_bitwise():
    p = fi.surface2d(48, 70, 90, seed=83)
    v = fi.random_velocity(p.shape, 84, 2000, 3000)
    d = np.random.default_rng(10).standard_normal((p.nt, p.receivers.count)).astype(np.float32)
    a = _image_gpu(p, v, d, 7)
    b = _image_gpu(p, v, d, p.nt)
    assert np.array_equal(a, b)


def test_image_linear_in_data_and_accumulates():
    p = fi.surface2d(40, 48, 50, seed=85)
    v = fi.random_velocity(p.shape, 86, 2000, 3000)
    rng = np.random.default_rng(11)
    d1 = rng.standard_normal((p.nt, p.receivers.count)).astype(np.float32)
    i1 = _image_gpu(p, v, d1, 10)
    # scaling the data by 2 scales every FP32 value by 2 exactly, except where
    # the receiver field decays into FP32 subnormals (rounded at a fixed
    # absolute step), which carry a negligible part of the image
    i2 = _image_gpu(p, v, 2 * d1, 10)
    assert rel_l2(i2, 2 * i1) <= 1e-12
    model, state, shot = setup(p, v)
    ck = model.checkpoint_buffer(p.nt, 10)
    model.run_shot(state, shot, ckpt=ck, ckpt_every=10)
    img = torch.zeros(p.ncells, dtype=torch.float64, device="cuda")
    dt = torch.from_numpy(d1).cuda()
    model.rtm_image(shot, dt, ck, 10, img)
    model.rtm_image(shot, dt, ck, 10, img)
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy().reshape(p.shape), 2 * i1)
