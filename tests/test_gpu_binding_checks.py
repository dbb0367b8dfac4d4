"""The Python binding hands the C calls raw device addresses, which carry no
size; it checks every buffer a caller supplies (device, element type,
contiguity, element count) and raises ValueError before anything is
launched.  Each case here passes one bad buffer and checks that the error
comes and that the state and the caller's tensors are untouched."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import setup

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prob():
    p = fi.surface2d(64, 96, 40, seed=5)
    model, state, shot = setup(p)
    return p, model, state, shot


def _bad_traces(p):
    nt, nrec = p.nt, p.receivers.count
    return {
        "short": torch.zeros(nt * nrec - 1, device="cuda"),
        "fp64": torch.zeros((nt, nrec), dtype=torch.float64, device="cuda"),
        "strided": torch.zeros((nrec, nt), device="cuda").t(),
        "host": torch.zeros((nt, nrec)),
    }


@pytest.mark.parametrize("kind", ["short", "fp64", "strided", "host"])
def test_run_shot_traces_checked(prob, kind):
    p, model, state, shot = prob
    print(f"run_shot traces {kind}", flush=True)
    state.begin(shot)
    before = state.wavefield(0).clone()
    bad = _bad_traces(p)[kind]
    keep = bad.clone()
    with pytest.raises(ValueError):
        model.run_shot(state, shot, bad)
    torch.cuda.synchronize()
    assert torch.equal(bad, keep)
    assert torch.equal(state.wavefield(0), before)


def test_step_row_and_wavefield_checked(prob):
    p, model, state, shot = prob
    state.begin(shot)
    before = state.wavefield(0).clone()
    with pytest.raises(ValueError):
        state.step(shot, 0, torch.zeros(p.receivers.count - 1, device="cuda"))
    with pytest.raises(ValueError):
        state.step_routines_noalloc(shot, 0, torch.zeros(p.receivers.count, dtype=torch.float16,
                                                         device="cuda"))
    with pytest.raises(ValueError):
        state.wavefield(0, out=torch.empty(int(np.prod(p.shape)) - 1, device="cuda"))
    with pytest.raises(ValueError):
        state.set_wavefield(0, torch.zeros(p.shape))
    with pytest.raises(ValueError):
        state.check_finite(torch.zeros(1, dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(state.wavefield(0), before)
    assert state.next == 0


def test_backward_inputs_checked(prob):
    import paper_2311_05038_amd as fd
    p, model, state, shot = prob
    every = 8
    sz = model.sizes_for(p.nt, every)
    ckpt = model.checkpoint_buffer(p.nt, every)
    tr = model.run_shot(state, shot, None, ckpt, every).clone()
    grad = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        model.adjoint_gradient(shot, tr.flatten()[:-1], ckpt, every, grad)
    # a short checkpoint buffer: its byte count goes to the library, which refuses it
    with pytest.raises(fd.FDError):
        model.rtm_image(shot, tr, ckpt[:-1], every, grad,
                        torch.empty(sz.adjoint_work, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert not grad.any()
    # and a good call still works after the refusals
    model.adjoint_gradient(shot, tr, ckpt, every, grad)
    torch.cuda.synchronize()
    assert torch.isfinite(grad).all() and grad.abs().max() > 0


def test_multi_shot_lists_checked(prob):
    p, model, state, shot = prob
    states = [model.new_state(), model.new_state()]
    with pytest.raises(ValueError):
        model.run_shots(states[:1], [shot, shot])
    with pytest.raises(ValueError):
        model.run_shots(states, [shot, shot],
                        torch.zeros((2, p.nt, p.receivers.count - 1), device="cuda"))
