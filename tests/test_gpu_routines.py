"""The step as one kernel per routine (fd_step_routines: z, x [, y]
derivative fields materialised, then the time update, then the source
addition) against the fused step and against the oracle.

Both forms perform the same FP32 operations in the same order, so traces and
fields must agree bit for bit; the oracle bound is the FP32 one (relative L2
<= 1e-4).  Shapes are ragged (nx not a multiple of 64, chunks that do not
divide the axes) so the padding, halo and chunk edges are exercised."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
import oracle
from helpers import rel_l2, setup

pytestmark = pytest.mark.gpu


def _cases():
    return [fi.surface2d(75, 133, 90, seed=61),
            fi.green2d().scaled(nt=60),
            fi.layered3d(nx=72, ny=41, nz=45, nt=40),
            fi.layered3d(nx=130, ny=66, nz=70, nt=25)]


def _routines_shot(p):
    model, state, shot = setup(p)
    work = torch.empty(model.sizes.routines_work, dtype=torch.uint8, device="cuda")
    tr = torch.zeros((p.nt, p.receivers.count), device="cuda")
    state.begin(shot)
    for n in range(p.nt):
        state.step_routines(shot, n, work, tr[n])
    return tr, state.wavefield(0)


@pytest.mark.parametrize("case", range(4))
def test_routines_equal_fused_step_bitwise(case):
    p = _cases()[case]
    print(f"case {p.name} {p.shape} nt={p.nt}", flush=True)
    tr_r, f_r = _routines_shot(p)
    model, state, shot = setup(p)
    tr_f = model.run_shot(state, shot)
    f_f = state.wavefield(0)
    torch.cuda.synchronize()
    assert torch.equal(tr_r, tr_f)
    assert torch.equal(f_r, f_f)


@pytest.mark.parametrize("case", [0, 2])
def test_routines_match_oracle(case):
    p = _cases()[case]
    tr, f = _routines_shot(p)
    torch.cuda.synchronize()
    out = oracle.forward(oracle.grid_of(p), p.velocity().reshape(p.nz, p.ny, p.nx), p.wavelet(),
                         p.nt, p.src, p.rec_index())
    e_tr = rel_l2(tr.cpu().numpy(), out["traces"])
    e_f = rel_l2(f.cpu().numpy().reshape(-1), out["cur"].reshape(-1))
    print("routines vs oracle", e_tr, e_f, flush=True)
    assert e_tr <= 1e-4 and e_f <= 1e-4


def test_routines_argument_errors():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd._abi import FDError, FD_ERR_INVALID_ARG, FD_ERR_UNSUPPORTED
    p = fi.surface2d(40, 70, 10, seed=62)
    model, state, shot = setup(p)
    state.begin(shot)
    small = torch.empty(model.sizes.routines_work - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(FDError) as e:
        state.step_routines(shot, 0, small)
    assert e.value.status == FD_ERR_INVALID_ARG
    work = torch.empty(model.sizes.routines_work, dtype=torch.uint8, device="cuda")
    with pytest.raises(FDError) as e:          # not the state's next step
        state.step_routines(shot, 1, work)
    assert e.value.status == FD_ERR_INVALID_ARG
    m16, s16, sh16 = setup(p, storage=1)
    s16.begin(sh16)
    with pytest.raises(FDError) as e:
        s16.step_routines(sh16, 0, work)
    assert e.value.status == FD_ERR_UNSUPPORTED
    # the failed calls left the state where it was: step 0 still runs
    state.step_routines(shot, 0, work)
    torch.cuda.synchronize()
    assert state.next == 1
