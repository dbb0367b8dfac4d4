"""The routine-per-kernel step without a work argument
(fd_step_routines_noalloc: the derivative fields live in the library's
static per-device area) against the same step with a caller-owned work
buffer (fd_step_routines), through the C ABI.

Both run the same kernels on the same inputs, so traces and fields must agree
bit for bit.  Two grids run back to back, the second smaller than the first,
so the second reuses an area that still holds the first one's fields; then
the largest 2D grid the area takes (2048 x 4096: two 32 MiB fields, exactly
the 64 MiB area), and a grid one tile wider, which must be refused before
anything is launched."""
import pytest
import torch

import fd_inputs as fi
from helpers import setup

pytestmark = pytest.mark.gpu


def _shot(p, noalloc, nt=None):
    nt = p.nt if nt is None else nt
    model, state, shot = setup(p)
    tr = torch.zeros((nt, p.receivers.count), device="cuda")
    work = None if noalloc else torch.empty(model.sizes.routines_work, dtype=torch.uint8, device="cuda")
    state.begin(shot)
    for n in range(nt):
        if noalloc:
            state.step_routines_noalloc(shot, n, tr[n])
        else:
            state.step_routines(shot, n, work, tr[n])
    f = state.wavefield(0)
    g = state.wavefield(1)
    torch.cuda.synchronize()
    return tr, f, g


def test_noalloc_equals_work_buffer_on_two_grids_in_a_row():
    import paper_2311_05038_amd as fd
    first = fi.layered3d(nx=130, ny=66, nz=70, nt=25)    # 3 fields of 3.5 MB
    second = fi.surface2d(75, 133, 40, seed=61)           # 2 fields of 77 KB
    for p in (first, second):
        print(f"case {p.name} {p.shape} nt={p.nt}", flush=True)
        model, _, _ = setup(p)
        assert model.sizes.routines_work <= fd._abi.ROUTINES_STATIC_BYTES
        a = _shot(p, noalloc=True)
        b = _shot(p, noalloc=False)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        assert float(a[1].abs().max()) > 0


def test_noalloc_largest_grid_and_refusal():
    import paper_2311_05038_amd as fd
    big = fi.surface2d(2048, 4096, 1000, seed=5050)
    model, _, _ = setup(big)
    assert model.sizes.routines_work == fd._abi.ROUTINES_STATIC_BYTES
    print(f"case {big.name} {big.shape} 6 steps", flush=True)
    a = _shot(big, noalloc=True, nt=6)
    b = _shot(big, noalloc=False, nt=6)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # one 64-column tile wider: 2 x 2048 x 4160 x 4 B > 64 MiB
    wide = fi.surface2d(2048, 4160, 10, seed=5051)
    model, state, shot = setup(wide)
    assert model.sizes.routines_work > fd._abi.ROUTINES_STATIC_BYTES
    state.begin(shot)
    with pytest.raises(fd.FDError) as e:
        state.step_routines_noalloc(shot, 0)
    assert e.value.status == fd._abi.FD_ERR_INVALID_ARG
    assert "static work area" in fd._abi.fd_last_error()
    # nothing ran: the state still takes step 0 (with a work buffer)
    work = torch.empty(model.sizes.routines_work, dtype=torch.uint8, device="cuda")
    state.step_routines(shot, 0, work)
    torch.cuda.synchronize()
