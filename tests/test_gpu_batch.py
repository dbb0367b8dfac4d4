"""Batched stepping of shots on different grids: one launch per global step
advances every shot in flight; each result must equal the shot run alone,
bit for bit (same kernel body, same arithmetic, no cross-shot data)."""
import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import setup

pytestmark = pytest.mark.gpu


def test_batch_equals_alone_bitwise():
    import paper_2311_05038_amd as fd
    probs = [fi.surface2d(70, 133, 90, seed=31), fi.surface2d(129, 64, 60, seed=32),
             fi.surface2d(40, 300, 120, seed=33), fi.green2d().scaled(nt=75)]
    alone = []
    for p in probs:
        m, s, sh = setup(p)
        tr = m.run_shot(s, sh).clone()
        alone.append((tr, s.wavefield(0).clone()))
    objs = [setup(p) for p in probs]
    traces = [torch.zeros((p.nt, p.receivers.count), device="cuda") for p in probs]
    # staggered admission: shots 0,1 start, 2 joins after 25 steps, 3 after 40
    entries = []
    for i in (0, 1):
        m, s, sh = objs[i]
        s.begin(sh)
        entries.append((m, s, sh, traces[i]))
    fd.step_batch(entries, 25)
    m, s, sh = objs[2]
    s.begin(sh)
    entries.append((m, s, sh, traces[2]))
    fd.step_batch(entries, 15)
    m, s, sh = objs[3]
    s.begin(sh)
    entries.append((m, s, sh, traces[3]))
    while any(e[1].next < e[2].nt for e in entries):
        fd.step_batch(entries, 7)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        assert objs[i][1].next == p.nt
        assert torch.equal(traces[i], alone[i][0]), i
        assert torch.equal(objs[i][1].wavefield(0), alone[i][1]), i
