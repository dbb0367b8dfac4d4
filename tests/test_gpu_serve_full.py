"""The serving stream's largest grid (2048 x 4096, 1000 steps, random-field
velocity) run through the batched step kernel in a mix with two smaller
shots, as the shot server runs it, against the FP64 oracle samples stored by
tests/golden/make_golden.py (every 16th receiver's trace, 8192 final cells,
16^2 block sums, the norms).  FP32 bound: relative L2 <= 1e-4 (measured:
traces 5.9e-6, cells 5.6e-5, blocks 7.4e-5, norms below 2e-6)."""
import os

import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import rel_l2, setup

pytestmark = pytest.mark.gpu

TOL = 1e-4


def test_serving_size_shot_in_a_batch_against_stored_oracle():
    import sys
    import paper_2311_05038_amd as fd
    path = os.path.join(os.path.dirname(__file__), "golden", "serving2d_2048x4096.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_golden import serving_shot
    gold = np.load(path)
    p = serving_shot()
    print(f"{p.name} nt={p.nt} in a batch of 3", flush=True)
    probs = [p, fi.surface2d(512, 700, 400, seed=5051), fi.surface2d(900, 512, 1000, seed=5052)]
    objs = [setup(q) for q in probs]
    big = objs[0]
    entries = []
    traces = []
    for q, (m, st, sh) in zip(probs, objs):
        st.begin(sh)
        tr = torch.zeros((q.nt, q.receivers.count), device="cuda")
        traces.append(tr)
        entries.append((m, st, sh, tr))
    while any(e[1].next < e[2].nt for e in entries):
        fd.step_batch(entries, 50)
    torch.cuda.synchronize()
    assert [e[1].next for e in entries] == [q.nt for q in probs]
    tr = traces[0].cpu().numpy()
    cur = big[1].wavefield(0).cpu().numpy().reshape(p.nz, p.nx)
    e_tr = rel_l2(tr[:, gold["traces_idx"]], gold["traces"])
    e_cells = rel_l2(cur.ravel()[gold["cells_idx"]], gold["cells"])
    b = 16
    blocks = cur.astype(np.float64).reshape(p.nz // b, b, p.nx // b, b).sum(axis=(1, 3))
    e_blocks = rel_l2(blocks, gold["blocks"])
    e_norm_f = abs(np.linalg.norm(cur.astype(np.float64)) / float(gold["field_norm"]) - 1)
    e_norm_t = abs(np.linalg.norm(tr.astype(np.float64)) / float(gold["trace_norm"]) - 1)
    print(f"2048x4096 errors vs FP64: traces {e_tr:.3e} cells {e_cells:.3e} blocks {e_blocks:.3e} "
          f"field norm {e_norm_f:.3e} trace norm {e_norm_t:.3e}", flush=True)
    assert max(e_tr, e_cells, e_blocks, e_norm_f, e_norm_t) <= TOL
