"""Full-size precision workload (768x768x512, 2000 steps, layered model,
256x256 receivers) in FP32, FP16 and BF16 field storage against the FP64
oracle values stored by tests/golden/make_golden.py (sampled traces, sampled
final cells, 16^3 block sums and the two norms; the oracle takes over two
hours for this run, so only samples are kept).

Errors are stated (printed) and bounded, per storage, for the traces (and
their norm), the field norm, and the sampled final cells and 16^3 block sums:
  FP32: 1e-4 / 1e-4 / 1e-4 (measured 7.7e-7, 7.9e-8, 3.2e-6 / 1.6e-6).
        The kernels take each axis's second difference as a weighted sum of
        differences from the centre value; with the centre weight summed
        against the taps instead, the cancellation error carried by the
        slowly decaying long-wavelength modes left the late-time field at
        1.5e-4 (cells) and 2.5e-4 (block sums).
  FP16: 1e-2 / 1e-2 / 5e-2 (measured 5.7e-3, 2.8e-4, 2.1e-2 / 2.6e-2).
  BF16: 8e-2 / 2e-1 / 1.0 (measured 6.4e-2, 1.0e-1, 0.52 / 0.89): with 8
        significand bits the stored fields lose the late-time field to
        accumulated quantisation error after 2000 steps; the traces, which
        record the early arrivals, keep 6% accuracy.
The 16-bit forms also run with c in 16-bit fixed point (8 bytes per cell),
under the same bounds.  The small whole-shot tests tie the 16-bit errors to
the oracle's own 16-bit emulation (within 1.5x); at this size the emulation
is out of reach."""
import os

import numpy as np
import pytest

import fd_inputs as fi
from helpers import rel_l2, run

pytestmark = pytest.mark.gpu

TRACE_BOUND = {0: 1e-4, 1: 1e-2, 2: 8e-2}
NORM_BOUND = {0: 1e-4, 1: 1e-2, 2: 2e-1}
FIELD_BOUND = {0: 1e-4, 1: 5e-2, 2: 1.0}
NAME = {0: "fp32", 1: "fp16", 2: "bf16"}


@pytest.mark.parametrize("storage,c16", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 1)])
def test_precision3d_768_against_stored_oracle(storage, c16):
    path = os.path.join(os.path.dirname(__file__), "golden", "precision3d_768.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle values not generated")
    gold = np.load(path)
    p = fi.precision3d()
    print(f"precision3d 768x768x512 nt={p.nt} storage={NAME[storage]} c16={c16}", flush=True)
    tr, cur = run(p, storage=storage, c_storage=c16)
    e_tr = rel_l2(tr[:, gold["traces_idx"]], gold["traces"])
    e_cells = rel_l2(cur.ravel()[gold["cells_idx"]], gold["cells"])
    b = 16
    blocks = cur.reshape(p.nz // b, b, p.ny // b, b, p.nx // b, b).astype(np.float64).sum(axis=(1, 3, 5))
    e_blocks = rel_l2(blocks, gold["blocks"])
    e_norm_f = abs(np.linalg.norm(cur.astype(np.float64)) / float(gold["field_norm"]) - 1)
    e_norm_t = abs(np.linalg.norm(tr.astype(np.float64)) / float(gold["trace_norm"]) - 1)
    print(f"768x768x512 {NAME[storage]}{'+c16' if c16 else ''} errors vs FP64: traces {e_tr:.3e} cells {e_cells:.3e} "
          f"blocks {e_blocks:.3e} field norm {e_norm_f:.3e} trace norm {e_norm_t:.3e}", flush=True)
    assert max(e_tr, e_norm_t) <= TRACE_BOUND[storage]
    assert e_norm_f <= NORM_BOUND[storage]
    assert max(e_cells, e_blocks) <= FIELD_BOUND[storage]
