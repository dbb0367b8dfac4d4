"""Every cell and every trace sample of the full-size FP32 shots: the GPU
library (libfd.so) against the host back-end (libfd_cpu.so), bit for bit.

The FP64 oracle takes tens of minutes to hours at these sizes, so the
full-size oracle checks compare samples (random cells, block sums, norms,
every 32nd receiver).  The two libraries compute the same FP32 operations in
the same order (pinned against each other and against the oracle on small
grids), so at full size every value must agree exactly: an error confined to
one plane, row, tile edge or z-chunk boundary of the GPU kernel, which
samples would likely miss, shows here.  Cases: the 512^3 / 1000-step
headline shot (65,536 receivers) and the 768x768x512 / 2000-step precision
grid in FP32 (about 10 s and 40 s of host time on 16 cores)."""
import os

import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import grid_of, receivers_of, run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpu():
    from paper_2311_05038_amd import cpu as c
    if not os.path.exists(c.LIB_PATH):
        pytest.fail("libfd_cpu.so is not built")
    c.lib()
    return c


@pytest.mark.parametrize("case", ["layered3d_512", "precision3d_768"])
def test_full_size_gpu_equals_host_everywhere(cpu, case):
    p = fi.layered3d() if case == "layered3d_512" else fi.precision3d()
    print(f"[case] {case} {p.shape} nt={p.nt}: GPU", flush=True)
    v = p.velocity()
    tr_g, cur_g = run(p, v)
    print(f"[case] {case}: host back-end, {cpu.threads()} threads", flush=True)
    m = cpu.Model(grid_of(p), v)
    s = m.new_state()
    tr_c = m.run_shot(s, cpu.Shot(p.src, p.wavelet(), receivers_of(p)))
    cur_c = s.wavefield(0).reshape(cur_g.shape)
    bad_tr = np.argwhere(tr_c != tr_g)
    bad_f = np.argwhere(cur_c != cur_g)
    print(f"[case] {case}: differing trace samples {len(bad_tr)}, differing cells {len(bad_f)}", flush=True)
    assert len(bad_tr) == 0, bad_tr[:10]
    assert len(bad_f) == 0, bad_f[:10]
    torch.cuda.synchronize()
