"""The host back-end (libfd_cpu.so) and the GPU library (libfd.so) compute
the same FP32 step operation for operation, so on the same inputs they give
the same bits: traces, final field and previous level, in 2D and 3D, with
damping, ragged rows and strided receivers."""
import os

import numpy as np
import pytest
import torch

import fd_inputs as fi
from helpers import receivers_of, run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpu():
    from paper_2311_05038_amd import cpu as c
    if not os.path.exists(c.LIB_PATH):
        pytest.fail("libfd_cpu.so is not built")
    c.lib()
    return c


@pytest.mark.parametrize("case", ["green2d", "surface2d", "layered3d", "ragged3d"])
def test_host_and_gpu_give_the_same_bits(cpu, case):
    from helpers import grid_of
    p = {"green2d": fi.green2d().scaled(nt=200),
         "surface2d": fi.surface2d(150, 333, 150, seed=9),
         "layered3d": fi.layered3d(nx=96, ny=72, nz=80, nt=60),
         "ragged3d": fi.layered3d(nx=101, ny=37, nz=45, nt=50).scaled(sponge_faces=fi.FACES_ALL),
         }[case]
    print(f"[case] {case} {p.shape} nt={p.nt}", flush=True)
    v = p.velocity()
    tr_g, cur_g = run(p, v)
    m = cpu.Model(grid_of(p), v)
    s = m.new_state()
    tr_c = m.run_shot(s, cpu.Shot(p.src, p.wavelet(), receivers_of(p)))
    assert np.array_equal(tr_c, tr_g)
    assert np.array_equal(s.wavefield(0).reshape(cur_g.shape), cur_g)
    torch.cuda.synchronize()
