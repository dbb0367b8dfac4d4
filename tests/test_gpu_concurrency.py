"""Several host threads, each with its own state of one shared model, its
own shot and its own stream, run shots at the same time through the C ABI:
every shot gives the bits it gives alone.  The model is only read while
stepping; each state, trace buffer and stream belongs to one thread."""
import threading

import pytest
import torch

import fd_inputs as fi
from helpers import receivers_of, setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ndim", [2, 3])
def test_threads_on_own_streams_give_the_bits_of_lone_shots(ndim):
    import paper_2311_05038_amd as fd
    p = fi.surface2d(160, 300, 120, seed=41) if ndim == 2 else fi.layered3d(nx=96, ny=48, nz=56, nt=50)
    print(f"case {p.name} shape={p.shape} nt={p.nt}", flush=True)
    model, _, shot0 = setup(p)
    nthreads = 4
    srcs = [(p.src[0] + 3 * k, p.src[1], p.src[2] - 5 * k) for k in range(nthreads)]
    shots = [fd.Shot(s, shot0.wavelet, receivers_of(p)) for s in srcs]
    ref = []
    for sh in shots:
        st = model.new_state()
        ref.append((model.run_shot(st, sh).clone(), st.wavefield(0).clone()))
    torch.cuda.synchronize()

    states = [model.new_state() for _ in range(nthreads)]
    streams = [torch.cuda.Stream() for _ in range(nthreads)]
    outs = [None] * nthreads
    errors = []
    barrier = threading.Barrier(nthreads)

    def worker(k):
        try:
            torch.cuda.set_device(0)
            with torch.cuda.stream(streams[k]):
                barrier.wait()
                for _ in range(3):
                    tr = model.run_shot(states[k], shots[k], stream=streams[k])
                cur = states[k].wavefield(0, stream=streams[k])
            streams[k].synchronize()
            outs[k] = (tr, cur)
        except Exception as e:          # reported below, in the main thread
            errors.append((k, repr(e)))

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(nthreads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    for k in range(nthreads):
        assert torch.equal(outs[k][0], ref[k][0]), k
        assert torch.equal(outs[k][1], ref[k][1]), k
