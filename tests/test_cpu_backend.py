"""The host back-end (libfd_cpu.so, include/fd_cpu.h): the forward time loop
of Listing 3 (Section 7) behind the C ABI of include/fd.h, on host memory
with OpenMP and AVX2/AVX-512.  Checked against the FP64 oracle at the FP32
parity bar (relative L2 <= 1e-4 on traces and the final field), and for the
properties the back-end promises: fd_step sequences equal fd_run_shot, and
neither the instruction set nor the thread count changes a bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import fd_inputs as fi
from helpers import grid_of, receivers_of

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 1e-4


@pytest.fixture(scope="module")
def cpu():
    from paper_2311_05038_amd import build, cpu as c
    if not os.path.exists(c.LIB_PATH):
        build.build_cpu()
    c.lib()
    return c


def run_cpu(cpu, p, v=None):
    v = p.velocity() if v is None else v
    m = cpu.Model(grid_of(p), v)
    s = m.new_state()
    shot = cpu.Shot(p.src, p.wavelet(), receivers_of(p))
    tr = m.run_shot(s, shot)
    return m, s, shot, tr


def oracle_run(orc, p, v=None):
    v = p.velocity() if v is None else v
    return orc.forward(orc.grid_of(p), v.reshape(p.nz, p.ny, p.nx), p.wavelet(), p.nt, p.src,
                       p.rec_index())


def declared(header):
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", header)).read(), flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:fd_status|const char\s*\*|int32_t)\s*(fd_\w+)\s*\(",
                                 text, flags=re.M)))


def test_exports_every_declared_symbol(cpu):
    names = declared("fd.h") + declared("fd_cpu.h")
    assert "fd_cpu_stream_probe" in names and "fd_run_shot" in names
    for n in names:
        assert hasattr(cpu.lib(), n), n
    assert cpu.isa() in ("avx512", "avx2", "scalar")
    assert "fd-cpu" in cpu.version()


@pytest.mark.parametrize("case", ["green2d", "surface2d", "layered3d", "ragged3d"])
def test_parity_with_oracle(cpu, orc, case):
    p = {"green2d": fi.green2d(),                                 # 256^2, 500 steps
         "surface2d": fi.surface2d(70, 93, 120, seed=3),          # damped, ragged rows
         "layered3d": fi.layered3d(nx=48, ny=40, nz=36, nt=80),   # 5 damped faces
         "ragged3d": fi.layered3d(nx=37, ny=23, nz=29, nt=60).scaled(sponge_faces=fi.FACES_ALL),
         }[case]
    _, s, _, tr = run_cpu(cpu, p)
    ref = oracle_run(orc, p)
    e_tr = orc.rel_l2(tr, ref["traces"])
    e_f = orc.rel_l2(s.wavefield(0).ravel(), ref["cur"].ravel())
    e_p = orc.rel_l2(s.wavefield(1).ravel(), ref["prev"].ravel())
    assert e_tr <= TOL and e_f <= TOL and e_p <= TOL, (e_tr, e_f, e_p)


def test_tiny_and_degenerate_grids(cpu, orc):
    """Grids thinner than the stencil, a one-row 3D grid, a receiver on the
    source cell, strided receivers, no receivers."""
    cases = [
        fi.Problem(name="t1", ndim=2, nz=5, ny=1, nx=3, dh=10.0, dt=1e-3, nt=30, src=(2, 0, 1),
                   receivers=fi.Receivers(0, 0, 0, 5, 1, 3), f0=25.0, v_const=1500.0),
        fi.Problem(name="t2", ndim=3, nz=6, ny=1, nx=9, dh=10.0, dt=1e-3, nt=30, src=(3, 0, 4),
                   receivers=fi.Receivers(3, 0, 4, 1, 1, 1), f0=25.0, v_const=1500.0),
        fi.Problem(name="t3", ndim=3, nz=13, ny=11, nx=17, dh=10.0, dt=1e-3, nt=40, src=(6, 5, 8),
                   receivers=fi.Receivers(1, 2, 3, 3, 2, 4, 4, 3, 3), f0=20.0, sponge_width=3,
                   sponge_faces=fi.FACES_ALL, velocity_kind="layered", velocity_seed=4),
        fi.Problem(name="t4", ndim=2, nz=21, ny=1, nx=19, dh=10.0, dt=1e-3, nt=40, src=(10, 0, 9),
                   receivers=fi.Receivers(0, 0, 0, 0, 0, 0), f0=20.0, v_const=2500.0),
    ]
    for p in cases:
        _, s, _, tr = run_cpu(cpu, p)
        ref = oracle_run(orc, p)
        if p.receivers.count:
            assert orc.rel_l2(tr, ref["traces"]) <= TOL, p.name
        assert orc.rel_l2(s.wavefield(0).ravel(), ref["cur"].ravel()) <= TOL, p.name


def test_step_sequence_equals_run_shot(cpu):
    for p in (fi.surface2d(40, 51, 30, seed=2), fi.layered3d(nx=33, ny=20, nz=18, nt=25)):
        m, s, shot, tr = run_cpu(cpu, p)
        s2 = m.new_state()
        s2.begin(shot)
        rows = np.empty_like(tr)
        for n in range(p.nt):
            s2.step(shot, n, rows[n])
        assert np.array_equal(rows, tr)
        for w in (0, 1):
            assert np.array_equal(s2.wavefield(w), s.wavefield(w))


def test_instruction_set_and_thread_count_do_not_change_bits(cpu):
    p = fi.layered3d(nx=45, ny=26, nz=30, nt=30)
    _, s, _, tr = run_cpu(cpu, p)
    f = s.wavefield(0)
    best, nthreads = cpu.isa(), cpu.threads()
    try:
        for isa in ("avx512", "avx2", "scalar"):
            try:
                cpu.set_isa(isa)
            except cpu.FDError as e:
                assert e.status == 5   # this processor lacks it
                continue
            for t in (1, 3, nthreads):
                cpu.threads(t)
                _, s2, _, tr2 = run_cpu(cpu, p)
                assert np.array_equal(tr2, tr), (isa, t)
                assert np.array_equal(s2.wavefield(0), f), (isa, t)
    finally:
        cpu.set_isa(best)
        cpu.threads(nthreads)


def test_set_and_get_wavefield(cpu, orc):
    """A state started from given levels (no source) steps like the oracle's
    time loop from the same levels."""
    p = fi.layered3d(nx=24, ny=20, nz=22, nt=12)
    v = p.velocity()
    m = cpu.Model(grid_of(p), v)
    s = m.new_state()
    rng = np.random.default_rng(3)
    P = rng.standard_normal(p.shape).astype(np.float32)
    Q = rng.standard_normal(p.shape).astype(np.float32)
    s.set_wavefield(0, P)
    s.set_wavefield(1, Q)
    assert np.array_equal(s.wavefield(0), P) and np.array_equal(s.wavefield(1), Q)
    import paper_2311_05038_amd as fd
    shot = cpu.Shot(p.src, np.zeros(p.nt, np.float32), fd.Receivers())
    for n in range(p.nt):
        s.step(shot, n)
    ref = orc.forward(orc.grid_of(p), v.reshape(p.nz, p.ny, p.nx), np.zeros(p.nt, np.float32),
                      p.nt, None, [], init_prev=Q.astype(np.float64), init_cur=P.astype(np.float64))
    assert orc.rel_l2(s.wavefield(0).ravel(), ref["cur"].ravel()) <= TOL


def test_validation_and_unsupported(cpu):
    import paper_2311_05038_amd as fd
    lib = cpu.lib()
    FD_INVALID, FD_UNSTABLE, FD_UNSUPPORTED = 1, 2, 5

    def query(**kw):
        base = dict(ndim=2, nz=10, ny=1, nx=10, dh=1.0, dt=1e-4)
        base.update(kw)
        out = fd._abi.fd_sizes()
        g = fd.Grid(**base).c()
        return lib.fd_query_bytes(ctypes.byref(g), 0, 0, ctypes.byref(out)), out

    for kw in (dict(ndim=4), dict(nz=0), dict(ny=2), dict(dh=0.0), dict(dt=-1.0), dict(storage=7),
               dict(sponge_width=-1)):
        assert query(**kw)[0] == FD_INVALID, kw
        assert lib.fd_last_error()
    for kw in (dict(radius=2), dict(storage=fd.FD_F16), dict(bc=1),
               dict(ndim=3, ny=8, nz=8, slab_nz_global=16)):
        assert query(**kw)[0] == FD_UNSUPPORTED, kw
    st, sizes = query()
    assert st == 0 and sizes.state > 0 and sizes.checkpoints == 0 and sizes.adjoint_work == 0

    p = fi.surface2d(32, 40, 6, seed=1)
    # unstable: 3000 m/s * 2 ms / 10 m = 0.6 > 0.5546
    with pytest.raises(fd.FDError) as e:
        cpu.Model(grid_of(p.scaled(dt=2e-3)), np.full(p.shape, 3000.0, np.float32))
    assert e.value.status == FD_UNSTABLE
    for bad in (0.0, -1.0, np.nan, np.inf):
        v = p.velocity().copy()
        v[5, 7] = bad
        with pytest.raises(fd.FDError) as e:
            cpu.Model(grid_of(p), v)
        assert e.value.status == FD_INVALID
    m = cpu.Model(grid_of(p), p.velocity())
    s = m.new_state()
    shot = cpu.Shot(p.src, p.wavelet(), receivers_of(p))
    with pytest.raises(fd.FDError):
        s.step(shot, 0)                      # before begin
    s.begin(shot)
    with pytest.raises(fd.FDError):
        s.step(shot, 1)                      # out of order
    for n in range(p.nt):
        s.step(shot, n)
    with pytest.raises(fd.FDError):
        s.step(shot, p.nt)                   # past nt
    with pytest.raises(fd.FDError):
        s.begin(cpu.Shot((32, 0, 0), p.wavelet(), receivers_of(p)))   # source outside
    ck = cpu._aligned(1024)
    st = lib.fd_run_shot(m.handle, s.handle, ctypes.byref(shot._c), None, ck.ctypes.data, 1024, 1,
                         None)
    assert st == FD_UNSUPPORTED
    for name in ("fd_adjoint_gradient", "fd_rtm_image", "fd_step_batch", "fd_step_routines",
                 "fd_slab_exchange"):
        assert getattr(lib, name).restype == ctypes.c_int
    assert lib.fd_slab_exchange(s.handle, s.handle, None) == FD_UNSUPPORTED
    assert lib.fd_step_batch(None, 0, 1, None) == FD_UNSUPPORTED


def test_stream_probe(cpu):
    gbs = cpu.stream_probe(1 << 20, 3)
    assert gbs > 0.1
    with pytest.raises(Exception):
        cpu.stream_probe(10, 1)


def test_check_finite_reports_planted_values(cpu):
    """fd_check_finite on the host back-end: a healthy shot reports 0; a NaN
    or an infinity planted in P through fd_set_wavefield spreads through the
    update and is still reported after further steps, in both levels."""
    p = fi.layered3d(nx=40, ny=36, nz=30, nt=30)
    m, s, shot, _ = run_cpu(cpu, p)
    assert s.check_finite() == 0
    for bad in (np.nan, np.inf, -np.inf):
        s2 = m.new_state()
        s2.begin(shot)
        for n in range(5):
            s2.step(shot, n)
        f = s2.wavefield(0).copy()
        f.reshape(-1)[f.size // 3] = bad
        s2.set_wavefield(0, f)
        assert s2.check_finite() == 5          # P, and a non-finite input
        for n in range(5, 9):
            s2.step(shot, n)
        assert s2.check_finite() == 7          # spread into both levels
        w = s2.wavefield(0)
        assert np.count_nonzero(~np.isfinite(w)) > 1
    s2.begin(shot)
    assert s2.check_finite() == 0              # a new shot clears the flags
    w = p.wavelet().copy()
    w[7] = np.nan
    s2.begin(cpu.Shot(p.src, w, receivers_of(p)))
    assert s2.check_finite() == 4              # a non-finite wavelet sample
    fresh = m.new_state()
    with pytest.raises(cpu.FDError):
        fresh.check_finite()                   # no shot begun


@pytest.mark.parametrize("seed", range(24))
def test_random_shapes_against_oracle(cpu, orc, seed):
    """Seeded small workloads of arbitrary shape (axes from 1 cell up, 1-13
    steps, source, receiver box and sponge faces anywhere): both levels and
    the traces at the FP32 parity bar, and fd_step equal to fd_run_shot."""
    p = fi.random_geometry(seed)
    v = p.velocity()
    m, s, shot, tr = run_cpu(cpu, p, v)
    ref = oracle_run(orc, p, v)
    n = p.receivers.count
    if n:
        assert orc.rel_l2(tr[:, :n], ref["traces"]) <= TOL
    assert orc.rel_l2(s.wavefield(0).reshape(-1), ref["cur"].reshape(-1)) <= TOL
    assert orc.rel_l2(s.wavefield(1).reshape(-1), ref["prev"].reshape(-1)) <= TOL
    s2 = m.new_state()
    s2.begin(shot)
    tr2 = np.zeros_like(tr)
    for k in range(p.nt):
        s2.step(shot, k, tr2[k] if n else None)
    assert np.array_equal(tr2, tr)
    assert np.array_equal(s2.wavefield(0), s.wavefield(0))
