"""The built C-ABI library loads and exports every function include/fd.h
declares; host-only entry points validate their arguments (no device needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:fd_status|const char\s*\*)\s*(fd_\w+)\s*\(", text,
                                 flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("fd_create_model", "fd_step", "fd_run_shot", "fd_adjoint_gradient",
              "fd_step_batch", "fd_query_bytes", "fd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2311_05038_amd import _abi
    lib = _abi.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    # the binding wraps exactly the declared set
    assert sorted(n for n, _, _ in _abi.SIGNATURES) == declared_functions()


def test_query_bytes_and_validation_on_host():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd import _abi
    g = fd.Grid(ndim=3, nz=512, ny=512, nx=512, dh=10.0, dt=1e-3, sponge_width=32).c()
    s = _abi.fd_query_bytes(g, 1000, 50)
    cells = 512 ** 3
    assert s.state >= 2 * cells * 4 and s.state < 2 * cells * 4 + 4096
    assert s.model >= cells * 4
    assert s.checkpoints == 20 * 2 * cells * 4
    g16 = fd.Grid(ndim=3, nz=512, ny=512, nx=512, dh=10.0, dt=1e-3, storage=fd.FD_F16).c()
    assert _abi.fd_query_bytes(g16).state < s.state // 2 + 4096
    bad = [dict(ndim=4), dict(nz=0), dict(ny=2, ndim=2), dict(dh=0.0), dict(dt=-1.0),
           dict(storage=7), dict(sponge_width=-1)]
    for kw in bad:
        base = dict(ndim=2, nz=10, ny=1, nx=10, dh=1.0, dt=1e-4)
        base.update(kw)
        with pytest.raises(fd.FDError) as e:
            _abi.fd_query_bytes(fd.Grid(**base).c())
        assert e.value.status == _abi.FD_ERR_INVALID_ARG, kw
        assert _abi.fd_last_error()
    with pytest.raises(fd.FDError) as e:
        _abi.fd_query_bytes(fd.Grid(ndim=2, nz=10, ny=1, nx=10, dh=1.0, dt=1e-4, radius=2).c())
    assert e.value.status == _abi.FD_ERR_UNSUPPORTED


def test_c_fixed16_sizes_and_validation_on_host():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd import _abi
    kw = dict(ndim=3, nz=512, ny=768, nx=768, dh=10.0, dt=1e-3, storage=fd.FD_BF16)
    s32 = _abi.fd_query_bytes(fd.Grid(**kw).c())
    s16 = _abi.fd_query_bytes(fd.Grid(c_storage=fd.FD_C_FIXED16, **kw).c())
    cells = 512 * 768 * 768
    assert s32.model - s16.model == cells * 2          # c: 4 -> 2 bytes per cell
    assert s16.state == s32.state
    # 16-bit c goes with 16-bit fields only; unknown kinds are rejected
    with pytest.raises(fd.FDError) as e:
        _abi.fd_query_bytes(fd.Grid(ndim=2, nz=10, ny=1, nx=10, dh=1.0, dt=1e-4,
                                    c_storage=fd.FD_C_FIXED16).c())
    assert e.value.status == _abi.FD_ERR_UNSUPPORTED
    with pytest.raises(fd.FDError) as e:
        _abi.fd_query_bytes(fd.Grid(ndim=2, nz=10, ny=1, nx=10, dh=1.0, dt=1e-4,
                                    storage=fd.FD_F16, c_storage=3).c())
    assert e.value.status == _abi.FD_ERR_INVALID_ARG


def test_null_handles_are_rejected_on_host():
    from paper_2311_05038_amd import _abi
    lib = _abi.lib()
    shot = _abi.fd_shot()
    assert lib.fd_step(None, None, ctypes.byref(shot), 0, None, None) == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_get_wavefield(None, 0, None, None) == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_step_batch(None, 99, 1, None) == _abi.FD_ERR_INVALID_ARG
    assert b"count" in lib.fd_last_error()


def test_z_slab_sizes_and_validation_on_host():
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd import _abi
    whole = fd.Grid(ndim=3, nz=512, ny=512, nx=512, dh=10.0, dt=1e-3, sponge_width=32)
    slabs = whole.slabs([64] * 8)
    assert [(g.slab_z0, g.nz, g.slab_nz_global) for g in slabs][3] == (192, 64, 512)
    s = _abi.fd_query_bytes(slabs[3].c(), 1000, 50)
    plane = 512 * 512 * 4
    # two levels of 64 owned + 2 x 4 ghost planes, and the 16-bit metadata words
    assert 2 * 72 * plane <= s.state < 2 * 72 * plane + 4096
    assert 64 * plane <= s.model < 64 * plane + 3 * 4096
    assert s.checkpoints == 0 and s.adjoint_work == 0 and s.routines_work == 0
    with pytest.raises(ValueError):
        whole.slabs([64] * 7)
    base = dict(ndim=3, nz=16, ny=8, nx=8, dh=1.0, dt=1e-4, slab_z0=0, slab_nz_global=40)
    for kw, status in [(dict(ndim=2, ny=1), _abi.FD_ERR_UNSUPPORTED),
                       (dict(storage=fd.FD_F16), _abi.FD_ERR_UNSUPPORTED),
                       (dict(nz=3), _abi.FD_ERR_INVALID_ARG),
                       (dict(slab_z0=30), _abi.FD_ERR_INVALID_ARG),
                       (dict(slab_z0=-1), _abi.FD_ERR_INVALID_ARG),
                       (dict(slab_nz_global=0, slab_z0=4), _abi.FD_ERR_INVALID_ARG)]:
        with pytest.raises(fd.FDError) as e:
            _abi.fd_query_bytes(fd.Grid(**{**base, **kw}).c())
        assert e.value.status == status, kw
    _abi.fd_query_bytes(fd.Grid(**{**base, "slab_z0": 24}).c())   # the last 16 planes
    assert _abi.lib().fd_slab_exchange(None, None, None) == _abi.FD_ERR_INVALID_ARG


def test_probe_health_noalloc_and_graph_validate_before_launching():
    """Argument errors of fd_stream_probe, fd_check_finite,
    fd_step_routines_noalloc and the recorded-shot calls come back as
    statuses before any launch (the pointers below are never dereferenced:
    every call fails validation)."""
    from paper_2311_05038_amd import _abi
    lib = _abi.lib()
    shot = _abi.fd_shot()
    A = 1 << 20                                 # a 16-byte aligned stand-in address
    for args, what in [((2, A, A, A, 16, None), b"kind"),
                       ((-1, A, A, A, 16, None), b"kind"),
                       ((0, None, None, A, 16, None), b"NULL"),
                       ((1, A, None, A, 16, None), b"NULL"),
                       ((0, A, None, None, 16, None), b"NULL"),
                       ((0, A, None, A, 18, None), b"multiple of 4"),
                       ((0, A + 4, None, A, 16, None), b"aligned"),
                       ((1, A, A + 8, A, 16, None), b"aligned"),
                       ((1, A, A, A + 12, 16, None), b"aligned")]:
        assert lib.fd_stream_probe(*args) == _abi.FD_ERR_INVALID_ARG, args
        assert what in lib.fd_last_error(), (args, lib.fd_last_error())
    out = ctypes.c_void_p(123)
    assert lib.fd_shot_graph_create(None, None, ctypes.byref(shot), None, ctypes.byref(out)) \
        == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_shot_graph_launch(None, None) == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_shot_graph_destroy(None) == _abi.FD_OK
    # an empty stream launches nothing and does not look at the arrays
    assert lib.fd_stream_probe(1, None, None, None, 0, None) == _abi.FD_OK
    assert lib.fd_stream_probe(2, None, None, None, 0, None) == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_check_finite(None, A, None) == _abi.FD_ERR_INVALID_ARG
    assert lib.fd_step_routines_noalloc(None, None, ctypes.byref(shot), 0, None, None) \
        == _abi.FD_ERR_INVALID_ARG
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "fd.h")).read()
    m = re.search(r"#define FD_ROUTINES_STATIC_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and _abi.ROUTINES_STATIC_BYTES == int(m.group(1)) << int(m.group(2))


def test_last_error_is_per_thread():
    """fd_last_error is thread-local: threads that fail different calls at
    the same time each read back their own message."""
    import threading
    import paper_2311_05038_amd as fd
    from paper_2311_05038_amd import _abi
    lib = _abi.lib()
    barrier = threading.Barrier(8)
    seen = {}

    def worker(k):
        g = fd.Grid(ndim=2, nz=10 + k, ny=1, nx=10, dh=1.0, dt=1e-4, storage=7 + k).c()
        barrier.wait()
        for _ in range(200):
            st = lib.fd_query_bytes(ctypes.byref(g), 1, 1, ctypes.byref(_abi.fd_sizes()))
            msg = lib.fd_last_error().decode()
            if st != _abi.FD_ERR_INVALID_ARG or f"storage kind {7 + k}" not in msg:
                seen[k] = (st, msg)
                return
        seen[k] = "ok"

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert all(v == "ok" for v in seen.values()) and len(seen) == 8, seen


def test_binding_buffer_checks_on_host():
    """The binding's buffer check refuses host tensors, the wrong element
    type, non-contiguous views and short tensors (no device needed)."""
    import torch
    import paper_2311_05038_amd as fd
    with pytest.raises(ValueError, match="device tensor"):
        fd._buf(torch.zeros(8), "x", torch.float32, 8)
    with pytest.raises(ValueError, match="device tensor"):
        fd._nbytes(torch.zeros(8))
    with pytest.raises(ValueError, match="entries"):
        fd._same_len([1, 2], states=[1])
    fd._same_len([1, 2], states=[1, 2], ckpts=None)
