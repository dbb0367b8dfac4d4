"""The C ABI from plain C.  On the host: include/fd.h and include/fd_cpu.h
compile as strict C99, and tests/native/abi_example.c (a whole shot through
fd.h with buffers from the HIP runtime API, no other layer) compiles and
links as strict C11 against libfd.so.  On the GPU: that program's traces and
final wavefield equal those of the Python binding on the same inputs, bit
for bit."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import fd_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2311_05038_amd")
ROCM = "/opt/rocm"
need_gcc = pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")


def _build(exe):
    cmd = ["gcc", "-std=c11", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "abi_example.c"), "-L", PKG, "-lfd",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-Wl,-rpath," + PKG, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@need_gcc
@pytest.mark.parametrize("header", ["fd.h", "fd_cpu.h"])
def test_headers_are_strict_c99(header):
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-x", "c", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "include", header)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@need_gcc
@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")), reason="no HIP runtime")
def test_c_example_builds(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libfd.so")):
        pytest.skip("libfd.so is not built")
    _build(str(tmp_path / "abi_example"))


@pytest.mark.gpu
@need_gcc
def test_c_example_equals_python_binding(tmp_path):
    import torch
    import paper_2311_05038_amd as fd
    exe = str(tmp_path / "abi_example")
    _build(exe)
    nz, nx, nt = 96, 160, 150
    src, rec_z0, rec_x0, rec_nx, rec_dx = (30, 0, 80), 3, 5, 50, 3
    dh, dt = 10.0, 1e-3
    v = fi.layered_velocity((nz, nx), 7)
    w = fi.ricker(15.0, dt, nt)
    with open(tmp_path / "in.bin", "wb") as f:
        f.write(struct.pack("<12q", 2, nz, 1, nx, nt, *src, rec_z0, rec_x0, rec_nx, rec_dx))
        f.write(struct.pack("<2d", dh, dt))
        f.write(np.ascontiguousarray(v, dtype=np.float32).tobytes())
        f.write(np.ascontiguousarray(w, dtype=np.float32).tobytes())
    print("case abi_example 96x160 nt=150", flush=True)
    r = subprocess.run([exe, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(tmp_path / "out.bin", dtype=np.float32)
    tr_c, p_c = out[:nt * rec_nx].reshape(nt, rec_nx), out[nt * rec_nx:].reshape(nz, nx)

    g = fd.Grid(ndim=2, nz=nz, ny=1, nx=nx, dh=dh, dt=dt, sponge_width=0)
    model = fd.Model(g, torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32).ravel()).cuda())
    state = model.new_state()
    shot = fd.Shot(src, torch.from_numpy(np.ascontiguousarray(w, dtype=np.float32)).cuda(),
                   fd.Receivers(rec_z0, 0, rec_x0, 1, 1, rec_nx, 1, 1, rec_dx))
    tr = model.run_shot(state, shot).cpu().numpy()
    p = state.wavefield(0).cpu().numpy()
    assert np.array_equal(tr, tr_c)
    assert np.array_equal(p, p_c)
    assert np.abs(tr).max() > 0
