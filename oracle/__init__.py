"""FP64 CPU oracle for explicit finite-difference acoustic time stepping.

TEST INFRASTRUCTURE ONLY.  This package is imported by the test-suite, by the
smoke check and by the CPU-baseline leg of the benchmark; the library never
imports it, and it imports nothing from the library.  The arithmetic lives in
``fd_oracle.c`` (plain loops, FP64, OpenMP over the slowest axis) and, for tiny
grids, in the independent NumPy twin ``oracle.np_twin``.

Parity status of each function (pins live in tests/test_oracle_*.py):
  coefficients  pinned: exact-rational moment solve, degree-10 error constant,
                symbol range
  laplacian     pinned: polynomial exactness, symmetry
  forward       pinned: 2D and 3D Green's functions (with dt-halving
                convergence; the 3D one at offsets along each axis and a
                diagonal), discrete energy conservation, growth above the
                stability limit and reciprocity, each in 2D and in 3D; NumPy
                twin
  sponge        pinned: a uniform damping factor g maps the damped update
                exactly onto the undamped one for P^n / g^n (forward_G);
                profile properties (1 off the band, decreasing into it,
                enabled faces only, G = product of the axis profiles)
  adjoint       pinned: dot-product test against the tangent-linear model and
                central finite differences
  image         pinned: dot-product test against the NumPy twin's
                tangent-linear model of the scatterer perturbation
                L -> L + diag(m), and central finite differences of the
                twin's forward map in m
  forward_half  pinned: conversions bit-exact against numpy float16 and torch
                bfloat16; the FP32 arithmetic against the NumPy twin's
                emulation (FP32 and 16-bit storage); the FP32-storage form
                against the FP64 forward within the FP32 rounding bound, and
                bit-identical to it on inputs whose arithmetic is exact in
                FP32 (dyadic c, an impulse source)
  c_fixed16     pinned: scale bracket, nearest code with ties to even, the
                cap, monotonicity; the twin's separate implementation; models
                whose c values are codes already run unchanged
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "fd_oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile fd_oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC,
           "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("sponge_width", ctypes.c_int32),
                ("nz", ctypes.c_int64), ("ny", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("dh", ctypes.c_double), ("dt", ctypes.c_double),
                ("sponge_alpha", ctypes.c_double), ("sponge_faces", ctypes.c_uint32),
                ("pad_", ctypes.c_uint32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_coefficients.argtypes = [ctypes.c_int, P]
        L.or_sponge_profile.argtypes = [i64, ctypes.c_int32, ctypes.c_double, ctypes.c_int, ctypes.c_int, P]
        L.or_laplacian.argtypes = [P, P, P]
        L.or_setup.argtypes = [P, P, P, P]
        L.or_forward.argtypes = [P, P, P, i64, i64, i64, P, P, P, P, P, P, P]
        L.or_forward.restype = ctypes.c_int
        L.or_adjoint.argtypes = [P, P, P, i64, i64, i64, P, P, P, P]
        L.or_adjoint.restype = ctypes.c_int
        L.or_image.argtypes = [P, P, P, i64, i64, i64, P, P, P]
        L.or_image.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = ctypes.c_int
        L.or_forward_G.argtypes = [P, P, P, P, i64, i64, i64, P, P, P, P, P, P]
        L.or_forward_G.restype = ctypes.c_int
        L.or_forward_half.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, i64, i64, i64, P, P, P, P, P]
        L.or_c_fixed16.argtypes = [P, i64, P, P, ctypes.c_int]
        L.or_forward_half.restype = ctypes.c_int
        L.or_encode_array.argtypes = [ctypes.c_int, P, P, i64]
        L.or_decode_array.argtypes = [ctypes.c_int, P, P, i64]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def grid_of(prob) -> OrGrid:
    """The oracle's grid record for a workload description (fd_inputs.Problem)."""
    return OrGrid(ndim=prob.ndim, radius=prob.radius, bc=prob.bc,
                  sponge_width=prob.sponge_width, nz=prob.nz, ny=prob.ny, nx=prob.nx,
                  dh=prob.dh, dt=prob.dt, sponge_alpha=prob.alpha(),
                  sponge_faces=prob.sponge_faces)


def coefficients(R: int) -> np.ndarray:
    a = np.zeros(9, dtype=np.float64)
    lib().or_coefficients(R, _p(a))
    return a[: R + 1].copy()


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count
    in effect."""
    return int(lib().or_set_threads(int(n)))


def sponge_profile(n: int, width: int, alpha: float, lo: bool, hi: bool) -> np.ndarray:
    g = np.zeros(n, dtype=np.float64)
    lib().or_sponge_profile(n, width, alpha, int(lo), int(hi), _p(g))
    return g


def laplacian(grid: OrGrid, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    lib().or_laplacian(ctypes.byref(grid), _p(u), _p(out))
    return out


def setup(grid: OrGrid, v: np.ndarray):
    v = np.ascontiguousarray(v, dtype=np.float32)
    c = np.empty(v.shape, dtype=np.float64)
    G = np.empty(v.shape, dtype=np.float64)
    lib().or_setup(ctypes.byref(grid), _p(v), _p(c), _p(G))
    return c, G


def _src_linear(grid: OrGrid, src) -> int:
    if src is None:
        return -1
    z, y, x = src
    return int((z * grid.ny + y) * grid.nx + x)


def forward(grid: OrGrid, v: np.ndarray, wavelet: np.ndarray, nt: int, src, rec_index,
            init_prev=None, init_cur=None, want_lap: bool = False):
    """Run nt steps.  Returns dict(traces [nt, nrec], prev, cur[, lap])."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    shape = v.shape
    N = v.size
    wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
    assert wavelet.size >= nt or src is None
    rec = np.ascontiguousarray(rec_index, dtype=np.int64)
    traces = np.zeros((nt, rec.size), dtype=np.float64)
    prev = np.empty(shape, dtype=np.float64)
    cur = np.empty(shape, dtype=np.float64)
    lap = np.empty((nt,) + shape, dtype=np.float64) if want_lap else None
    ip = None if init_prev is None else np.ascontiguousarray(init_prev, dtype=np.float64)
    ic = None if init_cur is None else np.ascontiguousarray(init_cur, dtype=np.float64)
    rc = lib().or_forward(ctypes.byref(grid), _p(v), _p(wavelet), nt, _src_linear(grid, src),
                          rec.size, _p(rec), _p(ip), _p(ic), _p(traces), _p(prev), _p(cur),
                          _p(lap))
    if rc != 0:
        raise MemoryError("oracle forward: allocation failed")
    out = dict(traces=traces, prev=prev, cur=cur)
    if want_lap:
        out["lap"] = lap
    assert N == prev.size
    return out


def forward_G(grid: OrGrid, v: np.ndarray, G: np.ndarray, nt: int, init_prev: np.ndarray,
              init_cur: np.ndarray, rec_index=()):
    """forward() from a given start state and no source, with the damping
    field G (one value per cell) given instead of built from the band."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    G = np.ascontiguousarray(G, dtype=np.float64)
    ip = np.ascontiguousarray(init_prev, dtype=np.float64)
    ic = np.ascontiguousarray(init_cur, dtype=np.float64)
    rec = np.ascontiguousarray(rec_index, dtype=np.int64)
    traces = np.zeros((nt, max(rec.size, 1)), dtype=np.float64)
    prev = np.empty(v.shape, dtype=np.float64)
    cur = np.empty(v.shape, dtype=np.float64)
    wav = np.zeros(max(nt, 1), dtype=np.float32)
    rc = lib().or_forward_G(ctypes.byref(grid), _p(v), _p(G), _p(wav), nt, -1, rec.size, _p(rec),
                            _p(ip), _p(ic), _p(traces), _p(prev), _p(cur))
    if rc != 0:
        raise MemoryError("oracle forward_G: allocation failed")
    return dict(traces=traces[:, :rec.size], prev=prev, cur=cur)


def adjoint(grid: OrGrid, v: np.ndarray, wavelet: np.ndarray, nt: int, src, rec_index,
            resid: np.ndarray):
    """Gradient of J with respect to v (and c) given resid = dJ/dtraces."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
    rec = np.ascontiguousarray(rec_index, dtype=np.int64)
    resid = np.ascontiguousarray(resid, dtype=np.float64)
    assert resid.shape == (nt, rec.size)
    gv = np.empty(v.shape, dtype=np.float64)
    gc = np.empty(v.shape, dtype=np.float64)
    rc = lib().or_adjoint(ctypes.byref(grid), _p(v), _p(wavelet), nt, _src_linear(grid, src),
                          rec.size, _p(rec), _p(resid), _p(gv), _p(gc))
    if rc != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return gv, gc


def image(grid: OrGrid, v: np.ndarray, wavelet: np.ndarray, nt: int, src, rec_index,
          resid: np.ndarray) -> np.ndarray:
    """Zero-lag correlation image sum_k z^k w^{k-1} of the source wavefield
    and the z-form receiver wavefield driven by resid (dJ/dm for L -> L +
    diag(m))."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
    rec = np.ascontiguousarray(rec_index, dtype=np.int64)
    resid = np.ascontiguousarray(resid, dtype=np.float64)
    assert resid.shape == (nt, rec.size)
    img = np.empty(v.shape, dtype=np.float64)
    rc = lib().or_image(ctypes.byref(grid), _p(v), _p(wavelet), nt, _src_linear(grid, src),
                        rec.size, _p(rec), _p(resid), _p(img))
    if rc != 0:
        raise MemoryError("oracle image: allocation failed")
    return img


def forward_half(grid: OrGrid, storage: int, v: np.ndarray, wavelet: np.ndarray, nt: int,
                 src, rec_index, init_prev=None, init_cur=None, c_fixed16: bool = False):
    """FP32-arithmetic emulation with FP32 (storage 0) or 16-bit storage
    (1 = binary16, 2 = bfloat16).  init_prev/init_cur (FP32) replace the start
    state and its s[0] addition; c_fixed16 (16-bit storage only) holds c in
    16-bit fixed point (c_fixed16())."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    ip = None if init_prev is None else np.ascontiguousarray(init_prev, dtype=np.float32)
    ic = None if init_cur is None else np.ascontiguousarray(init_cur, dtype=np.float32)
    wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
    rec = np.ascontiguousarray(rec_index, dtype=np.int64)
    traces = np.zeros((nt, rec.size), dtype=np.float32)
    cur = np.empty(v.shape, dtype=np.float32)
    rc = lib().or_forward_half(ctypes.byref(grid), storage, int(bool(c_fixed16)), _p(v), _p(wavelet), nt,
                               _src_linear(grid, src), rec.size, _p(rec), _p(ip), _p(ic),
                               _p(traces), _p(cur))
    if rc == -2:
        raise ValueError("oracle forward_half: storage must be 0, 1 or 2 (16-bit c needs 16-bit storage)")
    if rc != 0:
        raise MemoryError("oracle forward_half: allocation failed")
    return dict(traces=traces, cur=cur)


def c_fixed16(c: np.ndarray):
    """c (FP32) as 16-bit unsigned fixed point with one power-of-two scale:
    returns (codes, e, decoded) with decoded = codes * 2^(e-16) in FP32."""
    c = np.array(c, dtype=np.float32, copy=True, order="C")
    q = np.empty(c.shape, dtype=np.uint16)
    e = ctypes.c_int32(0)
    lib().or_c_fixed16(_p(c), c.size, _p(q), ctypes.byref(e), 1)
    return q, int(e.value), c


def encode(storage: int, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    q = np.empty(x.shape, dtype=np.uint16)
    lib().or_encode_array(storage, _p(x), _p(q), x.size)
    return q


def decode(storage: int, q: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.uint16)
    x = np.empty(q.shape, dtype=np.float32)
    lib().or_decode_array(storage, _p(q), _p(x), q.size)
    return x


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 evaluated in FP64."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((x - ref).ravel()) / (den if den > 0 else 1.0))


if __name__ == "__main__":  # pragma: no cover
    print(build())
    sys.exit(0)
