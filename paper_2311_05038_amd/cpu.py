"""The host back-end: libfd_cpu.so, the C ABI of include/fd.h over host
memory (include/fd_cpu.h), bound with ctypes under the same names.

It is chosen explicitly (``from paper_2311_05038_amd import cpu``) and never
loaded by the GPU package, which has no fallback.  Buffers are numpy arrays;
argument marshalling only, every step runs in the library.

    m = cpu.Model(grid, velocity)               # fd_create_model
    s = m.new_state()                           # fd_create_state
    traces = m.run_shot(s, cpu.Shot(src, wavelet, receivers))   # fd_run_shot
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from ._abi import SIGNATURES, FDError, FD_OK, fd_grid, fd_shot, fd_sizes

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfd_cpu.so")

_P = ctypes.c_void_p
EXTRA_SIGNATURES = [
    ("fd_cpu_threads", ctypes.c_int32, [ctypes.c_int32]),
    ("fd_cpu_isa", ctypes.c_char_p, []),
    ("fd_cpu_set_isa", ctypes.c_int, [ctypes.c_char_p]),
    ("fd_cpu_stream_probe", ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_double)]),
]

_lib = None


def lib():
    """The loaded host library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2311_05038_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES + EXTRA_SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != FD_OK:
        raise FDError(status, lib().fd_last_error().decode())


def threads(n: int = 0) -> int:
    """fd_cpu_threads: set (n >= 1) and return the thread count."""
    return int(lib().fd_cpu_threads(n))


def isa() -> str:
    return lib().fd_cpu_isa().decode()


def set_isa(name: str) -> None:
    check(lib().fd_cpu_set_isa(name.encode()))


def version() -> str:
    return lib().fd_version().decode()


def stream_probe(n_floats: int = 1 << 26, reps: int = 5) -> float:
    """fd_cpu_stream_probe: GB/s of the step's 3-read / 1-rewrite pattern."""
    out = ctypes.c_double()
    check(lib().fd_cpu_stream_probe(n_floats, reps, ctypes.byref(out)))
    return out.value


def _aligned(nbytes: int) -> np.ndarray:
    """A 256-byte aligned host byte buffer."""
    raw = np.zeros(int(nbytes) + 256, dtype=np.uint8)
    off = (-raw.ctypes.data) % 256
    return raw[off:off + max(int(nbytes), 1)]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Shot:
    """A point source with its wavelet (host FP32 array) and receivers (the
    package's Receivers)."""

    def __init__(self, src, wavelet: np.ndarray, receivers):
        self.wavelet = np.ascontiguousarray(wavelet, dtype=np.float32)
        self.src = tuple(int(v) for v in src)
        self.receivers = receivers
        self.nt = int(self.wavelet.size)
        self._c = fd_shot(src_z=self.src[0], src_y=self.src[1], src_x=self.src[2],
                          wavelet=self.wavelet.ctypes.data, nt=self.nt, rec=receivers.c())

    @property
    def nrec(self) -> int:
        return self.receivers.count


class Model:
    """fd_create_model over a host buffer; `grid` is the package's Grid."""

    def __init__(self, grid, velocity: np.ndarray):
        v = np.ascontiguousarray(velocity, dtype=np.float32).reshape(-1)
        if v.size != grid.ncells:
            raise ValueError(f"velocity has {v.size} cells, grid has {grid.ncells}")
        self.grid = grid
        self._g: fd_grid = grid.c()
        self.sizes = fd_sizes()
        check(lib().fd_query_bytes(ctypes.byref(self._g), 0, 0, ctypes.byref(self.sizes)))
        self.buf = _aligned(self.sizes.model)
        h = _P()
        check(lib().fd_create_model(ctypes.byref(self._g), v.ctypes.data, self.buf.ctypes.data,
                                    self.sizes.model, None, ctypes.byref(h)))
        self.handle = h.value

    def new_state(self) -> "State":
        return State(self)

    def run_shot(self, state: "State", shot: Shot, traces: Optional[np.ndarray] = None) -> np.ndarray:
        if traces is None:
            traces = np.empty((shot.nt, shot.nrec), dtype=np.float32)
        check(lib().fd_run_shot(self.handle, state.handle, ctypes.byref(shot._c),
                                _ptr(traces) if shot.nrec > 0 else None, None, 0, 0, None))
        state.next = shot.nt
        return traces

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.fd_destroy_model(h)
            self.handle = None


class State:
    """fd_create_state: the two time levels of one shot, in host memory."""

    def __init__(self, model: Model):
        self.model = model
        self.buf = _aligned(model.sizes.state)
        h = _P()
        check(lib().fd_create_state(model.handle, self.buf.ctypes.data, model.sizes.state,
                                    ctypes.byref(h)))
        self.handle = h.value
        self.next = -1

    def begin(self, shot: Shot) -> None:
        check(lib().fd_begin_shot(self.model.handle, self.handle, ctypes.byref(shot._c), None))
        self.next = 0

    def step(self, shot: Shot, n: int, trace_row: Optional[np.ndarray] = None) -> None:
        check(lib().fd_step(self.model.handle, self.handle, ctypes.byref(shot._c), n,
                            _ptr(trace_row), None))
        self.next = n + 1

    def wavefield(self, which: int = 0) -> np.ndarray:
        out = np.empty(self.model.grid.shape, dtype=np.float32)
        check(lib().fd_get_wavefield(self.handle, which, out.ctypes.data, None))
        return out

    def check_finite(self) -> int:
        """fd_check_finite: bit 0 (P) and bit 1 (Pold) set when that level
        holds a NaN or an infinity; 0 for a healthy shot."""
        flags = np.zeros(1, dtype=np.uint32)
        check(lib().fd_check_finite(self.handle, flags.ctypes.data, None))
        return int(flags[0])

    def set_wavefield(self, which: int, values: np.ndarray) -> None:
        v = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
        if v.size != self.model.grid.ncells:
            raise ValueError("values must have one entry per cell")
        check(lib().fd_set_wavefield(self.handle, which, v.ctypes.data, None))
        if self.next < 0:
            self.next = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.fd_destroy_state(h)
            self.handle = None
