"""ctypes binding of libfd.so, one Python function per C entry point of
include/fd.h, with the same names.  Argument marshalling only: every step of
the computation runs in the library's HIP kernels.  Device pointers are
passed as integers (torch's ``tensor.data_ptr()``), streams as the raw
``hipStream_t`` handle (torch's ``stream.cuda_stream``)."""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime first, so libfd.so binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfd.so")

FD_OK = 0
FD_ERR_INVALID_ARG = 1
FD_ERR_UNSTABLE = 2
FD_ERR_OUT_OF_MEMORY = 3
FD_ERR_DEVICE = 4
FD_ERR_UNSUPPORTED = 5
FD_F32, FD_F16, FD_BF16 = 0, 1, 2
FD_C_F32, FD_C_FIXED16 = 0, 1
FD_BC_ZERO, FD_BC_PERIODIC = 0, 1
FD_BATCH_MAX = 16

_STATUS_NAMES = {0: "FD_OK", 1: "FD_ERR_INVALID_ARG", 2: "FD_ERR_UNSTABLE",
                 3: "FD_ERR_OUT_OF_MEMORY", 4: "FD_ERR_DEVICE", 5: "FD_ERR_UNSUPPORTED"}


class fd_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("radius", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("sponge_width", ctypes.c_int32), ("nz", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nx", ctypes.c_int64), ("dh", ctypes.c_double), ("dt", ctypes.c_double),
                ("sponge_alpha", ctypes.c_double), ("sponge_faces", ctypes.c_uint32),
                ("storage", ctypes.c_int32), ("c_storage", ctypes.c_int32),
                ("slab_z0", ctypes.c_int64), ("slab_nz_global", ctypes.c_int64)]


class fd_receivers(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("z0", "y0", "x0", "nz", "ny", "nx", "dz", "dy", "dx")]


class fd_shot(ctypes.Structure):
    _fields_ = [("src_z", ctypes.c_int64), ("src_y", ctypes.c_int64), ("src_x", ctypes.c_int64),
                ("wavelet", ctypes.c_void_p), ("nt", ctypes.c_int64), ("rec", fd_receivers)]


class fd_sizes(ctypes.Structure):
    _fields_ = [("model", ctypes.c_size_t), ("state", ctypes.c_size_t),
                ("checkpoints", ctypes.c_size_t), ("adjoint_work", ctypes.c_size_t),
                ("routines_work", ctypes.c_size_t)]


class fd_batch_item(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("state", ctypes.c_void_p),
                ("shot", ctypes.POINTER(fd_shot)), ("n", ctypes.c_int64),
                ("traces", ctypes.c_void_p)]


class FDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# (name, restype, argtypes) of every symbol declared in include/fd.h
_P = ctypes.c_void_p
_I32, _I64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = [
    ("fd_query_bytes", ctypes.c_int, [ctypes.POINTER(fd_grid), _I64, _I32, ctypes.POINTER(fd_sizes)]),
    ("fd_create_model", ctypes.c_int, [ctypes.POINTER(fd_grid), _P, _P, _SZ, _P, ctypes.POINTER(_P)]),
    ("fd_destroy_model", ctypes.c_int, [_P]),
    ("fd_create_state", ctypes.c_int, [_P, _P, _SZ, ctypes.POINTER(_P)]),
    ("fd_destroy_state", ctypes.c_int, [_P]),
    ("fd_begin_shot", ctypes.c_int, [_P, _P, ctypes.POINTER(fd_shot), _P]),
    ("fd_step", ctypes.c_int, [_P, _P, ctypes.POINTER(fd_shot), _I64, _P, _P]),
    ("fd_run_shot", ctypes.c_int, [_P, _P, ctypes.POINTER(fd_shot), _P, _P, _SZ, _I32, _P]),
    ("fd_adjoint_gradient", ctypes.c_int,
     [_P, ctypes.POINTER(fd_shot), _P, _P, _SZ, _I32, _P, _SZ, _P, _P]),
    ("fd_rtm_image", ctypes.c_int,
     [_P, ctypes.POINTER(fd_shot), _P, _P, _SZ, _I32, _P, _SZ, _P, _P]),
    ("fd_run_shots", ctypes.c_int, [_P, _P, _P, _I32, _P, _P, _SZ, _I32, _P]),
    ("fd_adjoint_gradient_shots", ctypes.c_int, [_P, _P, _I32, _P, _P, _SZ, _I32, _P, _SZ, _P, _P]),
    ("fd_rtm_image_shots", ctypes.c_int, [_P, _P, _I32, _P, _P, _SZ, _I32, _P, _SZ, _P, _P]),
    ("fd_get_wavefield", ctypes.c_int, [_P, _I32, _P, _P]),
    ("fd_set_wavefield", ctypes.c_int, [_P, _I32, _P, _P]),
    ("fd_step_batch", ctypes.c_int, [ctypes.POINTER(fd_batch_item), _I32, _I32, _P]),
    ("fd_step_routines", ctypes.c_int, [_P, _P, ctypes.POINTER(fd_shot), _I64, _P, _P, _SZ, _P]),
    ("fd_step_routines_noalloc", ctypes.c_int, [_P, _P, ctypes.POINTER(fd_shot), _I64, _P, _P]),
    ("fd_slab_exchange", ctypes.c_int, [_P, _P, _P]),
    ("fd_check_finite", ctypes.c_int, [_P, _P, _P]),
    ("fd_stream_probe", ctypes.c_int, [_I32, _P, _P, _P, _SZ, _P]),
    ("fd_shot_graph_create", ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(_P)]),
    ("fd_shot_graph_launch", ctypes.c_int, [_P, _P]),
    ("fd_shot_graph_destroy", ctypes.c_int, [_P]),
    ("fd_last_error", ctypes.c_char_p, []),
    ("fd_version", ctypes.c_char_p, []),
]

_lib = None


def lib():
    """The loaded library.  Raises if libfd.so has not been built: there is
    no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2311_05038_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != FD_OK:
        raise FDError(status, fd_last_error())


def fd_last_error() -> str:
    return lib().fd_last_error().decode()


def fd_version() -> str:
    return lib().fd_version().decode()


def fd_query_bytes(grid: fd_grid, nt: int = 0, ckpt_every: int = 0) -> fd_sizes:
    out = fd_sizes()
    check(lib().fd_query_bytes(ctypes.byref(grid), nt, ckpt_every, ctypes.byref(out)))
    return out


def fd_create_model(grid: fd_grid, velocity_ptr: int, model_ptr: int, model_bytes: int,
                    stream: int) -> int:
    h = _P()
    check(lib().fd_create_model(ctypes.byref(grid), velocity_ptr, model_ptr, model_bytes, stream,
                                ctypes.byref(h)))
    return h.value


def fd_destroy_model(model: int) -> None:
    check(lib().fd_destroy_model(model))


def fd_create_state(model: int, state_ptr: int, state_bytes: int) -> int:
    h = _P()
    check(lib().fd_create_state(model, state_ptr, state_bytes, ctypes.byref(h)))
    return h.value


def fd_destroy_state(state: int) -> None:
    check(lib().fd_destroy_state(state))


def fd_begin_shot(model: int, state: int, shot: fd_shot, stream: int) -> None:
    check(lib().fd_begin_shot(model, state, ctypes.byref(shot), stream))


def fd_step(model: int, state: int, shot: fd_shot, n: int, trace_row_ptr, stream: int) -> None:
    check(lib().fd_step(model, state, ctypes.byref(shot), n, trace_row_ptr, stream))


def fd_step_routines(model: int, state: int, shot: fd_shot, n: int, trace_row_ptr, work_ptr: int,
                     work_bytes: int, stream: int) -> None:
    check(lib().fd_step_routines(model, state, ctypes.byref(shot), n, trace_row_ptr, work_ptr,
                                 work_bytes, stream))


def fd_step_routines_noalloc(model: int, state: int, shot: fd_shot, n: int, trace_row_ptr,
                             stream: int) -> None:
    check(lib().fd_step_routines_noalloc(model, state, ctypes.byref(shot), n, trace_row_ptr, stream))


def fd_stream_probe(kind: int, a_ptr: int, b_ptr, out_ptr: int, n: int, stream: int) -> None:
    check(lib().fd_stream_probe(kind, a_ptr, b_ptr, out_ptr, n, stream))


def fd_shot_graph_create(model: int, state: int, shot: fd_shot, traces_ptr) -> int:
    out = _P()
    check(lib().fd_shot_graph_create(model, state, ctypes.byref(shot), traces_ptr, ctypes.byref(out)))
    return out.value


def fd_shot_graph_launch(graph: int, stream: int) -> None:
    check(lib().fd_shot_graph_launch(graph, stream))


def fd_shot_graph_destroy(graph: int) -> None:
    check(lib().fd_shot_graph_destroy(graph))


def fd_check_finite(state: int, flags_ptr: int, stream: int) -> None:
    check(lib().fd_check_finite(state, flags_ptr, stream))


# size of the library's static work area (FD_ROUTINES_STATIC_BYTES)
ROUTINES_STATIC_BYTES = 64 << 20


def fd_run_shot(model: int, state: int, shot: fd_shot, traces_ptr, ckpt_ptr, ckpt_bytes: int,
                ckpt_every: int, stream: int) -> None:
    check(lib().fd_run_shot(model, state, ctypes.byref(shot), traces_ptr, ckpt_ptr, ckpt_bytes,
                            ckpt_every, stream))


def fd_adjoint_gradient(model: int, shot: fd_shot, adj_ptr: int, ckpt_ptr: int, ckpt_bytes: int,
                        ckpt_every: int, work_ptr: int, work_bytes: int, grad_v_ptr: int,
                        stream: int) -> None:
    check(lib().fd_adjoint_gradient(model, ctypes.byref(shot), adj_ptr, ckpt_ptr, ckpt_bytes,
                                    ckpt_every, work_ptr, work_bytes, grad_v_ptr, stream))


def fd_rtm_image(model: int, shot: fd_shot, data_ptr: int, ckpt_ptr: int, ckpt_bytes: int,
                 ckpt_every: int, work_ptr: int, work_bytes: int, image_ptr: int,
                 stream: int) -> None:
    check(lib().fd_rtm_image(model, ctypes.byref(shot), data_ptr, ckpt_ptr, ckpt_bytes,
                             ckpt_every, work_ptr, work_bytes, image_ptr, stream))


def _ptrs(values):
    """A C array of pointers (None -> NULL) and the array object to keep alive."""
    arr = (ctypes.c_void_p * len(values))(*[v if v else None for v in values])
    return ctypes.cast(arr, ctypes.c_void_p), arr


def fd_run_shots(model: int, states, shots, traces_ptrs, ckpt_ptrs, ckpt_bytes: int,
                 ckpt_every: int, stream: int) -> None:
    st, a1 = _ptrs(states)
    sh, a2 = _ptrs([ctypes.addressof(s) for s in shots])
    tr, a3 = _ptrs(traces_ptrs) if traces_ptrs is not None else (None, None)
    ck, a4 = _ptrs(ckpt_ptrs) if ckpt_ptrs is not None else (None, None)
    check(lib().fd_run_shots(model, st, sh, len(shots), tr, ck, ckpt_bytes, ckpt_every, stream))


def fd_adjoint_gradient_shots(model: int, shots, adj_ptrs, ckpt_ptrs, ckpt_bytes: int,
                              ckpt_every: int, work_ptrs, work_bytes: int, grad_v_ptr: int,
                              stream: int) -> None:
    sh, a1 = _ptrs([ctypes.addressof(s) for s in shots])
    ad, a2 = _ptrs(adj_ptrs)
    ck, a3 = _ptrs(ckpt_ptrs)
    wk, a4 = _ptrs(work_ptrs)
    check(lib().fd_adjoint_gradient_shots(model, sh, len(shots), ad, ck, ckpt_bytes, ckpt_every,
                                          wk, work_bytes, grad_v_ptr, stream))


def fd_rtm_image_shots(model: int, shots, data_ptrs, ckpt_ptrs, ckpt_bytes: int, ckpt_every: int,
                       work_ptrs, work_bytes: int, image_ptr: int, stream: int) -> None:
    sh, a1 = _ptrs([ctypes.addressof(s) for s in shots])
    dt, a2 = _ptrs(data_ptrs)
    ck, a3 = _ptrs(ckpt_ptrs)
    wk, a4 = _ptrs(work_ptrs)
    check(lib().fd_rtm_image_shots(model, sh, len(shots), dt, ck, ckpt_bytes, ckpt_every, wk,
                                   work_bytes, image_ptr, stream))


def fd_get_wavefield(state: int, which: int, out_ptr: int, stream: int) -> None:
    check(lib().fd_get_wavefield(state, which, out_ptr, stream))


def fd_set_wavefield(state: int, which: int, in_ptr: int, stream: int) -> None:
    check(lib().fd_set_wavefield(state, which, in_ptr, stream))


def fd_slab_exchange(upper: int, lower: int, stream: int) -> None:
    check(lib().fd_slab_exchange(upper, lower, stream))


def fd_step_batch(items, nsteps: int, stream: int) -> None:
    """items: a ctypes array of fd_batch_item (n fields are updated in place)."""
    check(lib().fd_step_batch(items, len(items), nsteps, stream))
