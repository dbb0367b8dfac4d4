"""Seeded synthetic inputs for the acoustic finite-difference workloads.

This module is shared by the oracle side and the GPU side of every test and
benchmark.  It holds no arithmetic of the time-stepping method itself: only
the things the method consumes — source wavelets, velocity models, source and
receiver placements, grid descriptions and request streams.  Everything is a
pure function of its arguments and a seed.

The paper (Section 7, Eq. 1) fixes only the equation
``P_tt = v(x,z)^2 (P_xx + P_zz) + S(t)`` with a space-dependent velocity and a
time-dependent source.  The concrete shapes below (grid sizes, spacing, time
step, wavelet, velocity statistics, receiver layouts) are the workload recipes
of this repository; the readings that fill the paper's silences are listed
with each generator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Sponge face bits: z-, z+, y-, y+, x-, x+ .  "All faces but z-" keeps the top
# (z = 0) as a zero-pressure free surface.
FACE_ZLO, FACE_ZHI, FACE_YLO, FACE_YHI, FACE_XLO, FACE_XHI = (1 << i for i in range(6))
FACES_ALL = 0x3F
FACES_NO_TOP = FACES_ALL & ~FACE_ZLO

BC_ZERO = 0
BC_PERIODIC = 1

STORE_F32 = 0
STORE_F16 = 1
STORE_BF16 = 2


@dataclasses.dataclass
class Receivers:
    """A regular receiver array: a box of cells sampled with a stride.

    Receiver r is ordered (rz, ry, rx) row-major with rx fastest; its cell is
    (z0 + rz*dz, y0 + ry*dy, x0 + rx*dx).
    """
    z0: int
    y0: int
    x0: int
    nz: int
    ny: int
    nx: int
    dz: int = 1
    dy: int = 1
    dx: int = 1

    @property
    def count(self) -> int:
        return self.nz * self.ny * self.nx

    def cells(self) -> np.ndarray:
        """(count, 3) int64 array of (z, y, x) in receiver order."""
        rz, ry, rx = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                                 np.arange(self.nx), indexing="ij")
        return np.stack([self.z0 + rz.ravel() * self.dz,
                         self.y0 + ry.ravel() * self.dy,
                         self.x0 + rx.ravel() * self.dx], axis=1).astype(np.int64)

    def linear(self, ny: int, nx: int) -> np.ndarray:
        """Linear cell indices (z*ny + y)*nx + x of every receiver, in order."""
        c = self.cells()
        return ((c[:, 0] * ny + c[:, 1]) * nx + c[:, 2]).astype(np.int64)


@dataclasses.dataclass
class Problem:
    """One forward-modelling workload: grid, model, source, receivers, steps."""
    name: str
    ndim: int
    nz: int
    ny: int
    nx: int
    dh: float
    dt: float
    nt: int
    src: Tuple[int, int, int]          # (z, y, x); y = 0 in 2D
    receivers: Receivers
    f0: float                          # Ricker peak frequency, Hz
    radius: int = 4
    bc: int = BC_ZERO
    sponge_width: int = 0
    sponge_alpha: float = 0.0          # 0 -> 0.3 / sponge_width
    sponge_faces: int = FACES_NO_TOP
    velocity_kind: str = "constant"
    velocity_seed: int = 0
    v_const: float = 2000.0

    @property
    def shape(self) -> Tuple[int, ...]:
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nz * self.ny * self.nx

    def alpha(self) -> float:
        if self.sponge_width <= 0:
            return 0.0
        return self.sponge_alpha if self.sponge_alpha > 0 else 0.3 / self.sponge_width

    def wavelet(self, nt: Optional[int] = None) -> np.ndarray:
        return ricker(self.f0, self.dt, self.nt if nt is None else nt)

    def velocity(self) -> np.ndarray:
        if self.velocity_kind == "constant":
            return np.full(self.shape, self.v_const, dtype=np.float32)
        if self.velocity_kind == "layered":
            return layered_velocity(self.shape, self.velocity_seed)
        if self.velocity_kind == "grf":
            return grf_velocity(self.shape, self.velocity_seed, corr_cells=200.0 / self.dh)
        if self.velocity_kind == "gradient":
            return gradient_velocity(self.shape)
        if self.velocity_kind == "random":
            return random_velocity(self.shape, self.velocity_seed, 1500.0, 3000.0)
        raise ValueError(self.velocity_kind)

    def rec_index(self) -> np.ndarray:
        return self.receivers.linear(self.ny, self.nx)

    def scaled(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Source wavelet
# --------------------------------------------------------------------------

def ricker(f0: float, dt: float, nt: int, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet sampled at t_n = n*dt, peak 1 at t0 (default 1.5/f0).

    The paper only says the source is time dependent (Section 7); the Ricker
    pulse is this repository's choice, delayed so that s(0) is ~1e-8.
    """
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


# --------------------------------------------------------------------------
# Velocity models
# --------------------------------------------------------------------------

def layered_velocity(shape: Tuple[int, ...], seed: int, vmin: float = 1500.0,
                     vmax: float = 4500.0, sigma: float = 50.0) -> np.ndarray:
    """Flat layers plus i.i.d. Gaussian noise, clipped to [vmin, vmax], FP32.

    10-20 layers; interfaces at sorted uniform fractional depths (so a seed
    gives the same structure at any nz); layer velocities are sorted uniform
    draws with the top layer at vmin.  Noise is drawn plane by plane in z order
    so memory stays bounded for the 768x768x512 grid.
    """
    rng = np.random.default_rng(seed)
    nlay = int(rng.integers(10, 21))
    interfaces = np.sort(rng.uniform(0.0, 1.0, nlay - 1))
    vel = np.sort(rng.uniform(vmin, vmax, nlay))
    vel[0] = vmin
    nz = shape[0]
    zf = (np.arange(nz) + 0.5) / nz
    layer_of_z = np.searchsorted(interfaces, zf, side="right")
    out = np.empty(shape, dtype=np.float32)
    plane = shape[1:]
    for z in range(nz):
        noise = rng.standard_normal(plane, dtype=np.float32) * np.float32(sigma)
        np.clip(noise + np.float32(vel[layer_of_z[z]]), vmin, vmax, out=out[z])
    return out


def grf_velocity(shape: Tuple[int, ...], seed: int, mean: float = 3000.0,
                 std: float = 500.0, corr_cells: float = 20.0,
                 vmin: float = 1500.0, vmax: float = 4500.0) -> np.ndarray:
    """Smoothed Gaussian random field, FP32.

    White N(0,1) noise is convolved (periodic FFT) with a Gaussian kernel of
    standard deviation corr_cells/sqrt(2), which makes the covariance
    exp(-r^2 / (2 corr^2)); the result is renormalised to the empirical std,
    shifted to the mean and clipped.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(shape)
    sk = corr_cells / math.sqrt(2.0)
    spec = np.fft.rfftn(white)
    # Fourier transform of a unit-mass Gaussian of std sk on each axis.
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = np.fft.rfftfreq(n)
        else:
            k = np.fft.fftfreq(n)
        g = np.exp(-2.0 * (math.pi * k * sk) ** 2)
        bshape = [1] * len(shape)
        bshape[ax] = g.size
        spec *= g.reshape(bshape)
    f = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    f = (f - f.mean()) / f.std()
    return np.clip(mean + std * f, vmin, vmax).astype(np.float32)


def grf_velocity_torch(shape: Tuple[int, ...], seed: int, device="cuda", mean: float = 3000.0,
                       std: float = 500.0, corr_cells: float = 20.0, vmin: float = 1500.0,
                       vmax: float = 4500.0):
    """The recipe of grf_velocity (white N(0,1) noise, periodic FFT smoothing
    with a Gaussian of std corr_cells/sqrt(2) per axis, renormalised, shifted,
    clipped, FP32) drawn with torch's generator on `device` on the
    power-of-two shape that holds `shape` and cropped to it: the same
    distribution (not the same numbers), in milliseconds per model, with a
    handful of FFT sizes for any mix of shapes."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    full = tuple(1 << max(0, int(n - 1).bit_length()) for n in shape)
    white = torch.randn(full, generator=g, device=device, dtype=torch.float32)
    sk = corr_cells / math.sqrt(2.0)
    spec = torch.fft.rfftn(white)
    for ax, n in enumerate(full):
        if ax == len(full) - 1:
            k = torch.fft.rfftfreq(n, device=device)
        else:
            k = torch.fft.fftfreq(n, device=device)
        w = torch.exp(-2.0 * (math.pi * k * sk) ** 2)
        bshape = [1] * len(full)
        bshape[ax] = w.numel()
        spec *= w.reshape(bshape)
    f = torch.fft.irfftn(spec, s=full, dim=tuple(range(len(full))))
    f = f[tuple(slice(0, n) for n in shape)]
    f = (f - f.mean()) / f.std(correction=0)
    return torch.clamp(mean + std * f, vmin, vmax).to(torch.float32).contiguous()


def gradient_velocity(shape: Tuple[int, ...], vtop: float = 2000.0,
                      vbot: float = 4000.0) -> np.ndarray:
    """1-D linear-in-depth start model v0(z) = vtop + (vbot-vtop) z/(nz-1)."""
    nz = shape[0]
    prof = vtop + (vbot - vtop) * np.arange(nz, dtype=np.float64) / (nz - 1)
    out = np.empty(shape, dtype=np.float32)
    out[...] = prof.reshape((nz,) + (1,) * (len(shape) - 1)).astype(np.float32)
    return out


def perturbation(shape: Tuple[int, ...], seed: int, scale: float = 1.0) -> np.ndarray:
    """Unit-rms random direction for derivative checks (FP64)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(shape)
    return scale * d / np.sqrt(np.mean(d * d))


def random_velocity(shape: Tuple[int, ...], seed: int, vmin: float = 1500.0,
                    vmax: float = 4500.0) -> np.ndarray:
    """Uniform i.i.d. velocities, FP32 (small test grids)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(vmin, vmax, shape).astype(np.float32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def random_geometry(seed: int) -> Problem:
    """A small seeded workload of arbitrary shape, for sweeps that look for
    shape-dependent mistakes (tile and chunk edges, axes shorter than the
    stencil, odd strides): 2D or 3D, each axis drawn from sizes between 1 and
    a few tiles (x up to 300), 1 to 13 steps, the source anywhere, a strided
    receiver box anywhere (sometimes empty), sponge width 0-5 on a random set
    of faces.  Velocities come from random_velocity(shape, seed, 1500, 3000)
    (Courant number at most 0.3 with dh = 10 m, dt = 1 ms)."""
    rng = np.random.default_rng(10_000 + seed)
    ndim = 2 if rng.random() < 0.4 else 3
    short = [1, 2, 3, 4, 5, 7, 8, 9, 12, 17, 31, 33, 40]
    nz = int(rng.choice(short))
    ny = 1 if ndim == 2 else int(rng.choice(short))
    nx = int(rng.choice(short + [63, 65, 130, 257, 300]))
    nt = int(rng.choice([1, 2, 5, 13]))
    src = (int(rng.integers(nz)), 0 if ndim == 2 else int(rng.integers(ny)), int(rng.integers(nx)))

    def axis(n):
        d = int(rng.integers(1, 4))
        o = int(rng.integers(n))
        return o, int(rng.integers(1, (n - 1 - o) // d + 2)), d

    (z0, cz, dz), (x0, cx, dx) = axis(nz), axis(nx)
    y0, cy, dy = (0, 1, 1) if ndim == 2 else axis(ny)
    rec = Receivers(z0, y0, x0, cz, cy, cx, dz, dy, dx)
    if rng.random() < 0.1:
        rec = Receivers(0, 0, 0, 0, 0, 0)
    return Problem(name=f"random{seed}", ndim=ndim, nz=nz, ny=ny, nx=nx, dh=10.0, dt=1e-3, nt=nt,
                   src=src, receivers=rec, f0=float(rng.choice([10.0, 20.0, 30.0])),
                   sponge_width=int(rng.integers(0, 6)), sponge_faces=int(rng.integers(0, 64)),
                   velocity_kind="random", velocity_seed=seed)


def green2d() -> Problem:
    """2D homogeneous medium: 256x256, dh=10 m, v=2000 m/s, dt=0.5 ms, 500
    steps, 15 Hz Ricker at the centre cell (128,128), a full receiver row
    through the source, zero edges, no sponge."""
    n = 256
    return Problem(name="green2d_256", ndim=2, nz=n, ny=1, nx=n, dh=10.0, dt=5e-4,
                   nt=500, src=(n // 2, 0, n // 2),
                   receivers=Receivers(n // 2, 0, 0, 1, 1, n), f0=15.0,
                   sponge_width=0, velocity_kind="constant", v_const=2000.0)


def layered3d(nx: int = 512, ny: int = 512, nz: int = 512, nt: int = 1000,
              seed: int = 2311) -> Problem:
    """3D layered model: dh=10 m, dt=1 ms, 12 Hz Ricker at (4, ny/2, nx/2),
    a 256x256 receiver block at depth index 2 centred laterally (clipped to
    the grid on small test grids), a 32-cell sponge on every face but the top
    (thinner on small grids)."""
    rny, rnx = min(256, ny), min(256, nx)
    width = 32 if min(nx, ny, nz) >= 128 else max(2, min(nx, ny, nz) // 8)
    return Problem(name=f"layered3d_{nx}x{ny}x{nz}", ndim=3, nz=nz, ny=ny, nx=nx,
                   dh=10.0, dt=1e-3, nt=nt, src=(min(4, nz - 1), ny // 2, nx // 2),
                   receivers=Receivers(min(2, nz - 1), ny // 2 - rny // 2,
                                       nx // 2 - rnx // 2, 1, rny, rnx),
                   f0=12.0, sponge_width=width, sponge_faces=FACES_NO_TOP,
                   velocity_kind="layered", velocity_seed=seed)


def precision3d(nt: int = 2000) -> Problem:
    """The 768x768x512 (x, y, z) precision workload: same generator, seed,
    source and receiver layout as layered3d, 2000 steps."""
    return layered3d(nx=768, ny=768, nz=512, nt=nt).scaled(name="precision3d_768x768x512")


def surface2d(nz: int, nx: int, nt: int, seed: int, src_x: Optional[int] = None,
              name: str = "surface2d", kind: str = "grf") -> Problem:
    """2D surface-acquisition shot: dh=10 m, dt=1 ms, 10 Hz Ricker at depth
    index 2, a receiver at every x on depth index 2, a 32-cell sponge on the
    bottom and both sides (narrower on small test grids)."""
    width = 32 if min(nx, nz) >= 128 else max(2, min(nx, nz) // 8)
    return Problem(name=name, ndim=2, nz=nz, ny=1, nx=nx, dh=10.0, dt=1e-3, nt=nt,
                   src=(2, 0, nx // 2 if src_x is None else src_x),
                   receivers=Receivers(2, 0, 0, 1, 1, nx), f0=10.0,
                   sponge_width=width, sponge_faces=FACES_NO_TOP,
                   velocity_kind=kind, velocity_seed=seed)


def adjoint2d(n: int = 1024, nt: int = 2000, nshots: int = 8, seed: int = 5038):
    """The gradient workload: n x n, 8 shots at depth index 2 and
    x = n/16 + k*n/8 (64 + 128 k at n = 1024), receivers at every x on depth
    index 2, checkpoint interval 50.  Returns (shots, true_v, start_v)."""
    shots = [surface2d(n, n, nt, seed, src_x=n // 16 + k * (n // 8),
                       name=f"adjoint2d_{n}_shot{k}") for k in range(nshots)]
    true_v = grf_velocity((n, n), seed, corr_cells=200.0 / 10.0)
    start_v = gradient_velocity((n, n))
    return shots, true_v, start_v


@dataclasses.dataclass
class Request:
    """One shot request of the serving stream."""
    rid: int
    arrival: float      # seconds from stream start
    nz: int
    nx: int
    nt: int
    seed: int


def serving_stream(n_requests: int, seed: int = 50, rate: float = 50.0,
                   nz_range=(512, 2048), nx_range=(512, 4096),
                   nt_range=(1000, 4000)) -> List[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate) of shots whose grid and
    step count are drawn uniformly from the given integer ranges."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        out.append(Request(i, t, int(rng.integers(nz_range[0], nz_range[1] + 1)),
                           int(rng.integers(nx_range[0], nx_range[1] + 1)),
                           int(rng.integers(nt_range[0], nt_range[1] + 1)),
                           int(rng.integers(0, 2**31 - 1))))
    return out


def request_problem(req: Request) -> Problem:
    return surface2d(req.nz, req.nx, req.nt, req.seed, name=f"req{req.rid}")
