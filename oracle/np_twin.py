"""NumPy twin of the FP64 oracle, for tiny grids.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  A second, independent
writing of the same definition: array slicing instead of loops, and the
stencil weights obtained by solving the moment conditions in exact rational
arithmetic instead of the closed form the C oracle uses.  Also holds the
tangent-linear model used by the adjoint dot-product test.

Definition (arXiv 2311.05038, Section 7, Eq. 1 and the step order of
Listing 3; readings as in oracle/fd_oracle.c):
  w^n     = y^n + dt^2/h^D s[n] e_src             (source added to P first)
  y^{n+1} = G (2 w^n + c L w^n) - G^2 w^{n-1}     (derivatives, time update)
  d^n     = y^{n+1}[receivers]
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

import numpy as np


def weights_exact(R: int) -> List[Fraction]:
    """a_0..a_R with sum_{k=-R..R} a_|k| k^(2m) = 2 delta_{m,1}, m = 0..R.

    Gauss-Jordan elimination over the rationals."""
    n = R + 1
    # unknowns a_0..a_R; row m: a_0 [m==0] + sum_{k>=1} 2 a_k k^(2m)
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for m in range(n):
        A[m][0] = Fraction(1 if m == 0 else 0)
        for k in range(1, n):
            A[m][k] = Fraction(2 * k ** (2 * m))
        b[m] = Fraction(2 if m == 1 else 0)
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        p = A[col][col]
        A[col] = [x / p for x in A[col]]
        b[col] = b[col] / p
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] = b[r] - f * b[col]
    return b


def _shift(u: np.ndarray, axis: int, k: int, periodic: bool) -> np.ndarray:
    """out[i] = u[i + k] along axis, zero (or wrapped) outside."""
    if periodic:
        return np.roll(u, -k, axis=axis)
    out = np.zeros_like(u)
    n = u.shape[axis]
    if abs(k) >= n:
        return out
    src = [slice(None)] * u.ndim
    dst = [slice(None)] * u.ndim
    if k > 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    out[tuple(dst)] = u[tuple(src)]
    return out


def laplacian(u: np.ndarray, R: int = 4, periodic: bool = False, dtype=np.float64) -> np.ndarray:
    a = [dtype(float(w)) for w in weights_exact(R)]
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        out = out + a[0] * u
        for k in range(1, R + 1):
            out = out + a[k] * (_shift(u, ax, k, periodic) + _shift(u, ax, -k, periodic))
    return out


def profile(n: int, width: int, alpha: float, lo: bool, hi: bool) -> np.ndarray:
    """One axis: exp(-(alpha d)^2), d = distance into the band of an enabled face."""
    i = np.arange(n, dtype=np.float64)
    d = np.zeros(n)
    if width > 0:
        if lo:
            d = np.maximum(d, width - i)
        if hi:
            d = np.maximum(d, i - (n - 1 - width))
    return np.exp(-(alpha * d) ** 2)


def sponge(shape: Sequence[int], width: int, alpha: float, faces: int) -> np.ndarray:
    """G = product of exp(-(alpha d)^2) axis profiles; face bits z-,z+,y-,y+,x-,x+."""
    G = np.ones(shape)
    axes_bits = [(0, 1)] + ([(2, 3)] if len(shape) == 3 else []) + [(4, 5)]
    for ax, (blo, bhi) in enumerate(axes_bits):
        n = shape[ax]
        g = profile(n, width, alpha, bool(faces >> blo & 1), bool(faces >> bhi & 1))
        bs = [1] * len(shape)
        bs[ax] = n
        G = G * g.reshape(bs)
    return G


class Twin:
    """The definition on a small grid (prob is an fd_inputs.Problem)."""

    def __init__(self, prob, v: np.ndarray):
        self.p = prob
        self.v = v.astype(np.float64)
        self.c = (self.v * prob.dt / prob.dh) ** 2
        self.G = sponge(prob.shape, prob.sponge_width, prob.alpha(), prob.sponge_faces)
        self.amp = prob.dt ** 2 / prob.dh ** prob.ndim
        self.periodic = prob.bc == 1
        src = prob.src if prob.ndim == 3 else (prob.src[0], prob.src[2])
        self.src = tuple(src)
        cells = prob.receivers.cells()
        if prob.ndim == 2:
            self.rec = (cells[:, 0], cells[:, 2])
        else:
            self.rec = (cells[:, 0], cells[:, 1], cells[:, 2])

    def L(self, u):
        return laplacian(u, self.p.radius, self.periodic)

    def forward(self, wavelet, nt, c=None, keep=False):
        c = self.c if c is None else c
        G = self.G
        prev = np.zeros(self.p.shape)
        cur = np.zeros(self.p.shape)
        traces = np.zeros((nt, len(self.rec[0])))
        ws = []
        for n in range(nt):
            cur = cur.copy()
            cur[self.src] += self.amp * float(wavelet[n])
            if keep:
                ws.append(cur.copy())
            new = G * (2 * cur + c * self.L(cur)) - G * G * prev
            traces[n] = new[self.rec]
            prev, cur = cur, new
        return traces, cur, prev, ws

    def tangent(self, wavelet, nt, dc):
        """Tangent-linear model: d traces for a perturbation dc of c."""
        G, c = self.G, self.c
        _, _, _, ws = self.forward(wavelet, nt, keep=True)
        dprev = np.zeros(self.p.shape)
        dcur = np.zeros(self.p.shape)
        dtr = np.zeros((nt, len(self.rec[0])))
        for n in range(nt):
            dnew = G * (2 * dcur + c * self.L(dcur) + dc * self.L(ws[n])) - G * G * dprev
            dtr[n] = dnew[self.rec]
            dprev, dcur = dcur, dnew
        return dtr

    def forward_m(self, wavelet, nt, m):
        """Forward map with the spatial operator L replaced by L + diag(m)
        (a field of point scatterers): traces only."""
        G, c = self.G, self.c
        prev = np.zeros(self.p.shape)
        cur = np.zeros(self.p.shape)
        traces = np.zeros((nt, len(self.rec[0])))
        for n in range(nt):
            cur = cur.copy()
            cur[self.src] += self.amp * float(wavelet[n])
            new = G * (2 * cur + c * (self.L(cur) + m * cur)) - G * G * prev
            traces[n] = new[self.rec]
            prev, cur = cur, new
        return traces

    def tangent_m(self, wavelet, nt, dm):
        """Tangent-linear model of forward_m at m = 0: d traces for dm."""
        G, c = self.G, self.c
        _, _, _, ws = self.forward(wavelet, nt, keep=True)
        dprev = np.zeros(self.p.shape)
        dcur = np.zeros(self.p.shape)
        dtr = np.zeros((nt, len(self.rec[0])))
        for n in range(nt):
            dnew = G * (2 * dcur + c * (self.L(dcur) + dm * ws[n])) - G * G * dprev
            dtr[n] = dnew[self.rec]
            dprev, dcur = dcur, dnew
        return dtr

    def adjoint_c(self, wavelet, nt, resid):
        """dJ/dc by back-propagation written directly from the forward map
        (ybar recursion, not the z-form used by the C oracle)."""
        G, c = self.G, self.c
        _, _, _, ws = self.forward(wavelet, nt, keep=True)
        ybar1 = np.zeros(self.p.shape)   # ybar^{k+1}
        ybar2 = np.zeros(self.p.shape)   # ybar^{k+2}
        gc = np.zeros(self.p.shape)
        for k in range(nt, 0, -1):
            # wbar^k = (dy^{k+1}/dw^k)^T ybar^{k+1} + (dy^{k+2}/dw^k)^T ybar^{k+2}
            wbar = 2 * G * ybar1 + self.L(c * G * ybar1) - G * G * ybar2
            ybar = wbar.copy()
            np.add.at(ybar, self.rec, resid[k - 1])
            gc += G * ybar * self.L(ws[k - 1])
            ybar2, ybar1 = ybar1, ybar
        return gc

    def forward_half(self, wavelet, nt, storage: int, c_fixed16: bool = False):
        """FP32 arithmetic with FP32 or 16-bit storage and power-of-two field
        scales.

        storage 0: FP32 storage (no rounding beyond the FP32 arithmetic);
        storage 1: numpy float16 (IEEE binary16, round to nearest even);
        storage 2: bfloat16 by round-to-nearest-even on the FP32 bit pattern.
        c_fixed16: c replaced by its 16-bit fixed-point value (codes
        rint(c 2^(16-e)) with e the least exponent that keeps every code
        below 2^16: 2^(e-1) <= max c < 2^e, plus one if max c rounds to 2^16)."""
        f32 = np.float32
        c = ((self.v * self.p.dt / self.p.dh) ** 2).astype(f32)
        if c_fixed16:
            e = int(np.frexp(c.max())[1])
            while np.rint(float(c.max()) * 2.0 ** (16 - e)) > 65535.0:
                e += 1
            codes = np.rint(c.astype(np.float64) * 2.0 ** (16 - e))
            assert codes.max() <= 65535.0
            c = (codes * 2.0 ** (e - 16)).astype(f32)
        shape = self.p.shape
        # axis profiles rounded to FP32, multiplied in z, y, x order
        axes_bits = [(0, 1)] + ([(2, 3)] if len(shape) == 3 else []) + [(4, 5)]
        profs = []
        for ax, (blo, bhi) in enumerate(axes_bits):
            n = shape[ax]
            f = self.p.sponge_faces
            g = profile(n, self.p.sponge_width, self.p.alpha(),
                        bool(f >> blo & 1), bool(f >> bhi & 1)).astype(f32)
            bs = [1] * len(shape)
            bs[ax] = n
            profs.append(g.reshape(bs))
        G = profs[0] * profs[1] if len(shape) == 2 else (profs[0] * profs[1]) * profs[2]
        G = np.broadcast_to(G, shape).astype(f32)
        a = [f32(float(w)) for w in weights_exact(self.p.radius)]
        amp = f32(self.amp)

        def enc(x):
            if storage == 0:
                return x.astype(f32)
            if storage == 1:
                return x.astype(np.float16)
            u = x.astype(f32).view(np.uint32).astype(np.uint64)
            kept = u >> 16
            rem = u & 0xFFFF
            up = (rem > 0x8000) | ((rem == 0x8000) & ((kept & 1) == 1))
            return (kept + up).astype(np.uint16)

        def dec(q):
            if storage == 0:
                return q.astype(f32)
            if storage == 1:
                return q.astype(f32)
            return (q.astype(np.uint32) << 16).view(f32)

        def expo(m):
            m = max(float(m), 2.0 ** -100)
            return int(np.frexp(f32(m))[1]) - 1 - 11

        def lap32(u):
            out = np.zeros_like(u)
            for ax in range(u.ndim):
                out = out + a[0] * u
                for k in range(1, self.p.radius + 1):
                    out = out + a[k] * (_shift(u, ax, k, False) + _shift(u, ax, -k, False))
            return out

        x0 = amp * f32(wavelet[0])
        ec = expo(abs(x0))
        tmp = np.zeros(shape, f32)
        tmp[self.src] = np.ldexp(x0, -ec)
        qc = enc(tmp)
        Mc = abs(x0)
        qp = enc(np.zeros(shape, f32))
        ep, Mp = 0, f32(0)
        traces = np.zeros((nt, len(self.rec[0])), dtype=f32)
        for n in range(nt):
            cur = np.ldexp(dec(qc), ec).astype(f32)
            prev = np.ldexp(dec(qp), ep).astype(f32)
            x = G * (f32(2) * cur + c * lap32(cur)) - (G * G) * prev
            traces[n] = x[self.rec]
            inj = amp * f32(wavelet[n + 1]) if n + 1 < nt else f32(0)
            x[self.src] += inj
            en = expo(max(Mc, Mp, abs(inj)))
            qn = enc(np.ldexp(x, -en).astype(f32))
            Mn = np.abs(x).max()
            qp, qc = qc, qn
            ep, ec = ec, en
            Mp, Mc = Mc, Mn
        return traces, np.ldexp(dec(qc), ec).astype(f32)
