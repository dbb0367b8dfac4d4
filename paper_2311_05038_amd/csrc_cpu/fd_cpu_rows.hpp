// Row loops of the host step, written once over a small vector-operations
// type and compiled once per instruction set (fd_cpu_avx2.cpp,
// fd_cpu_avx512.cpp, and the scalar form in fd_cpu.cpp).
//
// One call updates one grid row (fixed z, and y in 3D) in place:
//   new = G (2 P + c L P) - G^2 Pold,   G = gz(z) gy(y) gx(x),
// the fused form of Listing 3's fd_pzz, fd_pxx and fd_time (Section 7), with
// L the 8th-order second difference summed over the axes (weights
// a = (-205/72, 8/5, -1/5, 8/315, -1/560)).  Every multiply-add is an exact
// fused one and the order of operations is fixed (taps of one axis as
// a4 (u-4 + u+4) + (a3 (u-3 + u+3) + (a2 (u-2 + u+2) + a1 (u-1 + u+1))),
// axes as z + (y + x), then the centre), so the result does not depend on
// the vector width.
#pragma once

#include <cstddef>
#include <cstdint>

namespace fdcpu {

constexpr float kA0 = (float)(-205.0 / 72.0);
constexpr float kA1 = (float)(8.0 / 5.0);
constexpr float kA2 = (float)(-1.0 / 5.0);
constexpr float kA3 = (float)(8.0 / 315.0);
constexpr float kA4 = (float)(-1.0 / 560.0);

// One row's pointers.  P points at cell (z, y, x = 0) of the current level;
// neighbours at +-k along x are P[x +- k], along y P[x +- k*ys] and along z
// P[x +- k*zs] (the frame of zeros makes every one of them addressable).
// Q is the same cell of the other level: Pold on entry, Pnew on return.
struct Row {
    const float *P;
    float *Q;
    const float *c;   // c = (v dt / dh)^2 of the row
    const float *gx;  // damping factors along x (at least the rounded-up row length)
    float gzy;        // gz(z) gy(y) (gz(z) in 2D)
    ptrdiff_t ys, zs;
    int64_t nx;
};

template <class O>
inline typename O::V taps(typename O::V m4, typename O::V m3, typename O::V m2, typename O::V m1,
                          typename O::V p1, typename O::V p2, typename O::V p3, typename O::V p4)
{
    using V = typename O::V;
    const V t1 = O::mul(O::set1(kA1), O::add(m1, p1));
    const V t2 = O::fma(O::set1(kA2), O::add(m2, p2), t1);
    const V t3 = O::fma(O::set1(kA3), O::add(m3, p3), t2);
    return O::fma(O::set1(kA4), O::add(m4, p4), t3);
}

template <class O>
inline typename O::V axis_taps(const float *p, ptrdiff_t s)
{
    return taps<O>(O::ld(p - 4 * s), O::ld(p - 3 * s), O::ld(p - 2 * s), O::ld(p - s), O::ld(p + s),
                   O::ld(p + 2 * s), O::ld(p + 3 * s), O::ld(p + 4 * s));
}

template <class O, int NDIM>
inline void step_row(const Row &r)
{
    using V = typename O::V;
    const V kc = O::set1((float)NDIM * kA0);
    const V two = O::set1(2.0f);
    const V gzy = O::set1(r.gzy);
    for (int64_t x = 0; x < r.nx; x += O::W) {
        const float *p = r.P + x;
        const V ctr = O::ld(p);
        const V lx = axis_taps<O>(p, 1);
        const V lz = axis_taps<O>(p, r.zs);
        V sum;
        if constexpr (NDIM == 3)
            sum = O::add(lz, O::add(axis_taps<O>(p, r.ys), lx));
        else
            sum = O::add(lz, lx);
        const V lap = O::fma(kc, ctr, sum);
        const V G = O::mul(gzy, O::ld(r.gx + x));
        const V GG = O::neg(O::mul(G, G));
        V nw = O::fma(G, O::fma(O::ld(r.c + x), lap, O::mul(two, ctr)), O::mul(GG, O::ld(r.Q + x)));
        if (x + O::W > r.nx) nw = O::keep(nw, (int)(r.nx - x));  // cells past the row stay 0
        O::st(r.Q + x, nw);
    }
}

}  // namespace fdcpu
