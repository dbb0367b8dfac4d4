// Row loops of the host step, written once over a small vector-operations
// type and compiled once per instruction set (fd_cpu_avx2.cpp,
// fd_cpu_avx512.cpp, and the scalar form in fd_cpu.cpp).
//
// One call updates one grid row (fixed z, and y in 3D) in place:
//   new = G (2 P + c L P) - G^2 Pold,   G = gz(z) gy(y) gx(x),
// the fused form of Listing 3's fd_pzz, fd_pxx and fd_time (Section 7), with
// L the 8th-order second difference summed over the axes (weights
// a = (-205/72, 8/5, -1/5, 8/315, -1/560)).  Every multiply-add is an exact
// fused one and the order of operations is fixed, so the result does not
// depend on the vector width: each axis as
// c34 u + (a4 s4 + (a3 s3 + (a2 d2 + a1 d1))) with dk = (u-k - u) + (u+k - u),
// sk = u-k + u+k and c34 = -2 (a3 + a4) = -17/360 (the centre weight
// a0 = -2 (a1 + a2 + a3 + a4) folded into the two differences and c34),
// axes as z + (y + x), and the update as G (P + (c L + (P - G Pold))).
#pragma once

#include <cstddef>
#include <cstdint>

namespace fdcpu {

constexpr float kA1 = (float)(8.0 / 5.0);
constexpr float kA2 = (float)(-1.0 / 5.0);
constexpr float kA3 = (float)(8.0 / 315.0);
constexpr float kA4 = (float)(-1.0 / 560.0);
constexpr float kC34 = (float)(-17.0 / 360.0);

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
inline typename O::V dsum(typename O::V m, typename O::V u, typename O::V p)
{
    return O::add(O::sub(m, u), O::sub(p, u));
}

// The second difference along one axis, from the centre value u.
template <class O>
inline typename O::V axis_d2(const float *p, ptrdiff_t s, typename O::V u)
{
    using V = typename O::V;
    const V t1 = O::mul(O::set1(kA1), dsum<O>(O::ld(p - s), u, O::ld(p + s)));
    const V t2 = O::fma(O::set1(kA2), dsum<O>(O::ld(p - 2 * s), u, O::ld(p + 2 * s)), t1);
    const V t3 = O::fma(O::set1(kA3), O::add(O::ld(p - 3 * s), O::ld(p + 3 * s)), t2);
    const V t4 = O::fma(O::set1(kA4), O::add(O::ld(p - 4 * s), O::ld(p + 4 * s)), t3);
    return O::fma(O::set1(kC34), u, t4);
}

template <class O, int NDIM>
inline void step_row(const Row &r)
{
    using V = typename O::V;
    const V gzy = O::set1(r.gzy);
    for (int64_t x = 0; x < r.nx; x += O::W) {
        const float *p = r.P + x;
        const V ctr = O::ld(p);
        const V lx = axis_d2<O>(p, 1, ctr);
        const V lz = axis_d2<O>(p, r.zs, ctr);
        V lap;
        if constexpr (NDIM == 3)
            lap = O::add(lz, O::add(axis_d2<O>(p, r.ys, ctr), lx));
        else
            lap = O::add(lz, lx);
        const V G = O::mul(gzy, O::ld(r.gx + x));
        const V inc = O::fma(O::ld(r.c + x), lap, O::fma(O::neg(G), O::ld(r.Q + x), ctr));
        V nw = O::mul(G, O::add(ctr, inc));
        if (x + O::W > r.nx) nw = O::keep(nw, (int)(r.nx - x));  // cells past the row stay 0
        O::st(r.Q + x, nw);
    }
}

}  // namespace fdcpu
