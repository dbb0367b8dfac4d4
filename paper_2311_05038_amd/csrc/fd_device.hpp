// Device-side definitions shared by the step kernels (gfx950).
//
// One fused kernel computes one time step of the explicit scheme for the
// acoustic wave equation (arXiv 2311.05038, Section 7, Eq. 1), i.e. the
// routines of Listing 3 (source addition, z- and x-derivatives [and y],
// time update, level rotation) in a single pass over HBM:
//   new = G (2 cur + c L cur) - G^2 prev      (written over prev)
// with receivers sampled from `new` and the next source addition applied to
// `new` in the same pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd_args.hpp"

namespace fdk {

// 8th-order central second-difference weights (radius 4), h = 1.
constexpr float kA0 = (float)(-205.0 / 72.0);
constexpr float kA1 = (float)(8.0 / 5.0);
constexpr float kA2 = (float)(-1.0 / 5.0);
constexpr float kA3 = (float)(8.0 / 315.0);
constexpr float kA4 = (float)(-1.0 / 560.0);

// sum_k a_k (u_{-k} + u_{+k}), k = 1..4 (the 16-bit steps add a_0 u
// afterwards).  The library is built with -ffp-contract=off; every fused
// multiply-add is written out, so all kernel variants round identically.
__device__ __forceinline__ float stencil_taps(float m4, float m3, float m2, float m1, float p1,
                                              float p2, float p3, float p4)
{
    return fmaf(kA4, m4 + p4, fmaf(kA3, m3 + p3, fmaf(kA2, m2 + p2, kA1 * (m1 + p1))));
}

// The whole second difference along one axis, a_0 u + sum_k a_k (u_{-k} +
// u_{+k}), evaluated with the two large weights on differences from the
// centre value:
//   a_1 ((u_{-1} - u) + (u_{+1} - u)) + a_2 ((u_{-2} - u) + (u_{+2} - u))
//     + a_3 (u_{-3} + u_{+3}) + a_4 (u_{-4} + u_{+4}) - 2 (a_3 + a_4) u
// (equal, since a_0 = -2 (a_1 + a_2 + a_3 + a_4); -2 (a_3 + a_4) = -17/360).
// For a smooth field the differences are small and nearly exact, so the
// partial sums stay near the derivative (within 0.05 |u|) instead of reaching
// a_1 2 |u| = 3.2 |u| as when a_0 u is summed against all the taps; that
// cancellation error, carried by the leapfrog's slowly decaying
// long-wavelength modes, dominated the FP32 field error.  Differences on all
// four taps give the same accuracy at three more instructions per axis.
constexpr float kC34 = (float)(-17.0 / 360.0);
__device__ __forceinline__ float axis_d2(float m4, float m3, float m2, float m1, float u, float p1,
                                         float p2, float p3, float p4)
{
    return fmaf(kC34, u,
                fmaf(kA4, m4 + p4, fmaf(kA3, m3 + p3, fmaf(kA2, (m2 - u) + (p2 - u), kA1 * ((m1 - u) + (p1 - u))))));
}

// new = G (2 cur + c lap) - G^2 prev, evaluated as G (cur + (c lap + (cur -
// G prev))): the small increment c lap + (cur - G prev) is formed before the
// large cur is added (G = 1 off the damping band).
__device__ __forceinline__ float leapfrog(float G, float ctr, float c, float lap, float prev)
{
    return G * (ctr + fmaf(c, lap, fmaf(-G, prev, ctr)));
}

template <int ST> struct Stor { using T = uint16_t; };
template <> struct Stor<kF32> { using T = float; };

template <typename T, int VX>
struct alignas(sizeof(T) * VX) Pack {
    T v[VX];
};

template <typename T, int VX>
__device__ __forceinline__ Pack<T, VX> ldp(const T *p)
{
    return *reinterpret_cast<const Pack<T, VX> *>(p);
}

template <typename T, int VX>
__device__ __forceinline__ void stp(T *p, const Pack<T, VX> &x)
{
    *reinterpret_cast<Pack<T, VX> *>(p) = x;
}

// p + e elements with a 32-bit element offset: for a wave-uniform p the
// address is a scalar base plus a 32-bit lane offset, which the global
// load/store instructions take directly.
template <typename T>
__device__ __forceinline__ T *at(T *p, uint32_t e)
{
    return (T *)((char *)p + e * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T *at(const T *p, uint32_t e)
{
    return (const T *)((const char *)p + e * (uint32_t)sizeof(T));
}

// Raw integer vector of a given byte size, for the non-temporal builtins.
template <int B> struct Raw;
template <> struct Raw<2> { using type = unsigned short; };
template <> struct Raw<4> { using type = unsigned int; };
template <> struct Raw<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct Raw<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <> struct Raw<32> { typedef unsigned int type __attribute__((ext_vector_type(8))); };

// Streaming (read-once / write-once) accesses: Pold, c and Pnew are touched
// once per step, so they are marked non-temporal to leave the L2 to the
// current field, whose planes neighbouring tiles re-read as halos.
template <typename T, int VX>
__device__ __forceinline__ Pack<T, VX> ldp_stream(const T *p)
{
    using R = typename Raw<sizeof(T) * VX>::type;
    const R r = __builtin_nontemporal_load(reinterpret_cast<const R *>(p));
    Pack<T, VX> o;
    __builtin_memcpy(&o, &r, sizeof(o));
    return o;
}

template <typename T, int VX>
__device__ __forceinline__ void stp_stream(T *p, const Pack<T, VX> &x)
{
    using R = typename Raw<sizeof(T) * VX>::type;
    R r;
    __builtin_memcpy(&r, &x, sizeof(r));
    __builtin_nontemporal_store(r, reinterpret_cast<R *>(p));
}

template <int ST>
__device__ __forceinline__ float decode(typename Stor<ST>::T q, float scale)
{
    if constexpr (ST == kF32) {
        return q;
    } else if constexpr (ST == kF16) {
        return (float)__builtin_bit_cast(_Float16, q) * scale;
    } else {
        return __uint_as_float((uint32_t)q << 16) * scale;
    }
}

// Decode used inside the step kernels, before the power-of-two field scale:
// exact for every code (the hardware conversion for binary16, subnormals and
// non-finite codes included; a shift for bfloat16).
template <int ST>
__device__ __forceinline__ float decode_raw(typename Stor<ST>::T q)
{
    return decode<ST>(q, 1.0f);
}

// Round-to-nearest-even encode of x * inv_scale.
template <int ST>
__device__ __forceinline__ typename Stor<ST>::T encode(float x, float inv_scale)
{
    if constexpr (ST == kF32) {
        return x;
    } else if constexpr (ST == kF16) {
        return __builtin_bit_cast(uint16_t, (_Float16)(x * inv_scale));
    } else {
        uint32_t u = __float_as_uint(x * inv_scale);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
}

// Pairs of FP32 values rounded to nearest even into 16-bit codes with the
// gfx950 two-value conversions (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32); the
// values arrive already scaled by 2^-e.
template <int ST, int VX>
__device__ __forceinline__ void encode_pairs(const float (&x)[VX], uint16_t (&q)[VX])
{
    static_assert(VX % 2 == 0 || VX == 1, "pairs");
    if constexpr (VX == 1) {
        q[0] = encode<ST>(x[0], 1.0f);
    } else {
#pragma unroll
        for (int v = 0; v < VX; v += 2) {
            if constexpr (ST == kF16) {
                typedef _Float16 h2 __attribute__((ext_vector_type(2)));
                const h2 r = {(_Float16)x[v], (_Float16)x[v + 1]};
                const uint32_t u = __builtin_bit_cast(uint32_t, r);
                q[v] = (uint16_t)u;
                q[v + 1] = (uint16_t)(u >> 16);
            } else {
                typedef __bf16 b2 __attribute__((ext_vector_type(2)));
                const b2 r = {(__bf16)x[v], (__bf16)x[v + 1]};
                const uint32_t u = __builtin_bit_cast(uint32_t, r);
                q[v] = (uint16_t)u;
                q[v + 1] = (uint16_t)(u >> 16);
            }
        }
    }
}

// 2^e for e in [-126, 127].
__device__ __forceinline__ float pow2i(int e) { return __uint_as_float((uint32_t)(e + 127) << 23); }

// floor(log2(max(m, 2^-100))) - 11: the storage exponent of a field whose
// magnitude is bounded by 7 m (16x headroom below binary16's largest value).
__device__ __forceinline__ int storage_exponent(float m)
{
    const float floor_m = 7.888609052210118e-31f;  // 2^-100
    float t = m > floor_m ? m : floor_m;
    return (int)((__float_as_uint(t) >> 23) & 0xFFu) - 127 - 11;
}

// Per-launch quantities of the 16-bit storage form.  The step computes the
// new field directly in its storage units (value times 2^-en): the decode
// scales of cur and prev are multiplied by the encode scale 2^-en, which is
// exact for powers of two, so rounding the result to 16 bits needs no
// further multiply.
struct HalfCtx {
    float sc, sp;   // 2^(ec - en), 2^(ep - en)
    float sn;       // 2^en: storage units -> value (traces, magnitude)
    float sn_inv;   // 2^-en: value -> storage units (source term)
};

__device__ __forceinline__ float level_max(const int32_t *meta, int level)
{
    uint32_t m = 0;
#pragma unroll 16
    for (int k = 0; k < kMaxSlots; ++k) m = max(m, (uint32_t)meta[kMaxBase + level * kMaxSlots + k]);
    return __uint_as_float(m);
}

template <int ST>
__device__ __forceinline__ HalfCtx half_prologue(const StepArgs &a, float inj, bool block0)
{
    HalfCtx h{1.0f, 1.0f, 1.0f, 1.0f};
    if constexpr (ST != kF32) {
        const int ic = (int)(a.n & 3), ip = (int)((a.n + 3) & 3);
        const int in = (int)((a.n + 1) & 3), iz = (int)((a.n + 2) & 3);
        const int ec = a.meta[ic], ep = a.meta[ip];
        float m = fmaxf(level_max(a.meta, ic), level_max(a.meta, ip));
        m = fmaxf(m, fabsf(inj));
        const int en = storage_exponent(m);
        // ec - en and ep - en stay within a few units (the magnitude changes
        // by a bounded factor per step); the clamp only keeps 2^k finite.
        h.sc = pow2i(min(ec - en, 127));
        h.sp = pow2i(min(ep - en, 127));
        h.sn = pow2i(en);
        h.sn_inv = pow2i(-en);
        if (block0) {
            if (threadIdx.x == 0) a.meta[in] = en;
            // slots of level n+2 (not read by this step) are cleared for the next one
            if (threadIdx.x < kMaxSlots) a.meta[kMaxBase + iz * kMaxSlots + threadIdx.x] = 0;
        }
    }
    return h;
}

__device__ __forceinline__ int32_t *max_slot(int32_t *meta, int level)
{
    return &meta[kMaxBase + level * kMaxSlots + (blockIdx.x & (kMaxSlots - 1))];
}

// Folds a non-negative float into a slot by atomicMax on its bit pattern
// (order-independent, hence deterministic).  atomicMax is monotone, so a
// block whose value does not exceed what the slot already holds may skip
// the atomic: most blocks do, which keeps the atomics on one slot few.
__device__ __forceinline__ void fold_max(int32_t *slot, float m)
{
    const uint32_t bits = __float_as_uint(m);
    if (bits > (uint32_t)__atomic_load_n(slot, __ATOMIC_RELAXED))
        atomicMax((unsigned int *)slot, bits);
}

// Block-wide max of non-negative floats, folded into a slot.
template <int NT>
__device__ __forceinline__ void block_max_to(int32_t *slot, float v, float *red)
{
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    if constexpr (NT == 64) {
        if (threadIdx.x == 0) fold_max(slot, v);
    } else {
        const int w = threadIdx.x >> 6;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[w] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            float m = red[0];
            for (int i = 1; i < NT / 64; ++i) m = fmaxf(m, red[i]);
            fold_max(slot, m);
        }
    }
}

// Maps the hardware block index to a logical tile so that each XCD (blocks
// are dealt round-robin to the 8 XCDs) works on one contiguous range of
// tiles, which keeps neighbouring tiles' halo reads in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int per = nblocks >> 3;
    if (bid < (per << 3)) return (bid & 7) * per + (bid >> 3);
    return bid;
}

// 3D variant.  Blocks run in rounds of `resident` (the blocks the device
// holds at once; later blocks start, in index order, as earlier ones end).
// Within each round, XCD k gets the k-th eighth of the round's tiles
// (t = chunk * cols + column, so consecutive tiles are x/y neighbours at one
// depth), which keeps the blocks sharing an L2 neighbours whatever the
// chunk length.  A ragged tail (fewer than 8 blocks) keeps its index.
__device__ __forceinline__ int xcd_tile3d(int bid, int nblocks, int resident)
{
    if (resident < 8) return xcd_tile(bid, nblocks);
    const int base = bid / resident * resident;
    const int m8 = min(resident, nblocks - base) & ~7;
    const int w = bid - base;
    if (w >= m8) return bid;
    return base + (w & 7) * (m8 >> 3) + (w >> 3);
}

}  // namespace fdk
