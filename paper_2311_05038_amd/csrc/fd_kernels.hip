// Step kernels and set-up kernels for gfx950 (MI355X).
//
// 2D (z, x):  one wave per block.  A block owns a 64*VX-wide column strip and
//   a chunk of `zc` rows; each lane streams its VX columns down z keeping the
//   9 rows z-4..z+4 in registers, and the x-neighbours come from one LDS row
//   (plus 4 halo cells each side).  One HBM read of cur/prev/c and one write
//   per cell and step (16 B/cell in FP32, 10 B with 16-bit fields).
// 3D (z, y, x): NW waves per block.  A block owns a tile of the x-y plane
//   (256x8 cells for FP32 fields, 128x8 for 16-bit) and a chunk of `zc`
//   planes; lanes stream along z (the slow axis) with a 9-deep register queue
//   per cell, and x/y neighbours come from a double-buffered LDS copy of the
//   current plane with a 4-cell halo.
// Both follow the fused step of arXiv 2311.05038, Section 7 (Listing 3's
// add_source, fd_pzz, fd_pxx, fd_time and swap in one pass).
#include <algorithm>

#include <type_traits>

#include "fd_device.hpp"
#include "fd_launch.hpp"

// The 16-bit steps order their memory operations so that the next plane's
// loads overlap the compute: the z sponge factor travels with the
// prefetched data, the prefetch is unconditional (planes past the chunk are
// in bounds or read as zero), and each new plane is stored one plane late,
// right before the next prefetch.  Vector loads and stores share one
// completion counter, and the compiler waits for a load by waiting until
// every older memory operation has completed once both kinds are
// outstanding: a load issued after the prefetch and used at once, a
// skipped prefetch (the previous registers are then copied, which waits),
// or a store issued right after the compute would each make a plane wait
// for its own prefetch.  Measured at 768x768x512: BF16 649 -> 566 us.  The
// FP32 steps keep the plain order (stores right after the compute, the
// sponge factor loaded after the barrier), which measured faster for them
// (512^3 366 against 387 us): their loop is bandwidth-bound with more bytes
// in flight per wave already.
namespace fdk {

// --------------------------------------------------------------------------
// Epilogue shared by 2D and 3D: receivers, source, padding, store.
// --------------------------------------------------------------------------
// A row's outgoing values.  The 16-bit steps store them one plane (row)
// later, right before the next prefetch (see the ordering note above); the
// FP32 steps store them at once.
template <typename T, int VX>
struct Outgoing {
    Pack<T, VX> o;
    Pack<float, VX> L;  // history value (L cur or cur), history modes only
    T *dst;
    float *ldst;
    bool ok;
};

template <typename T, int VX, int MODE, bool STREAM>
__device__ __forceinline__ void flush(Outgoing<T, VX> &out)
{
    if (out.ok) {
        if constexpr (STREAM)
            stp_stream<T, VX>(out.dst, out.o);
        else
            stp<T, VX>(out.dst, out.o);
        if constexpr (stores_history(MODE)) stp<float, VX>(out.ldst, out.L);
    }
    out.ok = false;
}

// nw holds the new values (FP32 fields) or the new values in storage units
// (16-bit fields: value = h.sn * nw).  FULL: every cell of the lane lies
// inside the grid (x < nx), so no padding mask is needed.  The adjoint
// step (which reads lap and g here) stores at once; the forward steps leave
// their stores in `out`.  lp: the history value to store (history modes), or
// in the adjoint step the centre value of cur (the previous step's new
// value, for a deferred gradient term); pv: the centre value of prev (the
// new value of two steps back, for a second deferred term).
template <int ST, int VX, int MODE, bool STREAM, bool FULL>
__device__ __forceinline__ void finish_cells(const StepArgs &a, const HalfCtx &h, int z, int y,
                                             int x0, bool store_ok, size_t row, uint32_t eo,
                                             float (&nw)[VX],
                                             const float (&lp)[VX], const float (&pv)[VX],
                                             const float (&cc)[VX],
                                             const float (&G)[VX], float inj, float &bmax,
                                             Outgoing<typename Stor<ST>::T, VX> &out)
{
    using T = typename Stor<ST>::T;
    // Receiver box membership of this row (z, y).
    int rrow = -1;
    {
        const int zr = z - a.rec.z0, yr = y - a.rec.y0;
        if (zr >= 0 && yr >= 0 && zr % a.rec.dz == 0 && yr % a.rec.dy == 0 &&
            zr / a.rec.dz < a.rec.nz && yr / a.rec.dy < a.rec.ny)
            rrow = (zr / a.rec.dz) * a.rec.ny + yr / a.rec.dy;
    }
    if constexpr (MODE == kAdj) {
        if (a.resid_row != nullptr && rrow >= 0) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const int xr = x0 + v - a.rec.x0;
                if (x0 + v < a.nx && xr >= 0 && xr % a.rec.dx == 0 && xr / a.rec.dx < a.rec.nx)
                    nw[v] = fmaf(cc[v] * G[v], a.resid_row[(size_t)rrow * a.rec.nx + xr / a.rec.dx], nw[v]);
            }
        }
    } else {
        if (a.trace_row != nullptr && rrow >= 0) {
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const int xr = x0 + v - a.rec.x0;
                if (x0 + v < a.nx && xr >= 0 && xr % a.rec.dx == 0 && xr / a.rec.dx < a.rec.nx) {
                    if constexpr (ST == kF32)
                        a.trace_row[(size_t)rrow * a.rec.nx + xr / a.rec.dx] = nw[v];
                    else
                        a.trace_row[(size_t)rrow * a.rec.nx + xr / a.rec.dx] = nw[v] * h.sn;
                }
            }
        }
        if (z == a.sz && y == a.sy) {
            const float inj_s = ST == kF32 ? inj : inj * h.sn_inv;
#pragma unroll
            for (int v = 0; v < VX; ++v)
                if (x0 + v == a.sx) nw[v] += inj_s;
        }
    }
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        if (!FULL && x0 + v >= a.nx) nw[v] = 0.0f;
        if constexpr (ST != kF32) bmax = fmaxf(bmax, fabsf(nw[v]));
    }
    T *dst = (T *)(a.out != nullptr ? a.out : a.prev);
    if constexpr (ST == kF32) {
#pragma unroll
        for (int v = 0; v < VX; ++v) out.o.v[v] = nw[v];
    } else {
        encode_pairs<ST, VX>(nw, out.o.v);
    }
    out.dst = at(dst + row, eo);
    out.ok = store_ok;
    if constexpr (stores_history(MODE)) {
#pragma unroll
        for (int v = 0; v < VX; ++v) out.L.v[v] = (FULL || x0 + v < a.nx) ? lp[v] : 0.0f;
        out.ldst = at(a.lap + row, eo);
    }
    if constexpr (MODE == kAdj) {
        flush<T, VX, MODE, STREAM>(out);
        // the time sum in FP64, one term per level in descending level order
        // however many terms share a pass over g
        if (store_ok && a.gmode != 1) {
            const Pack<float, VX> lw = ldp<float, VX>(at(a.lap + row, eo));
            Pack<double, VX> gg = ldp<double, VX>(at(a.g + row, eo));
            if (a.gmode == 3) {
                const Pack<float, VX> lw3 = ldp<float, VX>(at(a.lap3 + row, eo));
#pragma unroll
                for (int v = 0; v < VX; ++v) gg.v[v] = fma((double)pv[v], (double)lw3.v[v], gg.v[v]);
            }
            if (a.gmode >= 2) {
                const Pack<float, VX> lw2 = ldp<float, VX>(at(a.lap2 + row, eo));
#pragma unroll
                for (int v = 0; v < VX; ++v) gg.v[v] = fma((double)lp[v], (double)lw2.v[v], gg.v[v]);
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) gg.v[v] = fma((double)nw[v], (double)lw.v[v], gg.v[v]);
            stp<double, VX>(at(a.g + row, eo), gg);
        }
    }
}


// The same update on 16-bit fields read as raw codes q (P = 2^ec q, Pold =
// 2^ep qp, and L q computed from the raw q), producing the new field in its
// storage units 2^-en: (G sc)(2 q + c L q) - (G^2 sp) qp with sc = 2^(ec-en)
// and sp = 2^(ep-en).  This is the scaled arithmetic exactly, since
// multiplying by 2^k does not round.
template <int ST>
__device__ __forceinline__ float update(float G, float ctr, float c, float lap, float prev,
                                        const HalfCtx &h)
{
    if constexpr (ST == kF32)
        return leapfrog(G, ctr, c, lap, prev);
    else
        return fmaf(G * h.sc, fmaf(c, lap, 2.0f * ctr), -((G * G) * h.sp) * prev);
}

// --------------------------------------------------------------------------
// 2D
// --------------------------------------------------------------------------
// CQ: c is read as 16-bit fixed-point codes (16-bit fields, forward step).
template <int ST, int VX, int MODE, bool CQ>
__device__ __forceinline__ void step2d_tile(const StepArgs &a, int tx, int tz,
                                            float (*row)[64 * VX + 8], const HalfCtx &h,
                                            float inj, float &bmax)
{
    static_assert(!CQ || (ST != kF32 && MODE == kFwd), "16-bit c: 16-bit fields, forward step");
    using T = typename Stor<ST>::T;
    using CT = std::conditional_t<CQ, uint16_t, float>;
    constexpr int TX = 64 * VX;
    const int lane = threadIdx.x & 63;
    const int xb = tx * TX;
    const int x0 = xb + lane * VX;
    const int zb = tz * a.zc;
    const int ze = min(zb + a.zc, a.nz);
    const T *__restrict__ cur = (const T *)a.cur;
    const T *__restrict__ prv = (const T *)a.prev;
    const size_t px = (size_t)a.px;
    const bool lane_in = x0 < a.px;
    const int nx = a.nx, nz = a.nz;

    float gxv[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) gxv[v] = (x0 + v < nx) ? a.gx[x0 + v] : 0.0f;

    int hx = -1, hslot = 0;
    if (lane < 4) {
        hx = xb - 4 + lane;
        hslot = lane;
    } else if (lane >= 60) {
        hx = xb + TX + (lane - 60);
        hslot = TX + 4 + (lane - 60);
    }
    const bool hlane = (lane < 4) || (lane >= 60);
    const bool hvalid = hx >= 0 && hx < nx;

    // Loads return raw packs (zero outside the grid); values are decoded
    // where they are consumed, so a prefetch never waits for its own load.
    using PT = Pack<T, VX>;
    using PC = Pack<CT, VX>;
    const CT *cbase;
    if constexpr (CQ)
        cbase = a.c16;
    else
        cbase = a.c;
    auto ld_cur = [&](int z) -> PT {
        PT p{};
        if (z >= 0 && z < nz && lane_in) p = ldp<T, VX>(cur + (size_t)z * px + x0);
        return p;
    };
    auto ld_prev = [&](int z) -> PT {
        PT p{};
        if (z < nz && lane_in) p = ldp<T, VX>(prv + (size_t)z * px + x0);
        return p;
    };
    auto ld_c = [&](int z) -> PC {
        PC p{};
        if (z < nz && lane_in) p = ldp<CT, VX>(cbase + (size_t)z * px + x0);
        return p;
    };
    auto ld_halo = [&](int z) -> T { return (hvalid && z < nz) ? cur[(size_t)z * px + hx] : (T)0; };

    float q[9][VX];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const PT p = ld_cur(zb - 4 + k);
#pragma unroll
        for (int v = 0; v < VX; ++v) q[k][v] = decode_raw<ST>(p.v[v]);
    }
    PT la = ld_cur(zb + 4), pv = ld_prev(zb);
    PC cv = ld_c(zb);
    T hv = ld_halo(zb);
    // the row's sponge factor travels with the prefetch: a load issued after
    // it and waited for in the same row would also wait for the prefetch
    constexpr bool LATE = ST != kF32;   // the 16-bit memory-op order (see top)
    float gn = a.gz[zb];
    Outgoing<T, VX> out;
    out.ok = false;

    for (int z = zb; z < ze; ++z) {
        float pc[VX], cc[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            q[8][v] = decode_raw<ST>(la.v[v]);
            pc[v] = decode_raw<ST>(pv.v[v]);
            if constexpr (CQ)
                cc[v] = (float)cv.v[v] * a.c16_scale;   // exact: a power-of-two scale
            else
                cc[v] = cv.v[v];
        }
        const float hc = decode_raw<ST>(hv);
        const float gzp = gn;
        // the previous row's stores go out after the wait for this row's
        // data and just before the next prefetch
        if constexpr (LATE) {
            __builtin_amdgcn_sched_barrier(0);
            flush<T, VX, MODE, false>(out);
        }
        if (LATE || z + 1 < ze) {
            la = ld_cur(z + 5);
            pv = ld_prev(z + 1);
            cv = ld_c(z + 1);
            hv = ld_halo(z + 1);
            if constexpr (LATE) gn = z + 1 < nz ? a.gz[z + 1] : 0.0f;
        }
        float *rw = row[z & 1];
#pragma unroll
        for (int v = 0; v < VX; ++v) rw[4 + lane * VX + v] = q[4][v];
        if (hlane) rw[hslot] = hc;
        __syncthreads();
        const float gzz = LATE ? gzp : a.gz[z];
        float nw[VX], lp[VX], G[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int li = 4 + lane * VX + v;
            float lap;
            if constexpr (ST == kF32) {
                const float lx = axis_d2(rw[li - 4], rw[li - 3], rw[li - 2], rw[li - 1], q[4][v],
                                         rw[li + 1], rw[li + 2], rw[li + 3], rw[li + 4]);
                const float lz = axis_d2(q[0][v], q[1][v], q[2][v], q[3][v], q[4][v], q[5][v],
                                         q[6][v], q[7][v], q[8][v]);
                lap = lz + lx;
            } else {
                const float lx = stencil_taps(rw[li - 4], rw[li - 3], rw[li - 2], rw[li - 1],
                                              rw[li + 1], rw[li + 2], rw[li + 3], rw[li + 4]);
                const float lz = stencil_taps(q[0][v], q[1][v], q[2][v], q[3][v], q[5][v], q[6][v],
                                              q[7][v], q[8][v]);
                lap = fmaf(2.0f * kA0, q[4][v], lz + lx);
            }
            G[v] = gzz * gxv[v];
            nw[v] = update<ST>(G[v], q[4][v], cc[v], lap, pc[v], h);
            lp[v] = MODE == kAdj ? q[4][v] : lap;
        }
        finish_cells<ST, VX, MODE, false, false>(a, h, z, 0, x0, lane_in, (size_t)z * px, (uint32_t)x0, nw,
                                                 lp, pc, cc, G, inj, bmax, out);
        if constexpr (!LATE) flush<T, VX, MODE, false>(out);
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int v = 0; v < VX; ++v) q[k][v] = q[k + 1][v];
    }
    flush<T, VX, MODE, false>(out);
}

template <int ST, int VX, int MODE, bool CQ>
__global__ __launch_bounds__(64) void k_step2d(StepArgs a)
{
    __shared__ float row[2][64 * VX + 8];
    const int nb = a.tiles_x * a.tiles_z;
    const int t = xcd_tile(blockIdx.x, nb);
    const int tx = t % a.tiles_x, tz = t / a.tiles_x;
    float inj = 0.0f;
    if constexpr (MODE != kAdj)
        if (a.n + 1 < a.nt) inj = a.amp * a.wavelet[a.n + 1];
    const HalfCtx h = half_prologue<ST>(a, inj, blockIdx.x == 0);
    float bmax = 0.0f;
    step2d_tile<ST, VX, MODE, CQ>(a, tx, tz, row, h, inj, bmax);
    if constexpr (ST != kF32)
        block_max_to<64>(max_slot(a.meta, (int)((a.n + 1) & 3)), bmax * h.sn, nullptr);
}

// Batched 2D FP32 step (any mode): block b belongs to the item whose tile
// range holds b; every item keeps its own grid, fields and step index.
template <int VX, int MODE>
__global__ __launch_bounds__(64) void k_step2d_batch(Batch2D b)
{
    __shared__ float row[2][64 * VX + 8];
    const int t = blockIdx.x;
    int i = 0;
    while (i + 1 < b.count && t >= b.begin[i + 1]) ++i;
    const StepArgs &a = b.it[i];
    const int lt = t - b.begin[i];
    const int tx = lt % a.tiles_x, tz = lt / a.tiles_x;
    float inj = 0.0f;
    if constexpr (MODE != kAdj)
        if (a.n + 1 < a.nt) inj = a.amp * a.wavelet[a.n + 1];
    const HalfCtx h{1.0f, 1.0f, 1.0f, 1.0f};
    float bmax = 0.0f;
    step2d_tile<kF32, VX, MODE, false>(a, tx, tz, row, h, inj, bmax);
}

// --------------------------------------------------------------------------
// 3D
// --------------------------------------------------------------------------
// A wave covers RPW rows of the tile at once (64/RPW lanes per row, VX
// cells per lane), so a lane's VX cells are contiguous in x; the block's NW
// waves stack NW*RPW rows, and each thread handles RY such row groups.
// CQ: c is read as 16-bit fixed-point codes q (16-bit fields, forward step):
// 2 P + c L P = s (2 P / s + q L P) with s = 2^(e-16), and s joins the
// other power-of-two factors of the update (exact; the Laplacian keeps the
// scale of the stored codes).
template <int ST, int VX, int RY, int NW, int RPW, int MODE, bool CQ>
__global__ __launch_bounds__(64 * NW) void k_step3d(StepArgs a)
{
    static_assert(!CQ || (ST != kF32 && MODE == kFwd), "16-bit c: 16-bit fields, forward step");
    using T = typename Stor<ST>::T;
    using CT = std::conditional_t<CQ, uint16_t, float>;
    static_assert(NW == 2 || NW == 4 || NW == 8, "waves per block");
    static_assert(RPW == 1 || RPW == 2, "rows per wave");
    static_assert(8 % (NW * RPW) == 0, "y-halo rows per wave");
    constexpr int LPR = 64 / RPW;   // lanes per row
    constexpr int TX = LPR * VX, TY = NW * RPW * RY, LW = TX + 8, LH = TY + 8, HH = 8 / (NW * RPW);
    __shared__ float pl[2][LH * LW];
    __shared__ float red[NW];
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    const int col = lane % LPR, trow = wy * RPW + lane / LPR;   // thread's column and row
    const int nb = a.tiles_x * a.tiles_y * a.tiles_z;
    const int t = xcd_tile3d(blockIdx.x, nb, a.resident);
    const int tx = t % a.tiles_x;
    const int t2 = t / a.tiles_x;
    const int ty = t2 % a.tiles_y, tz = t2 / a.tiles_y;
    const int xb = tx * TX, yb = ty * TY, x0 = xb + col * VX;
    const int zb = tz * a.zc, ze = min(zb + a.zc, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t px = (size_t)a.px, pp = (size_t)ny * px;
    const int zlo = ST == kF32 ? -a.zghost : 0, zhi = ST == kF32 ? nz + a.zghost : nz;
    const bool lane_in = x0 < a.px;
    const T *__restrict__ cur = (const T *)a.cur;
    const T *__restrict__ prv = (const T *)a.prev;

    float inj = 0.0f;
    if constexpr (MODE != kAdj)
        if (a.n + 1 < a.nt) inj = a.amp * a.wavelet[a.n + 1];
    const HalfCtx h = half_prologue<ST>(a, inj, blockIdx.x == 0);

    // FULL: every lane's cells, every row and every y-halo row of the tile
    // lie inside the grid, so loads need no per-lane or per-row tests (the z
    // tests are uniform); other tiles take the checked path.
    auto tile = [&](auto full_c) -> float {
        constexpr bool FULL = decltype(full_c)::value;
        int yj[RY];
        bool yin[RY];
        float gyv[RY];
    #pragma unroll
        for (int j = 0; j < RY; ++j) {
            yj[j] = yb + trow + NW * RPW * j;
            yin[j] = FULL || yj[j] < ny;
            gyv[j] = yin[j] ? a.gy[yj[j]] : 0.0f;
        }
        float gxv[VX], gxv2[VX];
    #pragma unroll
        for (int v = 0; v < VX; ++v) {
            gxv[v] = (FULL || x0 + v < nx) ? a.gx[x0 + v] : 0.0f;
            gxv2[v] = gxv[v] * gxv[v];
        }

        // y-halo rows handled by this thread: k = (wy + NW hh) RPW + its row
        // within the wave, hh < 8 / (NW RPW).
        int hy[HH], hyslot[HH];
        bool hyv[HH];
    #pragma unroll
        for (int hh = 0; hh < HH; ++hh) {
            const int k = (wy + NW * hh) * RPW + lane / LPR;
            const int ly = k < 4 ? k - 4 : TY + k - 4;
            hy[hh] = yb + ly;
            hyv[hh] = FULL || (hy[hh] >= 0 && hy[hh] < ny && lane_in);
            hyslot[hh] = (ly + 4) * LW + 4 + col * VX;
        }
        // x-halo cell handled by this thread (threads < 8 TY).
        const bool hxl = threadIdx.x < 8 * TY;
        int hxx = 0, hxy = 0, hxslot = 0;
        if (hxl) {
            const int lr = threadIdx.x >> 3, ci = threadIdx.x & 7;
            hxx = ci < 4 ? xb - 4 + ci : xb + TX + ci - 4;
            hxy = yb + lr;
            hxslot = (lr + 4) * LW + (ci < 4 ? ci : TX + ci);
        }
        const bool hxv = hxl && hxx >= 0 && hxx < nx && hxy < ny;

        // Element offsets within a plane (32-bit: a plane holds < 2^29
        // cells): each access is a wave-uniform plane pointer plus a lane
        // offset, which keeps the address arithmetic scalar.  (FP32 fields,
        // bandwidth-bound, measured faster with plain 64-bit addresses.)
        constexpr bool OFF32 = ST != kF32;
        constexpr bool LATE = ST != kF32;   // the 16-bit memory-op order (see top)
        auto addr = [&](auto *base, int z, uint32_t e, int y, int x) {
            if constexpr (OFF32)
                return at(base + (size_t)z * pp, e);
            else
                return base + (size_t)z * pp + (size_t)y * px + x;
        };
        uint32_t eo[RY], eohy[HH];
    #pragma unroll
        for (int j = 0; j < RY; ++j) eo[j] = (uint32_t)(yj[j] * a.px + x0);
    #pragma unroll
        for (int hh = 0; hh < HH; ++hh) eohy[hh] = (FULL || hyv[hh]) ? (uint32_t)(hy[hh] * a.px + x0) : 0u;
        const uint32_t eohx = hxv ? (uint32_t)(hxy * a.px + hxx) : 0u;

        // Loads return raw packs (zero outside the grid); values are decoded
        // where they are consumed, so a prefetch never waits for its own load.
        using PT = Pack<T, VX>;
        using PC = Pack<CT, VX>;
        const CT *cbase;
        if constexpr (CQ)
            cbase = a.c16;
        else
            cbase = a.c;
        // cur (the only field read off its own planes) is readable over
        // [-zghost, nz + zghost): a z-slab's ghost planes, or zero edges
        auto ld3 = [&](const T *base, int z, int j) -> PT {
            PT p{};
            if (z >= zlo && z < zhi && (FULL || (yin[j] && lane_in)))
                p = ldp<T, VX>(addr(base, z, eo[j], yj[j], x0));
            return p;
        };
        auto ld3nt = [&](const T *base, int z, int j) -> PT {
            PT p{};
            if (z < nz && (FULL || (yin[j] && lane_in)))
                p = ldp_stream<T, VX>(addr(base, z, eo[j], yj[j], x0));
            return p;
        };
        auto ldc3 = [&](int z, int j) -> PC {
            PC p{};
            if (z < nz && (FULL || (yin[j] && lane_in)))
                p = ldp_stream<CT, VX>(addr(cbase, z, eo[j], yj[j], x0));
            return p;
        };
        auto ldhy = [&](int z, int hh) -> PT {
            PT p{};
            if ((FULL || hyv[hh]) && z < nz) p = ldp<T, VX>(addr(cur, z, eohy[hh], hy[hh], x0));
            return p;
        };
        auto ldhx = [&](int z) -> T {
            return (hxv && z < nz) ? *addr(cur, z, eohx, hxy, hxx) : (T)0;
        };

        float q[RY][9][VX];
    #pragma unroll
        for (int j = 0; j < RY; ++j)
    #pragma unroll
            for (int k = 0; k < 8; ++k) {
                const PT p = ld3(cur, zb - 4 + k, j);
    #pragma unroll
                for (int v = 0; v < VX; ++v) q[j][k][v] = decode_raw<ST>(p.v[v]);
            }
        // Prefetched raw data of one plane zz: cur at zz + 4 (the queue's
        // next entry), prev and c at zz, and the halo cells of cur at zz.
        struct Ahead {
            PT la[RY], pv[RY], yh[HH];
            PC cv[RY];
            T xh;
            float gz;   // sponge factor of plane zz (16-bit steps)
        };
        auto fetch = [&](int zz, Ahead &r) {
    #pragma unroll
            for (int j = 0; j < RY; ++j) {
                r.la[j] = ld3(cur, zz + 4, j);
                r.pv[j] = ld3nt(prv, zz, j);
                r.cv[j] = ldc3(zz, j);
            }
    #pragma unroll
            for (int hh = 0; hh < HH; ++hh) r.yh[hh] = ldhy(zz, hh);
            r.xh = ldhx(zz);
            if constexpr (LATE) r.gz = zz < nz ? a.gz[zz] : 0.0f;
        };
        Ahead ah;
        fetch(zb, ah);
        float bmax = 0.0f;
        Outgoing<T, VX> out[RY];
    #pragma unroll
        for (int j = 0; j < RY; ++j) out[j].ok = false;

        // One plane: slot k of the register queue holds plane z - 4 + k; the
        // values shift down one slot per plane.
        auto plane_step = [&](int z) {
            float pc[RY][VX], cc[RY][VX], yhc[HH][VX];
    #pragma unroll
            for (int j = 0; j < RY; ++j)
    #pragma unroll
                for (int v = 0; v < VX; ++v) {
                    q[j][8][v] = decode_raw<ST>(ah.la[j].v[v]);
                    pc[j][v] = decode_raw<ST>(ah.pv[j].v[v]);
                    cc[j][v] = (float)ah.cv[j].v[v];
                }
    #pragma unroll
            for (int hh = 0; hh < HH; ++hh)
    #pragma unroll
                for (int v = 0; v < VX; ++v) yhc[hh][v] = decode_raw<ST>(ah.yh[hh].v[v]);
            const float xhc = decode_raw<ST>(ah.xh);
            const float gzp = ah.gz;
            // 16-bit: the previous plane's stores go out after the wait for
            // this plane's data and just before the next prefetch
            if constexpr (LATE) {
                __builtin_amdgcn_sched_barrier(0);
    #pragma unroll
                for (int j = 0; j < RY; ++j) flush<T, VX, MODE, true>(out[j]);
            }
            if (LATE || z + 1 < ze) fetch(z + 1, ah);
            float *P = pl[z & 1];
    #pragma unroll
            for (int j = 0; j < RY; ++j)
    #pragma unroll
                for (int v = 0; v < VX; ++v) P[(trow + NW * RPW * j + 4) * LW + 4 + col * VX + v] = q[j][4][v];
    #pragma unroll
            for (int hh = 0; hh < HH; ++hh)
    #pragma unroll
                for (int v = 0; v < VX; ++v) P[hyslot[hh] + v] = yhc[hh][v];
            if (hxl) P[hxslot] = xhc;
            __syncthreads();
            const float gzz = LATE ? gzp : a.gz[z];
    #pragma unroll
            for (int j = 0; j < RY; ++j) {
                float nw[VX], lp[VX], G[VX];
                if constexpr (ST != kF32) {
                    // 16-bit fields (VALU-bound): taps summed over the three
                    // axes before weighting, and the sponge factor's square
                    // taken per lane and per row, which saves instructions at
                    // a different FP32 rounding order.
                    const float gr = gzz * gyv[j];
                    const float sc = CQ ? h.sc * a.c16_scale : h.sc;
                    const float two = CQ ? 2.0f * a.c16_inv : 2.0f;
                    const float r1 = gr * sc, r2 = (gr * gr) * h.sp;
    #pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        const int li = (trow + NW * RPW * j + 4) * LW + 4 + col * VX + v;
                        const float(&qq)[9][VX] = q[j];
                        float sk[4];
    #pragma unroll
                        for (int k = 1; k <= 4; ++k)
                            sk[k - 1] = ((P[li - k] + P[li + k]) + (P[li - k * LW] + P[li + k * LW])) +
                                        (qq[4 - k][v] + qq[4 + k][v]);
                        const float ctr = qq[4][v];
                        const float lap = fmaf(3.0f * kA0, ctr,
                                               fmaf(kA4, sk[3], fmaf(kA3, sk[2], fmaf(kA2, sk[1], kA1 * sk[0]))));
                        G[v] = 0.0f;
                        nw[v] = fmaf(gxv[v] * r1, fmaf(cc[j][v], lap, two * ctr), -(gxv2[v] * r2) * pc[j][v]);
                        lp[v] = lap;
                    }
                } else {
    #pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const int li = (trow + NW * RPW * j + 4) * LW + 4 + col * VX + v;
                    const float u = q[j][4][v];
                    const float lx = axis_d2(P[li - 4], P[li - 3], P[li - 2], P[li - 1], u, P[li + 1],
                                             P[li + 2], P[li + 3], P[li + 4]);
                    const float lyv = axis_d2(P[li - 4 * LW], P[li - 3 * LW], P[li - 2 * LW], P[li - LW], u,
                                              P[li + LW], P[li + 2 * LW], P[li + 3 * LW], P[li + 4 * LW]);
                    const float lz = axis_d2(q[j][0][v], q[j][1][v], q[j][2][v], q[j][3][v], u,
                                             q[j][5][v], q[j][6][v], q[j][7][v], q[j][8][v]);
                    const float lap = lz + (lyv + lx);
                    G[v] = (gzz * gyv[j]) * gxv[v];
                    nw[v] = update<ST>(G[v], q[j][4][v], cc[j][v], lap, pc[j][v], h);
                    lp[v] = MODE == kAdj ? q[j][4][v] : lap;
                }
                }
                if constexpr (OFF32)
                    finish_cells<ST, VX, MODE, true, FULL>(a, h, z, yj[j], x0, lane_in && yin[j],
                                                           (size_t)z * pp, eo[j], nw, lp, pc[j], cc[j], G, inj,
                                                           bmax, out[j]);
                else
                    finish_cells<ST, VX, MODE, true, FULL>(a, h, z, yj[j], x0, lane_in && yin[j],
                                                           (size_t)z * pp + (size_t)yj[j] * px, (uint32_t)x0, nw,
                                                           lp, pc[j], cc[j], G, inj, bmax, out[j]);
                if constexpr (!LATE) flush<T, VX, MODE, true>(out[j]);
            }
        };
        using std::integral_constant;
        for (int z = zb; z < ze; ++z) {
            plane_step(z);
    #pragma unroll
            for (int j = 0; j < RY; ++j)
    #pragma unroll
                for (int k = 0; k < 8; ++k)
    #pragma unroll
                    for (int v = 0; v < VX; ++v) q[j][k][v] = q[j][k + 1][v];
        }
    #pragma unroll
        for (int j = 0; j < RY; ++j) flush<T, VX, MODE, true>(out[j]);
        return bmax;
    };
    // (measured: a small gain with 16-bit fields, a small loss with FP32)
    const bool full = ST != kF32 && xb + TX <= nx && yb >= 4 && yb + TY + 4 <= ny;
    const float bmax = full ? tile(std::true_type{}) : tile(std::false_type{});
    if constexpr (ST != kF32)
        block_max_to<64 * NW>(max_slot(a.meta, (int)((a.n + 1) & 3)), bmax * h.sn, red);
}

// --------------------------------------------------------------------------
// Set-up and utility kernels
// --------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t val)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = val;
}

// c = (v dt/h)^2 rounded from FP64 to FP32.
__device__ __forceinline__ float model_c(float v, double r)
{
    const double qq = (double)v * r;
    return (float)(qq * qq);
}

// c padded (skipped when c is null); also the velocity range (max as float
// bits) and a flag for non-positive or non-finite values.
__global__ void k_model_c(const float *__restrict__ v, float *__restrict__ c, int64_t nrows,
                          int32_t nx, int32_t px, double r, uint32_t *scratch)
{
    uint32_t vmax = 0, bad = 0;
    const size_t total = (size_t)nrows * nx;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)nx, x = i - rw * (size_t)nx;
        const float vi = v[i];
        if (!(vi > 0.0f) || !(vi < 3.0e38f)) bad = 1;
        vmax = max(vmax, __float_as_uint(fabsf(vi)));
        if (c != nullptr) c[rw * (size_t)px + x] = model_c(vi, r);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off, 64));
        bad |= (uint32_t)__shfl_xor((int)bad, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&scratch[0], vmax);
        if (bad) atomicOr(&scratch[1], 1u);
    }
}

// c in 16-bit unsigned fixed point: q = min(RNE(c 2^(16-e)), 65535), where
// inv_scale = 2^(16-e) and c < 2^e for every cell (the product is exact).
__global__ void k_model_c16(const float *__restrict__ v, uint16_t *__restrict__ c16, int64_t nrows,
                            int32_t nx, int32_t px, double r, float inv_scale)
{
    const size_t total = (size_t)nrows * nx;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)nx, x = i - rw * (size_t)nx;
        const float q = fminf(rintf(model_c(v[i], r) * inv_scale), 65535.0f);
        c16[rw * (size_t)px + x] = (uint16_t)q;
    }
}

// First source addition of a shot into the zeroed level-0 field (+ the
// storage exponent and magnitude of levels 0 and -1).  The wave also scans
// the shot's nt injected values amp * s[n] and records a non-finite one in
// the shot's health flags.
template <int ST>
__global__ void k_begin(void *cur, int64_t src_off, float amp, const float *wavelet, int64_t nt,
                        int32_t *meta)
{
    bool bad = false;
    for (int64_t i = threadIdx.x; i < nt; i += blockDim.x) bad |= !(fabsf(amp * wavelet[i]) <= 3.4028235e38f);
    if (__ballot(bad) != 0 && threadIdx.x == 0) atomicOr((uint32_t *)&meta[kHealth], kNonfiniteInput);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    using T = typename Stor<ST>::T;
    const float x0 = amp * wavelet[0];
    if constexpr (ST == kF32) {
        ((T *)cur)[src_off] = x0;
    } else {
        // the state was cleared: every exponent and magnitude slot is zero
        const int e0 = storage_exponent(fabsf(x0));
        ((T *)cur)[src_off] = encode<ST>(x0, pow2i(-e0));
        meta[0] = e0;
        meta[kMaxBase] = (int32_t)__float_as_uint(fabsf(x0));
    }
}

template <int ST>
__global__ void k_get_field(const void *buf, float *__restrict__ out, int64_t nrows, int32_t nx,
                            int32_t px, const int32_t *meta, int32_t level_slot)
{
    using T = typename Stor<ST>::T;
    float s = 1.0f;
    if constexpr (ST != kF32) s = pow2i(meta[level_slot]);
    const size_t total = (size_t)nrows * nx;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)nx, x = i - rw * (size_t)nx;
        out[i] = decode<ST>(((const T *)buf)[rw * (size_t)px + x], s);
    }
}

// max |x| over a dense array, folded into slots[blockIdx % kMaxSlots] as
// float bits.
__global__ void k_absmax(const float *__restrict__ x, size_t n, uint32_t *slots)
{
    uint32_t *slot = &slots[blockIdx.x & (kMaxSlots - 1)];
    float m = 0.0f;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) m = fmaxf(m, fabsf(x[i]));
    for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));
}

// Dense FP32 -> padded stored field; 16-bit storage takes its exponent from
// the magnitude in meta[4 + slot] and records it in meta[slot].
template <int ST>
__global__ void k_set_field(const float *__restrict__ in, void *buf, int64_t nrows, int32_t nx,
                            int32_t px, int32_t *meta, int32_t slot)
{
    using T = typename Stor<ST>::T;
    float inv = 1.0f;
    if constexpr (ST != kF32) {
        const int e = storage_exponent(level_max(meta, slot));
        inv = pow2i(-e);
        if (blockIdx.x == 0 && threadIdx.x == 0) meta[slot] = e;
    }
    const size_t total = (size_t)nrows * px;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)px, x = i - rw * (size_t)px;
        const float v = x < (size_t)nx ? in[rw * (size_t)nx + x] : 0.0f;
        bad |= !(fabsf(v) <= 3.4028235e38f);
        ((T *)buf)[i] = encode<ST>(v, inv);
    }
    // a non-finite value set into the shot is recorded in its health flags
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr((uint32_t *)&meta[kHealth], kNonfiniteInput);
}

// Sets `bit` in *flags when a stored level holds a non-finite value (NaN or
// infinity), and (health non-null) the shot's sticky non-finite-input flag: the exponent field of a code all ones (FP32 0x7F800000,
// binary16 0x7C00, bfloat16 0x7F80), tested on the raw codes 16 bytes at a
// time without decoding; one atomic per wave that found one.
template <int ST>
__global__ void k_nonfinite(const uint4 *__restrict__ p, size_t n16, uint32_t *flags, uint32_t bit,
                            const int32_t *health)
{
    if (health != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t hf = (uint32_t)*health & kNonfiniteInput;
        if (hf) atomicOr(flags, hf);
    }
    bool bad = false;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) {
        const uint4 q = p[i];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (ST == kF32)
                bad |= (w[k] & 0x7F800000u) == 0x7F800000u;
            else if constexpr (ST == kF16)
                bad |= ((w[k] & 0x7C00u) == 0x7C00u) | ((w[k] & 0x7C000000u) == 0x7C000000u);
            else
                bad |= ((w[k] & 0x7F80u) == 0x7F80u) | ((w[k] & 0x7F800000u) == 0x7F800000u);
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flags, bit);
}

// grad_v += dJ/dc * 2c/v with v = (h/dt) sqrt(c): 2 g dt / (h sqrt(c)).
__global__ void k_grad_finish(const double *__restrict__ g, const float *__restrict__ c,
                              double *__restrict__ grad_v, int64_t nrows, int32_t nx, int32_t px,
                              double two_dt_over_h)
{
    const size_t total = (size_t)nrows * nx;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)nx, x = i - rw * (size_t)nx;
        const size_t p = rw * (size_t)px + x;
        grad_v[i] += g[p] * two_dt_over_h / sqrt((double)c[p]);
    }
}

// image += the accumulated zero-lag correlation (padded -> dense).
__global__ void k_image_finish(const double *__restrict__ g, double *__restrict__ image,
                               int64_t nrows, int32_t nx, int32_t px)
{
    const size_t total = (size_t)nrows * nx;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const size_t rw = i / (size_t)nx, x = i - rw * (size_t)nx;
        image[i] += g[rw * (size_t)px + x];
    }
}

// --------------------------------------------------------------------------
// Host launchers
// --------------------------------------------------------------------------
static int grid_blocks(size_t n, int threads)
{
    size_t b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_fill_u32(void *p, size_t nwords, uint32_t val, hipStream_t s)
{
    if (nwords == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(nwords, 256)), dim3(256), 0, s,
                       (uint32_t *)p, nwords, val);
    return hipGetLastError();
}

hipError_t launch_model_c(const float *v, float *c, int64_t nrows, int32_t nx, int32_t px,
                          double r, uint32_t *scratch, hipStream_t s)
{
    hipLaunchKernelGGL(k_model_c, dim3(grid_blocks((size_t)nrows * nx, 256)), dim3(256), 0, s,
                       v, c, nrows, nx, px, r, scratch);
    return hipGetLastError();
}

hipError_t launch_model_c16(const float *v, uint16_t *c16, int64_t nrows, int32_t nx, int32_t px,
                            double r, float inv_scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_model_c16, dim3(grid_blocks((size_t)nrows * nx, 256)), dim3(256), 0, s,
                       v, c16, nrows, nx, px, r, inv_scale);
    return hipGetLastError();
}

hipError_t launch_begin(int storage, void *cur, int64_t src_off, float amp,
                        const float *wavelet, int64_t nt, int32_t *meta, hipStream_t s)
{
    switch (storage) {
    case kF32: hipLaunchKernelGGL(k_begin<kF32>, dim3(1), dim3(64), 0, s, cur, src_off, amp, wavelet, nt, meta); break;
    case kF16: hipLaunchKernelGGL(k_begin<kF16>, dim3(1), dim3(64), 0, s, cur, src_off, amp, wavelet, nt, meta); break;
    default: hipLaunchKernelGGL(k_begin<kBF16>, dim3(1), dim3(64), 0, s, cur, src_off, amp, wavelet, nt, meta); break;
    }
    return hipGetLastError();
}

hipError_t launch_get_field(int storage, const void *buf, float *out, int64_t nrows, int32_t nx,
                            int32_t px, const int32_t *meta, int32_t level_slot, hipStream_t s)
{
    const dim3 g(grid_blocks((size_t)nrows * nx, 256)), b(256);
    switch (storage) {
    case kF32: hipLaunchKernelGGL(k_get_field<kF32>, g, b, 0, s, buf, out, nrows, nx, px, meta, level_slot); break;
    case kF16: hipLaunchKernelGGL(k_get_field<kF16>, g, b, 0, s, buf, out, nrows, nx, px, meta, level_slot); break;
    default: hipLaunchKernelGGL(k_get_field<kBF16>, g, b, 0, s, buf, out, nrows, nx, px, meta, level_slot); break;
    }
    return hipGetLastError();
}

hipError_t launch_set_field(int storage, const float *in, void *buf, int64_t nrows, int32_t nx,
                            int32_t px, int32_t *meta, int32_t slot, hipStream_t s)
{
    if (storage != kF32) {
        uint32_t *slots = (uint32_t *)&meta[kMaxBase + slot * kMaxSlots];
        hipError_t e = launch_fill_u32(slots, kMaxSlots, 0u, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_absmax, dim3(grid_blocks((size_t)nrows * nx, 256)), dim3(256), 0, s,
                           in, (size_t)nrows * nx, slots);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 g(grid_blocks((size_t)nrows * px, 256)), b(256);
    switch (storage) {
    case kF32: hipLaunchKernelGGL(k_set_field<kF32>, g, b, 0, s, in, buf, nrows, nx, px, meta, slot); break;
    case kF16: hipLaunchKernelGGL(k_set_field<kF16>, g, b, 0, s, in, buf, nrows, nx, px, meta, slot); break;
    default: hipLaunchKernelGGL(k_set_field<kBF16>, g, b, 0, s, in, buf, nrows, nx, px, meta, slot); break;
    }
    return hipGetLastError();
}

hipError_t launch_nonfinite(int storage, const void *level, size_t bytes, uint32_t *flags, uint32_t bit,
                            const int32_t *health, hipStream_t s)
{
    if (bytes % 16 != 0) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const dim3 g(grid_blocks(n16, 256)), b(256);
    const uint4 *p = (const uint4 *)level;
    switch (storage) {
    case kF32: hipLaunchKernelGGL(k_nonfinite<kF32>, g, b, 0, s, p, n16, flags, bit, health); break;
    case kF16: hipLaunchKernelGGL(k_nonfinite<kF16>, g, b, 0, s, p, n16, flags, bit, health); break;
    default: hipLaunchKernelGGL(k_nonfinite<kBF16>, g, b, 0, s, p, n16, flags, bit, health); break;
    }
    return hipGetLastError();
}

hipError_t launch_image_finish(const double *g, double *image, int64_t nrows, int32_t nx,
                               int32_t px, hipStream_t s)
{
    hipLaunchKernelGGL(k_image_finish, dim3(grid_blocks((size_t)nrows * nx, 256)), dim3(256), 0, s,
                       g, image, nrows, nx, px);
    return hipGetLastError();
}

hipError_t launch_grad_finish(const double *g, const float *c, double *grad_v, int64_t nrows,
                              int32_t nx, int32_t px, double two_dt_over_h, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_finish, dim3(grid_blocks((size_t)nrows * nx, 256)), dim3(256), 0,
                       s, g, c, grad_v, nrows, nx, px, two_dt_over_h);
    return hipGetLastError();
}

// Tile shapes.  2D: one wave, 64*VX columns by zc rows.  3D: NW waves of
// RPW rows each, (64/RPW*VX) x (NW*RPW*RY) cells by zc planes: FP32 fields
// 256x8 (4 cells x 2 rows per lane) or, chosen per grid, 128x8 (below),
// 16-bit fields 128x8 (4 cells x 1 row per lane, two rows per wave: half the
// y-halo loads of a 256x4 tile, measured 568 -> 554 us at 768x768x512 BF16).
// (Overridable at build time for tuning.)
#ifndef FD_3D_VX32
#define FD_3D_VX32 4
#endif
#ifndef FD_3D_RY32
#define FD_3D_RY32 2
#endif
#ifndef FD_3D_VX16
#define FD_3D_VX16 4
#endif
#ifndef FD_3D_RY16
#define FD_3D_RY16 1
#endif
#ifndef FD_3D_NW32
#define FD_3D_NW32 4
#endif
#ifndef FD_3D_NW16
#define FD_3D_NW16 4
#endif
#ifndef FD_3D_RPW32
#define FD_3D_RPW32 1
#endif
#ifndef FD_3D_RPW16
#define FD_3D_RPW16 2
#endif
constexpr int k3dVX32 = FD_3D_VX32, k3dRY32 = FD_3D_RY32;   // FP32 fields
constexpr int k3dVX16 = FD_3D_VX16, k3dRY16 = FD_3D_RY16;   // 16-bit fields
constexpr int kBatchVX = 2;

// FP32 fields have two tile shapes: 256x8 (4 cells x 2 rows per lane, 2
// waves per SIMD) and 128x8 (4 cells x 1 row per lane, two rows per wave, 3
// waves per SIMD).  The wide tile is faster on large grids that it fits
// (512^3 369 against 390 us, 768x768x512 860 against 925: about 5.5% per
// column), the narrow one where the x size leaves much of the last 256-wide
// tile empty (384^3 210 -> 155 us, 320x512x512 328 -> 248, 640x640x256 358
// -> 310, 896x448x256 331 -> 305) and on small grids, which need short
// z-chunks to fill the device and gain from twice the columns (256^3 55 ->
// 51 us, 768x256x256 140 -> 135); same bits either way.
constexpr int k3dRYN32 = 1, k3dRPWN32 = 2;
constexpr int k3dTXW32 = 64 / FD_3D_RPW32 * k3dVX32, k3dTXN32 = 64 / k3dRPWN32 * k3dVX32;

// Whether an FP32 3D step takes the narrow tile: when its padded width, at
// 1.055 times the cost per column, is smaller, or when the grid (at the
// wide tile's padded width) holds fewer than 2^26 cells.
static bool narrow_tile_f32(int nx, int ny, int nz)
{
    const int64_t wide = ((int64_t)nx + k3dTXW32 - 1) / k3dTXW32 * k3dTXW32;
    const int64_t narrow = ((int64_t)nx + k3dTXN32 - 1) / k3dTXN32 * k3dTXN32;
    return 1000 * wide > 1055 * narrow || wide * ny * nz < ((int64_t)1 << 26);
}

// The 3D forward kernel of a storage kind (16-bit c or not; FP32: the
// narrow tile or not).
template <int ST, bool CQ, bool NARROW = false>
static const void *step3d_fwd_kernel()
{
    if constexpr (ST == kF32 && NARROW)
        return reinterpret_cast<const void *>(&k_step3d<kF32, k3dVX32, k3dRYN32, FD_3D_NW32, k3dRPWN32, kFwd, false>);
    else if constexpr (ST == kF32)
        return reinterpret_cast<const void *>(&k_step3d<kF32, k3dVX32, k3dRY32, FD_3D_NW32, FD_3D_RPW32, kFwd, false>);
    else
        return reinterpret_cast<const void *>(&k_step3d<ST, k3dVX16, k3dRY16, FD_3D_NW16, FD_3D_RPW16, kFwd, CQ>);
}

// Blocks of the 3D forward kernel that fit on the device at once (queried
// once per kernel; the CU count times the occupancy per CU).
static int64_t resident_blocks_3d(int storage, bool cq, bool narrow)
{
    static int64_t cache[6] = {0, 0, 0, 0, 0, 0};
    const int k = storage == kF32 ? (narrow ? 5 : 0) : (storage == kF16 ? 1 : 2) + (cq ? 2 : 0);
    if (cache[k] == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) {
            const void *f = storage == kF32 ? (narrow ? step3d_fwd_kernel<kF32, false, true>()
                                                      : step3d_fwd_kernel<kF32, false>())
                            : storage == kF16 ? (cq ? step3d_fwd_kernel<kF16, true>() : step3d_fwd_kernel<kF16, false>())
                                              : (cq ? step3d_fwd_kernel<kBF16, true>() : step3d_fwd_kernel<kBF16, false>());
            const int threads = 64 * (storage == kF32 ? FD_3D_NW32 : FD_3D_NW16);
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, threads, 0);
        }
        (void)hipGetLastError();
        cache[k] = (e == hipSuccess && cus > 0 && per_cu > 0) ? (int64_t)cus * per_cu : 512;
    }
    return cache[k];
}

// Tile shapes.  3D: NW waves of RPW rows, (64/RPW VX) x (NW RPW RY) cells by
// zc planes (the defaults come from a sweep of shapes on the 512^3 and
// 768x768x512 grids; FP32 grids pick the wide or the narrow tile with
// narrow_tile_f32).
// 2D: one wave, 64 VX columns by zc rows; the widest tile and tallest chunk
// that still give >= 2048 blocks (8 per CU) are taken from
// (VX, zc) = (2, 16), (2, 8), (1, 8), (1, 4).
void plan_tiles(StepArgs &a, int ndim, int storage, bool batched)
{
    if (ndim == 2) {
        static const int cand[4][2] = {{2, 16}, {2, 8}, {1, 8}, {1, 4}};
        for (int i = 0; i < 4; ++i) {
            if (batched && cand[i][0] != kBatchVX) continue;  // the batched kernel's width only
            a.vx = cand[i][0];
            a.zc = cand[i][1];
            a.tiles_x = (a.nx + 64 * a.vx - 1) / (64 * a.vx);
            a.tiles_z = (a.nz + a.zc - 1) / a.zc;
            if ((int64_t)a.tiles_x * a.tiles_z >= 2048) break;
        }
        a.tiles_y = 1;
    } else {
        // 3D: a.vx records the tile width in units of 64 cells, which picks
        // the FP32 kernel (4: 256 wide, 2: 128 wide)
        const bool narrow = storage == kF32 && narrow_tile_f32(a.nx, a.ny, a.nz);
        const int VX = storage == kF32 ? k3dVX32 : k3dVX16;
        const int RY = storage == kF32 ? (narrow ? k3dRYN32 : k3dRY32) : k3dRY16;
        const int NW = storage == kF32 ? FD_3D_NW32 : FD_3D_NW16;
        const int RPW = storage == kF32 ? (narrow ? k3dRPWN32 : FD_3D_RPW32) : FD_3D_RPW16;
        const int TX = 64 / RPW * VX, TY = NW * RPW * RY;
        a.vx = (int16_t)(TX / 64);
        a.tiles_x = (a.nx + TX - 1) / TX;
        a.tiles_y = (a.ny + TY - 1) / TY;
        // Planes per block: a block streams zc planes after priming 8 halo
        // planes, and blocks run in R = ceil(blocks / resident) rounds, so
        // the time goes as (R + 3/16) * (zc + 8), the fraction standing for
        // filling and draining the device, which a later round overlaps with
        // the blocks still running (512^3 FP32: two rounds of 64 planes 364
        // us against one round of 128 planes 371 us; 16-bit fields: one
        // round of 171 planes and two of 86 within 1%).  The column is cut
        // into k equal chunks (zc = ceil(nz / k) >= 4: short columns, such
        // as a z-slab's, need short chunks to fill the device: 32 planes of
        // 512^2 in chunks of 8 take 31 us against 40 in chunks of 16); ties
        // go to the longer chunk (less halo traffic).
        const int64_t cols = (int64_t)a.tiles_x * a.tiles_y;
        const int64_t resident = resident_blocks_3d(storage, a.c16 != nullptr, narrow);
        a.resident = (int32_t)std::min<int64_t>(resident, 1 << 30);
        int64_t best = -1;
        for (int k = 1; k <= std::max(1, a.nz / 4); ++k) {
            const int zc = (a.nz + k - 1) / k;
            const int64_t nb = cols * ((a.nz + zc - 1) / zc);
            const int64_t cost = (16 * ((nb + resident - 1) / resident) + 3) * (int64_t)(zc + 8);
            if (best < 0 || cost < best) {
                best = cost;
                a.zc = zc;
            }
        }
        a.tiles_z = (a.nz + a.zc - 1) / a.zc;
    }
}

template <int ST, int MODE, bool CQ = false>
static void launch3d(const StepArgs &a, int nb, hipStream_t s)
{
    if constexpr (ST == kF32) {
        if (a.vx * 64 == k3dTXN32)
            hipLaunchKernelGGL((k_step3d<ST, k3dVX32, k3dRYN32, FD_3D_NW32, k3dRPWN32, MODE, false>), dim3(nb),
                               dim3(64 * FD_3D_NW32), 0, s, a);
        else
            hipLaunchKernelGGL((k_step3d<ST, k3dVX32, k3dRY32, FD_3D_NW32, FD_3D_RPW32, MODE, false>), dim3(nb),
                               dim3(64 * FD_3D_NW32), 0, s, a);
    }
    else
        hipLaunchKernelGGL((k_step3d<ST, k3dVX16, k3dRY16, FD_3D_NW16, FD_3D_RPW16, MODE, CQ>), dim3(nb),
                           dim3(64 * FD_3D_NW16), 0, s, a);
}

template <int VX>
static void launch2d(const StepArgs &a, int storage, int mode, int nb, hipStream_t s)
{
    const dim3 g(nb), b(64);
    const bool cq = a.c16 != nullptr;
    if (storage == kF32) {
        if (mode == kFwd) hipLaunchKernelGGL((k_step2d<kF32, VX, kFwd, false>), g, b, 0, s, a);
        else if (mode == kFwdLap) hipLaunchKernelGGL((k_step2d<kF32, VX, kFwdLap, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<kF32, VX, kAdj, false>), g, b, 0, s, a);
    } else if (storage == kF16) {
        if (cq) hipLaunchKernelGGL((k_step2d<kF16, VX, kFwd, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<kF16, VX, kFwd, false>), g, b, 0, s, a);
    } else {
        if (cq) hipLaunchKernelGGL((k_step2d<kBF16, VX, kFwd, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_step2d<kBF16, VX, kFwd, false>), g, b, 0, s, a);
    }
}

hipError_t launch_step(StepArgs a, int ndim, int storage, int mode, hipStream_t s)
{
    // 16-bit c is built for the forward step on 16-bit fields only
    if (a.c16 != nullptr && (storage == kF32 || mode != kFwd)) return hipErrorInvalidValue;
    plan_tiles(a, ndim, storage, false);
    const int nb = a.tiles_x * a.tiles_y * a.tiles_z;
    if (ndim == 2) {
        if (a.vx == 2) launch2d<2>(a, storage, mode, nb, s);
        else launch2d<1>(a, storage, mode, nb, s);
    } else {
        if (storage == kF32) {
            if (mode == kFwd) launch3d<kF32, kFwd>(a, nb, s);
            else if (mode == kFwdLap) launch3d<kF32, kFwdLap>(a, nb, s);
            else launch3d<kF32, kAdj>(a, nb, s);
        } else if (storage == kF16) {
            if (a.c16 != nullptr) launch3d<kF16, kFwd, true>(a, nb, s);
            else launch3d<kF16, kFwd>(a, nb, s);
        } else {
            if (a.c16 != nullptr) launch3d<kBF16, kFwd, true>(a, nb, s);
            else launch3d<kBF16, kFwd>(a, nb, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_step_batch2d(Batch2D &b, int mode, hipStream_t s)
{
    int total = 0;
    for (int i = 0; i < b.count; ++i) {
        plan_tiles(b.it[i], 2, kF32, true);
        b.begin[i] = total;
        total += b.it[i].tiles_x * b.it[i].tiles_z;
    }
    b.begin[b.count] = total;
    if (total == 0) return hipSuccess;
    switch (mode) {
    case kFwd: hipLaunchKernelGGL((k_step2d_batch<kBatchVX, kFwd>), dim3(total), dim3(64), 0, s, b); break;
    case kFwdLap: hipLaunchKernelGGL((k_step2d_batch<kBatchVX, kFwdLap>), dim3(total), dim3(64), 0, s, b); break;
    default: hipLaunchKernelGGL((k_step2d_batch<kBatchVX, kAdj>), dim3(total), dim3(64), 0, s, b); break;
    }
    return hipGetLastError();
}

}  // namespace fdk
