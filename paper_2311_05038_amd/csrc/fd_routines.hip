// The time step laid out as the paper's routines, one kernel each
// (arXiv 2311.05038, Section 7, Listing 3: fd_pzz, fd_pxx, fd_time,
// add_source, then the level rotation), for FP32 fields in the padded layout
// of the fused kernels.  The second-derivative fields are materialised in
// HBM between the kernels (4 B read + 4 B written per cell per derivative,
// then 24 B read + 4 B written by the time update in 3D), which is what the
// fused step kernel avoids; the arithmetic is the fused kernel's, operation
// for operation, so both give the same bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fd_device.hpp"
#include "fd_launch.hpp"

namespace fdk {

namespace {

// Second difference along a strided axis (z, or y in 3D).  A
// thread owns 4 adjacent x cells of one line along the axis and walks a
// chunk of it with a 9-deep register queue, so each input value is read
// once.  Work item w = (outer line, chunk, x group), x group fastest, so the
// chunks that share halo planes run close together.
template <bool STREAM>
__global__ __launch_bounds__(256) void k_deriv_axis(const float *__restrict__ in,
                                                    float *__restrict__ out, int32_t n_axis,
                                                    int64_t axis_stride, int32_t n_outer,
                                                    int64_t outer_stride, int32_t px, int32_t chunk)
{
    const int32_t groups = px / 4;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t lines = (int64_t)n_outer * groups;
    const int64_t nchunks = (n_axis + chunk - 1) / chunk;
    if (w >= lines * nchunks) return;
    const int32_t g = (int32_t)(w % groups);
    const int32_t k0 = (int32_t)((w / groups) % nchunks) * chunk;
    const int64_t o = w / (groups * nchunks);
    const int32_t k1 = min(k0 + chunk, n_axis);
    const float *base = in + o * outer_stride + 4 * g;
    float *obase = out + o * outer_stride + 4 * g;
    auto ld = [&](int32_t k) -> float4 {
        if (k < 0 || k >= n_axis) return make_float4(0.f, 0.f, 0.f, 0.f);
        return *reinterpret_cast<const float4 *>(base + (int64_t)k * axis_stride);
    };
    float4 q[9];
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = ld(k0 - 4 + i);
    for (int32_t k = k0; k < k1; ++k) {
        q[8] = ld(k + 4);
        float4 r;
        r.x = axis_d2(q[0].x, q[1].x, q[2].x, q[3].x, q[4].x, q[5].x, q[6].x, q[7].x, q[8].x);
        r.y = axis_d2(q[0].y, q[1].y, q[2].y, q[3].y, q[4].y, q[5].y, q[6].y, q[7].y, q[8].y);
        r.z = axis_d2(q[0].z, q[1].z, q[2].z, q[3].z, q[4].z, q[5].z, q[6].z, q[7].z, q[8].z);
        r.w = axis_d2(q[0].w, q[1].w, q[2].w, q[3].w, q[4].w, q[5].w, q[6].w, q[7].w, q[8].w);
        if constexpr (STREAM)
            stp_stream<float, 4>(obase + (int64_t)k * axis_stride, Pack<float, 4>{{r.x, r.y, r.z, r.w}});
        else
            *reinterpret_cast<float4 *>(obase + (int64_t)k * axis_stride) = r;
#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
    }
}

// Second difference along x: a thread owns 4 adjacent cells of
// a row and loads only those; the 4 values on each side come from the
// neighbouring lanes through the wave (lanes hold consecutive groups of a
// row), and only the wave's first and last lanes load them.  Cells past nx
// hold zeros in every field, and taps past the padded row read zero.
template <bool STREAM>
__global__ __launch_bounds__(256) void k_deriv_x(const float *__restrict__ in, float *__restrict__ out,
                                                 int64_t nrows, int32_t px)
{
    const int32_t groups = px / 4;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = w < nrows * groups;   // every lane takes part in the shuffles
    const int64_t row = valid ? w / groups : 0;
    const int32_t x0 = valid ? (int32_t)(w % groups) * 4 : 0;
    const int lane = threadIdx.x & 63;
    const float *r = in + row * px;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = valid ? *reinterpret_cast<const float4 *>(r + x0) : zero;
    float4 a, c;
    a.x = __shfl_up(b.x, 1, 64);
    a.y = __shfl_up(b.y, 1, 64);
    a.z = __shfl_up(b.z, 1, 64);
    a.w = __shfl_up(b.w, 1, 64);
    c.x = __shfl_down(b.x, 1, 64);
    c.y = __shfl_down(b.y, 1, 64);
    c.z = __shfl_down(b.z, 1, 64);
    c.w = __shfl_down(b.w, 1, 64);
    if (!valid) return;
    // the previous group is in this row when x0 >= 4, and in this wave
    // unless this is its first lane (likewise for the next group)
    if (x0 < 4) a = zero;
    else if (lane == 0) a = *reinterpret_cast<const float4 *>(r + x0 - 4);
    if (x0 + 4 >= px) c = zero;
    else if (lane == 63) c = *reinterpret_cast<const float4 *>(r + x0 + 4);
    const float u[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
    float o[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        o[v] = axis_d2(u[v], u[v + 1], u[v + 2], u[v + 3], u[v + 4], u[v + 5], u[v + 6], u[v + 7], u[v + 8]);
    if constexpr (STREAM)
        stp_stream<float, 4>(out + row * px + x0, Pack<float, 4>{{o[0], o[1], o[2], o[3]}});
    else
        *reinterpret_cast<float4 *>(out + row * px + x0) = make_float4(o[0], o[1], o[2], o[3]);
}

// Time update with the sponge, from the materialised derivative fields:
//   L = Pzz + (Pyy + Pxx)      (2D: Pzz + Pxx)
//   new = G (2 cur + c L) - G^2 prev,  G = gz gy gx,
// written over prev, with the receivers sampling `new`.
// STREAM (all three kinds of routine kernels): non-temporal accesses, for
// steps whose fields cannot stay in the Infinity Cache anyway (512^3: the
// routine step 1,373 -> 1,229 us, fd_time 715 -> 591 us); on smaller grids
// the cache keeps each kernel's output for the next kernel, and the ordinary
// accesses are faster (2048x4096: fd_pzz 14.7 against 18.0 us).
template <int NDIM, bool STREAM>
__global__ __launch_bounds__(256) void k_time(StepArgs a, const float *__restrict__ dzz,
                                              const float *__restrict__ dxx,
                                              const float *__restrict__ dyy)
{
    const int32_t groups = a.px / 4;
    const int64_t nrows = (int64_t)a.nz * a.ny;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nrows * groups) return;
    const int64_t row = w / groups;
    const int32_t x0 = (int32_t)(w % groups) * 4;
    const int32_t z = (int32_t)(row / a.ny), y = (int32_t)(row % a.ny);
    const int64_t off = row * a.px + x0;
    const float *cur = (const float *)a.cur;
    float *prv = (float *)a.prev;
    using P4 = Pack<float, 4>;
    auto ld = [&](const float *p) -> P4 {
        if constexpr (STREAM)
            return ldp_stream<float, 4>(p);
        else
            return ldp<float, 4>(p);
    };
    const P4 P = ld(cur + off), Q = ld(prv + off), C = ld(a.c + off), Z = ld(dzz + off);
    const P4 X = ld(dxx + off);
    P4 Y{};
    if constexpr (NDIM == 3) Y = ld(dyy + off);
    const float(&pv)[4] = P.v, (&qv)[4] = Q.v, (&cv)[4] = C.v, (&zv)[4] = Z.v, (&xv)[4] = X.v,
               (&yv)[4] = Y.v;
    const float gzz = a.gz[z];
    const float gzy = NDIM == 3 ? gzz * a.gy[y] : gzz;
    float nw[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int32_t x = x0 + v;
        const float gx = x < a.nx ? a.gx[x] : 0.0f;
        float lap;
        if constexpr (NDIM == 3)
            lap = zv[v] + (yv[v] + xv[v]);
        else
            lap = zv[v] + xv[v];
        nw[v] = x < a.nx ? leapfrog(gzy * gx, pv[v], cv[v], lap, qv[v]) : 0.0f;
    }
    if (a.trace_row != nullptr) {
        const int32_t zr = z - a.rec.z0, yr = y - a.rec.y0;
        if (zr >= 0 && yr >= 0 && zr % a.rec.dz == 0 && yr % a.rec.dy == 0 && zr / a.rec.dz < a.rec.nz &&
            yr / a.rec.dy < a.rec.ny) {
            const int64_t rrow = (int64_t)(zr / a.rec.dz) * a.rec.ny + yr / a.rec.dy;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t xr = x0 + v - a.rec.x0;
                if (x0 + v < a.nx && xr >= 0 && xr % a.rec.dx == 0 && xr / a.rec.dx < a.rec.nx)
                    a.trace_row[rrow * a.rec.nx + xr / a.rec.dx] = nw[v];
            }
        }
    }
    if constexpr (STREAM)
        stp_stream<float, 4>(prv + off, P4{{nw[0], nw[1], nw[2], nw[3]}});
    else
        stp<float, 4>(prv + off, P4{{nw[0], nw[1], nw[2], nw[3]}});
}

// The source addition of step n + 1 into the new field (none after the last
// step).
__global__ void k_add_source(StepArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || a.n + 1 >= a.nt) return;
    float *p = (float *)a.prev;
    const int64_t off = ((int64_t)a.sz * a.ny + a.sy) * a.px + a.sx;
    p[off] += a.amp * a.wavelet[a.n + 1];
}

int blocks_for(int64_t items, int threads) { return (int)((items + threads - 1) / threads); }

constexpr int kMaxDevices = 64;

}  // namespace

// The work area of the routine-per-kernel step for callers that cannot
// allocate: every GPU the library is loaded on holds its own copy.  In host
// code this name stands for the symbol only; the device address comes from
// routines_scratch().
static __device__ __align__(256) unsigned char scratch[kRoutinesScratchBytes];

hipError_t routines_scratch(hipStream_t s, void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = s != nullptr ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        // the symbol's address on `dev`, looked up with `dev` current
        int cur = 0;
        e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (p == nullptr || (uintptr_t)p % 256 != 0) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_routines(const StepArgs &a, int ndim, float *dzz, float *dxx, float *dyy,
                           hipStream_t s)
{
    const int64_t groups = a.px / 4;
    const int64_t nrows = (int64_t)a.nz * a.ny;
    const int64_t pp = (int64_t)a.ny * a.px;
    const float *cur = (const float *)a.cur;
    // streaming accesses when the step's fields (ndim + 3 read by fd_time,
    // one written) exceed the 256 MiB Infinity Cache
    const bool stream = (double)nrows * (double)a.px * 4.0 * (ndim + 4) > 256.0 * 1048576.0;
    // chunk of an axis walk: the longest (<= 64) that still gives >= 2^19
    // threads, at least 8
    auto chunk_for = [&](int64_t n_axis, int64_t lines) {
        int64_t c = 64;
        while (c > 8 && lines * ((n_axis + c - 1) / c) < ((int64_t)1 << 19)) c /= 2;
        return (int32_t)c;
    };
    // fd_pzz: along z, lines over (y, x)
    {
        const int32_t ch = chunk_for(a.nz, (int64_t)a.ny * groups);
        const int64_t items = (int64_t)a.ny * groups * ((a.nz + ch - 1) / ch);
        if (stream)
            hipLaunchKernelGGL(k_deriv_axis<true>, dim3(blocks_for(items, 256)), dim3(256), 0, s, cur, dzz,
                               a.nz, pp, a.ny, (int64_t)a.px, a.px, ch);
        else
            hipLaunchKernelGGL(k_deriv_axis<false>, dim3(blocks_for(items, 256)), dim3(256), 0, s, cur, dzz,
                               a.nz, pp, a.ny, (int64_t)a.px, a.px, ch);
    }
    // fd_pxx: along x, rows
    if (stream)
        hipLaunchKernelGGL(k_deriv_x<true>, dim3(blocks_for(nrows * groups, 256)), dim3(256), 0, s, cur, dxx,
                           nrows, a.px);
    else
        hipLaunchKernelGGL(k_deriv_x<false>, dim3(blocks_for(nrows * groups, 256)), dim3(256), 0, s, cur, dxx,
                           nrows, a.px);
    // the y derivative of the 3D form: along y, lines over (z, x)
    if (ndim == 3) {
        const int32_t ch = chunk_for(a.ny, (int64_t)a.nz * groups);
        const int64_t items = (int64_t)a.nz * groups * ((a.ny + ch - 1) / ch);
        if (stream)
            hipLaunchKernelGGL(k_deriv_axis<true>, dim3(blocks_for(items, 256)), dim3(256), 0, s, cur, dyy,
                               a.ny, (int64_t)a.px, a.nz, pp, a.px, ch);
        else
            hipLaunchKernelGGL(k_deriv_axis<false>, dim3(blocks_for(items, 256)), dim3(256), 0, s, cur, dyy,
                               a.ny, (int64_t)a.px, a.nz, pp, a.px, ch);
    }
    // fd_time
    const dim3 tg(blocks_for(nrows * groups, 256)), tb(256);
    if (ndim == 3) {
        if (stream) hipLaunchKernelGGL((k_time<3, true>), tg, tb, 0, s, a, dzz, dxx, dyy);
        else hipLaunchKernelGGL((k_time<3, false>), tg, tb, 0, s, a, dzz, dxx, dyy);
    } else {
        if (stream) hipLaunchKernelGGL((k_time<2, true>), tg, tb, 0, s, a, dzz, dxx, dyy);
        else hipLaunchKernelGGL((k_time<2, false>), tg, tb, 0, s, a, dzz, dxx, dyy);
    }
    // add_source
    hipLaunchKernelGGL(k_add_source, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace fdk
