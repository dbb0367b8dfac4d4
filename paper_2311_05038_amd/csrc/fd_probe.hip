// Memory-roof probes: plain streams with the access patterns of the step
// kernels and no stencil, which measure the HBM bandwidth those kernels can
// reach on this GPU (the role the measured stream bandwidth plays under the
// roofline of arXiv 2311.05038, Section 7).
#include <hip/hip_runtime.h>

#include "fd_device.hpp"
#include "fd_launch.hpp"

namespace fdk {

namespace {

// kind 0: out = a (8 bytes per element); kind 1: out = a + b * out in place
// (three streams read, one rewritten: the FP32 step's 16 bytes per cell).
// Each thread issues all its loads (U float4 per stream, 256 apart) before
// it computes and stores; blocks take consecutive ranges in launch order.
// The configuration of each kind is the fastest of a sweep on MI355X (1 GiB
// copy / 512^3 three-stream update): kind 0 one float4 per thread with
// ordinary loads (6.26 TB/s; 4 per thread 5.68, non-temporal loads 6.11),
// kind 1 four float4 per stream with non-temporal loads (6.13 TB/s;
// ordinary loads 5.40, two per thread 6.01, eight per thread 1.14 (register
// pressure), XCD-contiguous block ranges 5.83, grid-stride loops <= 5.79);
// stores are non-temporal in both.
constexpr int kProbeThreads = 256;

template <int KIND, int U, bool NTL>
__global__ __launch_bounds__(kProbeThreads) void k_stream(const float4 *__restrict__ a,
                                                          const float4 *__restrict__ b,
                                                          float4 *__restrict__ out, size_t n4)
{
    const size_t base = (size_t)blockIdx.x * (kProbeThreads * U) + threadIdx.x;
    Pack<float, 4> x[U], y[U], z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * kProbeThreads;
        if (i < n4) {
            x[u] = NTL ? ldp_stream<float, 4>((const float *)(a + i)) : ldp<float, 4>((const float *)(a + i));
            if constexpr (KIND == 1) {
                y[u] = NTL ? ldp_stream<float, 4>((const float *)(b + i)) : ldp<float, 4>((const float *)(b + i));
                z[u] = NTL ? ldp_stream<float, 4>((const float *)(out + i)) : ldp<float, 4>((const float *)(out + i));
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * kProbeThreads;
        if (i < n4) {
            Pack<float, 4> r = x[u];
            if constexpr (KIND == 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) r.v[k] = fmaf(y[u].v[k], z[u].v[k], x[u].v[k]);
            }
            stp_stream<float, 4>((float *)(out + i), r);
        }
    }
}

constexpr int kCopyU = 1, kStepU = 4;

}  // namespace

hipError_t launch_stream_probe(int kind, const float *a, const float *b, float *out, size_t n,
                               hipStream_t s)
{
    const size_t n4 = n / 4;
    const size_t per_block = (size_t)kProbeThreads * (kind == 0 ? kCopyU : kStepU);
    const size_t blocks = (n4 + per_block - 1) / per_block;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), t(kProbeThreads);
    if (kind == 0)
        hipLaunchKernelGGL((k_stream<0, kCopyU, false>), g, t, 0, s, (const float4 *)a, (const float4 *)nullptr,
                           (float4 *)out, n4);
    else
        hipLaunchKernelGGL((k_stream<1, kStepU, true>), g, t, 0, s, (const float4 *)a, (const float4 *)b,
                           (float4 *)out, n4);
    return hipGetLastError();
}

}  // namespace fdk
