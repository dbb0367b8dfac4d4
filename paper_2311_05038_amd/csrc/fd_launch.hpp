// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd_device.hpp"

namespace fdk {

constexpr int kBatchMax = 16;

// Kernel-argument table of one batched launch (passed by value, < 4 KiB).
struct Batch2D {
    int32_t count;
    int32_t begin[kBatchMax + 1];
    StepArgs it[kBatchMax];
};
static_assert(sizeof(Batch2D) <= 4096, "batched step arguments must fit the kernel-argument segment");

// Fills tiles_x/y/z, zc and vx of `a` for the kernel variant that runs it
// (batched: the tile width of the batched 2D kernel).
void plan_tiles(StepArgs &a, int ndim, int storage, bool batched);

hipError_t launch_step(StepArgs a, int ndim, int storage, int mode, hipStream_t s);
hipError_t launch_step_batch2d(Batch2D &b, int mode, hipStream_t s);
// The step as separate routine kernels (derivative fields dzz, dxx and, in
// 3D, dyy materialised in HBM); FP32 fields only.
hipError_t launch_routines(const StepArgs &a, int ndim, float *dzz, float *dxx, float *dyy,
                           hipStream_t s);
// Size of the routine step's static work area (one per device, held from
// load to process end), and its device address on the stream's device
// (looked up once per device; nothing is allocated).
constexpr size_t kRoutinesScratchBytes = (size_t)64 << 20;
hipError_t routines_scratch(hipStream_t s, void **ptr);
hipError_t launch_fill_u32(void *p, size_t nwords, uint32_t val, hipStream_t s);
// Memory-roof probe: kind 0 out = a, kind 1 out = a + b * out (n floats,
// a multiple of 4, 16-byte aligned arrays).
hipError_t launch_stream_probe(int kind, const float *a, const float *b, float *out, size_t n,
                               hipStream_t s);
// c = (v r)^2 into `c` (padded FP32; null: velocity range only), with the
// largest |v| and a flag for bad velocities in scratch[0..1].
hipError_t launch_model_c(const float *v, float *c, int64_t nrows, int32_t nx, int32_t px,
                          double r, uint32_t *scratch, hipStream_t s);
// c as 16-bit fixed point: min(RNE(c inv_scale), 65535), padded.
hipError_t launch_model_c16(const float *v, uint16_t *c16, int64_t nrows, int32_t nx, int32_t px,
                            double r, float inv_scale, hipStream_t s);
// The first source addition (s[0]), and the shot's health flag when any of
// its nt injected values is non-finite.
hipError_t launch_begin(int storage, void *cur, int64_t src_off, float amp,
                        const float *wavelet, int64_t nt, int32_t *meta, hipStream_t s);
hipError_t launch_get_field(int storage, const void *buf, float *out, int64_t nrows, int32_t nx,
                            int32_t px, const int32_t *meta, int32_t level_slot, hipStream_t s);
hipError_t launch_set_field(int storage, const float *in, void *buf, int64_t nrows, int32_t nx,
                            int32_t px, int32_t *meta, int32_t slot, hipStream_t s);
// Sets `bit` in *flags if the `bytes` (a multiple of 16) of a stored level
// at `level` (16-byte aligned) hold a non-finite value; with `health`, also
// the shot's sticky non-finite-input flag.
hipError_t launch_nonfinite(int storage, const void *level, size_t bytes, uint32_t *flags, uint32_t bit,
                            const int32_t *health, hipStream_t s);
hipError_t launch_image_finish(const double *g, double *image, int64_t nrows, int32_t nx,
                               int32_t px, hipStream_t s);
hipError_t launch_grad_finish(const double *g, const float *c, double *grad_v, int64_t nrows,
                              int32_t nx, int32_t px, double two_dt_over_h, hipStream_t s);

}  // namespace fdk
