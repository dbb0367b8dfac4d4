// Plain data shared by the host logic and the step kernels: the kernel
// argument record of one step and the layout of the 16-bit storage
// bookkeeping.  No device code and no HIP types, so the host logic that
// fills these records builds without the GPU toolchain.
#pragma once

#include <stdint.h>

namespace fdk {

enum Mode : int {
    kFwd = 0,     // forward step
    kFwdLap = 1,  // forward step that also stores L(cur) (gradient recompute)
    kAdj = 2      // adjoint step: receiver injection of c G r, g += new * hist
};

// Forward modes that write a per-step history field (StepArgs::lap).
constexpr bool stores_history(int mode) { return mode == kFwdLap; }

enum StorageKind : int { kF32 = 0, kF16 = 1, kBF16 = 2 };

struct RecBox {
    int32_t z0, y0, x0;
    int32_t nz, ny, nx;
    int32_t dz, dy, dx;
};

// Arguments of one step on one grid.  Field buffers use a padded layout:
// element (z, y, x) sits at (z * ny + y) * px + x with px a multiple of 64;
// cells with x >= nx are zero in every field.
struct StepArgs {
    const void *cur;      // level n
    void *prev;           // level n-1 in, level n+1 out (unless `out` is set)
    void *out;            // forward steps: level n+1 here instead, prev only read
    const float *c;       // (v dt / h)^2, padded, zero in padding (FP32 c)
    const uint16_t *c16;  // or 16-bit fixed point: c = c16 * c16_scale (else null)
    float c16_scale;      // 2^(e - 16)
    float c16_inv;        // 2^(16 - e)
    const float *gz, *gy, *gx;  // damping profiles (nz, ny, nx entries)
    int32_t nz, ny, nx, px;
    int32_t zc;           // planes (rows in 2D) per block
    int16_t vx;           // 2D: cells per lane along x (tile width 64 * vx);
                          // 3D: tile width / 64 (FP32: 4 or 2, the kernel)
    int16_t zghost;       // 3D FP32: planes of cur readable past each z end (the
                          // ghost planes of a z-slab), else 0 (zero edges)
    int32_t tiles_x, tiles_y, tiles_z;
    int32_t resident;     // 3D: blocks resident at once (tile mapping)
    int32_t sz, sy, sx;   // source cell
    float amp;            // dt^2 / h^D
    const float *wavelet; // device, nt samples
    int64_t n, nt;
    RecBox rec;
    int32_t gmode;        // (fills the padding after rec)
                          // kAdj: 0 g += new lap; 1 no g update (deferred to a later
                          // step); 2 g += cur lap2, then new lap; 3 g += prev lap3,
                          // then cur lap2, then new lap (the deferred terms first:
                          // descending level order)
    float *trace_row;     // nrec floats of row n, or null
    int32_t *meta;        // 16-bit storage: e[4] exponents then max|.|[4] bits
    float *lap;           // kFwdLap: out (L cur);  kAdj: in (history of level k-1),
                          // padded FP32
    const float *lap2;    // kAdj, gmode 2 and 3: history of level k
    const float *lap3;    // kAdj, gmode 3: history of level k+1
    const float *resid_row;  // kAdj: dJ/dtraces row k-1 (nrec), or null
    double *g;            // kAdj: FP64 accumulator, padded
};

// Layout of the 16-bit storage bookkeeping ("meta", in the state buffer):
// meta[l] (l < 4) is the exponent of time level l mod 4; the largest
// magnitude of level l is the maximum over kMaxSlots words at
// meta[kMaxBase + l * kMaxSlots + k] (float bit patterns; blocks fold their
// maxima into slot blockIdx % kMaxSlots, which spreads the atomics).
constexpr int kMaxSlots = 64;
constexpr int kMaxBase = 16;
constexpr int kMetaWords = kMaxBase + 4 * kMaxSlots;
// meta[kHealth]: sticky flags of the shot (every storage kind); bit 2 is set
// when a non-finite value entered it (a wavelet sample times the source
// amplitude, or a value given to fd_set_wavefield)
constexpr int kHealth = 8;
constexpr uint32_t kNonfiniteInput = 4u;

}  // namespace fdk
