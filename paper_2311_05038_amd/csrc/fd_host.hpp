// Host-side logic of the C ABI that needs no device: the error text behind
// fd_last_error, buffer layouts, argument validation, the stability check,
// the damping profiles and the kernel arguments of a shot's step.  Free of
// HIP, so it also builds with a plain host compiler (the sanitizer test
// builds it with AddressSanitizer and UBSan and drives every function here).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/fd.h"
#include "fd_args.hpp"

namespace fdh {

// Records a printf-style message for fd_last_error and returns st.
fd_status fail(fd_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// Clears the message and returns FD_OK.
fd_status ok();
// The calling thread's last message ("" after ok()).
const char *last_error();

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Largest magnitude of the 8th-order second-difference symbol, 4096/630.
constexpr double kSymbolMax = 4096.0 / 630.0;
constexpr int64_t kMaxDim = (int64_t)1 << 30;

struct Layout {
    int32_t ndim, storage, c_storage;
    int64_t nz, ny, nx;
    int32_t px;        // row pitch in elements (multiple of 64)
    size_t npad;       // nz * ny * px
    size_t elem;       // bytes per stored field element
    size_t field;      // bytes of one stored field, aligned
    size_t f32field;   // bytes of one FP32 padded field, aligned
    size_t cfield;     // bytes of the stored c (FP32 or 16-bit fixed point), aligned
    size_t c_off, gz_off, gy_off, gx_off, scratch_off, model_bytes;
    size_t state_bytes, meta_off;
    // z-slab of a larger grid: global index of plane 0, global plane count
    // (nz for an ordinary grid), and the bytes of the 4 ghost planes that
    // precede (and follow) a slab's stored level (0 for an ordinary grid)
    int64_t z0, nzg;
    size_t ghost;
};

constexpr int kGhost = 4;  // the stencil radius

bool is_slab(const Layout &L);
// Sizes and offsets of every buffer for a grid that passed check_grid.
Layout make_layout(const fd_grid &g);
size_t ckpt_slot_bytes(const Layout &L);
int64_t n_ckpt(int64_t nt, int32_t every);
size_t adjoint_work_bytes(const Layout &L, int32_t every);
fd_status check_grid(const fd_grid *g);

// Damping factors g(i) = exp(-(alpha d)^2), d the distance into the band of
// width W on the enabled faces (0 off the band), FP64 rounded to FP32.
std::vector<float> damping_profile(int64_t n, int32_t W, double alpha, bool lo, bool hi);
// dt^2 / dh^D, the source amplitude factor.
float source_amp(const fd_grid &g);
// FD_OK, or FD_ERR_UNSTABLE when vmax dt/dh breaks the stability limit of
// the 8th-order scheme in ndim dimensions.
fd_status check_stability(const fd_grid &g, float vmax);
// The exponent e of the 16-bit fixed-point c (codes c 2^(16-e)) for the
// largest velocity: e = floor(log2 cmax) + 1, raised by one when cmax lies
// within half a code of 2^e.
int c16_exponent(float vmax, double dt_over_dh);

}  // namespace fdh

// The opaque handles of include/fd.h.
struct fd_model {
    fd_grid grid;
    fdh::Layout L;
    float *c;          // FP32 c, or null when c is stored in 16-bit fixed point
    uint16_t *c16;     // 16-bit fixed-point c (value c16 * c16_scale), or null
    float c16_scale;   // 2^(e - 16)
    float c16_inv;     // 2^(16 - e)
    float *gz, *gy, *gx;
    uint32_t *scratch;
    float amp;  // dt^2 / h^D
};

struct fd_state {
    const fd_model *m;
    void *base;    // the state buffer
    void *buf[2];  // plane 0 of each stored level (past a slab's leading ghosts)
    int32_t *meta;
    int64_t next;  // next step index, -1 before fd_begin_shot
};

namespace fdh {

fd_status check_shot(const fd_model *m, const fd_shot *s);
int64_t nrec_of(const fd_shot *s);
// Step arguments for a shot.  On a z-slab the global source plane and
// receiver rows are made local: a source off the slab's planes gets plane
// -1 (never matched), and only the receiver rows on the slab's planes stay,
// *rec_skip being the entries of the full trace row that precede them (-1:
// none on the slab).
fdk::StepArgs base_args(const fd_model *m, const fd_shot *s, int64_t *rec_skip = nullptr);
// Element offset of the source cell in a stored level.
size_t src_offset(const Layout &L, const fd_shot *s);

}  // namespace fdh
