// C ABI of the finite-difference engine: validation, buffer layouts, handle
// management and kernel dispatch.  Declarations and semantics: include/fd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fd.h"
#include "fd_launch.hpp"

using fdk::StepArgs;

namespace {

thread_local std::string g_err;

fd_status fail(fd_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

fd_status ok()
{
    g_err.clear();
    return FD_OK;
}

fd_status hip_fail(hipError_t e, const char *what)
{
    return fail(FD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

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

bool is_slab(const Layout &L) { return L.nzg != L.nz || L.z0 != 0 || L.ghost != 0; }

Layout make_layout(const fd_grid &g)
{
    Layout L{};
    L.ndim = g.ndim;
    L.storage = g.storage;
    L.c_storage = g.c_storage;
    L.nz = g.nz;
    L.ny = g.ny;
    L.nx = g.nx;
    L.px = (int32_t)((g.nx + 63) / 64 * 64);
    L.npad = (size_t)g.nz * (size_t)g.ny * (size_t)L.px;
    L.elem = g.storage == FD_F32 ? 4 : 2;
    const bool slab = g.slab_nz_global > 0;
    L.z0 = slab ? g.slab_z0 : 0;
    L.nzg = slab ? g.slab_nz_global : g.nz;
    L.ghost = slab ? (size_t)kGhost * (size_t)g.ny * (size_t)L.px * L.elem : 0;
    L.field = align_up(L.npad * L.elem + 2 * L.ghost);
    L.f32field = align_up(L.npad * 4);
    L.cfield = g.c_storage == FD_C_FIXED16 ? align_up(L.npad * 2) : L.f32field;
    L.c_off = 0;
    L.gz_off = L.c_off + L.cfield;
    L.gy_off = L.gz_off + align_up((size_t)g.nz * 4);
    L.gx_off = L.gy_off + align_up((size_t)g.ny * 4);
    L.scratch_off = L.gx_off + align_up((size_t)g.nx * 4);
    L.model_bytes = L.scratch_off + kAlign;
    L.meta_off = 2 * L.field;
    L.state_bytes = L.meta_off + align_up(fdk::kMetaWords * 4);
    return L;
}

size_t ckpt_slot_bytes(const Layout &L) { return 2 * L.field; }

int64_t n_ckpt(int64_t nt, int32_t every) { return (nt + every - 1) / every; }

size_t adjoint_work_bytes(const Layout &L, int32_t every)
{
    // recompute state (2) + history fields (every) + adjoint fields (2) + FP64 sum
    return 2 * L.f32field + (size_t)every * L.f32field + 2 * L.f32field +
           align_up(L.npad * 8);
}

fd_status check_grid(const fd_grid *g)
{
    if (!g) return fail(FD_ERR_INVALID_ARG, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(FD_ERR_INVALID_ARG, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->nz < 1 || g->ny < 1 || g->nx < 1 || g->nz > kMaxDim || g->ny > kMaxDim || g->nx > kMaxDim)
        return fail(FD_ERR_INVALID_ARG, "grid sizes must be in [1, 2^30] (nz=%lld ny=%lld nx=%lld)",
                    (long long)g->nz, (long long)g->ny, (long long)g->nx);
    if (g->ndim == 2 && g->ny != 1) return fail(FD_ERR_INVALID_ARG, "2D grids need ny == 1");
    if (!(g->dh > 0.0) || !std::isfinite(g->dh)) return fail(FD_ERR_INVALID_ARG, "dh must be > 0");
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return fail(FD_ERR_INVALID_ARG, "dt must be > 0");
    if (g->radius < 1) return fail(FD_ERR_INVALID_ARG, "radius must be >= 1");
    if (g->radius != 4) return fail(FD_ERR_UNSUPPORTED, "only radius 4 (8th order) is built");
    if (g->bc == FD_BC_PERIODIC) return fail(FD_ERR_UNSUPPORTED, "periodic edges are not built");
    if (g->bc != FD_BC_ZERO) return fail(FD_ERR_INVALID_ARG, "unknown boundary kind %d", g->bc);
    if (g->sponge_width < 0) return fail(FD_ERR_INVALID_ARG, "sponge_width must be >= 0");
    if (g->sponge_faces & ~0x3Fu) return fail(FD_ERR_INVALID_ARG, "unknown sponge face bits");
    if (!std::isfinite(g->sponge_alpha)) return fail(FD_ERR_INVALID_ARG, "sponge_alpha must be finite");
    if (g->storage != FD_F32 && g->storage != FD_F16 && g->storage != FD_BF16)
        return fail(FD_ERR_INVALID_ARG, "unknown storage kind %d", g->storage);
    if (g->c_storage != FD_C_F32 && g->c_storage != FD_C_FIXED16)
        return fail(FD_ERR_INVALID_ARG, "unknown c storage kind %d", g->c_storage);
    if (g->c_storage == FD_C_FIXED16 && g->storage == FD_F32)
        return fail(FD_ERR_UNSUPPORTED, "16-bit c is built for 16-bit fields only");
    if (g->slab_nz_global < 0 || g->slab_z0 < 0)
        return fail(FD_ERR_INVALID_ARG, "slab_z0 and slab_nz_global must be >= 0");
    if (g->slab_nz_global == 0 && g->slab_z0 != 0)
        return fail(FD_ERR_INVALID_ARG, "slab_z0 needs slab_nz_global > 0");
    if (g->slab_nz_global > 0) {
        if (g->ndim != 3) return fail(FD_ERR_UNSUPPORTED, "z-slabs are built for 3D grids");
        if (g->storage != FD_F32 || g->c_storage != FD_C_F32)
            return fail(FD_ERR_UNSUPPORTED, "z-slabs are built for FP32 fields and FP32 c");
        if (g->nz < kGhost) return fail(FD_ERR_INVALID_ARG, "a z-slab needs at least %d planes", kGhost);
        if (g->slab_nz_global > kMaxDim || g->slab_z0 + g->nz > g->slab_nz_global)
            return fail(FD_ERR_INVALID_ARG, "slab planes [%lld, %lld) leave the %lld-plane grid",
                        (long long)g->slab_z0, (long long)(g->slab_z0 + g->nz),
                        (long long)g->slab_nz_global);
    }
    const double cells = (double)(g->nz + 2 * kGhost) * (double)g->ny * (double)((g->nx + 63) / 64 * 64);
    if (cells > 4.0e9) return fail(FD_ERR_INVALID_ARG, "grid too large");
    // the 16-bit 3D kernels address a plane with 32-bit byte offsets
    if ((double)g->ny * (double)((g->nx + 63) / 64 * 64) >= 1073741824.0)
        return fail(FD_ERR_INVALID_ARG, "an x-y plane must hold fewer than 2^30 cells");
    return FD_OK;
}

}  // namespace

struct fd_model {
    fd_grid grid;
    Layout L;
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

namespace {

fd_status check_shot(const fd_model *m, const fd_shot *s)
{
    if (!s) return fail(FD_ERR_INVALID_ARG, "shot is NULL");
    const Layout &L = m->L;
    if (s->nt < 1) return fail(FD_ERR_INVALID_ARG, "shot nt must be >= 1");
    if (!s->wavelet) return fail(FD_ERR_INVALID_ARG, "shot wavelet is NULL");
    if (s->src_z < 0 || s->src_z >= L.nzg || s->src_y < 0 || s->src_y >= L.ny || s->src_x < 0 ||
        s->src_x >= L.nx)
        return fail(FD_ERR_INVALID_ARG, "source cell (%lld, %lld, %lld) outside the grid",
                    (long long)s->src_z, (long long)s->src_y, (long long)s->src_x);
    const fd_receivers &r = s->rec;
    const int64_t nrec = r.nz * r.ny * r.nx;
    if (r.nz < 0 || r.ny < 0 || r.nx < 0) return fail(FD_ERR_INVALID_ARG, "negative receiver counts");
    if (nrec == 0) {
        if (r.nz || r.ny || r.nx) return fail(FD_ERR_INVALID_ARG, "receiver counts must be all zero or all positive");
        return FD_OK;
    }
    if (nrec > ((int64_t)1 << 30)) return fail(FD_ERR_INVALID_ARG, "too many receivers");
    if (r.dz < 1 || r.dy < 1 || r.dx < 1) return fail(FD_ERR_INVALID_ARG, "receiver strides must be >= 1");
    if (r.z0 < 0 || r.y0 < 0 || r.x0 < 0 || r.z0 + (r.nz - 1) * r.dz >= L.nzg ||
        r.y0 + (r.ny - 1) * r.dy >= L.ny || r.x0 + (r.nx - 1) * r.dx >= L.nx)
        return fail(FD_ERR_INVALID_ARG, "receiver array leaves the grid");
    return FD_OK;
}

int64_t nrec_of(const fd_shot *s) { return s->rec.nz * s->rec.ny * s->rec.nx; }

// Step arguments for a shot.  On a z-slab the global source plane and
// receiver rows are made local: a source off the slab's planes gets plane
// -1 (never matched), and only the receiver rows on the slab's planes stay,
// *rec_skip being the entries of the full trace row that precede them.
StepArgs base_args(const fd_model *m, const fd_shot *s, int64_t *rec_skip = nullptr)
{
    StepArgs a{};
    const Layout &L = m->L;
    a.c = m->c;
    a.c16 = m->c16;
    a.c16_scale = m->c16_scale;
    a.c16_inv = m->c16_inv;
    a.gz = m->gz;
    a.gy = m->gy;
    a.gx = m->gx;
    a.nz = (int32_t)L.nz;
    a.ny = (int32_t)L.ny;
    a.nx = (int32_t)L.nx;
    a.px = L.px;
    a.amp = m->amp;
    if (s) {
        const int64_t lz = s->src_z - L.z0;
        a.sz = (lz >= 0 && lz < L.nz) ? (int32_t)lz : -1;
        a.sy = (int32_t)s->src_y;
        a.sx = (int32_t)s->src_x;
        a.wavelet = s->wavelet;
        a.nt = s->nt;
        const fd_receivers &r = s->rec;
        // receiver rows i in [i0, i1) lie on planes [z0, z0 + nz)
        int64_t i0 = 0, i1 = r.nz;
        if (nrec_of(s) > 0 && is_slab(L)) {
            i0 = std::max<int64_t>(0, (L.z0 - r.z0 + r.dz - 1) / r.dz);
            const int64_t zl = L.z0 + L.nz - 1 - r.z0;  // the slab's last plane, from row 0
            i1 = zl < 0 ? 0 : std::min<int64_t>(r.nz, zl / r.dz + 1);
        }
        if (nrec_of(s) > 0 && i1 > i0) {
            a.rec = fdk::RecBox{(int32_t)(r.z0 + i0 * r.dz - L.z0), (int32_t)r.y0, (int32_t)r.x0,
                                (int32_t)(i1 - i0), (int32_t)r.ny, (int32_t)r.nx, (int32_t)r.dz,
                                (int32_t)r.dy, (int32_t)r.dx};
            if (rec_skip) *rec_skip = i0 * r.ny * r.nx;
        } else {
            a.rec = fdk::RecBox{0, 0, 0, 0, 0, 0, 1, 1, 1};
            if (rec_skip) *rec_skip = -1;
        }
    }
    return a;
}

size_t src_offset(const Layout &L, const fd_shot *s)
{
    return ((size_t)s->src_z * (size_t)L.ny + (size_t)s->src_y) * (size_t)L.px + (size_t)s->src_x;
}

fd_status do_begin(const fd_model *m, fd_state *st, const fd_shot *s, hipStream_t stream)
{
    const Layout &L = m->L;
    hipError_t e = fdk::launch_fill_u32(st->base, L.state_bytes / 4, 0u, stream);
    if (e != hipSuccess) return hip_fail(e, "fd_begin_shot fill");
    // a z-slab adds the source only on its own planes
    if (s->src_z >= L.z0 && s->src_z < L.z0 + L.nz) {
        fd_shot local = *s;
        local.src_z -= L.z0;
        e = fdk::launch_begin(L.storage, st->buf[0], (int64_t)src_offset(L, &local), m->amp,
                              s->wavelet, st->meta, stream);
        if (e != hipSuccess) return hip_fail(e, "fd_begin_shot");
    }
    st->next = 0;
    return FD_OK;
}

fd_status do_step(const fd_model *m, fd_state *st, const fd_shot *s, int64_t n, float *trace_row,
                  hipStream_t stream)
{
    int64_t skip = 0;
    StepArgs a = base_args(m, s, &skip);
    a.cur = st->buf[n & 1];
    a.prev = st->buf[(n + 1) & 1];
    a.n = n;
    a.trace_row = (nrec_of(s) > 0 && trace_row && skip >= 0) ? trace_row + skip : nullptr;
    a.meta = st->meta;
    a.zghost = is_slab(m->L) ? (int16_t)kGhost : (int16_t)0;
    hipError_t e = fdk::launch_step(a, m->L.ndim, m->L.storage, fdk::kFwd, stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    st->next = n + 1;
    return FD_OK;
}

}  // namespace

extern "C" {

const char *fd_last_error(void) { return g_err.c_str(); }

const char *fd_version(void) { return "fd-mi355x 0.1 (gfx950, radius 4)"; }

fd_status fd_query_bytes(const fd_grid *grid, int64_t nt, int32_t ckpt_every, fd_sizes *out)
{
    fd_status st = check_grid(grid);
    if (st != FD_OK) return st;
    if (!out) return fail(FD_ERR_INVALID_ARG, "out is NULL");
    if (nt < 0 || ckpt_every < 0) return fail(FD_ERR_INVALID_ARG, "nt and ckpt_every must be >= 0");
    const Layout L = make_layout(*grid);
    out->model = L.model_bytes;
    out->state = L.state_bytes;
    const bool whole = !is_slab(L);  // slabs step one call at a time only
    out->checkpoints = (whole && nt > 0 && ckpt_every > 0) ? (size_t)n_ckpt(nt, ckpt_every) * ckpt_slot_bytes(L) : 0;
    out->adjoint_work = (whole && ckpt_every > 0) ? adjoint_work_bytes(L, ckpt_every) : 0;
    out->routines_work = whole ? (size_t)L.ndim * L.f32field : 0;
    return ok();
}

fd_status fd_create_model(const fd_grid *grid, const float *velocity, void *model_buf,
                          size_t model_bytes, void *stream, fd_model **out)
{
    fd_status st = check_grid(grid);
    if (st != FD_OK) return st;
    if (!velocity || !model_buf || !out) return fail(FD_ERR_INVALID_ARG, "NULL velocity, buffer or out");
    const Layout L = make_layout(*grid);
    if (model_bytes < L.model_bytes)
        return fail(FD_ERR_INVALID_ARG, "model buffer too small (%zu < %zu bytes)", model_bytes, L.model_bytes);
    if ((uintptr_t)model_buf % kAlign) return fail(FD_ERR_INVALID_ARG, "model buffer must be 256-byte aligned");

    fd_model *m = new (std::nothrow) fd_model;
    if (!m) return fail(FD_ERR_OUT_OF_MEMORY, "host allocation failed");
    m->grid = *grid;
    if (m->grid.sponge_width > 0 && !(m->grid.sponge_alpha > 0.0))
        m->grid.sponge_alpha = 0.3 / m->grid.sponge_width;
    m->L = L;
    char *base = (char *)model_buf;
    const bool fixed16 = L.c_storage == FD_C_FIXED16;
    m->c = fixed16 ? nullptr : (float *)(base + L.c_off);
    m->c16 = fixed16 ? (uint16_t *)(base + L.c_off) : nullptr;
    m->c16_scale = 1.0f;
    m->c16_inv = 1.0f;
    m->gz = (float *)(base + L.gz_off);
    m->gy = (float *)(base + L.gy_off);
    m->gx = (float *)(base + L.gx_off);
    m->scratch = (uint32_t *)(base + L.scratch_off);
    m->amp = (float)(grid->dt * grid->dt / std::pow(grid->dh, (double)grid->ndim));

    // Damping profiles g(i) = exp(-(alpha d)^2), FP64 on the host, stored FP32.
    const double alpha = m->grid.sponge_alpha;
    const int32_t W = m->grid.sponge_width;
    const uint32_t f = m->grid.sponge_faces;
    auto profile = [&](int64_t n, bool lo, bool hi) {
        std::vector<float> g((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            double d = 0.0;
            if (W > 0) {
                if (lo && (double)(W - i) > d) d = (double)(W - i);
                if (hi && (double)(i - (n - 1 - W)) > d) d = (double)(i - (n - 1 - W));
            }
            g[(size_t)i] = (float)std::exp(-(alpha * d) * (alpha * d));
        }
        return g;
    };
    // a z-slab takes its planes' factors from the whole grid's profile
    const std::vector<float> gzg = profile(L.nzg, f & FD_FACE_ZLO, f & FD_FACE_ZHI);
    const std::vector<float> gz(gzg.begin() + L.z0, gzg.begin() + L.z0 + L.nz);
    const std::vector<float> gy = grid->ndim == 3 ? profile(L.ny, f & FD_FACE_YLO, f & FD_FACE_YHI)
                                                  : std::vector<float>(1, 1.0f);
    const std::vector<float> gx = profile(L.nx, f & FD_FACE_XLO, f & FD_FACE_XHI);

    hipStream_t s = (hipStream_t)stream;
    uint32_t host_scratch[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(m->gz, gz.data(), gz.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(m->gy, gy.data(), gy.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(m->gx, gx.data(), gx.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = fdk::launch_fill_u32((uint32_t *)(base + L.c_off), L.cfield / 4, 0u, s);
    if (e == hipSuccess) e = fdk::launch_fill_u32(m->scratch, 2, 0u, s);
    // FP32 c, or (16-bit c) only the velocity range: the fixed-point scale
    // depends on the largest c
    if (e == hipSuccess)
        e = fdk::launch_model_c(velocity, m->c, L.nz * L.ny, (int32_t)L.nx, L.px,
                                grid->dt / grid->dh, m->scratch, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host_scratch, m->scratch, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "fd_create_model");
    }
    if (host_scratch[1]) {
        delete m;
        return fail(FD_ERR_INVALID_ARG, "velocity must be positive and finite everywhere");
    }
    float vmax;
    std::memcpy(&vmax, &host_scratch[0], 4);
    const double cfl = (double)vmax * grid->dt / grid->dh;
    const double lhs = cfl * cfl * grid->ndim * kSymbolMax;
    if (!(lhs <= 4.0)) {
        delete m;
        return fail(FD_ERR_UNSTABLE,
                    "unstable: vmax*dt/dh = %.6f exceeds the %dD limit %.6f", cfl, grid->ndim,
                    std::sqrt(4.0 / (grid->ndim * kSymbolMax)));
    }
    if (fixed16) {
        // the largest c, rounded to FP32 exactly as the kernels round every c
        // (the product is monotone in v), fixes e = floor(log2 cmax) + 1
        const double qq = (double)vmax * (grid->dt / grid->dh);
        const float cmax = (float)(qq * qq);
        int ex = 0;
        std::frexp(cmax, &ex);  // cmax = f 2^ex with f in [0.5, 1)
        // a cmax within half a code of 2^ex would round to code 2^16: the
        // next binade keeps every code in 16 bits and the error <= 2^(e-17)
        if (std::nearbyint(std::ldexp((double)cmax, 16 - ex)) > 65535.0) ex += 1;
        m->c16_scale = std::ldexp(1.0f, ex - 16);
        m->c16_inv = std::ldexp(1.0f, 16 - ex);
        e = fdk::launch_model_c16(velocity, m->c16, L.nz * L.ny, (int32_t)L.nx, L.px,
                                  grid->dt / grid->dh, std::ldexp(1.0f, 16 - ex), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete m;
            return hip_fail(e, "fd_create_model");
        }
    }
    *out = m;
    return ok();
}

fd_status fd_destroy_model(fd_model *model)
{
    delete model;
    return ok();
}

fd_status fd_create_state(const fd_model *model, void *state_buf, size_t state_bytes, fd_state **out)
{
    if (!model || !state_buf || !out) return fail(FD_ERR_INVALID_ARG, "NULL model, buffer or out");
    if (state_bytes < model->L.state_bytes)
        return fail(FD_ERR_INVALID_ARG, "state buffer too small (%zu < %zu bytes)", state_bytes,
                    model->L.state_bytes);
    if ((uintptr_t)state_buf % kAlign) return fail(FD_ERR_INVALID_ARG, "state buffer must be 256-byte aligned");
    fd_state *st = new (std::nothrow) fd_state;
    if (!st) return fail(FD_ERR_OUT_OF_MEMORY, "host allocation failed");
    st->m = model;
    st->base = state_buf;
    st->buf[0] = (char *)state_buf + model->L.ghost;
    st->buf[1] = (char *)state_buf + model->L.field + model->L.ghost;
    st->meta = (int32_t *)((char *)state_buf + model->L.meta_off);
    st->next = -1;
    *out = st;
    return ok();
}

fd_status fd_destroy_state(fd_state *state)
{
    delete state;
    return ok();
}

fd_status fd_begin_shot(const fd_model *model, fd_state *state, const fd_shot *shot, void *stream)
{
    if (!model || !state) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    st = do_begin(model, state, shot, (hipStream_t)stream);
    return st == FD_OK ? ok() : st;
}

fd_status fd_step(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                  float *trace_row, void *stream)
{
    if (!model || !state) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    if (n != state->next) return fail(FD_ERR_INVALID_ARG, "step %lld requested, next step is %lld",
                                      (long long)n, (long long)state->next);
    if (n >= shot->nt) return fail(FD_ERR_INVALID_ARG, "step %lld beyond the shot's %lld steps",
                                   (long long)n, (long long)shot->nt);
    st = do_step(model, state, shot, n, trace_row, (hipStream_t)stream);
    return st == FD_OK ? ok() : st;
}

fd_status fd_run_shot(const fd_model *model, fd_state *state, const fd_shot *shot, float *traces,
                      void *ckpt, size_t ckpt_bytes, int32_t ckpt_every, void *stream)
{
    if (!model || !state) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    const Layout &L = model->L;
    if (is_slab(L)) return fail(FD_ERR_UNSUPPORTED, "a z-slab steps with fd_step and fd_slab_exchange");
    if (ckpt) {
        if (ckpt_every < 1) return fail(FD_ERR_INVALID_ARG, "ckpt_every must be >= 1");
        const size_t need = (size_t)n_ckpt(shot->nt, ckpt_every) * ckpt_slot_bytes(L);
        if (ckpt_bytes < need)
            return fail(FD_ERR_INVALID_ARG, "checkpoint buffer too small (%zu < %zu bytes)", ckpt_bytes, need);
        if ((uintptr_t)ckpt % kAlign) return fail(FD_ERR_INVALID_ARG, "checkpoint buffer must be 256-byte aligned");
    }
    hipStream_t s = (hipStream_t)stream;
    st = do_begin(model, state, shot, s);
    if (st != FD_OK) return st;
    const int64_t nrec = nrec_of(shot);
    for (int64_t n = 0; n < shot->nt; ++n) {
        if (ckpt && n % ckpt_every == 0) {
            char *slot = (char *)ckpt + (size_t)(n / ckpt_every) * ckpt_slot_bytes(L);
            hipError_t e = hipMemcpyAsync(slot, state->buf[n & 1], L.field, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(slot + L.field, state->buf[(n + 1) & 1], L.field,
                                   hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
        }
        st = do_step(model, state, shot, n, traces ? traces + (size_t)n * (size_t)nrec : nullptr, s);
        if (st != FD_OK) return st;
    }
    return ok();
}

fd_status fd_run_shots(const fd_model *model, fd_state *const *states, const fd_shot *const *shots,
                       int32_t count, float *const *traces, void *const *ckpt, size_t ckpt_bytes,
                       int32_t ckpt_every, void *stream)
{
    if (!model) return fail(FD_ERR_INVALID_ARG, "NULL model");
    if (count < 1 || count > 4096) return fail(FD_ERR_INVALID_ARG, "count must be in [1, 4096]");
    if (!states || !shots) return fail(FD_ERR_INVALID_ARG, "NULL states or shots array");
    const Layout &L = model->L;
    if (is_slab(L)) return fail(FD_ERR_UNSUPPORTED, "a z-slab steps with fd_step and fd_slab_exchange");
    for (int32_t i = 0; i < count; ++i) {
        if (!states[i] || states[i]->m != model) return fail(FD_ERR_INVALID_ARG, "shot %d: state missing or of another model", i);
        fd_status st = check_shot(model, shots[i]);
        if (st != FD_OK) return st;
        if (shots[i]->nt != shots[0]->nt) return fail(FD_ERR_INVALID_ARG, "shot %d: all shots must share nt", i);
        for (int32_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return fail(FD_ERR_INVALID_ARG, "shot %d repeats a state", i);
        if (ckpt && ckpt[i]) {
            if (ckpt_every < 1) return fail(FD_ERR_INVALID_ARG, "ckpt_every must be >= 1");
            const size_t need = (size_t)n_ckpt(shots[i]->nt, ckpt_every) * ckpt_slot_bytes(L);
            if (ckpt_bytes < need)
                return fail(FD_ERR_INVALID_ARG, "checkpoint buffer too small (%zu < %zu bytes)", ckpt_bytes, need);
            if ((uintptr_t)ckpt[i] % kAlign) return fail(FD_ERR_INVALID_ARG, "checkpoint buffer must be 256-byte aligned");
        }
    }
    hipStream_t s = (hipStream_t)stream;
    const bool batched = L.ndim == 2 && L.storage == FD_F32 && count > 1;
    if (!batched) {
        for (int32_t i = 0; i < count; ++i) {
            fd_status st = fd_run_shot(model, states[i], shots[i], traces ? traces[i] : nullptr,
                                       ckpt ? ckpt[i] : nullptr, ckpt_bytes, ckpt_every, stream);
            if (st != FD_OK) return st;
        }
        return ok();
    }
    for (int32_t i = 0; i < count; ++i) {
        fd_status st = do_begin(model, states[i], shots[i], s);
        if (st != FD_OK) return st;
    }
    const int64_t nt = shots[0]->nt;
    for (int64_t n = 0; n < nt; ++n) {
        for (int32_t i0 = 0; i0 < count; i0 += FD_BATCH_MAX) {
            fdk::Batch2D b;
            b.count = 0;
            for (int32_t i = i0; i < std::min<int32_t>(count, i0 + FD_BATCH_MAX); ++i) {
                fd_state *st = states[i];
                if (ckpt && ckpt[i] && n % ckpt_every == 0) {
                    char *slot = (char *)ckpt[i] + (size_t)(n / ckpt_every) * ckpt_slot_bytes(L);
                    hipError_t e = hipMemcpyAsync(slot, st->buf[n & 1], L.field, hipMemcpyDeviceToDevice, s);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(slot + L.field, st->buf[(n + 1) & 1], L.field, hipMemcpyDeviceToDevice, s);
                    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
                }
                StepArgs a = base_args(model, shots[i]);
                a.cur = st->buf[n & 1];
                a.prev = st->buf[(n + 1) & 1];
                a.n = n;
                const int64_t nrec = nrec_of(shots[i]);
                a.trace_row = (traces && traces[i] && nrec > 0) ? traces[i] + (size_t)n * (size_t)nrec : nullptr;
                a.meta = st->meta;
                b.it[b.count++] = a;
            }
            hipError_t e = fdk::launch_step_batch2d(b, fdk::kFwd, s);
            if (e != hipSuccess) return hip_fail(e, "batched step launch");
        }
        for (int32_t i = 0; i < count; ++i) states[i]->next = n + 1;
    }
    return ok();
}

}  // extern "C"

namespace {

// Checkpointed backward pass shared by the gradient and the image, for
// `count` shots on one model: each segment is recomputed storing the
// history field of every step (L w^n for the gradient, w^n for the image),
// then the z-form adjoint field is stepped back through the segment
// accumulating sum_k z^k * hist^{k-1} in FP64, one sum per shot (acc[i],
// padded, inside work[i]).  In 2D FP32 every step of all shots is one
// launch of the batched kernel (groups of FD_BATCH_MAX shots); otherwise
// the shots' steps are launched one by one.  Per shot and cell the
// arithmetic is the same either way.
struct ShotIO {
    const fd_shot *shot;
    const float *adj;
    const void *ckpt;
    void *work;
};

fd_status backward_pass(const fd_model *model, const ShotIO *io, int32_t count, size_t ckpt_bytes,
                        int32_t ckpt_every, size_t work_bytes, bool image, hipStream_t s,
                        double **acc)
{
    const Layout &L = model->L;
    if (L.storage != FD_F32) return fail(FD_ERR_UNSUPPORTED, "the adjoint needs FP32 storage");
    if (ckpt_every < 1) return fail(FD_ERR_INVALID_ARG, "ckpt_every must be >= 1");
    if (count < 1) return fail(FD_ERR_INVALID_ARG, "count must be >= 1");
    for (int32_t i = 0; i < count; ++i) {
        fd_status st = check_shot(model, io[i].shot);
        if (st != FD_OK) return st;
        if (!io[i].adj || !io[i].ckpt || !io[i].work) return fail(FD_ERR_INVALID_ARG, "shot %d: NULL adj, ckpt or work", i);
        if (io[i].shot->nt != io[0].shot->nt) return fail(FD_ERR_INVALID_ARG, "shot %d: all shots must share nt", i);
        if ((uintptr_t)io[i].work % kAlign) return fail(FD_ERR_INVALID_ARG, "work buffer must be 256-byte aligned");
        for (int32_t j = 0; j < i; ++j)
            if (io[j].work == io[i].work) return fail(FD_ERR_INVALID_ARG, "shot %d repeats a work buffer", i);
    }
    const int64_t nt = io[0].shot->nt;
    const int64_t nseg = n_ckpt(nt, ckpt_every);
    if (ckpt_bytes < (size_t)nseg * ckpt_slot_bytes(L))
        return fail(FD_ERR_INVALID_ARG, "checkpoint buffer too small");
    if (work_bytes < adjoint_work_bytes(L, ckpt_every))
        return fail(FD_ERR_INVALID_ARG, "adjoint work buffer too small (%zu < %zu bytes)", work_bytes,
                    adjoint_work_bytes(L, ckpt_every));
    // work layout: recompute state (2), history (K), adjoint state (2), FP64 sum
    auto fw = [&](int32_t i, int64_t n) -> void * { return (char *)io[i].work + (size_t)(n & 1) * L.f32field; };
    auto hist = [&](int32_t i, int64_t slot) -> float * {
        return (float *)((char *)io[i].work + (2 + (size_t)slot) * L.f32field);
    };
    auto zf = [&](int32_t i, int64_t k) -> void * {
        return (char *)io[i].work + (2 + (size_t)ckpt_every + (size_t)(k & 1)) * L.f32field;
    };
    auto gsum = [&](int32_t i) -> double * {
        return (double *)((char *)io[i].work + (4 + (size_t)ckpt_every) * L.f32field);
    };
    const bool batched = L.ndim == 2 && count > 1;
    // one step of every shot: batched launches in 2D, one launch per shot otherwise
    auto launch_all = [&](auto make_args, int mode) -> hipError_t {
        if (!batched) {
            for (int32_t i = 0; i < count; ++i) {
                hipError_t e = fdk::launch_step(make_args(i), L.ndim, L.storage, mode, s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        for (int32_t i0 = 0; i0 < count; i0 += FD_BATCH_MAX) {
            fdk::Batch2D b;
            b.count = 0;
            for (int32_t i = i0; i < std::min<int32_t>(count, i0 + FD_BATCH_MAX); ++i) b.it[b.count++] = make_args(i);
            hipError_t e = fdk::launch_step_batch2d(b, mode, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };

    for (int32_t i = 0; i < count; ++i) {
        hipError_t e = fdk::launch_fill_u32(zf(i, 0), (2 * L.f32field + align_up(L.npad * 8)) / 4, 0u, s);
        if (e != hipSuccess) return hip_fail(e, "adjoint clear");
    }
    auto ckpt_slot = [&](int32_t i, int64_t seg) -> char * {
        return (char *)io[i].ckpt + (size_t)seg * ckpt_slot_bytes(L);
    };
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t n0 = seg * ckpt_every;
        const int64_t n1 = std::min<int64_t>(nt, n0 + ckpt_every);
        if (image) {
            // The image's history is the field itself: slot s holds w^(n0+s).
            // Slot 0 is the checkpoint's P; each recompute step reads its
            // Pold from the checkpoint or the slot before and writes the next
            // level into the next slot (out of place), a plain forward step.
            for (int32_t i = 0; i < count; ++i) {
                hipError_t e = hipMemcpyAsync(hist(i, 0), ckpt_slot(i, seg), L.field, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return hip_fail(e, "checkpoint restore");
            }
            for (int64_t n = n0; n + 1 < n1; ++n) {
                hipError_t e = launch_all(
                    [&](int32_t i) {
                        StepArgs a = base_args(model, io[i].shot);
                        a.cur = hist(i, n - n0);
                        a.prev = n == n0 ? (void *)(ckpt_slot(i, seg) + L.field) : (void *)hist(i, n - 1 - n0);
                        a.out = hist(i, n + 1 - n0);
                        a.n = n;
                        a.trace_row = nullptr;
                        return a;
                    },
                    fdk::kFwd);
                if (e != hipSuccess) return hip_fail(e, "recompute step");
            }
        } else {
            for (int32_t i = 0; i < count; ++i) {
                const char *slot = ckpt_slot(i, seg);
                hipError_t e = hipMemcpyAsync(fw(i, n0), slot, L.field, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess) e = hipMemcpyAsync(fw(i, n0 + 1), slot + L.field, L.field, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return hip_fail(e, "checkpoint restore");
            }
            for (int64_t n = n0; n < n1; ++n) {
                hipError_t e = launch_all(
                    [&](int32_t i) {
                        StepArgs a = base_args(model, io[i].shot);
                        a.cur = fw(i, n);
                        a.prev = fw(i, n + 1);
                        a.n = n;
                        a.trace_row = nullptr;
                        a.lap = hist(i, n - n0);
                        return a;
                    },
                    fdk::kFwdLap);
                if (e != hipSuccess) return hip_fail(e, "recompute step");
            }
        }
        // Adjoint steps k = n1 .. n0+1 in groups of three from the top of the
        // segment: the first two of a group leave their gradient terms to the
        // last, which adds all three (z^(k+2) is its prev and z^(k+1) its cur,
        // both read anyway), so g is read and written once per three steps.
        // A shorter last group (two or one steps) works the same way.  The
        // history of the segment is rebuilt by the next recompute, so groups
        // stay inside it.
        const int64_t m = n1 - n0;
        for (int64_t k = n1; k >= n0 + 1; --k) {
            const int64_t j = n1 - k;
            const int64_t size = std::min<int64_t>(3, m - j / 3 * 3);
            const int32_t gmode = j % 3 < size - 1 ? 1 : (size == 1 ? 0 : (int32_t)size);
            hipError_t e = launch_all(
                [&](int32_t i) {
                    StepArgs a = base_args(model, io[i].shot);
                    const int64_t nrec = nrec_of(io[i].shot);
                    a.cur = zf(i, k + 1);
                    a.prev = zf(i, k);
                    a.n = k;
                    a.nt = 0;  // no source in the adjoint recursion
                    a.lap = hist(i, k - 1 - n0);
                    a.lap2 = gmode >= 2 ? hist(i, k - n0) : nullptr;
                    a.lap3 = gmode == 3 ? hist(i, k + 1 - n0) : nullptr;
                    a.gmode = gmode;
                    a.resid_row = nrec > 0 ? io[i].adj + (size_t)(k - 1) * (size_t)nrec : nullptr;
                    a.g = gsum(i);
                    return a;
                },
                fdk::kAdj);
            if (e != hipSuccess) return hip_fail(e, "adjoint step");
        }
    }
    for (int32_t i = 0; i < count; ++i) acc[i] = gsum(i);
    return FD_OK;
}

}  // namespace

extern "C" {

fd_status fd_adjoint_gradient(const fd_model *model, const fd_shot *shot, const float *adj,
                              const void *ckpt, size_t ckpt_bytes, int32_t ckpt_every, void *work,
                              size_t work_bytes, double *grad_v, void *stream)
{
    return fd_adjoint_gradient_shots(model, &shot, 1, &adj, &ckpt, ckpt_bytes, ckpt_every, &work,
                                     work_bytes, grad_v, stream);
}

fd_status fd_rtm_image(const fd_model *model, const fd_shot *shot, const float *data,
                       const void *ckpt, size_t ckpt_bytes, int32_t ckpt_every, void *work,
                       size_t work_bytes, double *image, void *stream)
{
    return fd_rtm_image_shots(model, &shot, 1, &data, &ckpt, ckpt_bytes, ckpt_every, &work,
                              work_bytes, image, stream);
}

namespace {

fd_status backward_shots(const fd_model *model, const fd_shot *const *shots, int32_t count,
                         const float *const *adj, const void *const *ckpt, size_t ckpt_bytes,
                         int32_t ckpt_every, void *const *work, size_t work_bytes, double *out,
                         bool image, void *stream)
{
    if (!model) return fail(FD_ERR_INVALID_ARG, "NULL model");
    if (!out) return fail(FD_ERR_INVALID_ARG, image ? "NULL image" : "NULL grad_v");
    if (count < 1 || count > 4096) return fail(FD_ERR_INVALID_ARG, "count must be in [1, 4096]");
    if (!shots || !adj || !ckpt || !work) return fail(FD_ERR_INVALID_ARG, "NULL shots, adj, ckpt or work array");
    if (is_slab(model->L)) return fail(FD_ERR_UNSUPPORTED, "the adjoint and the image are not built for z-slabs");
    std::vector<ShotIO> io((size_t)count);
    for (int32_t i = 0; i < count; ++i) io[i] = ShotIO{shots[i], adj[i], ckpt[i], work[i]};
    hipStream_t s = (hipStream_t)stream;
    std::vector<double *> acc((size_t)count, nullptr);
    fd_status st = backward_pass(model, io.data(), count, ckpt_bytes, ckpt_every, work_bytes,
                                 image, s, acc.data());
    if (st != FD_OK) return st;
    const Layout &L = model->L;
    // shot after shot, so the FP64 sum has the order of one call per shot
    for (int32_t i = 0; i < count; ++i) {
        hipError_t e = image ? fdk::launch_image_finish(acc[i], out, L.nz * L.ny, (int32_t)L.nx, L.px, s)
                             : fdk::launch_grad_finish(acc[i], model->c, out, L.nz * L.ny, (int32_t)L.nx,
                                                       L.px, 2.0 * model->grid.dt / model->grid.dh, s);
        if (e != hipSuccess) return hip_fail(e, image ? "image finish" : "gradient finish");
    }
    return ok();
}

}  // namespace

fd_status fd_adjoint_gradient_shots(const fd_model *model, const fd_shot *const *shots,
                                    int32_t count, const float *const *adj,
                                    const void *const *ckpt, size_t ckpt_bytes, int32_t ckpt_every,
                                    void *const *work, size_t work_bytes, double *grad_v,
                                    void *stream)
{
    return backward_shots(model, shots, count, adj, ckpt, ckpt_bytes, ckpt_every, work, work_bytes,
                          grad_v, false, stream);
}

fd_status fd_rtm_image_shots(const fd_model *model, const fd_shot *const *shots, int32_t count,
                             const float *const *data, const void *const *ckpt, size_t ckpt_bytes,
                             int32_t ckpt_every, void *const *work, size_t work_bytes,
                             double *image, void *stream)
{
    return backward_shots(model, shots, count, data, ckpt, ckpt_bytes, ckpt_every, work, work_bytes,
                          image, true, stream);
}

fd_status fd_get_wavefield(const fd_state *state, int32_t which, float *out, void *stream)
{
    if (!state || !out) return fail(FD_ERR_INVALID_ARG, "NULL state or out");
    if (which != 0 && which != 1) return fail(FD_ERR_INVALID_ARG, "which must be 0 (P) or 1 (Pold)");
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    const Layout &L = state->m->L;
    const int64_t lvl = which == 0 ? state->next : state->next - 1;
    const void *buf = state->buf[lvl & 1];
    hipError_t e = fdk::launch_get_field(L.storage, buf, out, L.nz * L.ny, (int32_t)L.nx, L.px,
                                         state->meta, (int32_t)(lvl & 3), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fd_get_wavefield");
    return ok();
}

fd_status fd_set_wavefield(fd_state *state, int32_t which, const float *in, void *stream)
{
    if (!state || !in) return fail(FD_ERR_INVALID_ARG, "NULL state or in");
    if (which != 0 && which != 1) return fail(FD_ERR_INVALID_ARG, "which must be 0 (P) or 1 (Pold)");
    const Layout &L = state->m->L;
    hipStream_t s = (hipStream_t)stream;
    if (state->next < 0) {
        hipError_t e = fdk::launch_fill_u32(state->base, L.state_bytes / 4, 0u, s);
        if (e != hipSuccess) return hip_fail(e, "fd_set_wavefield clear");
        state->next = 0;
    }
    const int64_t lvl = which == 0 ? state->next : state->next - 1;
    hipError_t e = fdk::launch_set_field(L.storage, in, state->buf[lvl & 1], L.nz * L.ny,
                                         (int32_t)L.nx, L.px, state->meta, (int32_t)(lvl & 3), s);
    if (e != hipSuccess) return hip_fail(e, "fd_set_wavefield");
    return ok();
}

fd_status fd_slab_exchange(const fd_state *upper, const fd_state *lower, void *stream)
{
    if (!upper || !lower) return fail(FD_ERR_INVALID_ARG, "NULL state");
    if (upper == lower) return fail(FD_ERR_INVALID_ARG, "a slab cannot exchange with itself");
    const Layout &U = upper->m->L, &D = lower->m->L;
    if (!is_slab(U) || !is_slab(D)) return fail(FD_ERR_INVALID_ARG, "both states must be z-slabs");
    if (U.nzg != D.nzg || U.ny != D.ny || U.nx != D.nx || U.storage != D.storage)
        return fail(FD_ERR_INVALID_ARG, "the slabs belong to different grids");
    if (U.z0 + U.nz != D.z0)
        return fail(FD_ERR_INVALID_ARG, "upper's planes [%lld, %lld) do not end where lower's begin (%lld)",
                    (long long)U.z0, (long long)(U.z0 + U.nz), (long long)D.z0);
    if (upper->next < 0 || lower->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    if (upper->next != lower->next)
        return fail(FD_ERR_INVALID_ARG, "the slabs are at different steps (%lld, %lld)",
                    (long long)upper->next, (long long)lower->next);
    const size_t plane = (size_t)U.ny * (size_t)U.px * U.elem;
    const int64_t lvl = upper->next;  // P, the level the next step reads
    const char *u = (const char *)upper->buf[lvl & 1];
    const char *d = (const char *)lower->buf[lvl & 1];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync((char *)d - kGhost * plane, u + (size_t)(U.nz - kGhost) * plane,
                                  kGhost * plane, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)u + (size_t)U.nz * plane, d, kGhost * plane, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "fd_slab_exchange");
    return ok();
}

fd_status fd_step_routines(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                           float *trace_row, void *work, size_t work_bytes, void *stream)
{
    if (!model || !state) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    const Layout &L = model->L;
    if (L.storage != FD_F32) return fail(FD_ERR_UNSUPPORTED, "the routine-per-kernel step is built for FP32 fields only");
    if (is_slab(L)) return fail(FD_ERR_UNSUPPORTED, "the routine-per-kernel step is not built for z-slabs");
    if (!work) return fail(FD_ERR_INVALID_ARG, "work is NULL");
    if (work_bytes < (size_t)L.ndim * L.f32field)
        return fail(FD_ERR_INVALID_ARG, "work holds %zu bytes, %zu needed", work_bytes,
                    (size_t)L.ndim * L.f32field);
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    if (n != state->next) return fail(FD_ERR_INVALID_ARG, "step %lld requested, next step is %lld",
                                      (long long)n, (long long)state->next);
    if (n >= shot->nt) return fail(FD_ERR_INVALID_ARG, "step %lld beyond the shot's %lld steps",
                                   (long long)n, (long long)shot->nt);
    StepArgs a = base_args(model, shot);
    a.cur = state->buf[n & 1];
    a.prev = state->buf[(n + 1) & 1];
    a.n = n;
    a.trace_row = nrec_of(shot) > 0 ? trace_row : nullptr;
    char *w = (char *)work;
    float *dzz = (float *)w, *dxx = (float *)(w + L.f32field);
    float *dyy = L.ndim == 3 ? (float *)(w + 2 * L.f32field) : nullptr;
    hipError_t e = fdk::launch_routines(a, L.ndim, dzz, dxx, dyy, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "routine kernels launch");
    state->next = n + 1;
    return ok();
}

fd_status fd_step_batch(fd_batch_item *items, int32_t count, int32_t nsteps, void *stream)
{
    if (count < 0 || count > FD_BATCH_MAX) return fail(FD_ERR_INVALID_ARG, "count must be in [0, %d]", FD_BATCH_MAX);
    if (count > 0 && !items) return fail(FD_ERR_INVALID_ARG, "items is NULL");
    if (nsteps < 0) return fail(FD_ERR_INVALID_ARG, "nsteps must be >= 0");
    for (int32_t i = 0; i < count; ++i) {
        const fd_batch_item &it = items[i];
        if (!it.model || !it.state) return fail(FD_ERR_INVALID_ARG, "item %d: NULL model or state", i);
        if (it.state->m != it.model) return fail(FD_ERR_INVALID_ARG, "item %d: state of another model", i);
        if (it.model->L.ndim != 2 || it.model->L.storage != FD_F32 || is_slab(it.model->L))
            return fail(FD_ERR_UNSUPPORTED, "item %d: batching is built for 2D FP32 grids", i);
        fd_status st = check_shot(it.model, it.shot);
        if (st != FD_OK) return st;
        if (it.state->next < 0) return fail(FD_ERR_INVALID_ARG, "item %d: fd_begin_shot has not been called", i);
        if (it.n != it.state->next) return fail(FD_ERR_INVALID_ARG, "item %d: n is not the state's next step", i);
        for (int32_t j = 0; j < i; ++j)
            if (items[j].state == it.state) return fail(FD_ERR_INVALID_ARG, "item %d repeats a state", i);
    }
    hipStream_t s = (hipStream_t)stream;
    for (int32_t step = 0; step < nsteps; ++step) {
        fdk::Batch2D b;
        b.count = 0;
        int32_t which[FD_BATCH_MAX];
        for (int32_t i = 0; i < count; ++i) {
            fd_batch_item &it = items[i];
            if (it.n >= it.shot->nt) continue;
            StepArgs a = base_args(it.model, it.shot);
            a.cur = it.state->buf[it.n & 1];
            a.prev = it.state->buf[(it.n + 1) & 1];
            a.n = it.n;
            a.trace_row = (it.traces && nrec_of(it.shot) > 0)
                              ? it.traces + (size_t)it.n * (size_t)nrec_of(it.shot) : nullptr;
            a.meta = it.state->meta;
            b.it[b.count] = a;
            which[b.count] = i;
            ++b.count;
        }
        if (b.count == 0) break;
        hipError_t e = fdk::launch_step_batch2d(b, fdk::kFwd, s);
        if (e != hipSuccess) return hip_fail(e, "batched step launch");
        for (int32_t k = 0; k < b.count; ++k) {
            fd_batch_item &it = items[which[k]];
            it.n += 1;
            it.state->next = it.n;
        }
    }
    return ok();
}

}  // extern "C"
