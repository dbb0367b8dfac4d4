// Host back-end of the finite-difference engine (libfd_cpu.so): the C ABI of
// include/fd.h over host memory, OpenMP threads over blocks of rows and
// AVX2/AVX-512 vectors along x.  Semantics and the built subset:
// include/fd_cpu.h.
//
// A time step is the fused form of Listing 3's routines (Section 7):
// add_source, fd_pzz, fd_pxx (and y), fd_time and the level rotation in one
// pass over the fields, i.e. per cell
//   Pnew = G (2 P + c L P) - G^2 Pold      (written over Pold)
// then the receivers sample Pnew and the source of the next step is added to
// it (which is the addition Listing 3 makes to P at the start of that step).
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fd_cpu.h"
#include "fd_cpu_rows.hpp"

namespace fdcpu {
void step_rows_avx2(const Row *rows, int64_t count, int ndim);
void step_rows_avx512(const Row *rows, int64_t count, int ndim);
}  // namespace fdcpu

using fdcpu::Row;

namespace {

// ---- errors ---------------------------------------------------------------
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

fd_status unsupported(const char *what)
{
    return fail(FD_ERR_UNSUPPORTED, "%s is not built in the host back-end (libfd_cpu.so)", what);
}

// ---- row loops per instruction set -----------------------------------------
struct Scalar {
    using V = float;
    static constexpr int W = 1;
    static V ld(const float *p) { return *p; }
    static void st(float *p, V v) { *p = v; }
    static V set1(float a) { return a; }
    static V add(V a, V b) { return a + b; }
    static V sub(V a, V b) { return a - b; }
    static V mul(V a, V b) { return a * b; }
    static V fma(V a, V b, V c) { return std::fma(a, b, c); }
    static V neg(V a) { return -a; }
    static V keep(V v, int n) { return n > 0 ? v : 0.0f; }
};

void step_rows_scalar(const Row *rows, int64_t count, int ndim)
{
    if (ndim == 3)
        for (int64_t i = 0; i < count; ++i) fdcpu::step_row<Scalar, 3>(rows[i]);
    else
        for (int64_t i = 0; i < count; ++i) fdcpu::step_row<Scalar, 2>(rows[i]);
}

using RowsFn = void (*)(const Row *, int64_t, int);

struct Isa {
    const char *name;
    RowsFn fn;
    bool (*available)();
};

bool has_avx512() { return __builtin_cpu_supports("avx512f"); }
bool has_avx2() { return __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma"); }
bool has_scalar() { return true; }

const Isa kIsas[] = {{"avx512", fdcpu::step_rows_avx512, has_avx512},
                     {"avx2", fdcpu::step_rows_avx2, has_avx2},
                     {"scalar", step_rows_scalar, has_scalar}};

const Isa *best_isa()
{
    __builtin_cpu_init();
    for (const Isa &i : kIsas)
        if (i.available()) return &i;
    return &kIsas[2];
}

const Isa *g_isa = best_isa();
int32_t g_threads = 0;  // 0 until first use: the OpenMP default

int32_t threads()
{
    if (g_threads < 1) g_threads = std::max(1, omp_get_max_threads());
    return g_threads;
}

// ---- layout ----------------------------------------------------------------
constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }
constexpr int64_t kR = 4;        // stencil radius: frame planes and rows
constexpr int64_t kXoff = 16;    // zero cells left of each row (keeps rows 64-byte aligned)
constexpr int64_t kVec = 16;     // widest vector: rows are processed in multiples of it
constexpr double kSymbolMax = 4096.0 / 630.0;
constexpr int64_t kMaxDim = (int64_t)1 << 30;

struct Layout {
    int32_t ndim;
    int64_t nz, ny, nx;
    int64_t hy;       // frame rows on each y side (4 in 3D, 0 in 2D)
    int64_t pitch;    // floats per stored row
    int64_t ys, zs;   // row and plane strides (floats)
    size_t origin;    // float index of cell (0, 0, 0)
    size_t elems;     // floats per stored field
    size_t field;     // bytes per stored field, aligned
    size_t gz_off, gy_off, gx_off, model_bytes, state_bytes;
};

Layout make_layout(const fd_grid &g)
{
    Layout L{};
    L.ndim = g.ndim;
    L.nz = g.nz;
    L.ny = g.ny;
    L.nx = g.nx;
    L.hy = g.ndim == 3 ? kR : 0;
    L.pitch = kXoff + (g.nx + kVec - 1) / kVec * kVec + kVec;
    L.ys = L.pitch;
    L.zs = (g.ny + 2 * L.hy) * L.pitch;
    L.origin = (size_t)(kR * L.zs + L.hy * L.ys + kXoff);
    L.elems = (size_t)(g.nz + 2 * kR) * (size_t)L.zs;
    L.field = align_up(L.elems * 4);
    L.gz_off = L.field;  // the model buffer: c (a stored field), gz, gy, gx
    L.gy_off = L.gz_off + align_up((size_t)g.nz * 4);
    L.gx_off = L.gy_off + align_up((size_t)g.ny * 4);
    L.model_bytes = L.gx_off + align_up((size_t)L.pitch * 4);
    L.state_bytes = 2 * L.field;
    return L;
}

size_t index_of(const Layout &L, int64_t z, int64_t y, int64_t x)
{
    return L.origin + (size_t)(z * L.zs + y * L.ys + x);
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
    if (g->bc != FD_BC_ZERO && g->bc != FD_BC_PERIODIC)
        return fail(FD_ERR_INVALID_ARG, "unknown boundary kind %d", g->bc);
    if (g->sponge_width < 0) return fail(FD_ERR_INVALID_ARG, "sponge_width must be >= 0");
    if (g->sponge_faces & ~0x3Fu) return fail(FD_ERR_INVALID_ARG, "unknown sponge face bits");
    if (!std::isfinite(g->sponge_alpha)) return fail(FD_ERR_INVALID_ARG, "sponge_alpha must be finite");
    if (g->storage != FD_F32 && g->storage != FD_F16 && g->storage != FD_BF16)
        return fail(FD_ERR_INVALID_ARG, "unknown storage kind %d", g->storage);
    if (g->c_storage != FD_C_F32 && g->c_storage != FD_C_FIXED16)
        return fail(FD_ERR_INVALID_ARG, "unknown c storage kind %d", g->c_storage);
    if (g->slab_nz_global < 0 || g->slab_z0 < 0)
        return fail(FD_ERR_INVALID_ARG, "slab_z0 and slab_nz_global must be >= 0");
    if (g->slab_nz_global == 0 && g->slab_z0 != 0)
        return fail(FD_ERR_INVALID_ARG, "slab_z0 needs slab_nz_global > 0");
    const double cells = (double)(g->nz + 2 * kR) * (double)(g->ny + 2 * kR) *
                         (double)(g->nx + kXoff + 2 * kVec);
    if (cells > 4.0e9) return fail(FD_ERR_INVALID_ARG, "grid too large");
    // valid requests this back-end does not build
    if (g->radius != 4) return fail(FD_ERR_UNSUPPORTED, "only radius 4 (8th order) is built");
    if (g->bc == FD_BC_PERIODIC) return fail(FD_ERR_UNSUPPORTED, "periodic edges are not built");
    if (g->storage != FD_F32) return unsupported("16-bit field storage");
    if (g->c_storage != FD_C_F32) return unsupported("16-bit c");
    if (g->slab_nz_global > 0) return unsupported("a z-slab grid");
    return FD_OK;
}

}  // namespace

struct fd_model {
    fd_grid grid;
    Layout L;
    float *c;  // stored-field layout, frame and padding zero
    float *gz, *gy, *gx;
    float amp;  // dt^2 / dh^D
};

struct fd_state {
    const fd_model *m;
    float *buf[2];  // the two stored levels
    int64_t next;   // next step, -1 before fd_begin_shot
    uint32_t health;  // bit 2: a non-finite value entered the shot (as in fd.h)
};

namespace {

fd_status check_shot(const fd_model *m, const fd_shot *s)
{
    if (!s) return fail(FD_ERR_INVALID_ARG, "shot is NULL");
    const Layout &L = m->L;
    if (s->nt < 1) return fail(FD_ERR_INVALID_ARG, "shot nt must be >= 1");
    if (!s->wavelet) return fail(FD_ERR_INVALID_ARG, "shot wavelet is NULL");
    if (s->src_z < 0 || s->src_z >= L.nz || s->src_y < 0 || s->src_y >= L.ny || s->src_x < 0 ||
        s->src_x >= L.nx)
        return fail(FD_ERR_INVALID_ARG, "source cell (%lld, %lld, %lld) outside the grid",
                    (long long)s->src_z, (long long)s->src_y, (long long)s->src_x);
    const fd_receivers &r = s->rec;
    if (r.nz < 0 || r.ny < 0 || r.nx < 0) return fail(FD_ERR_INVALID_ARG, "negative receiver counts");
    if (r.nz == 0 || r.ny == 0 || r.nx == 0) {
        if (r.nz || r.ny || r.nx) return fail(FD_ERR_INVALID_ARG, "receiver counts must be all zero or all positive");
        return FD_OK;
    }
    if ((double)r.nz * (double)r.ny * (double)r.nx > (double)((int64_t)1 << 30))
        return fail(FD_ERR_INVALID_ARG, "too many receivers");
    if (r.dz < 1 || r.dy < 1 || r.dx < 1) return fail(FD_ERR_INVALID_ARG, "receiver strides must be >= 1");
    // the array's last cell along an axis of n cells, tested by division (no
    // overflow for any int64 input): x0 + (cnt - 1) d <= n - 1
    auto inside = [](int64_t x0, int64_t cnt, int64_t d, int64_t n) {
        return x0 >= 0 && x0 < n && (cnt - 1) <= (n - 1 - x0) / d;
    };
    if (!inside(r.z0, r.nz, r.dz, L.nz) || !inside(r.y0, r.ny, r.dy, L.ny) || !inside(r.x0, r.nx, r.dx, L.nx))
        return fail(FD_ERR_INVALID_ARG, "receiver array leaves the grid");
    return FD_OK;
}

int64_t nrec_of(const fd_shot *s) { return s->rec.nz * s->rec.ny * s->rec.nx; }

// Blocks of rows that the threads share out in every step: a task is the
// rows [y0, y1) of the planes [z0, z1) (2D: rows [z0, z1) of the one
// plane).  In 3D a task streams down its planes, so the 9 planes of the z
// stencil stay cached for a block of y rows; the block height keeps those
// planes within about 768 KiB.  Tasks are numbered plane-block-major and
// handed out statically, so each thread touches the same memory in every
// step (and first touched it when the state was cleared).
struct Tasks {
    int64_t by, nyb, bz, nzb;
    int64_t count() const { return nyb * nzb; }
};

Tasks plan(const Layout &L, int32_t T)
{
    Tasks t{};
    if (L.ndim == 3) {
        const int64_t row_bytes = L.pitch * 4;
        int64_t by = (768 * 1024) / (9 * row_bytes) - 2 * kR;
        by = std::max<int64_t>(8, std::min<int64_t>(by, 64));
        t.by = std::min<int64_t>(by, L.ny);
        t.nyb = (L.ny + t.by - 1) / t.by;
        int64_t nzb = std::max<int64_t>(1, (2 * T + t.nyb - 1) / t.nyb);
        nzb = std::min<int64_t>(nzb, std::max<int64_t>(1, L.nz / 8));
        t.bz = (L.nz + nzb - 1) / nzb;
    } else {
        t.by = 1;
        t.nyb = 1;
        const int64_t nzb = std::min<int64_t>(L.nz, 4 * (int64_t)T);
        t.bz = (L.nz + nzb - 1) / nzb;
    }
    t.nzb = (L.nz + t.bz - 1) / t.bz;
    return t;
}

struct StepIO {
    const float *cur;
    float *prev;       // Pold in, Pnew out
    float *trace_row;  // nrec floats or null
    float inj;         // source amplitude of step n+1 (0: none)
};

// The rows of task `t` for one step, then their receivers and the source.
void run_task(const fd_model *m, const fd_shot *s, const StepIO &io, const Tasks &tk, int64_t t)
{
    const Layout &L = m->L;
    const int64_t zb = t / tk.nyb, yb = t % tk.nyb;
    const int64_t z0 = zb * tk.bz, z1 = std::min<int64_t>(L.nz, z0 + tk.bz);
    const int64_t y0 = L.ndim == 3 ? yb * tk.by : 0;
    const int64_t y1 = L.ndim == 3 ? std::min<int64_t>(L.ny, y0 + tk.by) : 1;
    const fd_receivers &r = s->rec;
    const bool has_rec = io.trace_row != nullptr && nrec_of(s) > 0;
    for (int64_t z = z0; z < z1; ++z) {
        for (int64_t y = y0; y < y1; ++y) {
            const size_t i0 = index_of(L, z, y, 0);
            Row row;
            row.P = io.cur + i0;
            row.Q = io.prev + i0;
            row.c = m->c + i0;
            row.gx = m->gx;
            row.gzy = L.ndim == 3 ? m->gz[z] * m->gy[y] : m->gz[z];
            row.ys = L.ys;
            row.zs = L.zs;
            row.nx = L.nx;
            g_isa->fn(&row, 1, L.ndim);
            // receivers sample Pnew before the next source addition
            if (has_rec) {
                const int64_t zr = z - r.z0, yr = y - r.y0;
                if (zr >= 0 && yr >= 0 && zr % r.dz == 0 && yr % r.dy == 0 && zr / r.dz < r.nz &&
                    yr / r.dy < r.ny) {
                    float *out = io.trace_row + ((zr / r.dz) * r.ny + yr / r.dy) * r.nx;
                    for (int64_t k = 0; k < r.nx; ++k) out[k] = row.Q[r.x0 + k * r.dx];
                }
            }
            if (z == s->src_z && y == s->src_y) row.Q[s->src_x] += io.inj;
        }
    }
}

StepIO step_io(const fd_model *m, fd_state *st, const fd_shot *s, int64_t n, float *trace_row)
{
    StepIO io;
    io.cur = st->buf[n & 1];
    io.prev = st->buf[(n + 1) & 1];
    io.trace_row = trace_row;
    io.inj = n + 1 < s->nt ? m->amp * s->wavelet[n + 1] : 0.0f;
    return io;
}

// Both levels to zero (the frame included), the bytes of each task's rows
// first touched by the thread that steps them, then P[src] = amp s[0].
void do_begin(const fd_model *m, fd_state *st, const fd_shot *s)
{
    const Layout &L = m->L;
    const int32_t T = threads();
    const int64_t nplanes = L.nz + 2 * kR;
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t p = 0; p < nplanes; ++p)
        for (int lvl = 0; lvl < 2; ++lvl)
            std::memset(st->buf[lvl] + (size_t)p * L.zs, 0, (size_t)L.zs * 4);
    if (s) st->buf[0][index_of(L, s->src_z, s->src_y, s->src_x)] = m->amp * s->wavelet[0];
    st->health = 0;
    if (s)
        for (int64_t n = 0; n < s->nt; ++n)
            if (!std::isfinite(m->amp * s->wavelet[n])) st->health |= 4u;
    st->next = 0;
}

fd_status check_step(const fd_model *m, const fd_state *st, const fd_shot *s)
{
    if (!m || !st) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (st->m != m) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    return check_shot(m, s);
}

}  // namespace

extern "C" {

const char *fd_last_error(void) { return g_err.c_str(); }

const char *fd_version(void)
{
    static thread_local std::string v;
    v = std::string("fd-cpu 0.1 (OpenMP, ") + g_isa->name + ", radius 4)";
    return v.c_str();
}

int32_t fd_cpu_threads(int32_t n)
{
    if (n >= 1) g_threads = n;
    return threads();
}

const char *fd_cpu_isa(void) { return g_isa->name; }

fd_status fd_cpu_set_isa(const char *name)
{
    if (!name) return fail(FD_ERR_INVALID_ARG, "name is NULL");
    for (const Isa &i : kIsas) {
        if (std::strcmp(i.name, name) == 0) {
            if (!i.available()) return fail(FD_ERR_UNSUPPORTED, "this processor lacks %s", name);
            g_isa = &i;
            return ok();
        }
    }
    return fail(FD_ERR_INVALID_ARG, "unknown instruction set '%s' (avx512, avx2, scalar)", name);
}

fd_status fd_cpu_stream_probe(size_t n_floats, int32_t reps, double *gbs)
{
    if (n_floats < 1024 || reps < 1 || !gbs) return fail(FD_ERR_INVALID_ARG, "n_floats >= 1024, reps >= 1 and gbs are required");
    const size_t bytes = (n_floats * 4 + kAlign - 1) / kAlign * kAlign;
    float *a = (float *)std::aligned_alloc(kAlign, bytes);
    float *b = (float *)std::aligned_alloc(kAlign, bytes);
    float *p = (float *)std::aligned_alloc(kAlign, bytes);
    if (!a || !b || !p) {
        std::free(a);
        std::free(b);
        std::free(p);
        return fail(FD_ERR_OUT_OF_MEMORY, "probe arrays (3 x %zu bytes)", bytes);
    }
    const int64_t n = (int64_t)n_floats;
    const int32_t T = threads();
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t i = 0; i < n; ++i) {
        a[i] = 1.0f;
        b[i] = 0.5f;
        p[i] = 0.0f;
    }
    double best = 0.0;
    for (int32_t r = 0; r < reps; ++r) {
        const double t0 = omp_get_wtime();
#pragma omp parallel for schedule(static) num_threads(T)
        for (int64_t i = 0; i < n; ++i) p[i] = 2.0f * a[i] + b[i] * p[i];
        const double dt = omp_get_wtime() - t0;
        if (dt > 0.0) best = std::max(best, 16.0 * (double)n / dt / 1e9);
    }
    volatile float sink = p[n / 2];
    (void)sink;
    std::free(a);
    std::free(b);
    std::free(p);
    *gbs = best;
    return ok();
}

fd_status fd_query_bytes(const fd_grid *grid, int64_t nt, int32_t ckpt_every, fd_sizes *out)
{
    fd_status st = check_grid(grid);
    if (st != FD_OK) return st;
    if (!out) return fail(FD_ERR_INVALID_ARG, "out is NULL");
    if (nt < 0 || ckpt_every < 0) return fail(FD_ERR_INVALID_ARG, "nt and ckpt_every must be >= 0");
    const Layout L = make_layout(*grid);
    out->model = L.model_bytes;
    out->state = L.state_bytes;
    out->checkpoints = 0;  // checkpoints, the adjoint and the routine split are not built here
    out->adjoint_work = 0;
    out->routines_work = 0;
    return ok();
}

fd_status fd_create_model(const fd_grid *grid, const float *velocity, void *model_buf,
                          size_t model_bytes, void *stream, fd_model **out)
{
    (void)stream;
    fd_status st = check_grid(grid);
    if (st != FD_OK) return st;
    if (!velocity || !model_buf || !out) return fail(FD_ERR_INVALID_ARG, "NULL velocity, buffer or out");
    const Layout L = make_layout(*grid);
    if (model_bytes < L.model_bytes)
        return fail(FD_ERR_INVALID_ARG, "model buffer too small (%zu < %zu bytes)", model_bytes, L.model_bytes);
    if ((uintptr_t)model_buf % kAlign) return fail(FD_ERR_INVALID_ARG, "model buffer must be 256-byte aligned");

    // velocity range first: nothing is written for a rejected model
    const int64_t ncell = L.nz * L.ny * L.nx;
    float vmax = 0.0f;
    int bad = 0;
    const int32_t T = threads();
#pragma omp parallel for schedule(static) num_threads(T) reduction(max : vmax) reduction(| : bad)
    for (int64_t i = 0; i < ncell; ++i) {
        const float v = velocity[i];
        if (!(v > 0.0f) || !(v < 3.0e38f)) bad |= 1;
        else vmax = std::max(vmax, v);
    }
    if (bad) return fail(FD_ERR_INVALID_ARG, "velocity must be positive and finite everywhere");
    const double cfl = (double)vmax * grid->dt / grid->dh;
    if (!(cfl * cfl * grid->ndim * kSymbolMax <= 4.0))
        return fail(FD_ERR_UNSTABLE, "unstable: vmax*dt/dh = %.6f exceeds the %dD limit %.6f", cfl,
                    grid->ndim, std::sqrt(4.0 / (grid->ndim * kSymbolMax)));

    fd_model *m = new (std::nothrow) fd_model;
    if (!m) return fail(FD_ERR_OUT_OF_MEMORY, "host allocation failed");
    m->grid = *grid;
    if (m->grid.sponge_width > 0 && !(m->grid.sponge_alpha > 0.0))
        m->grid.sponge_alpha = 0.3 / m->grid.sponge_width;
    m->L = L;
    char *base = (char *)model_buf;
    m->c = (float *)base;
    m->gz = (float *)(base + L.gz_off);
    m->gy = (float *)(base + L.gy_off);
    m->gx = (float *)(base + L.gx_off);
    m->amp = (float)(grid->dt * grid->dt / std::pow(grid->dh, (double)grid->ndim));

    // c = (v dt/dh)^2, the FP64 product rounded to FP32; zero outside the grid
    const double r = grid->dt / grid->dh;
    const int64_t nplanes = L.nz + 2 * kR;
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t p = 0; p < nplanes; ++p) {
        float *plane = m->c + (size_t)p * L.zs;
        std::memset(plane, 0, (size_t)L.zs * 4);
        const int64_t z = p - kR;
        if (z < 0 || z >= L.nz) continue;
        for (int64_t y = 0; y < L.ny; ++y) {
            float *row = m->c + index_of(L, z, y, 0);
            const float *v = velocity + (size_t)(z * L.ny + y) * (size_t)L.nx;
            for (int64_t x = 0; x < L.nx; ++x) {
                const double q = (double)v[x] * r;
                row[x] = (float)(q * q);
            }
        }
    }
    // damping profiles g(i) = exp(-(alpha d)^2), FP64, stored FP32
    const double alpha = m->grid.sponge_alpha;
    const int32_t W = m->grid.sponge_width;
    const uint32_t f = m->grid.sponge_faces;
    auto profile = [&](float *g, int64_t n, int64_t len, bool lo, bool hi) {
        for (int64_t i = 0; i < len; ++i) {
            if (i >= n) {
                g[i] = 0.0f;
                continue;
            }
            double d = 0.0;
            if (W > 0) {
                if (lo && (double)(W - i) > d) d = (double)(W - i);
                if (hi && (double)(i - (n - 1 - W)) > d) d = (double)(i - (n - 1 - W));
            }
            g[i] = (float)std::exp(-(alpha * d) * (alpha * d));
        }
    };
    profile(m->gz, L.nz, L.nz, f & FD_FACE_ZLO, f & FD_FACE_ZHI);
    if (L.ndim == 3)
        profile(m->gy, L.ny, L.ny, f & FD_FACE_YLO, f & FD_FACE_YHI);
    else
        m->gy[0] = 1.0f;
    profile(m->gx, L.nx, L.pitch, f & FD_FACE_XLO, f & FD_FACE_XHI);
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
    st->buf[0] = (float *)state_buf;
    st->buf[1] = (float *)((char *)state_buf + model->L.field);
    st->next = -1;
    st->health = 0;
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
    (void)stream;
    fd_status st = check_step(model, state, shot);
    if (st != FD_OK) return st;
    do_begin(model, state, shot);
    return ok();
}

fd_status fd_step(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                  float *trace_row, void *stream)
{
    (void)stream;
    fd_status st = check_step(model, state, shot);
    if (st != FD_OK) return st;
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    if (n != state->next) return fail(FD_ERR_INVALID_ARG, "step %lld requested, next step is %lld",
                                      (long long)n, (long long)state->next);
    if (n >= shot->nt) return fail(FD_ERR_INVALID_ARG, "step %lld beyond the shot's %lld steps",
                                   (long long)n, (long long)shot->nt);
    const int32_t T = threads();
    const Tasks tk = plan(model->L, T);
    const StepIO io = step_io(model, state, shot, n, trace_row);
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t t = 0; t < tk.count(); ++t) run_task(model, shot, io, tk, t);
    state->next = n + 1;
    return ok();
}

fd_status fd_run_shot(const fd_model *model, fd_state *state, const fd_shot *shot, float *traces,
                      void *ckpt, size_t ckpt_bytes, int32_t ckpt_every, void *stream)
{
    (void)stream;
    (void)ckpt_bytes;
    (void)ckpt_every;
    fd_status st = check_step(model, state, shot);
    if (st != FD_OK) return st;
    if (ckpt) return unsupported("a checkpoint buffer (the adjoint)");
    do_begin(model, state, shot);
    const int32_t T = threads();
    const Tasks tk = plan(model->L, T);
    const int64_t nrec = nrec_of(shot), nt = shot->nt;
    // one parallel region for the whole time loop; the implicit barrier at
    // the end of each step's task loop orders the steps
#pragma omp parallel num_threads(T)
    for (int64_t n = 0; n < nt; ++n) {
        const StepIO io = step_io(model, state, shot, n, traces ? traces + (size_t)n * (size_t)nrec : nullptr);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < tk.count(); ++t) run_task(model, shot, io, tk, t);
    }
    state->next = nt;
    return ok();
}

fd_status fd_run_shots(const fd_model *model, fd_state *const *states, const fd_shot *const *shots,
                       int32_t count, float *const *traces, void *const *ckpt, size_t ckpt_bytes,
                       int32_t ckpt_every, void *stream)
{
    if (!model) return fail(FD_ERR_INVALID_ARG, "NULL model");
    if (count < 1 || count > 4096) return fail(FD_ERR_INVALID_ARG, "count must be in [1, 4096]");
    if (!states || !shots) return fail(FD_ERR_INVALID_ARG, "NULL states or shots array");
    for (int32_t i = 0; i < count; ++i) {
        fd_status st = check_step(model, states[i], shots[i]);
        if (st != FD_OK) return st;
        if (shots[i]->nt != shots[0]->nt) return fail(FD_ERR_INVALID_ARG, "shot %d: all shots must share nt", i);
        for (int32_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return fail(FD_ERR_INVALID_ARG, "shot %d repeats a state", i);
        if (ckpt && ckpt[i]) return unsupported("a checkpoint buffer (the adjoint)");
    }
    for (int32_t i = 0; i < count; ++i) {
        fd_status st = fd_run_shot(model, states[i], shots[i], traces ? traces[i] : nullptr, nullptr,
                                   ckpt_bytes, ckpt_every, stream);
        if (st != FD_OK) return st;
    }
    return ok();
}

fd_status fd_get_wavefield(const fd_state *state, int32_t which, float *out, void *stream)
{
    (void)stream;
    if (!state || !out) return fail(FD_ERR_INVALID_ARG, "NULL state or out");
    if (which != 0 && which != 1) return fail(FD_ERR_INVALID_ARG, "which must be 0 (P) or 1 (Pold)");
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    const Layout &L = state->m->L;
    const int64_t lvl = which == 0 ? state->next : state->next - 1;
    const float *buf = state->buf[lvl & 1];
    const int32_t T = threads();
#pragma omp parallel for schedule(static) num_threads(T)
    for (int64_t z = 0; z < L.nz; ++z)
        for (int64_t y = 0; y < L.ny; ++y)
            std::memcpy(out + (size_t)(z * L.ny + y) * (size_t)L.nx, buf + index_of(L, z, y, 0),
                        (size_t)L.nx * 4);
    return ok();
}

fd_status fd_set_wavefield(fd_state *state, int32_t which, const float *in, void *stream)
{
    (void)stream;
    if (!state || !in) return fail(FD_ERR_INVALID_ARG, "NULL state or in");
    if (which != 0 && which != 1) return fail(FD_ERR_INVALID_ARG, "which must be 0 (P) or 1 (Pold)");
    const Layout &L = state->m->L;
    if (state->next < 0) do_begin(state->m, state, nullptr);
    const int64_t lvl = which == 0 ? state->next : state->next - 1;
    float *buf = state->buf[lvl & 1];
    const int32_t T = threads();
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(T) reduction(| : bad)
    for (int64_t z = 0; z < L.nz; ++z)
        for (int64_t y = 0; y < L.ny; ++y) {
            const float *src = in + (size_t)(z * L.ny + y) * (size_t)L.nx;
            std::memcpy(buf + index_of(L, z, y, 0), src, (size_t)L.nx * 4);
            for (int64_t x = 0; x < L.nx; ++x) bad |= !std::isfinite(src[x]);
        }
    if (bad) state->health |= 4u;
    return ok();
}

fd_status fd_check_finite(const fd_state *state, uint32_t *flags, void *stream)
{
    (void)stream;
    if (!state || !flags) return fail(FD_ERR_INVALID_ARG, "NULL state or flags");
    if ((uintptr_t)flags % 4) return fail(FD_ERR_INVALID_ARG, "flags must be 4-byte aligned");
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    const Layout &L = state->m->L;
    uint32_t f = 0;
    for (int lvl = 0; lvl < 2; ++lvl) {
        const float *buf = state->buf[(state->next + lvl) & 1];
        int bad = 0;
        const int32_t T = threads();
#pragma omp parallel for schedule(static) num_threads(T) reduction(| : bad)
        for (int64_t z = 0; z < L.nz; ++z)
            for (int64_t y = 0; y < L.ny; ++y) {
                const float *row = buf + index_of(L, z, y, 0);
                for (int64_t x = 0; x < L.nx; ++x) bad |= !std::isfinite(row[x]);
            }
        if (bad) f |= 1u << lvl;
    }
    *flags = f | (state->health & 4u);
    return ok();
}

// ---- calls this back-end does not build -------------------------------------
fd_status fd_adjoint_gradient(const fd_model *, const fd_shot *, const float *, const void *, size_t,
                              int32_t, void *, size_t, double *, void *)
{
    return unsupported("fd_adjoint_gradient");
}

fd_status fd_rtm_image(const fd_model *, const fd_shot *, const float *, const void *, size_t,
                       int32_t, void *, size_t, double *, void *)
{
    return unsupported("fd_rtm_image");
}

fd_status fd_adjoint_gradient_shots(const fd_model *, const fd_shot *const *, int32_t,
                                    const float *const *, const void *const *, size_t, int32_t,
                                    void *const *, size_t, double *, void *)
{
    return unsupported("fd_adjoint_gradient_shots");
}

fd_status fd_rtm_image_shots(const fd_model *, const fd_shot *const *, int32_t, const float *const *,
                             const void *const *, size_t, int32_t, void *const *, size_t, double *,
                             void *)
{
    return unsupported("fd_rtm_image_shots");
}

fd_status fd_slab_exchange(const fd_state *, const fd_state *, void *)
{
    return unsupported("fd_slab_exchange");
}

fd_status fd_step_batch(fd_batch_item *, int32_t, int32_t, void *)
{
    return unsupported("fd_step_batch");
}

fd_status fd_step_routines(const fd_model *, fd_state *, const fd_shot *, int64_t, float *, void *,
                           size_t, void *)
{
    return unsupported("fd_step_routines");
}

fd_status fd_step_routines_noalloc(const fd_model *, fd_state *, const fd_shot *, int64_t, float *, void *)
{
    return unsupported("fd_step_routines_noalloc");
}

fd_status fd_stream_probe(int32_t, const float *, const float *, float *, size_t, void *)
{
    return unsupported("fd_stream_probe (the host roof is fd_cpu_stream_probe)");
}

fd_status fd_shot_graph_create(const fd_model *, fd_state *, const fd_shot *, float *, fd_shot_graph **out)
{
    if (out) *out = nullptr;
    return unsupported("fd_shot_graph_create (a host shot has no launches to record)");
}

fd_status fd_shot_graph_launch(fd_shot_graph *, void *)
{
    return unsupported("fd_shot_graph_launch");
}

fd_status fd_shot_graph_destroy(fd_shot_graph *)
{
    return FD_OK;
}

}  // extern "C"
