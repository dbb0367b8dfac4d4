// Host-side logic of the C ABI (declarations: fd_host.hpp).  No HIP here.
#include "fd_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

namespace fdh {

namespace {
thread_local std::string g_err;
}  // namespace

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

const char *last_error() { return g_err.c_str(); }


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
        if (g->slab_nz_global > kMaxDim || g->nz > g->slab_nz_global || g->slab_z0 > g->slab_nz_global - g->nz)
            return fail(FD_ERR_INVALID_ARG, "slab of %lld planes from plane %lld leaves the %lld-plane grid",
                        (long long)g->nz, (long long)g->slab_z0, (long long)g->slab_nz_global);
    }
    const double cells = (double)(g->nz + 2 * kGhost) * (double)g->ny * (double)((g->nx + 63) / 64 * 64);
    if (cells > 4.0e9) return fail(FD_ERR_INVALID_ARG, "grid too large");
    // the 16-bit 3D kernels address a plane with 32-bit byte offsets
    if ((double)g->ny * (double)((g->nx + 63) / 64 * 64) >= 1073741824.0)
        return fail(FD_ERR_INVALID_ARG, "an x-y plane must hold fewer than 2^30 cells");
    return FD_OK;
}

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
    // every test below is free of overflow for any int64 input: the counts
    // are bounded before they are multiplied, and the far end of each axis
    // is tested by division
    if (r.nz < 0 || r.ny < 0 || r.nx < 0) return fail(FD_ERR_INVALID_ARG, "negative receiver counts");
    if (r.nz == 0 || r.ny == 0 || r.nx == 0) {
        if (r.nz || r.ny || r.nx) return fail(FD_ERR_INVALID_ARG, "receiver counts must be all zero or all positive");
        return FD_OK;
    }
    const int64_t kMaxRec = (int64_t)1 << 30;
    if (r.nz > kMaxRec || r.ny > kMaxRec || r.nx > kMaxRec || r.nz * r.ny > kMaxRec || r.nz * r.ny * r.nx > kMaxRec)
        return fail(FD_ERR_INVALID_ARG, "too many receivers");
    if (r.dz < 1 || r.dy < 1 || r.dx < 1) return fail(FD_ERR_INVALID_ARG, "receiver strides must be >= 1");
    // the array's last cell along an axis of n cells: x0 + (cnt - 1) d <= n - 1
    auto inside = [](int64_t x0, int64_t cnt, int64_t d, int64_t n) {
        return x0 >= 0 && x0 < n && (cnt - 1) <= (n - 1 - x0) / d;
    };
    if (!inside(r.z0, r.nz, r.dz, L.nzg) || !inside(r.y0, r.ny, r.dy, L.ny) || !inside(r.x0, r.nx, r.dx, L.nx))
        return fail(FD_ERR_INVALID_ARG, "receiver array leaves the grid");
    return FD_OK;
}

int64_t nrec_of(const fd_shot *s) { return s->rec.nz * s->rec.ny * s->rec.nx; }

fdk::StepArgs base_args(const fd_model *m, const fd_shot *s, int64_t *rec_skip)
{
    fdk::StepArgs a{};
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

std::vector<float> damping_profile(int64_t n, int32_t W, double alpha, bool lo, bool hi)
{
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
}

float source_amp(const fd_grid &g) { return (float)(g.dt * g.dt / std::pow(g.dh, (double)g.ndim)); }

fd_status check_stability(const fd_grid &g, float vmax)
{
    const double cfl = (double)vmax * g.dt / g.dh;
    const double lhs = cfl * cfl * g.ndim * kSymbolMax;
    if (!(lhs <= 4.0))
        return fail(FD_ERR_UNSTABLE, "unstable: vmax*dt/dh = %.6f exceeds the %dD limit %.6f", cfl, g.ndim,
                    std::sqrt(4.0 / (g.ndim * kSymbolMax)));
    return FD_OK;
}

int c16_exponent(float vmax, double dt_over_dh)
{
    // the largest c, rounded to FP32 exactly as the kernels round every c
    // (the product is monotone in v)
    const double qq = (double)vmax * dt_over_dh;
    const float cmax = (float)(qq * qq);
    int ex = 0;
    std::frexp(cmax, &ex);  // cmax = f 2^ex with f in [0.5, 1)
    // a cmax within half a code of 2^ex would round to code 2^16: the next
    // binade keeps every code in 16 bits and the error <= 2^(e-17)
    if (std::nearbyint(std::ldexp((double)cmax, 16 - ex)) > 65535.0) ex += 1;
    return ex;
}

}  // namespace fdh
