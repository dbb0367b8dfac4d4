// Drives the library's host-side logic (paper_2311_05038_amd/csrc/fd_host.cpp:
// validation, layouts, stability check, damping profiles, step arguments)
// over ordinary, edge and hostile inputs.  Built with AddressSanitizer and
// UBSan by tests/test_sanitize.py; any out-of-bounds access, overflow or
// other undefined behaviour aborts the run, and every expectation below is
// checked.  No device is involved.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2311_05038_amd/csrc/fd_host.hpp"

using namespace fdh;

static int failures = 0;
#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                                \
        }                                                                              \
    } while (0)

static fd_grid grid3(int64_t nz, int64_t ny, int64_t nx)
{
    fd_grid g{};
    g.ndim = 3;
    g.nz = nz;
    g.ny = ny;
    g.nx = nx;
    g.dh = 10.0;
    g.dt = 1e-3;
    g.radius = 4;
    g.bc = FD_BC_ZERO;
    g.sponge_width = 8;
    g.sponge_faces = 0x3E;
    g.storage = FD_F32;
    g.c_storage = FD_C_F32;
    return g;
}

static fd_grid grid2(int64_t nz, int64_t nx)
{
    fd_grid g = grid3(nz, 1, nx);
    g.ndim = 2;
    return g;
}

static void check_layout(const fd_grid &g)
{
    const Layout L = make_layout(g);
    EXPECT(L.px % 64 == 0 && L.px >= L.nx && L.px < L.nx + 64);
    EXPECT(L.npad == (size_t)L.nz * (size_t)L.ny * (size_t)L.px);
    EXPECT(L.field % kAlign == 0 && L.field >= L.npad * L.elem + 2 * L.ghost);
    EXPECT(L.f32field % kAlign == 0 && L.f32field >= L.npad * 4);
    EXPECT(L.cfield >= L.npad * (g.c_storage == FD_C_FIXED16 ? 2 : 4));
    EXPECT(L.c_off == 0 && L.gz_off >= L.c_off + L.cfield);
    EXPECT(L.gy_off >= L.gz_off + (size_t)L.nz * 4 && L.gx_off >= L.gy_off + (size_t)L.ny * 4);
    EXPECT(L.scratch_off >= L.gx_off + (size_t)L.nx * 4 && L.model_bytes >= L.scratch_off + 8);
    for (size_t off : {L.gz_off, L.gy_off, L.gx_off, L.scratch_off, L.meta_off}) EXPECT(off % kAlign == 0);
    EXPECT(L.meta_off == 2 * L.field && L.state_bytes >= L.meta_off + fdk::kMetaWords * 4);
    EXPECT(adjoint_work_bytes(L, 50) >= 56 * L.f32field);
    EXPECT(ckpt_slot_bytes(L) == 2 * L.field);
}

static fd_shot shot_at(int64_t z, int64_t y, int64_t x, const float *wav, int64_t nt)
{
    fd_shot s{};
    s.src_z = z;
    s.src_y = y;
    s.src_x = x;
    s.wavelet = wav;
    s.nt = nt;
    return s;
}

// A host-only model handle: layout and scalars, no device buffers.
static fd_model model_of(const fd_grid &g)
{
    fd_model m{};
    m.grid = g;
    m.L = make_layout(g);
    m.amp = source_amp(g);
    return m;
}

int main()
{
    // ---- grid validation -------------------------------------------------
    EXPECT(check_grid(nullptr) == FD_ERR_INVALID_ARG && *last_error());
    {
        const fd_grid ok3 = grid3(40, 30, 70);
        EXPECT(check_grid(&ok3) == FD_OK);
        check_layout(ok3);
        const fd_grid ok2 = grid2(1, 1);
        EXPECT(check_grid(&ok2) == FD_OK);
        check_layout(ok2);
    }
    struct Bad {
        fd_grid g;
        fd_status want;
    };
    std::vector<Bad> bad;
    auto add = [&](fd_grid g, fd_status w) { bad.push_back({g, w}); };
    {
        fd_grid g = grid3(8, 8, 8);
        g.ndim = 4; add(g, FD_ERR_INVALID_ARG);
        g = grid3(0, 8, 8); add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, -1, 8); add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, ((int64_t)1 << 30) + 1); add(g, FD_ERR_INVALID_ARG);
        g = grid3(INT64_MAX, INT64_MAX, INT64_MAX); add(g, FD_ERR_INVALID_ARG);
        g = grid3((int64_t)1 << 30, (int64_t)1 << 30, (int64_t)1 << 30); add(g, FD_ERR_INVALID_ARG);
        g = grid2(8, 8); g.ny = 2; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.dh = 0.0; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.dh = NAN; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.dt = -1.0; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.dt = INFINITY; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.radius = 0; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.radius = 2; add(g, FD_ERR_UNSUPPORTED);
        g = grid3(8, 8, 8); g.bc = FD_BC_PERIODIC; add(g, FD_ERR_UNSUPPORTED);
        g = grid3(8, 8, 8); g.bc = (fd_bc)7; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.sponge_width = -3; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.sponge_faces = 0x40; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.sponge_alpha = NAN; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.storage = 9; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.c_storage = (fd_c_storage)5; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.c_storage = FD_C_FIXED16; add(g, FD_ERR_UNSUPPORTED);
        g = grid3(8, 8, 8); g.slab_nz_global = -1; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.slab_z0 = 3; add(g, FD_ERR_INVALID_ARG);
        g = grid2(8, 8); g.slab_nz_global = 16; add(g, FD_ERR_UNSUPPORTED);
        g = grid3(3, 8, 8); g.slab_nz_global = 16; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.slab_nz_global = 16; g.slab_z0 = 9; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.slab_nz_global = 16; g.storage = FD_F16; add(g, FD_ERR_UNSUPPORTED);
        g = grid3(4, 32768, 32768 + 64); add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.slab_nz_global = 16; g.slab_z0 = INT64_MAX; add(g, FD_ERR_INVALID_ARG);
        g = grid3(8, 8, 8); g.slab_nz_global = INT64_MAX; add(g, FD_ERR_INVALID_ARG);
        g = grid3(20, 8, 8); g.slab_nz_global = 16; add(g, FD_ERR_INVALID_ARG);
    }
    for (size_t i = 0; i < bad.size(); ++i) {
        const fd_status st = check_grid(&bad[i].g);
        if (st != bad[i].want) std::fprintf(stderr, "bad grid %zu: status %d, want %d\n", i, (int)st, (int)bad[i].want);
        EXPECT(st == bad[i].want);
        EXPECT(*last_error() != '\0');
    }
    EXPECT(ok() == FD_OK && *last_error() == '\0');
    // a message longer than the buffer is cut, not overrun
    {
        std::string longname(2000, 'x');
        EXPECT(fail(FD_ERR_INVALID_ARG, "%s", longname.c_str()) == FD_ERR_INVALID_ARG);
        EXPECT(std::string(last_error()).size() < 600);
    }

    // ---- layouts over random valid grids (incl. 16-bit forms and slabs) --
    std::mt19937_64 rng(12345);
    for (int it = 0; it < 3000; ++it) {
        const int nd = 2 + (int)(rng() % 2);
        fd_grid g = nd == 3 ? grid3(1 + rng() % 300, 1 + rng() % 300, 1 + rng() % 700)
                            : grid2(1 + rng() % 5000, 1 + rng() % 9000);
        g.storage = (int32_t)(rng() % 3);
        if (g.storage != FD_F32 && rng() % 2) g.c_storage = FD_C_FIXED16;
        if (nd == 3 && g.storage == FD_F32 && g.nz >= 4 && rng() % 3 == 0) {
            g.slab_nz_global = g.nz + (int64_t)(rng() % 200);
            g.slab_z0 = (int64_t)(rng() % (uint64_t)(g.slab_nz_global - g.nz + 1));
        }
        EXPECT(check_grid(&g) == FD_OK);
        check_layout(g);
        const Layout L = make_layout(g);
        EXPECT(is_slab(L) == (g.slab_nz_global > 0));
    }

    // ---- damping profiles ------------------------------------------------
    for (int64_t n : {1, 2, 9, 64, 65, 300}) {
        for (int32_t W : {0, 1, 4, 32}) {
            for (int f = 0; f < 4; ++f) {
                const std::vector<float> p = damping_profile(n, W, W > 0 ? 0.3 / W : 0.0, f & 1, f & 2);
                EXPECT((int64_t)p.size() == n);
                for (int64_t i = 0; i < n; ++i) {
                    EXPECT(p[i] > 0.0f && p[i] <= 1.0f);
                    const bool in_lo = (f & 1) && i < W, in_hi = (f & 2) && i > n - 1 - W;
                    if (!in_lo && !in_hi) EXPECT(p[i] == 1.0f);
                    if ((f & 1) && i + 1 < n && i + 1 <= W && !(f & 2)) EXPECT(p[i] <= p[i + 1]);
                }
            }
        }
    }

    // ---- stability limit and 16-bit c exponent ---------------------------
    {
        fd_grid g = grid3(8, 8, 8);
        const double limit3 = std::sqrt(4.0 / (3 * kSymbolMax));   // 0.45286
        EXPECT(check_stability(g, (float)(0.999 * limit3 * g.dh / g.dt)) == FD_OK);
        EXPECT(check_stability(g, (float)(1.001 * limit3 * g.dh / g.dt)) == FD_ERR_UNSTABLE);
        EXPECT(check_stability(g, NAN) == FD_ERR_UNSTABLE);
        EXPECT(check_stability(g, INFINITY) == FD_ERR_UNSTABLE);
        fd_grid g2 = grid2(8, 8);
        const double limit2 = std::sqrt(4.0 / (2 * kSymbolMax));   // 0.55463
        EXPECT(check_stability(g2, (float)(0.999 * limit2 * g2.dh / g2.dt)) == FD_OK);
        EXPECT(check_stability(g2, (float)(1.001 * limit2 * g2.dh / g2.dt)) == FD_ERR_UNSTABLE);
        for (int it = 0; it < 20000; ++it) {
            const float v = 100.0f + (float)(rng() % 1000000) * 0.01f;
            const int e = c16_exponent(v, 1e-4);
            const double qq = (double)v * 1e-4;
            const float cmax = (float)(qq * qq);
            EXPECT(std::ldexp(1.0, e - 2) <= cmax && (double)cmax < std::ldexp(1.0, e));
            EXPECT(std::nearbyint(std::ldexp((double)cmax, 16 - e)) <= 65535.0);
        }
    }

    // ---- shot validation and step arguments ------------------------------
    std::vector<float> wav(64, 1.0f);
    {
        const fd_grid g = grid3(20, 24, 70);
        const fd_model m = model_of(g);
        fd_shot s = shot_at(3, 5, 7, wav.data(), 64);
        EXPECT(check_shot(&m, &s) == FD_OK);
        EXPECT(check_shot(&m, nullptr) == FD_ERR_INVALID_ARG);
        fd_shot t = s; t.nt = 0; EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t = s; t.wavelet = nullptr; EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        const int64_t srcs[][3] = {{-1, 0, 0}, {20, 0, 0}, {0, 24, 0}, {0, 0, 70}, {0, -5, 0},
                                   {INT64_MIN, 0, 0}, {0, 0, INT64_MAX}};
        for (const auto &b : srcs) {
            t = shot_at(b[0], b[1], b[2], wav.data(), 64);
            EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        }
        // receivers: a strided box touching the far corner is fine; one past it is not
        t = s;
        t.rec = fd_receivers{1, 3, 5, 4, 3, 11, 6, 10, 6};   // z0 y0 x0, nz ny nx, dz dy dx
        EXPECT(check_shot(&m, &t) == FD_OK);   // last: z 19, y 23, x 65
        t.rec.nx = 12;                          // x 71: off the grid
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t.rec = fd_receivers{0, 0, 0, 1, 1, 1, 0, 1, 1};   // stride 0
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t.rec = fd_receivers{0, 0, 0, 0, 1, 1, 1, 1, 1};   // some counts zero
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t.rec = fd_receivers{0, 0, 0, -1, -1, 1, 1, 1, 1};
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t.rec = fd_receivers{0, 0, 0, (int64_t)1 << 40, (int64_t)1 << 40, 1, 1, 1, 1};
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        t.rec = fd_receivers{0, 0, INT64_MAX - 2, 1, 1, 2, 1, 1, 1};
        EXPECT(check_shot(&m, &t) == FD_ERR_INVALID_ARG);
        // arguments of a whole grid
        t = s;
        t.rec = fd_receivers{2, 4, 1, 3, 5, 17, 5, 3, 4};
        EXPECT(check_shot(&m, &t) == FD_OK);
        int64_t skip = 99;
        const fdk::StepArgs a = base_args(&m, &t, &skip);
        EXPECT(a.nz == 20 && a.ny == 24 && a.nx == 70 && a.px == 128 && a.sz == 3 && a.sy == 5 && a.sx == 7);
        EXPECT(a.rec.z0 == 2 && a.rec.nz == 3 && a.rec.ny == 5 && a.rec.nx == 17 && skip == 0);
        EXPECT(a.amp == m.amp && a.nt == 64);
        EXPECT(src_offset(m.L, &t) == (size_t)((3 * 24 + 5) * 128 + 7));
    }
    // z-slabs: the receiver rows on the slab's planes and their offset in the
    // full trace row, against a brute-force count
    for (int it = 0; it < 4000; ++it) {
        const int64_t nzg = 8 + (int64_t)(rng() % 120);
        const int64_t nz = 4 + (int64_t)(rng() % (uint64_t)(nzg - 3));
        fd_grid g = grid3(nz, 6 + rng() % 20, 10 + rng() % 100);
        g.slab_nz_global = nzg;
        g.slab_z0 = (int64_t)(rng() % (uint64_t)(nzg - nz + 1));
        EXPECT(check_grid(&g) == FD_OK);
        const fd_model m = model_of(g);
        fd_shot s = shot_at((int64_t)(rng() % (uint64_t)nzg), (int64_t)(rng() % (uint64_t)g.ny),
                            (int64_t)(rng() % (uint64_t)g.nx), wav.data(), 64);
        fd_receivers r{};
        r.dz = 1 + (int64_t)(rng() % 7);
        r.dy = 1 + (int64_t)(rng() % 3);
        r.dx = 1 + (int64_t)(rng() % 5);
        r.z0 = (int64_t)(rng() % (uint64_t)nzg);
        r.nz = 1 + (nzg - 1 - r.z0) / r.dz;
        r.nz = 1 + (int64_t)(rng() % (uint64_t)r.nz);
        r.y0 = (int64_t)(rng() % (uint64_t)g.ny);
        r.ny = 1 + (int64_t)(rng() % (uint64_t)(1 + (g.ny - 1 - r.y0) / r.dy));
        r.x0 = (int64_t)(rng() % (uint64_t)g.nx);
        r.nx = 1 + (int64_t)(rng() % (uint64_t)(1 + (g.nx - 1 - r.x0) / r.dx));
        s.rec = r;
        EXPECT(check_shot(&m, &s) == FD_OK);
        int64_t skip = 0;
        const fdk::StepArgs a = base_args(&m, &s, &skip);
        int64_t first = -1, rows = 0;
        for (int64_t i = 0; i < r.nz; ++i) {
            const int64_t zg = r.z0 + i * r.dz;
            if (zg >= g.slab_z0 && zg < g.slab_z0 + nz) {
                if (first < 0) first = i;
                ++rows;
            }
        }
        if (rows == 0) {
            EXPECT(skip == -1 && a.rec.nz == 0);
        } else {
            EXPECT(skip == first * r.ny * r.nx);
            EXPECT(a.rec.nz == rows && a.rec.z0 == r.z0 + first * r.dz - g.slab_z0);
            EXPECT(a.rec.z0 >= 0 && a.rec.z0 + (a.rec.nz - 1) * a.rec.dz < nz);
        }
        const bool on = s.src_z >= g.slab_z0 && s.src_z < g.slab_z0 + nz;
        EXPECT(on ? a.sz == s.src_z - g.slab_z0 : a.sz == -1);
    }
    if (failures) {
        std::fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
