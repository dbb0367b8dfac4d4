/*
 * Oracle: plain, slow, FP64 CPU definition of explicit finite-difference
 * acoustic time stepping.  TEST INFRASTRUCTURE ONLY: it is called by the
 * test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the library.  It shares no code with the GPU path.
 *
 * What it follows (arXiv 2311.05038):
 *   - Eq. 1 (Section 7): P_tt = v^2 (P_xx + P_zz) + S(t); extended here to a
 *     third axis (y) in the same form.
 *   - Listing 3 (Section 7): each time step applies, in order, the source
 *     addition to P, the second z- and x-derivatives, the time update to
 *     Pnew, then rotates (Pold, P, Pnew).  Fields P, Pold, Pnew, velocity V,
 *     scalars dt and one grid spacing dh.
 * Readings of what the paper leaves open (order, weights, source scaling,
 * sponge, receivers) are those of this repository's design notes:
 *   - second derivative: central weights of order 2R (closed form below),
 *     taps outside the grid read zero (zero edges) or wrap (periodic);
 *   - c = (v dt / dh)^2 folds 1/dh^2 into the velocity term, so the
 *     Laplacian sum L is dimensionless;
 *   - the source adds dt^2/dh^D * s[n] to one cell of P before the
 *     derivatives, with no v^2 factor (Eq. 1 puts S outside v^2);
 *   - damping: new = G (2 cur + c L cur) - G^2 prev with G = product over
 *     axes of exp(-(alpha d)^2), d the distance into the band on enabled
 *     faces.  How G enters the update is pinned by an exact identity (a
 *     uniform G = g maps the scheme onto the undamped one for P^n / g^n);
 *     the profile's shape is a reading, checked by its properties (1 off
 *     the band, strictly decreasing into it, enabled faces only, G the
 *     product of the axis profiles).
 *   - receivers sample the new field before the next source addition.
 *
 * Layout: arrays are row-major [nz][ny][nx], x fastest, ny = 1 in 2D.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the parallel loops from here on (timing on a given core
 * count); returns the count in effect. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t radius;        /* R: stencil half-width (1..8) */
    int32_t bc;            /* 0 zero edges, 1 periodic */
    int32_t sponge_width;  /* cells, 0 = no damping band */
    int64_t nz, ny, nx;
    double dh, dt;
    double sponge_alpha;
    uint32_t sponge_faces; /* bits: z-, z+, y-, y+, x-, x+ */
    uint32_t pad_;
} or_grid;

/* Central second-derivative weights of order 2R (h = 1):
 *   a_k = 2 (-1)^(k+1) (R!)^2 / (k^2 (R-k)! (R+k)!),  k = 1..R,
 *   a_0 = -2 sum_k a_k.
 * This is the classical closed form of the maximal-order symmetric
 * second-difference weights. */
void or_coefficients(int R, double *a)
{
    double fR = 1.0;
    for (int i = 2; i <= R; ++i) fR *= i;
    double sum = 0.0;
    for (int k = 1; k <= R; ++k) {
        double fm = 1.0, fp = 1.0;
        for (int i = 2; i <= R - k; ++i) fm *= i;
        for (int i = 2; i <= R + k; ++i) fp *= i;
        double ak = 2.0 * fR * fR / ((double)k * k * fm * fp);
        if (k % 2 == 0) ak = -ak;
        a[k] = ak;
        sum += ak;
    }
    a[0] = -2.0 * sum;
}

/* One axis of the damping profile: g(i) = exp(-(alpha d)^2). */
void or_sponge_profile(int64_t n, int32_t width, double alpha, int lo, int hi, double *g)
{
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        if (width > 0) {
            if (lo && (double)(width - i) > d) d = (double)(width - i);
            if (hi && (double)(i - (n - 1 - width)) > d) d = (double)(i - (n - 1 - width));
        }
        g[i] = exp(-(alpha * d) * (alpha * d));
    }
}

static double fetch(const or_grid *g, const double *u, int64_t z, int64_t y, int64_t x)
{
    if (g->bc == 1) {
        z = ((z % g->nz) + g->nz) % g->nz;
        y = ((y % g->ny) + g->ny) % g->ny;
        x = ((x % g->nx) + g->nx) % g->nx;
    } else if (z < 0 || z >= g->nz || y < 0 || y >= g->ny || x < 0 || x >= g->nx) {
        return 0.0;
    }
    return u[(z * g->ny + y) * g->nx + x];
}

/* (L u)_i = sum over axes of [a_0 u_i + sum_k a_k (u_{i+k e} + u_{i-k e})]. */
void or_laplacian(const or_grid *g, const double *u, double *out)
{
    double a[9];
    or_coefficients(g->radius, a);
    const int R = g->radius;
    const int naxes = g->ndim;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < g->nz; ++z)
        for (int64_t y = 0; y < g->ny; ++y)
            for (int64_t x = 0; x < g->nx; ++x) {
                double s = 0.0;
                /* z axis */
                s += a[0] * fetch(g, u, z, y, x);
                for (int k = 1; k <= R; ++k)
                    s += a[k] * (fetch(g, u, z + k, y, x) + fetch(g, u, z - k, y, x));
                /* y axis (3D only) */
                if (naxes == 3) {
                    s += a[0] * fetch(g, u, z, y, x);
                    for (int k = 1; k <= R; ++k)
                        s += a[k] * (fetch(g, u, z, y + k, x) + fetch(g, u, z, y - k, x));
                }
                /* x axis */
                s += a[0] * fetch(g, u, z, y, x);
                for (int k = 1; k <= R; ++k)
                    s += a[k] * (fetch(g, u, z, y, x + k) + fetch(g, u, z, y, x - k));
                out[(z * g->ny + y) * g->nx + x] = s;
            }
}

/* c = (v dt/h)^2 and G = gz * gy * gx, FP64. */
void or_setup(const or_grid *g, const float *v, double *c, double *G)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *gz = malloc(sizeof(double) * g->nz);
    double *gy = malloc(sizeof(double) * g->ny);
    double *gx = malloc(sizeof(double) * g->nx);
    const uint32_t f = g->sponge_faces;
    or_sponge_profile(g->nz, g->sponge_width, g->sponge_alpha, f & 1, (f >> 1) & 1, gz);
    if (g->ndim == 3)
        or_sponge_profile(g->ny, g->sponge_width, g->sponge_alpha, (f >> 2) & 1, (f >> 3) & 1, gy);
    else
        gy[0] = 1.0;
    or_sponge_profile(g->nx, g->sponge_width, g->sponge_alpha, (f >> 4) & 1, (f >> 5) & 1, gx);
    const double r = g->dt / g->dh;
    for (int64_t i = 0; i < N; ++i) {
        double q = (double)v[i] * r;
        c[i] = q * q;
    }
    for (int64_t z = 0; z < g->nz; ++z)
        for (int64_t y = 0; y < g->ny; ++y)
            for (int64_t x = 0; x < g->nx; ++x)
                G[(z * g->ny + y) * g->nx + x] = gz[z] * gy[y] * gx[x];
    free(gz);
    free(gy);
    free(gx);
}

static double source_amp(const or_grid *g)
{
    return g->dt * g->dt / pow(g->dh, (double)g->ndim);
}

/*
 * Forward modelling, nt steps.  Step n:
 *   1. cur[src] += dt^2/h^D * s[n]
 *   2. lap = L(cur)
 *   3. new = G (2 cur + c lap) - G^2 prev
 *   4. traces[n][r] = new[rec[r]]
 *   5. (prev, cur) <- (cur, new)
 * Optional: start from (init_prev, init_cur) instead of rest; store
 * lap_hist[n] = L(w^n) with w^n the field after step 1 of step n.
 * Returns 0, or -1 on allocation failure.
 */
/* The time loop of or_forward for given c and damping field G. */
static int forward_loop(const or_grid *g, const double *c, const double *G, const float *wavelet,
                        int64_t nt, int64_t src, int64_t nrec, const int64_t *rec,
                        const double *init_prev, const double *init_cur, double *traces,
                        double *final_prev, double *final_cur, double *lap_hist)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *prev = calloc(N, sizeof(double)), *cur = calloc(N, sizeof(double));
    double *nw = malloc(sizeof(double) * N), *lap = malloc(sizeof(double) * N);
    if (!prev || !cur || !nw || !lap) {
        free(prev); free(cur); free(nw); free(lap);
        return -1;
    }
    if (init_prev) memcpy(prev, init_prev, sizeof(double) * N);
    if (init_cur) memcpy(cur, init_cur, sizeof(double) * N);
    const double amp = source_amp(g);
    for (int64_t n = 0; n < nt; ++n) {
        if (src >= 0) cur[src] += amp * (double)wavelet[n];
        or_laplacian(g, cur, lap);
        if (lap_hist) memcpy(lap_hist + n * N, lap, sizeof(double) * N);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i)
            nw[i] = G[i] * (2.0 * cur[i] + c[i] * lap[i]) - G[i] * G[i] * prev[i];
        if (traces)
            for (int64_t r = 0; r < nrec; ++r) traces[n * nrec + r] = nw[rec[r]];
        double *t = prev;
        prev = cur;
        cur = nw;
        nw = t;
    }
    if (final_prev) memcpy(final_prev, prev, sizeof(double) * N);
    if (final_cur) memcpy(final_cur, cur, sizeof(double) * N);
    free(prev); free(cur); free(nw); free(lap);
    return 0;
}

int or_forward(const or_grid *g, const float *v, const float *wavelet, int64_t nt,
               int64_t src, int64_t nrec, const int64_t *rec,
               const double *init_prev, const double *init_cur,
               double *traces, double *final_prev, double *final_cur, double *lap_hist)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *c = malloc(sizeof(double) * N), *G = malloc(sizeof(double) * N);
    if (!c || !G) {
        free(c); free(G);
        return -1;
    }
    or_setup(g, v, c, G);
    int rc = forward_loop(g, c, G, wavelet, nt, src, nrec, rec, init_prev, init_cur, traces,
                          final_prev, final_cur, lap_hist);
    free(c); free(G);
    return rc;
}

/* or_forward with a caller-given damping field G (N values) in place of the
 * one built from the grid's band: the handle for pinning how the damping
 * enters the update (a spatially uniform G = g turns the scheme into the
 * undamped one for P^n / g^n). */
int or_forward_G(const or_grid *g, const float *v, const double *G, const float *wavelet, int64_t nt,
                 int64_t src, int64_t nrec, const int64_t *rec, const double *init_prev,
                 const double *init_cur, double *traces, double *final_prev, double *final_cur)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *c = malloc(sizeof(double) * N), *G0 = malloc(sizeof(double) * N);
    if (!c || !G0) {
        free(c); free(G0);
        return -1;
    }
    or_setup(g, v, c, G0);
    int rc = forward_loop(g, c, G, wavelet, nt, src, nrec, rec, init_prev, init_cur, traces,
                          final_prev, final_cur, NULL);
    free(c); free(G0);
    return rc;
}

/*
 * Exact discrete adjoint of or_forward with respect to c, then v.
 * With y^{n+1} the new field of step n, w^n the field after the source
 * addition, the forward map is y^{n+1} = G (2 + c L) w^n - G^2 w^{n-1} and
 * d^n = R y^{n+1}.  For symmetric L (zero or periodic edges), z^k = c G ybar^k
 * obeys
 *   z^k = G (2 z^{k+1} + c L z^{k+1}) - G^2 z^{k+2} + c G R^T r^{k-1},
 *   k = nt .. 1, z^{nt+1} = z^{nt+2} = 0,
 * and dJ/dc = sum_k (z^k / c) * L w^{k-1},  dJ/dv = dJ/dc * 2 c / v.
 * resid[n][r] = dJ/d traces[n][r].  Stores the whole forward history of
 * L w^n (nt * N doubles): for small and medium grids only.
 * grad_v and grad_c (either may be NULL) are overwritten.
 */
int or_adjoint(const or_grid *g, const float *v, const float *wavelet, int64_t nt,
               int64_t src, int64_t nrec, const int64_t *rec, const double *resid,
               double *grad_v, double *grad_c)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *hist = malloc(sizeof(double) * N * nt);
    double *c = malloc(sizeof(double) * N), *G = malloc(sizeof(double) * N);
    double *z1 = calloc(N, sizeof(double)), *z2 = calloc(N, sizeof(double));
    double *zk = malloc(sizeof(double) * N), *lapz = malloc(sizeof(double) * N);
    double *gc = calloc(N, sizeof(double));
    if (!hist || !c || !G || !z1 || !z2 || !zk || !lapz || !gc) {
        free(hist); free(c); free(G); free(z1); free(z2); free(zk); free(lapz); free(gc);
        return -1;
    }
    int rc = or_forward(g, v, wavelet, nt, src, nrec, rec, NULL, NULL, NULL, NULL, NULL, hist);
    if (rc == 0) {
        or_setup(g, v, c, G);
        for (int64_t k = nt; k >= 1; --k) {
            or_laplacian(g, z1, lapz);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i)
                zk[i] = G[i] * (2.0 * z1[i] + c[i] * lapz[i]) - G[i] * G[i] * z2[i];
            for (int64_t r = 0; r < nrec; ++r) {
                int64_t i = rec[r];
                zk[i] += c[i] * G[i] * resid[(k - 1) * nrec + r];
            }
            const double *lw = hist + (k - 1) * N;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) gc[i] += zk[i] / c[i] * lw[i];
            double *t = z2;
            z2 = z1;
            z1 = zk;
            zk = t;
        }
        for (int64_t i = 0; i < N; ++i) {
            if (grad_c) grad_c[i] = gc[i];
            if (grad_v) grad_v[i] = gc[i] * 2.0 * c[i] / (double)v[i];
        }
    }
    free(hist); free(c); free(G); free(z1); free(z2); free(zk); free(lapz); free(gc);
    return rc;
}

/*
 * Imaging condition (reverse-time migration of one shot).  The source
 * wavefield w^n (the field after the source addition of step n) is
 * correlated at zero lag with the receiver wavefield z^k, the z-form
 * adjoint field of or_adjoint driven by resid (the recorded data, or any
 * dJ/dtraces):
 *   image = sum_{k=1..nt} z^k * w^{k-1}.
 * It is dJ/dm for the spatial operator L -> L + diag(m) at m = 0 (a point
 * scatterer: the scheme becomes y = G (2 w + c (L w + m w)) - G^2 w_old), by
 * the same argument as dJ/dc with (L w) replaced by w.  Stores the whole
 * forward history (nt * N doubles).  image is overwritten.
 */
int or_image(const or_grid *g, const float *v, const float *wavelet, int64_t nt, int64_t src,
             int64_t nrec, const int64_t *rec, const double *resid, double *image)
{
    const int64_t N = g->nz * g->ny * g->nx;
    double *hist = malloc(sizeof(double) * N * nt);
    double *c = malloc(sizeof(double) * N), *G = malloc(sizeof(double) * N);
    double *prev = calloc(N, sizeof(double)), *cur = calloc(N, sizeof(double));
    double *nw = malloc(sizeof(double) * N), *lap = malloc(sizeof(double) * N);
    double *z1 = calloc(N, sizeof(double)), *z2 = calloc(N, sizeof(double));
    double *zk = malloc(sizeof(double) * N);
    if (!hist || !c || !G || !prev || !cur || !nw || !lap || !z1 || !z2 || !zk) {
        free(hist); free(c); free(G); free(prev); free(cur); free(nw); free(lap);
        free(z1); free(z2); free(zk);
        return -1;
    }
    or_setup(g, v, c, G);
    const double amp = source_amp(g);
    /* forward: keep w^n */
    for (int64_t n = 0; n < nt; ++n) {
        if (src >= 0) cur[src] += amp * (double)wavelet[n];
        memcpy(hist + n * N, cur, sizeof(double) * N);
        or_laplacian(g, cur, lap);
        for (int64_t i = 0; i < N; ++i)
            nw[i] = G[i] * (2.0 * cur[i] + c[i] * lap[i]) - G[i] * G[i] * prev[i];
        double *t = prev;
        prev = cur;
        cur = nw;
        nw = t;
    }
    /* backward: z-form adjoint recursion and the zero-lag correlation */
    for (int64_t i = 0; i < N; ++i) image[i] = 0.0;
    for (int64_t k = nt; k >= 1; --k) {
        or_laplacian(g, z1, lap);
        for (int64_t i = 0; i < N; ++i)
            zk[i] = G[i] * (2.0 * z1[i] + c[i] * lap[i]) - G[i] * G[i] * z2[i];
        for (int64_t r = 0; r < nrec; ++r) {
            const int64_t i = rec[r];
            zk[i] += c[i] * G[i] * resid[(k - 1) * nrec + r];
        }
        const double *w = hist + (k - 1) * N;
        for (int64_t i = 0; i < N; ++i) image[i] += zk[i] * w[i];
        double *t = z2;
        z2 = z1;
        z1 = zk;
        zk = t;
    }
    free(hist); free(c); free(G); free(prev); free(cur); free(nw); free(lap);
    free(z1); free(z2); free(zk);
    return 0;
}

/* ------------------------------------------------------------------------
 * 16-bit storage emulation: FP32 arithmetic, fields stored as IEEE binary16
 * or bfloat16 codes q with one power-of-two exponent e per stored field
 * (value = q * 2^e).  Rounding is round-to-nearest-even from the FP32 value.
 * ---------------------------------------------------------------------- */

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* binary32 -> binary16, round to nearest, ties to even (IEEE 754-2008). */
uint16_t or_f32_to_f16(float f)
{
    uint32_t u = f2u(f);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    int32_t exp = (int32_t)((u >> 23) & 0xFFu);
    uint32_t man = u & 0x7FFFFFu;
    if (exp == 0xFF) /* inf or NaN */
        return (uint16_t)(sign | 0x7C00u | (man ? 0x200u : 0u));
    int32_t e = exp - 127; /* unbiased */
    if (e > 15) return (uint16_t)(sign | 0x7C00u);
    /* Full significand with the implicit bit (normal inputs). */
    uint32_t sig = exp ? (man | 0x800000u) : man;
    int32_t shift; /* bits of sig dropped to reach a 10-bit half mantissa */
    uint32_t hexp;
    if (e >= -14) { /* normal half */
        shift = 13;
        hexp = (uint32_t)(e + 15);
        sig &= 0x7FFFFFu; /* implicit bit kept in hexp */
    } else {          /* subnormal half: value = m * 2^-24 */
        if (exp == 0) return sign; /* FP32 subnormals are far below 2^-25 */
        shift = 13 + (-14 - e);
        if (shift > 24) return sign;
        hexp = 0;
    }
    uint32_t kept = sig >> shift;
    uint32_t rem = sig & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1);
    if (rem > half || (rem == half && (kept & 1u))) kept += 1u;
    /* A mantissa carry rolls into the exponent field, which is exactly the
     * correctly rounded next binade (and the infinity code on overflow). */
    uint32_t out = (hexp << 10) + kept;
    return (uint16_t)(sign | out);
}

float or_f16_to_f32(uint16_t h)
{
    uint32_t sign = ((uint32_t)h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1Fu, m = h & 0x3FFu;
    if (e == 0x1F) return u2f(sign | 0x7F800000u | (m << 13));
    if (e == 0) return (sign ? -1.0f : 1.0f) * ldexpf((float)m, -24);
    return u2f(sign | ((e + 112u) << 23) | (m << 13));
}

/* binary32 -> bfloat16 (upper 16 bits), round to nearest, ties to even. */
uint16_t or_f32_to_bf16(float f)
{
    uint32_t u = f2u(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu))
        return (uint16_t)((u >> 16) | 0x40u); /* quiet NaN */
    uint32_t rem = u & 0xFFFFu, kept = u >> 16;
    if (rem > 0x8000u || (rem == 0x8000u && (kept & 1u))) kept += 1u;
    return (uint16_t)kept;
}

float or_bf16_to_f32(uint16_t b) { return u2f((uint32_t)b << 16); }

static uint16_t enc(int storage, float x) { return storage == 1 ? or_f32_to_f16(x) : or_f32_to_bf16(x); }
static float dec(int storage, uint16_t q) { return storage == 1 ? or_f16_to_f32(q) : or_bf16_to_f32(q); }

/* floor(log2(m)) - 11 for the largest magnitude m a field may reach; a floor
 * of 2^-100 stands in for an all-zero field. */
static int32_t storage_exponent(float m)
{
    float t = m > ldexpf(1.0f, -100) ? m : ldexpf(1.0f, -100);
    int ex;
    frexpf(t, &ex);
    return (int32_t)(ex - 1 - 11);
}

/* The integer nearest t >= 0, ties to even. */
static double rne(double t)
{
    double k = floor(t);
    double frac = t - k;
    if (frac > 0.5 || (frac == 0.5 && fmod(k, 2.0) != 0.0)) k += 1.0;
    return k;
}

/*
 * The model term c = (v dt/dh)^2 held as unsigned 16-bit fixed point with one
 * power-of-two scale (the 16-bit storage form's option to store the model in
 * 16 bits as well): with M the largest c, e is the least exponent for which
 * every code fits 16 bits, i.e. the one with 2^(e-1) <= M < 2^e, raised by
 * one when M 2^(16-e) rounds up to 2^16 (M within half a code of 2^e).  Each
 * code is the integer nearest c 2^(16-e) (ties to even) and stands for
 * code * 2^(e-16), so |c - code 2^(e-16)| <= 2^(e-17) for every cell.  The
 * rounding decision is taken on the FP32 value of c, as the kernels take it.
 * Writes the codes to q (may be NULL) and e to *e; replaces c by its decoded
 * value when `decode_in_place` is set.
 */
void or_c_fixed16(float *c, int64_t n, uint16_t *q, int32_t *e, int decode_in_place)
{
    float M = 0.0f;
    for (int64_t i = 0; i < n; ++i)
        if (c[i] > M) M = c[i];
    int ex = 0;
    frexpf(M, &ex); /* M = f 2^ex, 1/2 <= f < 1 */
    if (rne(ldexp((double)M, 16 - ex)) > 65535.0) ex += 1;
    *e = ex;
    for (int64_t i = 0; i < n; ++i) {
        double k = rne(ldexp((double)c[i], 16 - ex)); /* the product is exact */
        if (q) q[i] = (uint16_t)k;
        if (decode_in_place) c[i] = (float)ldexp(k, ex - 16);
    }
}

/*
 * The value a field holds once stored with exponent e: x itself in FP32
 * storage (storage 0), else the 16-bit code RNE16(x 2^-e) decoded and scaled
 * back by 2^e (exact: a power-of-two scale of a representable value).
 */
static float stored(int storage, float x, int32_t e)
{
    if (storage == 0) return x;
    return ldexpf(dec(storage, enc(storage, ldexpf(x, -e))), e);
}

/*
 * The reduced-precision forms of or_forward: arithmetic in FP32, the order of
 * the terms as in or_forward, fields stored in FP32 (storage 0: the scheme's
 * own FP32 rounding, nothing else) or in 16 bits (1 binary16, 2 bfloat16).
 * Per step n:
 *   cur, prev = the stored levels; lap = L(cur); x = G (2 cur + c lap) - G^2 prev;
 *   traces[n] sample x; x[src] += amp * s[n+1] (if n+1 < nt);
 *   e_new = floor(log2(max(M_cur, M_prev, |amp s[n+1]|))) - 11;
 *   store x (16-bit: q = RNE16(x * 2^-e_new)); M_new = max |x|.
 * The start state holds amp*s[0] at the source (stored the same way), so the
 * source addition happens once per level, as in or_forward.  Given
 * (init_prev, init_cur) instead, the start state is those FP32 fields, each
 * stored with exponent floor(log2 max|field|) - 11, and no s[0] is added.
 * c and G are the FP64 setup rounded to FP32, G as a product of FP32 axis
 * profiles (z, y, x order); with c_fixed16 set (16-bit fields only), c then
 * takes its 16-bit fixed-point value (or_c_fixed16).
 */
int or_forward_half(const or_grid *g, int storage, int c_fixed16, const float *v,
                    const float *wavelet, int64_t nt, int64_t src, int64_t nrec,
                    const int64_t *rec, const float *init_prev, const float *init_cur,
                    float *traces, float *final_cur)
{
    if (storage < 0 || storage > 2 || (storage == 0 && c_fixed16)) return -2;
    const int64_t N = g->nz * g->ny * g->nx;
    float *c = malloc(sizeof(float) * N), *G = malloc(sizeof(float) * N);
    float *cur = malloc(sizeof(float) * N), *prev = calloc(N, sizeof(float));
    float *lap = malloc(sizeof(float) * N), *x = malloc(sizeof(float) * N);
    double *gz = malloc(sizeof(double) * g->nz), *gy = malloc(sizeof(double) * g->ny);
    double *gx = malloc(sizeof(double) * g->nx);
    if (!c || !G || !cur || !prev || !lap || !x || !gz || !gy || !gx) {
        free(c); free(G); free(cur); free(prev); free(lap); free(x);
        free(gz); free(gy); free(gx);
        return -1;
    }
    const uint32_t f = g->sponge_faces;
    or_sponge_profile(g->nz, g->sponge_width, g->sponge_alpha, f & 1, (f >> 1) & 1, gz);
    if (g->ndim == 3)
        or_sponge_profile(g->ny, g->sponge_width, g->sponge_alpha, (f >> 2) & 1, (f >> 3) & 1, gy);
    else
        gy[0] = 1.0;
    or_sponge_profile(g->nx, g->sponge_width, g->sponge_alpha, (f >> 4) & 1, (f >> 5) & 1, gx);
    const double r = g->dt / g->dh;
    for (int64_t z = 0; z < g->nz; ++z)
        for (int64_t y = 0; y < g->ny; ++y)
            for (int64_t xx = 0; xx < g->nx; ++xx) {
                int64_t i = (z * g->ny + y) * g->nx + xx;
                double q = (double)v[i] * r;
                c[i] = (float)(q * q);
                G[i] = ((float)gz[z] * (float)gy[y]) * (float)gx[xx];
            }
    if (c_fixed16) {
        int32_t ec16;
        or_c_fixed16(c, N, NULL, &ec16, 1);
    }
    double a64[9];
    or_coefficients(g->radius, a64);
    float a[9];
    for (int k = 0; k <= g->radius; ++k) a[k] = (float)a64[k];
    const float amp = (float)source_amp(g);
    const int R = g->radius;

    /* start state: cur and prev hold the stored levels (prev starts at zero) */
    float Mc, Mp = 0.0f;
    if (init_cur || init_prev) {
        Mc = 0.0f;
        for (int64_t i = 0; i < N; ++i) {
            if (init_cur && fabsf(init_cur[i]) > Mc) Mc = fabsf(init_cur[i]);
            if (init_prev && fabsf(init_prev[i]) > Mp) Mp = fabsf(init_prev[i]);
        }
        const int32_t ec = storage_exponent(Mc), ep = storage_exponent(Mp);
        for (int64_t i = 0; i < N; ++i) {
            cur[i] = stored(storage, init_cur ? init_cur[i] : 0.0f, ec);
            prev[i] = stored(storage, init_prev ? init_prev[i] : 0.0f, ep);
        }
    } else {
        float x0 = (nt > 0 && src >= 0) ? amp * wavelet[0] : 0.0f;
        for (int64_t i = 0; i < N; ++i) cur[i] = 0.0f;
        if (src >= 0) cur[src] = stored(storage, x0, storage_exponent(fabsf(x0)));
        Mc = fabsf(x0);
    }
    for (int64_t n = 0; n < nt; ++n) {
        /* FP32 Laplacian, zero edges, same term order as or_laplacian. */
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < g->nz; ++z)
            for (int64_t y = 0; y < g->ny; ++y)
                for (int64_t xx = 0; xx < g->nx; ++xx) {
#define AT(zz, yy, xv) (((zz) < 0 || (zz) >= g->nz || (yy) < 0 || (yy) >= g->ny || (xv) < 0 || (xv) >= g->nx) \
                            ? 0.0f : cur[((zz) * g->ny + (yy)) * g->nx + (xv)])
                    float s = 0.0f;
                    s += a[0] * AT(z, y, xx);
                    for (int k = 1; k <= R; ++k) s += a[k] * (AT(z + k, y, xx) + AT(z - k, y, xx));
                    if (g->ndim == 3) {
                        s += a[0] * AT(z, y, xx);
                        for (int k = 1; k <= R; ++k) s += a[k] * (AT(z, y + k, xx) + AT(z, y - k, xx));
                    }
                    s += a[0] * AT(z, y, xx);
                    for (int k = 1; k <= R; ++k) s += a[k] * (AT(z, y, xx + k) + AT(z, y, xx - k));
#undef AT
                    lap[(z * g->ny + y) * g->nx + xx] = s;
                }
        for (int64_t i = 0; i < N; ++i)
            x[i] = G[i] * (2.0f * cur[i] + c[i] * lap[i]) - (G[i] * G[i]) * prev[i];
        if (traces)
            for (int64_t rr = 0; rr < nrec; ++rr) traces[n * nrec + rr] = x[rec[rr]];
        float inj = (n + 1 < nt && src >= 0) ? amp * wavelet[n + 1] : 0.0f;
        if (src >= 0) x[src] += inj;
        float m = Mc > Mp ? Mc : Mp;
        if (fabsf(inj) > m) m = fabsf(inj);
        const int32_t en = storage_exponent(m);
        float Mn = 0.0f;
        /* the new level is stored over prev, which becomes the current level */
        for (int64_t i = 0; i < N; ++i) {
            float ax = fabsf(x[i]);
            if (ax > Mn) Mn = ax;
            prev[i] = stored(storage, x[i], en);
        }
        float *t = prev;
        prev = cur;
        cur = t;
        Mp = Mc;
        Mc = Mn;
    }
    if (final_cur)
        for (int64_t i = 0; i < N; ++i) final_cur[i] = cur[i];
    free(c); free(G); free(cur); free(prev); free(lap); free(x);
    free(gz); free(gy); free(gx);
    return 0;
}

/* Vectorised conversions for the tests. */
void or_encode_array(int storage, const float *x, uint16_t *q, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) q[i] = enc(storage, x[i]);
}

void or_decode_array(int storage, const uint16_t *q, float *x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) x[i] = dec(storage, q[i]);
}
