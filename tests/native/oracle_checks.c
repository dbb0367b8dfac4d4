/* Drives every entry point of the oracle (oracle/fd_oracle.c) over small
 * grids and edge cases -- 2D and 3D, radius 1..8, zero and periodic edges,
 * with and without a damping band, no source, no receivers, one step,
 * receivers on the grid's corners, every storage form of the
 * reduced-precision emulation, the 16-bit c quantiser and the conversions
 * over all 16-bit codes -- so that AddressSanitizer and UBSan (the build of
 * tests/test_sanitize.py) see each loop and index computation run.  Checks
 * return codes and that results are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t ndim, radius, bc, sponge_width;
    int64_t nz, ny, nx;
    double dh, dt, sponge_alpha;
    uint32_t sponge_faces, pad_;
} or_grid;

void or_coefficients(int R, double *a);
void or_sponge_profile(int64_t n, int32_t width, double alpha, int lo, int hi, double *g);
void or_laplacian(const or_grid *g, const double *u, double *out);
void or_setup(const or_grid *g, const float *v, double *c, double *G);
int or_forward(const or_grid *g, const float *v, const float *wavelet, int64_t nt, int64_t src,
               int64_t nrec, const int64_t *rec, const double *init_prev, const double *init_cur,
               double *traces, double *final_prev, double *final_cur, double *lap_hist);
int or_forward_G(const or_grid *g, const float *v, const double *G, const float *wavelet, int64_t nt,
                 int64_t src, int64_t nrec, const int64_t *rec, const double *init_prev,
                 const double *init_cur, double *traces, double *final_prev, double *final_cur);
int or_adjoint(const or_grid *g, const float *v, const float *wavelet, int64_t nt, int64_t src,
               int64_t nrec, const int64_t *rec, const double *resid, double *grad_v, double *grad_c);
int or_image(const or_grid *g, const float *v, const float *wavelet, int64_t nt, int64_t src,
             int64_t nrec, const int64_t *rec, const double *resid, double *image);
uint16_t or_f32_to_f16(float f);
float or_f16_to_f32(uint16_t h);
uint16_t or_f32_to_bf16(float f);
float or_bf16_to_f32(uint16_t b);
void or_c_fixed16(float *c, int64_t n, uint16_t *q, int32_t *e, int decode_in_place);
int or_forward_half(const or_grid *g, int storage, int c_fixed16, const float *v, const float *wavelet,
                    int64_t nt, int64_t src, int64_t nrec, const int64_t *rec, const float *init_prev,
                    const float *init_cur, float *traces, float *final_cur);
void or_encode_array(int storage, const float *x, uint16_t *q, int64_t n);
void or_decode_array(int storage, const uint16_t *q, float *x, int64_t n);

static int failures = 0;
#define EXPECT(c)                                                                   \
    do {                                                                            \
        if (!(c)) {                                                                 \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

static int finite_d(const double *x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static int finite_f(const float *x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static uint64_t rng_state = 88172645463325252ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static void one_case(int ndim, int R, int bc, int width, int64_t nz, int64_t ny, int64_t nx, int64_t nt,
                     int with_src, int nrec_kind)
{
    or_grid g;
    memset(&g, 0, sizeof(g));
    g.ndim = ndim;
    g.radius = R;
    g.bc = bc;
    g.sponge_width = width;
    g.nz = nz;
    g.ny = ndim == 3 ? ny : 1;
    g.nx = nx;
    g.dh = 10.0;
    g.dt = 5e-4;
    g.sponge_alpha = width > 0 ? 0.3 / width : 0.0;
    g.sponge_faces = 0x3E;
    const int64_t N = g.nz * g.ny * g.nx;
    float *v = malloc(sizeof(float) * N), *wav = malloc(sizeof(float) * nt);
    for (int64_t i = 0; i < N; ++i) v[i] = (float)(1500.0 + 1500.0 * urand());
    for (int64_t n = 0; n < nt; ++n) wav[n] = (float)sin(0.3 * (double)n);
    const int64_t src = with_src ? N / 2 : -1;
    /* receivers: none, the four corners of the first and last plane, or all cells */
    int64_t nrec = nrec_kind == 0 ? 0 : (nrec_kind == 1 ? 4 : N);
    int64_t *rec = malloc(sizeof(int64_t) * (nrec > 0 ? nrec : 1));
    if (nrec_kind == 1) {
        rec[0] = 0;
        rec[1] = g.nx - 1;
        rec[2] = N - g.nx;
        rec[3] = N - 1;
    } else {
        for (int64_t i = 0; i < nrec; ++i) rec[i] = i;
    }
    double *traces = malloc(sizeof(double) * (nt * nrec + 1));
    double *prev = malloc(sizeof(double) * N), *cur = malloc(sizeof(double) * N);
    double *lap_hist = malloc(sizeof(double) * N * nt);
    EXPECT(or_forward(&g, v, wav, nt, src, nrec, rec, NULL, NULL, traces, prev, cur, lap_hist) == 0);
    EXPECT(finite_d(cur, N) && finite_d(prev, N) && finite_d(traces, nt * nrec) && finite_d(lap_hist, N * nt));
    /* restart from the final state with a caller-given G */
    double *G = malloc(sizeof(double) * N), *c = malloc(sizeof(double) * N);
    or_setup(&g, v, c, G);
    EXPECT(or_forward_G(&g, v, G, wav, nt, src, nrec, rec, prev, cur, traces, prev, cur) == 0);
    EXPECT(finite_d(cur, N));
    double *lap = malloc(sizeof(double) * N);
    or_laplacian(&g, cur, lap);
    EXPECT(finite_d(lap, N));
    if (bc == 0) {
        double *resid = malloc(sizeof(double) * (nt * nrec + 1));
        for (int64_t i = 0; i < nt * nrec; ++i) resid[i] = urand() - 0.5;
        double *gv = malloc(sizeof(double) * N), *gc = malloc(sizeof(double) * N), *img = malloc(sizeof(double) * N);
        EXPECT(or_adjoint(&g, v, wav, nt, src, nrec, rec, resid, gv, gc) == 0);
        EXPECT(or_adjoint(&g, v, wav, nt, src, nrec, rec, resid, NULL, gc) == 0);
        EXPECT(or_image(&g, v, wav, nt, src, nrec, rec, resid, img) == 0);
        EXPECT(finite_d(gv, N) && finite_d(gc, N) && finite_d(img, N));
        if (R == 4) {
            float *tr32 = malloc(sizeof(float) * (nt * nrec + 1)), *f32 = malloc(sizeof(float) * N);
            float *ip = malloc(sizeof(float) * N), *ic = malloc(sizeof(float) * N);
            for (int64_t i = 0; i < N; ++i) {
                ip[i] = (float)(urand() - 0.5);
                ic[i] = (float)(urand() - 0.5);
            }
            for (int storage = 0; storage <= 2; ++storage)
                for (int c16 = 0; c16 <= (storage ? 1 : 0); ++c16) {
                    EXPECT(or_forward_half(&g, storage, c16, v, wav, nt, src, nrec, rec, NULL, NULL, tr32, f32) == 0);
                    EXPECT(finite_f(f32, N) && finite_f(tr32, nt * nrec));
                    EXPECT(or_forward_half(&g, storage, c16, v, wav, nt, src, nrec, rec, ip, ic, tr32, f32) == 0);
                    EXPECT(or_forward_half(&g, storage, c16, v, wav, nt, src, nrec, rec, NULL, ic, NULL, NULL) == 0);
                }
            EXPECT(or_forward_half(&g, 0, 1, v, wav, nt, src, nrec, rec, NULL, NULL, tr32, f32) == -2);
            EXPECT(or_forward_half(&g, 3, 0, v, wav, nt, src, nrec, rec, NULL, NULL, tr32, f32) == -2);
            free(tr32); free(f32); free(ip); free(ic);
        }
        free(resid); free(gv); free(gc); free(img);
    }
    free(v); free(wav); free(rec); free(traces); free(prev); free(cur); free(lap_hist); free(G); free(c); free(lap);
}

int main(void)
{
    double a[9];
    for (int R = 1; R <= 8; ++R) {
        or_coefficients(R, a);
        double s = a[0];
        for (int k = 1; k <= R; ++k) s += 2.0 * a[k];
        EXPECT(fabs(s) < 1e-12);
    }
    double prof[70];
    for (int lo = 0; lo <= 1; ++lo)
        for (int hi = 0; hi <= 1; ++hi) {
            or_sponge_profile(70, 0, 0.0, lo, hi, prof);
            or_sponge_profile(70, 32, 0.3 / 32, lo, hi, prof);
            or_sponge_profile(1, 32, 0.3 / 32, lo, hi, prof);
            EXPECT(finite_d(prof, 1));
        }
    /* grids no wider than the stencil, radius 1..8, both edge kinds */
    for (int R = 1; R <= 8; ++R) {
        one_case(2, R, 0, 0, 3, 1, 5, 3, 1, 1);
        one_case(3, R, 1, 0, 4, 3, 2, 2, 1, 2);
    }
    one_case(2, 4, 0, 4, 17, 1, 23, 12, 1, 1);
    one_case(2, 4, 0, 0, 9, 1, 9, 1, 0, 0);      /* one step, no source, no receivers */
    one_case(3, 4, 0, 3, 11, 10, 13, 8, 1, 2);    /* every cell a receiver */
    one_case(3, 4, 1, 0, 12, 9, 10, 6, 1, 1);
    one_case(3, 4, 0, 2, 10, 9, 12, 5, 0, 1);
    /* the 16-bit c quantiser: an all-zero model, a constant one, a maximum
     * just under a power of two, random values */
    {
        float c[257];
        uint16_t q[257];
        int32_t e = 0;
        memset(c, 0, sizeof(c));
        or_c_fixed16(c, 257, q, &e, 1);
        for (int i = 0; i < 257; ++i) c[i] = 0.2f;
        or_c_fixed16(c, 257, q, &e, 1);
        for (int i = 0; i < 257; ++i) c[i] = (float)urand() * 0.25f;
        c[100] = nextafterf(0.5f, 0.0f);
        or_c_fixed16(c, 257, q, &e, 0);
        EXPECT(e == 0);   /* 0.5 - ulp is within half a code of 2^-1 at e = -1: next binade */
        or_c_fixed16(c, 257, NULL, &e, 1);
        EXPECT(finite_f(c, 257));
    }
    /* conversions over every 16-bit code and a spread of FP32 values */
    {
        for (uint32_t h = 0; h < 65536; ++h) {
            const float f = or_f16_to_f32((uint16_t)h), b = or_bf16_to_f32((uint16_t)h);
            if (isfinite(f)) EXPECT(or_f32_to_f16(f) == (uint16_t)h || f == 0.0f);
            if (isfinite(b)) EXPECT(or_f32_to_bf16(b) == (uint16_t)h || b == 0.0f);
        }
        float x[4096];
        uint16_t q[4096];
        for (int i = 0; i < 4096; ++i) x[i] = (float)((urand() - 0.5) * pow(10.0, 20.0 * urand() - 10.0));
        x[0] = INFINITY;
        x[1] = -INFINITY;
        x[2] = NAN;
        x[3] = 1e30f;
        for (int s = 1; s <= 2; ++s) {
            or_encode_array(s, x, q, 4096);
            or_decode_array(s, q, x, 4096);
        }
    }
    if (failures) {
        fprintf(stderr, "%d expectation(s) failed\n", failures);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
