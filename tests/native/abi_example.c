/* A whole shot through the C ABI from plain C (C11), with device memory
 * from the HIP runtime API and no other layer: size query, model and state
 * creation in caller-owned buffers, fd_run_shot, the final wavefield read
 * back, handles destroyed, every status checked.
 *
 * Usage: abi_example <in.bin> <out.bin>
 *   in.bin:  int64 ndim, nz, ny, nx, nt, src_z, src_y, src_x, rec_z0,
 *            rec_x0, rec_nx, rec_dx; float64 dh, dt; then float32
 *            velocity[nz*ny*nx] and wavelet[nt]
 *   out.bin: float32 traces[nt][rec_nx], then P[nz*ny*nx]
 * Receivers: one row along x at depth rec_z0 (y = 0); no damping band. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "fd.h"

#define FD_OR_FAIL(call)                                                           \
    do {                                                                           \
        const fd_status st_ = (call);                                              \
        if (st_ != FD_OK) {                                                        \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, fd_last_error()); \
            return 1;                                                              \
        }                                                                          \
    } while (0)
#define HIP_OR_FAIL(call)                                                          \
    do {                                                                           \
        const hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));       \
            return 1;                                                              \
        }                                                                          \
    } while (0)

static int read_all(FILE *f, void *dst, size_t bytes)
{
    return fread(dst, 1, bytes, f) == bytes ? 0 : -1;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t h[12];
    double dhdt[2];
    if (read_all(in, h, sizeof h) || read_all(in, dhdt, sizeof dhdt)) return 2;
    const int64_t ncells = h[1] * h[2] * h[3], nt = h[4], nrec = h[10];
    float *v = malloc((size_t)ncells * sizeof(float));
    float *w = malloc((size_t)nt * sizeof(float));
    float *tr = malloc((size_t)(nt * nrec + ncells) * sizeof(float));
    if (!v || !w || !tr) return 2;
    if (read_all(in, v, (size_t)ncells * 4) || read_all(in, w, (size_t)nt * 4)) return 2;
    fclose(in);

    fd_grid g = {0};
    g.ndim = (int32_t)h[0];
    g.radius = 4;
    g.bc = FD_BC_ZERO;
    g.nz = h[1];
    g.ny = h[2];
    g.nx = h[3];
    g.dh = dhdt[0];
    g.dt = dhdt[1];
    g.storage = FD_F32;
    g.c_storage = FD_C_F32;

    fd_sizes sz;
    FD_OR_FAIL(fd_query_bytes(&g, nt, 0, &sz));
    void *model_buf = NULL, *state_buf = NULL;
    float *dv = NULL, *dw = NULL, *dtr = NULL, *dp = NULL;
    HIP_OR_FAIL(hipMalloc(&model_buf, sz.model));
    HIP_OR_FAIL(hipMalloc(&state_buf, sz.state));
    HIP_OR_FAIL(hipMalloc((void **)&dv, (size_t)ncells * 4));
    HIP_OR_FAIL(hipMalloc((void **)&dw, (size_t)nt * 4));
    HIP_OR_FAIL(hipMalloc((void **)&dtr, (size_t)(nt * nrec) * 4));
    HIP_OR_FAIL(hipMalloc((void **)&dp, (size_t)ncells * 4));
    HIP_OR_FAIL(hipMemcpy(dv, v, (size_t)ncells * 4, hipMemcpyHostToDevice));
    HIP_OR_FAIL(hipMemcpy(dw, w, (size_t)nt * 4, hipMemcpyHostToDevice));
    hipStream_t s;
    HIP_OR_FAIL(hipStreamCreate(&s));

    fd_model *m = NULL;
    fd_state *st = NULL;
    FD_OR_FAIL(fd_create_model(&g, dv, model_buf, sz.model, s, &m));
    FD_OR_FAIL(fd_create_state(m, state_buf, sz.state, &st));
    fd_shot shot = {0};
    shot.src_z = h[5];
    shot.src_y = h[6];
    shot.src_x = h[7];
    shot.wavelet = dw;
    shot.nt = nt;
    shot.rec.z0 = h[8];
    shot.rec.y0 = 0;
    shot.rec.x0 = h[9];
    shot.rec.nz = 1;
    shot.rec.ny = 1;
    shot.rec.nx = nrec;
    shot.rec.dz = 1;
    shot.rec.dy = 1;
    shot.rec.dx = h[11];
    FD_OR_FAIL(fd_run_shot(m, st, &shot, dtr, NULL, 0, 0, s));
    FD_OR_FAIL(fd_get_wavefield(st, 0, dp, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    HIP_OR_FAIL(hipMemcpy(tr, dtr, (size_t)(nt * nrec) * 4, hipMemcpyDeviceToHost));
    HIP_OR_FAIL(hipMemcpy(tr + nt * nrec, dp, (size_t)ncells * 4, hipMemcpyDeviceToHost));
    FD_OR_FAIL(fd_destroy_state(st));
    FD_OR_FAIL(fd_destroy_model(m));
    HIP_OR_FAIL(hipStreamDestroy(s));
    HIP_OR_FAIL(hipFree(model_buf));
    HIP_OR_FAIL(hipFree(state_buf));
    HIP_OR_FAIL(hipFree(dv));
    HIP_OR_FAIL(hipFree(dw));
    HIP_OR_FAIL(hipFree(dtr));
    HIP_OR_FAIL(hipFree(dp));

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    const size_t n = (size_t)(nt * nrec + ncells);
    if (fwrite(tr, sizeof(float), n, out) != n) return 2;
    fclose(out);
    free(v);
    free(w);
    free(tr);
    printf("abi_example: %s, version %s\n", "shot done", fd_version());
    return 0;
}
