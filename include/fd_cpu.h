/*
 * fd_cpu.h - the host (CPU) back-end of the finite-difference engine:
 * libfd_cpu.so, OpenMP threads over the cores and AVX2/AVX-512 vectors along
 * x.  It is the multi-core column of the paper's roofline comparison
 * (Section 7, the OpenMP back-end on a Xeon beside the GPUs) and the
 * "specialise the kernels for AVX" direction of its Discussion (Section 8).
 *
 * libfd_cpu.so exports every function of fd.h under the same name and with
 * the same arguments, so a program written against fd.h switches back-end by
 * linking (or loading) one library or the other.  It is a separate library:
 * nothing loads it implicitly, and the GPU library never falls back to it.
 *
 * What differs from fd.h:
 *   - every pointer fd.h calls "device" is ordinary host memory here (the
 *     caller still owns every buffer, sized by fd_query_bytes; buffers are
 *     256-byte aligned as in fd.h);
 *   - `stream` arguments are ignored and every call returns when its work is
 *     done;
 *   - built: fd_query_bytes, fd_create_model / fd_destroy_model,
 *     fd_create_state / fd_destroy_state, fd_begin_shot, fd_step,
 *     fd_run_shot (without checkpoints), fd_run_shots, fd_get_wavefield,
 *     fd_set_wavefield, fd_check_finite, fd_last_error, fd_version - the
 *     forward time loop of Listing 3 (Section 7) in 2D and 3D with FP32
 *     fields, radius 4, zero edges and the damping band; every other call,
 *     16-bit fields, 16-bit c, z-slabs and checkpoint buffers return
 *     FD_ERR_UNSUPPORTED;
 *   - the arithmetic is that of the GPU library's FP32 step, operation for
 *     operation (the same fused multiply-adds in the same order), so on the
 *     same inputs both give the same bits; the vector width does not change
 *     any result either.
 *
 * Layout (private, as in fd.h): each field carries a frame of zero cells (4
 * planes above and below, 4 rows on each y side in 3D, 16 cells left of each
 * row and at least 16 right of it) that the step reads as the zero edges and
 * never writes, so the inner loops have no bounds tests.
 */
#ifndef FD_CPU_H
#define FD_CPU_H

#include "fd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* OpenMP threads used by the steps: n >= 1 sets the count, n = 0 leaves it;
 * returns the count in effect (initially the OpenMP default, i.e.
 * OMP_NUM_THREADS or the cores this process may use). */
int32_t fd_cpu_threads(int32_t n);

/* Instruction set of the step loops: "avx512", "avx2" or "scalar".  The
 * best one the processor supports is chosen when the library loads;
 * fd_cpu_set_isa selects another by name (for tests: every choice gives the
 * same bits) and returns FD_ERR_UNSUPPORTED if this processor lacks it. */
const char *fd_cpu_isa(void);
fd_status fd_cpu_set_isa(const char *name);

/* Host memory bandwidth of the access pattern the step has: three FP32
 * streams read and one of them rewritten in place (p = 2 a + b p, 16 bytes
 * per element), over n_floats elements per stream (its own allocation, first
 * touched by the threads that use it), `reps` passes; *gbs receives the best
 * pass in GB/s (1e9 bytes).  The roof the step's bandwidth is measured
 * against.  FD_ERR_INVALID_ARG for n_floats < 1024, reps < 1 or NULL gbs;
 * FD_ERR_OUT_OF_MEMORY if the arrays cannot be allocated. */
fd_status fd_cpu_stream_probe(size_t n_floats, int32_t reps, double *gbs);

#ifdef __cplusplus
}
#endif

#endif /* FD_CPU_H */
