/*
 * fd.h - C ABI of the MI355X (gfx950) finite-difference acoustic wave engine.
 *
 * The library advances the acoustic wave equation of arXiv 2311.05038,
 * Section 7, Eq. 1 (P_tt = v^2 (P_xx + P_zz) + S(t)), in 2D (z, x) and in 3D
 * (z, y, x), by explicit finite differences: one time step is the sequence
 * of Listing 3 (source addition to P, second derivatives along each axis,
 * time update to Pnew, rotation of Pold/P/Pnew), fused here into one kernel
 * per step.  Readings of what the paper leaves open:
 *   - second derivatives: 8th-order central weights (radius R = 4)
 *     a = (-205/72, 8/5, -1/5, 8/315, -1/560); taps outside the grid read 0;
 *   - one grid spacing dh on every axis (the paper's single dh); the
 *     velocity term c = (v dt / dh)^2;
 *   - the source adds dt^2 / dh^D * s[n] to one cell of P before the
 *     derivatives (S sits outside v^2 in Eq. 1);
 *   - damping band ("sponge"): new = G (2 P + c L P) - G^2 Pold, with
 *     G = gz(z) gy(y) gx(x), g(i) = exp(-(alpha d)^2) and d the distance
 *     into the band of an enabled face;
 *   - receivers sample the new field of each step before the next source
 *     addition: traces[n][r] = Pnew_n[cell r].
 *
 * Conventions.
 *   - Every function returns an fd_status; nothing throws across the ABI.
 *     A non-OK status leaves outputs untouched unless stated, and
 *     fd_last_error() gives a message (thread-local, valid until the next
 *     call on that thread).
 *   - "device" pointers are HIP device (HBM) addresses; "host" pointers are
 *     ordinary process memory.  The library never allocates device memory:
 *     the caller provides every buffer, sized by fd_query_bytes.  Handles
 *     (fd_model, fd_state) are small host objects owned by the library,
 *     released by the matching destroy call; they borrow the caller's
 *     device buffers, which must outlive them.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return without waiting, except fd_create_model, which
 *     waits for its own work (it reads the velocity range back).
 *   - Dense arrays that cross the ABI are row-major [nz][ny][nx] (ny = 1 in
 *     2D), x fastest, FP32 unless stated.  Internal buffers use a private
 *     padded layout and are only read or written through this API.
 *   - Work on one fd_state must stay on one stream; an fd_model may be used
 *     from several streams at once.
 */
#ifndef FD_H
#define FD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FD_OK = 0,
    FD_ERR_INVALID_ARG = 1,   /* null pointer, out-of-range size/index, buffer too small */
    FD_ERR_UNSTABLE = 2,      /* velocity/time step violate the stability bound */
    FD_ERR_OUT_OF_MEMORY = 3, /* host allocation of a handle failed */
    FD_ERR_DEVICE = 4,        /* a HIP call or kernel launch failed */
    FD_ERR_UNSUPPORTED = 5    /* valid request this library does not implement */
} fd_status;

typedef enum { FD_F32 = 0, FD_F16 = 1, FD_BF16 = 2 } fd_storage;
/* Storage of the model term c = (v dt / dh)^2.  FD_C_FIXED16 (with 16-bit
 * fields only) keeps c as unsigned 16-bit fixed point with one power-of-two
 * scale, q = RNE(c 2^(16-e)) with e = floor(log2 max c) + 1, raised by one
 * when max c lies within half a code of 2^e (so that every code fits 16
 * bits), so the step reads 8 bytes per cell instead of 10; |c - q 2^(e-16)|
 * is at most 2^(e-17) for every cell (c is first rounded to FP32 from the
 * FP64 product), a relative error of at most (max c / c) 2^-17 in c
 * (2^-16 in the raised case): 6.9e-5 for a 3:1 velocity contrast, 7.6e-4
 * for 10:1.  Models with far larger contrasts should keep FD_C_F32. */
typedef enum { FD_C_F32 = 0, FD_C_FIXED16 = 1 } fd_c_storage;
typedef enum { FD_BC_ZERO = 0, FD_BC_PERIODIC = 1 } fd_bc;

/* Sponge face bits. */
#define FD_FACE_ZLO 0x01u
#define FD_FACE_ZHI 0x02u
#define FD_FACE_YLO 0x04u
#define FD_FACE_YHI 0x08u
#define FD_FACE_XLO 0x10u
#define FD_FACE_XHI 0x20u

/* Largest batch accepted by fd_step_batch. */
#define FD_BATCH_MAX 16

/* The computational grid and its discretisation (Section 7: dh, dt). */
typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t radius;        /* stencil half-width; this library: 4 */
    int32_t bc;            /* fd_bc; this library: FD_BC_ZERO */
    int32_t sponge_width;  /* cells in the damping band, 0 = none */
    int64_t nz, ny, nx;    /* cells; ny must be 1 when ndim == 2 */
    double dh;             /* grid spacing, m (> 0) */
    double dt;             /* time step, s (> 0) */
    double sponge_alpha;   /* damping constant; <= 0 selects 0.3 / sponge_width */
    uint32_t sponge_faces; /* FD_FACE_* bits of the faces that damp */
    int32_t storage;       /* fd_storage of the wavefields (arithmetic is FP32) */
    int32_t c_storage;     /* fd_c_storage of c; FD_C_FIXED16 needs 16-bit fields */
    /* z-slab of a larger grid: one share of a model cut along z (the slow
     * axis) into consecutive slabs, each of which would sit on its own
     * device.  slab_nz_global = 0 (the default) means an ordinary grid.
     * Otherwise this grid is the planes [slab_z0, slab_z0 + nz) of a grid
     * of slab_nz_global planes with the same ny, nx, dh, dt and sponge:
     *  - the velocity given to fd_create_model covers the slab's nz planes;
     *  - the damping band is placed in global z (the slab's planes get the
     *    factors those planes have in the whole grid);
     *  - each stored level carries 4 ghost planes on either side, which the
     *    step reads (the stencil radius) and never writes; they are zero
     *    after fd_begin_shot and are refilled from the neighbouring slabs by
     *    fd_slab_exchange after fd_begin_shot, after fd_set_wavefield of P
     *    and after every step (ghosts beyond the global top and bottom stay
     *    zero: the grid's zero edges);
     *  - shot coordinates (source, receivers) are global: a slab adds the
     *    source only if it owns the source plane and writes only the trace
     *    entries of the receivers in its own planes;
     *  - fd_step, fd_begin_shot, fd_get_wavefield and fd_set_wavefield
     *    (owned planes only) work on slabs; the whole-shot, adjoint, image,
     *    batched and per-routine calls return FD_ERR_UNSUPPORTED.
     * Slabs need ndim = 3, FP32 fields and FP32 c, and nz >= 4.  Stepping
     * every slab of a grid with an exchange after each step gives the
     * whole-grid fd_step results bit for bit. */
    int64_t slab_z0;
    int64_t slab_nz_global;
} fd_grid;

/* A regular receiver array: cells (z0 + i*dz, y0 + j*dy, x0 + k*dx) for
 * i < nz, j < ny, k < nx; receiver r = (i*ny + j)*nx + k.  nz = ny = nx = 0
 * means no receivers.  Every cell must lie inside the grid (y0 = 0, ny = 1
 * in 2D). */
typedef struct {
    int64_t z0, y0, x0;
    int64_t nz, ny, nx;
    int64_t dz, dy, dx;
} fd_receivers;

/* One shot: a point source and its wavelet, plus the receivers. */
typedef struct {
    int64_t src_z, src_y, src_x; /* source cell (src_y = 0 in 2D) */
    const float *wavelet;        /* device, nt samples s[0..nt-1] (Eq. 1's S(t) at t = n dt) */
    int64_t nt;                  /* time steps of the shot (>= 1) */
    fd_receivers rec;
} fd_shot;

/* Device bytes the caller provides. */
typedef struct {
    size_t model;        /* fd_create_model's buffer */
    size_t state;        /* fd_create_state's buffer (two time levels) */
    size_t checkpoints;  /* fd_run_shot's checkpoint buffer for (nt, ckpt_every) */
    size_t adjoint_work; /* fd_adjoint_gradient's work buffer for ckpt_every */
    size_t routines_work; /* fd_step_routines' work buffer (ndim FP32 fields) */
} fd_sizes;

typedef struct fd_model fd_model;
typedef struct fd_state fd_state;

/* Bytes of every caller-provided buffer for this grid (Section 5, Start and
 * stop: the containers the algorithms work on live in the device memory
 * space and are filled from, and emptied to, the host by explicit copies;
 * here the caller allocates that device memory, so it needs the sizes).
 * nt and ckpt_every only affect `checkpoints` and `adjoint_work` (pass 0 to
 * skip them).  For a z-slab, `state` includes the ghost planes and the
 * buffers of the calls slabs do not support are 0.  Host-only; no device
 * work.  Errors: FD_ERR_INVALID_ARG for a NULL grid or out, an invalid grid
 * or negative nt / ckpt_every; FD_ERR_UNSUPPORTED for a valid grid this
 * library does not build (*out is then untouched). */
fd_status fd_query_bytes(const fd_grid *grid, int64_t nt, int32_t ckpt_every, fd_sizes *out);

/* Model setup (velocity V, dt, dh of Listing 3's WaveSimulator): computes
 * c = (v dt / dh)^2 and the damping profiles into `model_buf` (device,
 * >= fd_sizes.model bytes), then checks stability
 *     (vmax dt / dh)^2 * ndim * 6.5015873 <= 4
 * (the largest magnitude of the 8th-order second-difference symbol is
 * 4096/630), returning FD_ERR_UNSTABLE if it fails and FD_ERR_INVALID_ARG if
 * some velocity is not a positive finite number.  `velocity` is device,
 * dense FP32 m/s, read only during this call.  Synchronises `stream`. */
fd_status fd_create_model(const fd_grid *grid, const float *velocity, void *model_buf,
                          size_t model_bytes, void *stream, fd_model **out);
fd_status fd_destroy_model(fd_model *model);

/* Binds a state (the two time levels P and Pold of Listing 3's
 * WaveSimulator, Section 7) to `state_buf` (device, >= fd_sizes.state
 * bytes, 256-byte aligned, owned by the caller and borrowed until
 * fd_destroy_state): the device-resident container of Section 5 (Start and
 * stop).  Host-only; call fd_begin_shot (or fd_set_wavefield) before
 * stepping.  Errors: FD_ERR_INVALID_ARG for NULL arguments, a short or
 * misaligned buffer; FD_ERR_OUT_OF_MEMORY if the host handle cannot be
 * allocated. */
fd_status fd_create_state(const fd_model *model, void *state_buf, size_t state_bytes,
                          fd_state **out);
fd_status fd_destroy_state(fd_state *state);

/* Puts the state at rest and performs the first source addition
 * (P[src] = dt^2/dh^D * s[0]).  The next step is n = 0. */
fd_status fd_begin_shot(const fd_model *model, fd_state *state, const fd_shot *shot,
                        void *stream);

/* Time step n (must be the state's next step, 0 <= n < shot->nt): the
 * derivatives and time update of Listing 3 on P, then trace_row[r] =
 * Pnew[rec r] (device, nrec floats, or NULL), then the source addition of
 * step n+1 (none after the last step), then the rotation of levels.
 * fd_step n = 0..nt-1 after fd_begin_shot equals fd_run_shot bit for bit. */
fd_status fd_step(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                  float *trace_row, void *stream);

/* A whole shot: the time loop of Listing 3's run() (Section 7), i.e.
 * fd_begin_shot then steps 0..nt-1, all enqueued on `stream`.  traces:
 * device [nt][nrec] or NULL.  ckpt: device buffer of ckpt_bytes bytes (at
 * least fd_sizes.checkpoints for (nt, ckpt_every)), or NULL; when given,
 * the state before steps 0, K, 2K, ... (K = ckpt_every >= 1) is saved for
 * fd_adjoint_gradient.  Errors (nothing is enqueued): FD_ERR_INVALID_ARG for
 * NULL model/state/shot, a state of another model, an invalid shot, a short
 * or misaligned checkpoint buffer; FD_ERR_UNSUPPORTED on a z-slab;
 * FD_ERR_DEVICE if a launch fails (the state is then undefined). */
fd_status fd_run_shot(const fd_model *model, fd_state *state, const fd_shot *shot,
                      float *traces, void *ckpt, size_t ckpt_bytes, int32_t ckpt_every,
                      void *stream);

/* A recorded shot: the launches of fd_run_shot (without checkpoints) for
 * one (model, state, shot, traces) captured once into a HIP graph, so that
 * a shot on a grid too small to fill the GPU pays one graph launch instead
 * of one kernel launch per step.  Section 7's roofline places the step at
 * the memory bound; on small grids (e.g. 256^2) a step streams its bytes in
 * less time than a kernel launch takes, and the launches, not the memory,
 * set the pace.  Opaque handle. */
typedef struct fd_shot_graph fd_shot_graph;

/* Records fd_begin_shot and steps 0..nt-1 of `shot` on (model, state), with
 * trace rows written to `traces` (device [nt][nrec], or NULL), into a graph
 * and instantiates it.  Nothing runs on the device, and the state's step
 * counter is left as it was.  The graph keeps addresses, not contents:
 * every launch reads the model's buffer and the shot's wavelet as they are
 * then, and rewrites the state and `traces`; the fd_shot struct itself
 * (source cell, receivers, nt, wavelet address) is read only here.  The
 * model and state handles, their buffers, the wavelet and `traces` must
 * outlive the graph.  Errors (nothing recorded): FD_ERR_INVALID_ARG for NULL
 * arguments, a state of another model or an invalid shot; FD_ERR_UNSUPPORTED
 * on a z-slab; FD_ERR_DEVICE if the capture or instantiation fails;
 * FD_ERR_OUT_OF_MEMORY for the host handle. */
fd_status fd_shot_graph_create(const fd_model *model, fd_state *state, const fd_shot *shot, float *traces,
                               fd_shot_graph **out);

/* Enqueues the recorded shot on `stream`: the same work as fd_run_shot(model,
 * state, shot, traces, NULL, 0, 0, stream), with the same bits.  Afterwards
 * the state's next step is nt.  Launches that use one state must be ordered
 * (they rewrite it).  Errors: FD_ERR_INVALID_ARG for NULL; FD_ERR_DEVICE if
 * the launch fails. */
fd_status fd_shot_graph_launch(fd_shot_graph *graph, void *stream);
fd_status fd_shot_graph_destroy(fd_shot_graph *graph);

/* Exact discrete adjoint of fd_run_shot: accumulates into grad_v (device,
 * dense FP64, +=) the gradient dJ/dv of a scalar J of the traces, given
 * adj = dJ/dtraces (device FP32 [nt][nrec]) and the checkpoints fd_run_shot
 * saved for this model and shot with the same ckpt_every (ckpt_bytes as
 * given to fd_run_shot).  Each checkpoint
 * segment is recomputed, then the adjoint field is stepped backward:
 *   z^k = G (2 z^{k+1} + c L z^{k+1}) - G^2 z^{k+2} + c G R^T adj[k-1],
 *   dJ/dc += z^k / c * L(P^{k-1}),   dJ/dv = dJ/dc * 2 c / v,
 * with the time sum accumulated in FP64 on the device.
 * work: device, >= fd_sizes.adjoint_work bytes.  FP32 storage only. */
fd_status fd_adjoint_gradient(const fd_model *model, const fd_shot *shot, const float *adj,
                              const void *ckpt, size_t ckpt_bytes, int32_t ckpt_every,
                              void *work, size_t work_bytes, double *grad_v, void *stream);

/* Reverse-time-migration image of one shot (the imaging use the paper
 * names for this solver in its Discussion, Section 8): accumulates into image (device, dense
 * FP64, +=) the zero-lag correlation of the source wavefield w^n (the
 * field after the source addition of step n, recomputed from the
 * checkpoints) with the receiver wavefield z^k back-propagated from `data`
 * (device FP32 [nt][nrec]: the recorded traces, or any dJ/dtraces) by the
 * recursion of fd_adjoint_gradient:
 *   image += sum_{k=1..nt} z^k * w^{k-1}.
 * This is dJ/dm for J = <data, traces> with the spatial operator L
 * replaced by L + diag(m) (a field of point scatterers) at m = 0.  Same
 * checkpoints, ckpt_every, work buffer (fd_sizes.adjoint_work) and errors
 * as fd_adjoint_gradient.  FP32 storage only. */
fd_status fd_rtm_image(const fd_model *model, const fd_shot *shot, const float *data,
                       const void *ckpt, size_t ckpt_bytes, int32_t ckpt_every, void *work,
                       size_t work_bytes, double *image, void *stream);

/* Several shots on one model at once (the shots of one survey: a
 * gradient or an image sums over them).  `count` entries in each array;
 * all shots share nt.  In 2D with FP32 storage every time step of all the
 * shots is one launch of the batched step kernel (groups of FD_BATCH_MAX),
 * which keeps the device full on grids too small to fill it alone; otherwise
 * the shots run one after another.  Per shot, the results are those of the
 * single-shot call, bit for bit:
 *   fd_run_shots               = fd_run_shot on each (states[i], shots[i],
 *                                traces[i], ckpt[i]); traces or ckpt (the
 *                                arrays or entries) may be NULL.
 *   fd_adjoint_gradient_shots  = fd_adjoint_gradient on each shot in turn
 *                                (grad_v += shot 0, then shot 1, ...).
 *   fd_rtm_image_shots         = fd_rtm_image on each shot in turn.
 * Every shot needs its own state, checkpoint buffer and work buffer
 * (sizes as for the single-shot calls); 1 <= count <= 4096. */
fd_status fd_run_shots(const fd_model *model, fd_state *const *states, const fd_shot *const *shots,
                       int32_t count, float *const *traces, void *const *ckpt, size_t ckpt_bytes,
                       int32_t ckpt_every, void *stream);
fd_status fd_adjoint_gradient_shots(const fd_model *model, const fd_shot *const *shots,
                                    int32_t count, const float *const *adj,
                                    const void *const *ckpt, size_t ckpt_bytes, int32_t ckpt_every,
                                    void *const *work, size_t work_bytes, double *grad_v,
                                    void *stream);
fd_status fd_rtm_image_shots(const fd_model *model, const fd_shot *const *shots, int32_t count,
                             const float *const *data, const void *const *ckpt, size_t ckpt_bytes,
                             int32_t ckpt_every, void *const *work, size_t work_bytes,
                             double *image, void *stream);

/* Copies P (which = 0) or Pold (which = 1) of the state, decoded to FP32,
 * into `out` (device, dense [nz][ny][nx], caller-owned): the "get" accessor
 * of Listing 3's WaveSimulator (Section 7) and the first half of how an
 * application ends in Section 5 (Start and stop: results leave the device
 * container through an explicit copy; the caller then copies `out` to the
 * host).  After k steps P holds the new field of step k-1 plus the source
 * addition of step k (none after the last step, so after a whole shot it is
 * the final wavefield).  Stream-ordered.  Errors: FD_ERR_INVALID_ARG for
 * NULL arguments, `which` not 0 or 1, or a state that has not begun a shot;
 * FD_ERR_DEVICE if the copy kernel fails to launch. */
fd_status fd_get_wavefield(const fd_state *state, int32_t which, float *out, void *stream);

/* Sets P (which = 0) or Pold (which = 1) of the state from `in` (device,
 * dense FP32 [nz][ny][nx]): the "set" accessor beside fd_get_wavefield
 * (Listing 3's WaveSimulator exposes set/get methods).  With 16-bit storage
 * the level's scale is 2^(floor(log2 max|in|) - 11) and the values are
 * rounded to nearest even.  On a state that has not begun a shot, the state
 * is first put at rest with next step 0.  No source addition is made.
 * Resuming a shot: a shot stopped after k steps (P and Pold read with
 * fd_get_wavefield) continues on a fresh state given both levels here, with
 * a shot whose wavelet starts at sample k (its step n is step k + n of the
 * original, trace row n is row k + n); with FP32 storage the continuation
 * equals the uninterrupted shot bit for bit (16-bit storage re-derives the
 * levels' scales from their values). */
fd_status fd_set_wavefield(fd_state *state, int32_t which, const float *in, void *stream);

/* Health of a shot.  Writes *flags (device, one 4-byte-aligned uint32):
 * bit 0 set if the state's P holds a non-finite value (NaN or infinity),
 * bit 1 if its Pold does (on a z-slab: the owned planes), bit 2 if a
 * non-finite value entered the shot (one of the nt values amp * s[n] the
 * shot injects, found when fd_begin_shot runs, or a value given to
 * fd_set_wavefield); 0 for a healthy shot.  Stream-ordered like the steps,
 * so after fd_run_shot it reports on the finished shot.  A non-finite value
 * never becomes finite again under the update of Eq. 1 (it, or a non-finite
 * stencil neighbour, makes the new value non-finite; the grid's edges and
 * padding hold zeros; 16-bit codes decode exactly, non-finite ones
 * included), so bits 0 and 1 after the last step cover every step, overflow
 * included (16-bit fields keep 16x headroom in their storage scale, so the
 * scheme itself cannot overflow them).  A shot corrupted this way is
 * reported here instead of ending with FD_OK and meaningless traces.  Cost:
 * one read of the two levels (8 bytes per cell with FP32 fields).  Errors:
 * FD_ERR_INVALID_ARG for NULL or misaligned arguments or a state that has
 * not begun a shot. */
fd_status fd_check_finite(const fd_state *state, uint32_t *flags, void *stream);

/* Refreshes the ghost planes between two neighbouring slabs of one grid
 * (see fd_grid: `upper` owns the planes just above `lower`'s, i.e.
 * upper's slab_z0 + nz == lower's slab_z0): the current level P's last 4
 * owned planes of `upper` go into `lower`'s 4 leading ghost planes, and
 * lower's first 4 owned planes into upper's 4 trailing ghost planes.  Both
 * states must have begun the same shot and be at the same next step.  With
 * one device per slab this is the per-step halo exchange between
 * neighbouring devices; here both states are on the current device and the
 * planes move by two device-to-device copies on `stream` (2 x 4 planes of
 * ny * ceil(nx / 64) * 64 FP32 cells).  Stream-ordered; nothing else is
 * changed. */
fd_status fd_slab_exchange(const fd_state *upper, const fd_state *lower, void *stream);

/* One batch entry for fd_step_batch: a shot in flight with its own model,
 * state and next step n; traces is device [nt][nrec] or NULL (row n is
 * written). */
typedef struct {
    const fd_model *model;
    fd_state *state;
    const fd_shot *shot;
    int64_t n;
    float *traces;
} fd_batch_item;

/* Advances every item by up to `nsteps` steps with ONE kernel launch per
 * step covering all items (continuous batching of shots on grids of
 * different sizes).  An item stops at its last step; items[i].n is updated
 * (host) to the next step of each item.  Results equal fd_step on each
 * item alone, bit for bit.  2D, FP32 storage, count <= FD_BATCH_MAX. */
fd_status fd_step_batch(fd_batch_item *items, int32_t count, int32_t nsteps, void *stream);

/* Time step n computed as Listing 3 lays it out, one kernel per routine:
 * fd_pzz (the second difference of P along z into a Pzz field), fd_pxx
 * (along x, into Pxx), in 3D the same along y (Pyy), fd_time (Pnew =
 * G (2 P + c (Pzz + Pyy + Pxx)) - G^2 Pold over Pold, receivers sampled into
 * trace_row as in fd_step), add_source (the source addition of step n+1
 * into Pnew), then the rotation.  The derivative fields live in `work`
 * (device, >= fd_sizes.routines_work bytes, contents undefined on return).
 * Same preconditions and the same results as fd_step, bit for bit; it moves
 * 40 (2D) or 52 (3D) bytes per cell instead of 16.  It exists to measure the
 * routines one by one against the fused step.  FP32 storage only
 * (FD_ERR_UNSUPPORTED otherwise). */
fd_status fd_step_routines(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                           float *trace_row, void *work, size_t work_bytes, void *stream);

/* FD_ROUTINES_STATIC_BYTES: the size of the library's static work area. */
#define FD_ROUTINES_STATIC_BYTES ((size_t)64 << 20)

/* fd_step_routines for callers that cannot allocate device memory (code
 * under stream or graph capture, serving loops that forbid allocation,
 * harnesses without an allocator): the derivative fields live in a work
 * area of FD_ROUTINES_STATIC_BYTES (64 MiB) that the library holds in each
 * GPU's memory from the time it is loaded until the process ends, instead of
 * a `work` argument.  Nothing is allocated or freed: its address on a
 * device is looked up once and kept, by fd_create_model on that device (so
 * before a capture that uses the model) or else by the first call that
 * needs it.  Grids whose routine work (fd_sizes.routines_work: ndim padded FP32
 * fields) exceeds the area are rejected with FD_ERR_INVALID_ARG before any
 * launch (e.g. 2D up to 2048 x 4096, 3D up to about 5.5 M padded cells).
 * Every call on one GPU shares that GPU's area: calls that overlap on one
 * GPU (different streams, or threads without ordering) race and give
 * undefined results; calls ordered on one stream are safe.  The area starts
 * undefined and nothing in it needs clearing (every step rewrites what it
 * reads).  Otherwise identical to fd_step_routines, bit for bit. */
fd_status fd_step_routines_noalloc(const fd_model *model, fd_state *state, const fd_shot *shot,
                                   int64_t n, float *trace_row, void *stream);

/* The practical memory roof the step kernels are measured against (the
 * role the measured stream bandwidth plays under the roofline of Section
 * 7): streams n floats through HBM with no stencil, kind 0 a copy (out = a;
 * 8 bytes per element) and kind 1 the FP32 step's access pattern (out = a +
 * b * out: three streams read and one of them rewritten in place; 16 bytes
 * per element), each in the configuration of its access pattern that
 * streams fastest on gfx950 (non-temporal stores; non-temporal loads for
 * kind 1, as in the step kernels).  a, b, out: device, 16-byte
 * aligned (b unused by kind 0), n a multiple of 4; n = 0 launches nothing
 * and the arrays are not examined (they may be NULL).  Stream-ordered; the
 * caller times it with events on `stream`.  Errors: FD_ERR_INVALID_ARG for
 * an unknown kind, NULL or misaligned arrays or n not a multiple of 4. */
fd_status fd_stream_probe(int32_t kind, const float *a, const float *b, float *out, size_t n, void *stream);

/* Message for the last non-OK status on this thread ("" if none): the error
 * side of the host/device boundary of Section 5 (Start and stop), across
 * which every call above reports a status instead of throwing.  The string
 * is owned by the library and valid until the next call on this thread. */
const char *fd_last_error(void);

/* Library version string. */
const char *fd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
