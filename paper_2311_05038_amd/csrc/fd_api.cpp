// C ABI of the finite-difference engine: validation, buffer layouts, handle
// management and kernel dispatch.  Declarations and semantics: include/fd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fd.h"
#include "fd_host.hpp"
#include "fd_launch.hpp"

using fdk::StepArgs;
using namespace fdh;

namespace {

fd_status hip_fail(hipError_t e, const char *what)
{
    return fail(FD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
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
                              s->wavelet, s->nt, st->meta, stream);
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

const char *fd_last_error(void) { return last_error(); }

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
    m->amp = source_amp(*grid);

    // Damping profiles, FP64 on the host, stored FP32; a z-slab takes its
    // planes' factors from the whole grid's profile.
    const double alpha = m->grid.sponge_alpha;
    const int32_t W = m->grid.sponge_width;
    const uint32_t f = m->grid.sponge_faces;
    const std::vector<float> gzg = damping_profile(L.nzg, W, alpha, f & FD_FACE_ZLO, f & FD_FACE_ZHI);
    const std::vector<float> gz(gzg.begin() + L.z0, gzg.begin() + L.z0 + L.nz);
    const std::vector<float> gy = grid->ndim == 3 ? damping_profile(L.ny, W, alpha, f & FD_FACE_YLO, f & FD_FACE_YHI)
                                                  : std::vector<float>(1, 1.0f);
    const std::vector<float> gx = damping_profile(L.nx, W, alpha, f & FD_FACE_XLO, f & FD_FACE_XHI);

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
    st = check_stability(*grid, vmax);
    if (st != FD_OK) {
        delete m;
        return st;
    }
    if (fixed16) {
        const int ex = c16_exponent(vmax, grid->dt / grid->dh);
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
    // Settle, outside any stream capture, what later launches on this device
    // look up once and cache: the device address of the static routine work
    // area of fd_step_routines_noalloc, and the 3D launch plan's occupancy.
    // A failure here is left to the calls that need them, which report it.
    {
        void *area = nullptr;
        (void)fdk::routines_scratch(s, &area);
        StepArgs a = base_args(m, nullptr, nullptr);
        fdk::plan_tiles(a, L.ndim, L.storage, false);
        (void)hipGetLastError();
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

struct fd_shot_graph {
    hipGraphExec_t exec;
    fd_state *state;
    int64_t nt;
};

fd_status fd_shot_graph_create(const fd_model *model, fd_state *state, const fd_shot *shot, float *traces,
                               fd_shot_graph **out)
{
    if (!model || !state || !out) return fail(FD_ERR_INVALID_ARG, "NULL model, state or output handle");
    *out = nullptr;
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    if (is_slab(model->L)) return fail(FD_ERR_UNSUPPORTED, "a z-slab steps with fd_step and fd_slab_exchange");
    fd_shot_graph *h = new (std::nothrow) fd_shot_graph{};
    if (!h) return fail(FD_ERR_OUT_OF_MEMORY, "cannot allocate the graph handle");
    const int64_t next_before = state->next;  // recording advances the host counter only
    {
        // the tile plan of a 3D step asks the runtime for the kernel's
        // occupancy once per storage kind; ask before the capture starts
        int64_t skip = 0;
        StepArgs a = base_args(model, shot, &skip);
        fdk::plan_tiles(a, model->L.ndim, model->L.storage, false);
    }
    // The launches are recorded on a private stream (default priority) and
    // replayed on the caller's: the capture itself runs nothing.
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        if (cs) (void)hipStreamDestroy(cs);
        delete h;
        return hip_fail(e, "graph capture start");
    }
    st = do_begin(model, state, shot, cs);
    const int64_t nrec = nrec_of(shot);
    for (int64_t n = 0; st == FD_OK && n < shot->nt; ++n)
        st = do_step(model, state, shot, n, traces ? traces + (size_t)n * (size_t)nrec : nullptr, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);  // ends the capture whether or not recording succeeded
    if (st == FD_OK && e == hipSuccess) e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (st == FD_OK && e != hipSuccess) st = hip_fail(e, "graph capture");
    state->next = next_before;  // nothing ran on the device
    if (st != FD_OK) {
        delete h;
        return st;
    }
    h->state = state;
    h->nt = shot->nt;
    *out = h;
    return ok();
}

fd_status fd_shot_graph_launch(fd_shot_graph *g, void *stream)
{
    if (!g) return fail(FD_ERR_INVALID_ARG, "NULL graph");
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    g->state->next = g->nt;
    return ok();
}

fd_status fd_shot_graph_destroy(fd_shot_graph *g)
{
    if (g) (void)hipGraphExecDestroy(g->exec);
    delete g;
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

fd_status fd_check_finite(const fd_state *state, uint32_t *flags, void *stream)
{
    if (!state || !flags) return fail(FD_ERR_INVALID_ARG, "NULL state or flags");
    if ((uintptr_t)flags % 4) return fail(FD_ERR_INVALID_ARG, "flags must be 4-byte aligned");
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    const Layout &L = state->m->L;
    hipStream_t s = (hipStream_t)stream;
    // the owned cells of each level (padding included: it holds zeros)
    const size_t bytes = L.npad * L.elem;
    hipError_t e = fdk::launch_fill_u32(flags, 1, 0u, s);
    if (e == hipSuccess)
        e = fdk::launch_nonfinite(L.storage, state->buf[state->next & 1], bytes, flags, 1u,
                                  state->meta + fdk::kHealth, s);
    if (e == hipSuccess)
        e = fdk::launch_nonfinite(L.storage, state->buf[(state->next + 1) & 1], bytes, flags, 2u, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "fd_check_finite");
    return ok();
}

fd_status fd_stream_probe(int32_t kind, const float *a, const float *b, float *out, size_t n, void *stream)
{
    if (kind != 0 && kind != 1) return fail(FD_ERR_INVALID_ARG, "kind must be 0 (copy) or 1 (out = a + b * out)");
    if (n == 0) return ok();  // nothing to stream; the arrays are not examined
    if (!a || !out || (kind == 1 && !b)) return fail(FD_ERR_INVALID_ARG, "NULL array");
    if (n % 4) return fail(FD_ERR_INVALID_ARG, "n must be a multiple of 4");
    if ((uintptr_t)a % 16 || (uintptr_t)out % 16 || (kind == 1 && (uintptr_t)b % 16))
        return fail(FD_ERR_INVALID_ARG, "arrays must be 16-byte aligned");
    const hipError_t e = fdk::launch_stream_probe(kind, a, b, out, n, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fd_stream_probe");
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

}  // extern "C"

namespace {

fd_status step_routines(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                        float *trace_row, void *work, size_t work_bytes, bool static_work, hipStream_t s)
{
    if (!model || !state) return fail(FD_ERR_INVALID_ARG, "NULL model or state");
    if (state->m != model) return fail(FD_ERR_INVALID_ARG, "state was created for another model");
    fd_status st = check_shot(model, shot);
    if (st != FD_OK) return st;
    const Layout &L = model->L;
    if (L.storage != FD_F32) return fail(FD_ERR_UNSUPPORTED, "the routine-per-kernel step is built for FP32 fields only");
    if (is_slab(L)) return fail(FD_ERR_UNSUPPORTED, "the routine-per-kernel step is not built for z-slabs");
    const size_t need = (size_t)L.ndim * L.f32field;
    if (static_work) {
        if (need > fdk::kRoutinesScratchBytes)
            return fail(FD_ERR_INVALID_ARG,
                        "the grid's routine work (%zu bytes) exceeds the static work area (%zu bytes); "
                        "fd_step_routines takes a work buffer of any size",
                        need, fdk::kRoutinesScratchBytes);
    } else {
        if (!work) return fail(FD_ERR_INVALID_ARG, "work is NULL");
        if (work_bytes < need) return fail(FD_ERR_INVALID_ARG, "work holds %zu bytes, %zu needed", work_bytes, need);
    }
    if (state->next < 0) return fail(FD_ERR_INVALID_ARG, "fd_begin_shot has not been called");
    if (n != state->next) return fail(FD_ERR_INVALID_ARG, "step %lld requested, next step is %lld",
                                      (long long)n, (long long)state->next);
    if (n >= shot->nt) return fail(FD_ERR_INVALID_ARG, "step %lld beyond the shot's %lld steps",
                                   (long long)n, (long long)shot->nt);
    if (static_work) {
        const hipError_t e = fdk::routines_scratch(s, &work);
        if (e != hipSuccess) return hip_fail(e, "static work area of the routine step");
    }
    StepArgs a = base_args(model, shot);
    a.cur = state->buf[n & 1];
    a.prev = state->buf[(n + 1) & 1];
    a.n = n;
    a.trace_row = nrec_of(shot) > 0 ? trace_row : nullptr;
    char *w = (char *)work;
    float *dzz = (float *)w, *dxx = (float *)(w + L.f32field);
    float *dyy = L.ndim == 3 ? (float *)(w + 2 * L.f32field) : nullptr;
    hipError_t e = fdk::launch_routines(a, L.ndim, dzz, dxx, dyy, s);
    if (e != hipSuccess) return hip_fail(e, "routine kernels launch");
    state->next = n + 1;
    return ok();
}

}  // namespace

extern "C" {

fd_status fd_step_routines(const fd_model *model, fd_state *state, const fd_shot *shot, int64_t n,
                           float *trace_row, void *work, size_t work_bytes, void *stream)
{
    return step_routines(model, state, shot, n, trace_row, work, work_bytes, false, (hipStream_t)stream);
}

fd_status fd_step_routines_noalloc(const fd_model *model, fd_state *state, const fd_shot *shot,
                                   int64_t n, float *trace_row, void *stream)
{
    static_assert(fdk::kRoutinesScratchBytes == FD_ROUTINES_STATIC_BYTES, "static work area size");
    return step_routines(model, state, shot, n, trace_row, nullptr, 0, true, (hipStream_t)stream);
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
