// Resident context (hs_ctx) and the continuous-batching serving loop
// (hs_server) for many k-points of one atom set.
//
// The context keeps the k-independent part of Alg. 1 on the device: the
// per-atom Cholesky factors / failure flags and operand forms (M1, M2), the
// per-row metadata of the reductions, and a copy of T^AB. One k-point then
// costs the per-atom products and the two reductions only.
//
// The server owns one device arena and n_slots HIP streams (default
// priority). Requests are admitted when a slot is free and their footprint
// fits in the arena (first fit over a free list), in arrival order or, with
// the bypass policy, letting later requests that fit pass a waiting one a
// bounded number of times (serving_sched.h); each admitted request copies its
// A, B (2-D copies from the caller's host rows), builds on its slot's stream,
// and a host callback on that stream stamps the completion time. Results
// stay in the arena until released.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/hs_build.h"
#include "hs_internal.h"
#include "serving_sched.h"

struct hs_ctx {
    hs::AtomPlan plan;
    char *mem = nullptr;          // atom buffers, then the T^AB copy
    hs::AtomBufs ab;
    double2 *T_AB = nullptr;
    int device = 0;
};

namespace {

using hs::serve::align_up;

size_t footprint(const hs::AtomPlan &p, int n_g, int mode) {
    const size_t ab = align_up(16 * (size_t)p.K * (size_t)n_g);
    const size_t hs = align_up(16 * (size_t)n_g * (size_t)n_g);
    return 2 * ab + 2 * hs + p.kpoint_bytes(n_g, mode);
}

}  // namespace

extern "C" {

int hs_ctx_create(const hs_complex *T_AA, const hs_complex *T_AB, const hs_complex *T_BB,
                  const hs_complex *U, int N_A, int N_L, const int32_t *nl_per_atom,
                  void *stream, hs_ctx **out) {
    if (!T_AA) return -1;
    if (!T_AB) return -2;
    if (!T_BB) return -3;
    if (!U) return -4;
    if (N_A < 1) return -5;
    if (!nl_per_atom && (N_L < 1 || N_L > HS_MAX_NL)) return -6;
    if (!out) return -9;
    *out = nullptr;
    std::unique_ptr<hs_ctx> c(new hs_ctx);
    if (c->plan.make(N_A, nl_per_atom, N_L) != 0) return nl_per_atom ? -7 : -6;
    int rc = hs::check_device();
    if (rc != HS_OK) return rc;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return hs::hip_fail(e, "hipGetDevice");
    const size_t abytes = c->plan.atom_bytes();
    const size_t tbytes = 16 * (size_t)c->plan.t_total;
    e = hipMalloc(&c->mem, abytes + tbytes);
    if (e == hipErrorOutOfMemory) {
        hs::set_error(HS_ERR_NOMEM, "context allocation");
        return HS_ERR_NOMEM;
    }
    if (e != hipSuccess) return hs::hip_fail(e, "hipMalloc");
    c->ab.carve(c->plan, c->mem);
    c->T_AB = reinterpret_cast<double2 *>(c->mem + abytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(c->T_AB, T_AB, tbytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hs::enqueue_atoms(c->plan, c->ab, reinterpret_cast<const double2 *>(T_AA),
                              reinterpret_cast<const double2 *>(T_BB),
                              reinterpret_cast<const double2 *>(U), nullptr, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(c->mem);
        return hs::hip_fail(e, "context preparation");
    }
    *out = c.release();
    return HS_OK;
}

int hs_ctx_rows(const hs_ctx *ctx) { return ctx ? ctx->plan.K : 0; }

int hs_ctx_info(const hs_ctx *ctx, int32_t *info_host) {
    if (!ctx) return -1;
    if (!info_host) return -2;
    hipError_t e = hipMemcpy(info_host, ctx->ab.info, sizeof(int32_t) * ctx->plan.n_atoms,
                             hipMemcpyDeviceToHost);
    return e == hipSuccess ? HS_OK : hs::hip_fail(e, "hs_ctx_info");
}

size_t hs_ctx_workspace_bytes(const hs_ctx *ctx, int N_G, int mode) {
    if (!ctx || N_G < 1 || !hs::valid_mode(mode)) return 0;
    return ctx->plan.kpoint_bytes(N_G, mode);
}

size_t hs_ctx_footprint_bytes(const hs_ctx *ctx, int N_G, int mode) {
    if (!ctx || N_G < 1 || !hs::valid_mode(mode)) return 0;
    return footprint(ctx->plan, N_G, mode);
}

int hs_ctx_build(const hs_ctx *ctx, const hs_complex *A, const hs_complex *B, int N_G,
                 hs_complex *H, hs_complex *S, const hs_options *opt) {
    if (!ctx) return -1;
    if (!A) return -2;
    if (!B) return -3;
    if (N_G < 1) return -4;
    if (!H) return -5;
    if (!S) return -6;
    if (!opt || !hs::valid_mode(opt->mode) || (opt->batch != 0 && opt->batch != 1)) return -7;
    if (opt->batch && !hs::BatchPlan::valid(ctx->plan, opt->tuning ? opt->tuning->cfg : nullptr))
        return -7;
    if (!opt->workspace || opt->workspace_bytes < ctx->plan.kpoint_bytes(N_G, opt->mode)) {
        hs::set_error(HS_ERR_WORKSPACE, "workspace too small: the k-point needs " +
                      std::to_string(ctx->plan.kpoint_bytes(N_G, opt->mode)) + " bytes, " +
                      std::to_string(opt->workspace ? opt->workspace_bytes : 0) + " given");
        return HS_ERR_WORKSPACE;
    }
    hipStream_t st = static_cast<hipStream_t>(opt->stream);
    hipEvent_t ev[HS_NUM_PHASE_EVENTS] = {};
    if (opt->phase_events)
        for (int i = 0; i < HS_NUM_PHASE_EVENTS; ++i)
            ev[i] = static_cast<hipEvent_t>(opt->phase_events[i]);
    hipError_t e;
    if (ev[0] && (e = hipEventRecord(ev[0], st)) != hipSuccess) return hs::hip_fail(e, "phase event");
    hs::KpointBufs kb;
    kb.carve(ctx->plan, N_G, opt->mode, static_cast<char *>(opt->workspace));
    hs::AtomStage stage;   // batched: products only, the preparation is cached
    stage.batch = opt->batch != 0;
    stage.cfg = opt->tuning ? opt->tuning->cfg : nullptr;
    e = hs::enqueue_kpoint(ctx->plan, ctx->ab, N_G, opt->mode, reinterpret_cast<const double2 *>(A),
                           reinterpret_cast<const double2 *>(B), ctx->T_AB, kb,
                           reinterpret_cast<double2 *>(H), reinterpret_cast<double2 *>(S), st, ev,
                           stage);
    return e == hipSuccess ? HS_OK : hs::hip_fail(e, "hs_ctx_build launch");
}

void hs_ctx_destroy(hs_ctx *ctx) {
    if (!ctx) return;
    if (ctx->mem) (void)hipFree(ctx->mem);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Server: the device side of the serving loop. Admission, the arena's free
// list and the completion bookkeeping are serving_sched.h's Scheduler; this
// part copies an admitted request's inputs, enqueues its build on its slot's
// stream and stamps its completion from a host callback on that stream.

namespace {

using Clock = std::chrono::steady_clock;

struct Live : hs::serve::Request {
    hs_request req;
    Clock::time_point epoch;
};

void on_done(void *p) {
    Live *l = static_cast<Live *>(p);
    l->finish(std::chrono::duration<double>(Clock::now() - l->epoch).count());
}

}  // namespace

struct hs_server {
    hs_ctx *ctx = nullptr;
    int mode = HS_FP64;
    char *arena_mem = nullptr;
    std::unique_ptr<hs::serve::Scheduler> sched;
    std::vector<hipStream_t> streams;
    Clock::time_point epoch;
    double now() const { return std::chrono::duration<double>(Clock::now() - epoch).count(); }
};

namespace {

// Device addresses of an admitted request's A, B, H, S and workspace.
struct Placement {
    hs_complex *A, *B, *H, *S;
    char *ws;
};
Placement place(const hs_server *s, const Live *l) {
    const hs::AtomPlan &p = s->ctx->plan;
    const int n_g = l->req.N_G;
    char *base = s->arena_mem + l->off;
    const size_t ab = align_up(16 * (size_t)p.K * (size_t)n_g);
    const size_t hsz = align_up(16 * (size_t)n_g * (size_t)n_g);
    return {reinterpret_cast<hs_complex *>(base), reinterpret_cast<hs_complex *>(base + ab),
            reinterpret_cast<hs_complex *>(base + 2 * ab),
            reinterpret_cast<hs_complex *>(base + 2 * ab + hsz), base + 2 * ab + 2 * hsz};
}

// Launch one admitted request on its slot; returns a status. On failure the
// slot's stream is drained first, so nothing of the request is still running.
int launch(hs_server *s, Live *l) {
    const hs::AtomPlan &p = s->ctx->plan;
    const int n_g = l->req.N_G;
    const Placement d = place(s, l);
    hipStream_t st = s->streams[l->slot];
    const size_t row = 16 * (size_t)n_g, pitch = 16 * (size_t)l->req.ld;
    int rc = HS_OK;
    hipError_t e = hipMemcpy2DAsync(d.A, row, l->req.A_host, pitch, row, p.K, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(d.B, row, l->req.B_host, pitch, row, p.K, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = hs::hip_fail(e, "request input copy");
    if (rc == HS_OK) {
        hs_options opt;
        std::memset(&opt, 0, sizeof(opt));
        opt.stream = st;
        opt.workspace = d.ws;
        opt.workspace_bytes = p.kpoint_bytes(n_g, s->mode);
        opt.mode = s->mode;
        rc = hs_ctx_build(s->ctx, d.A, d.B, n_g, d.H, d.S, &opt);
    }
    if (rc == HS_OK) {
        e = hipLaunchHostFunc(st, on_done, l);
        if (e != hipSuccess) rc = hs::hip_fail(e, "completion callback");
    }
    if (rc != HS_OK) (void)hipStreamSynchronize(st);
    return rc;
}

}  // namespace

extern "C" {

int hs_server_create(hs_ctx *ctx, int n_slots, size_t arena_bytes, int mode, hs_server **out) {
    if (!ctx) return -1;
    if (n_slots < 1 || n_slots > 64) return -2;
    if (arena_bytes == 0) return -3;
    if (!hs::valid_mode(mode)) return -4;
    if (!out) return -5;
    *out = nullptr;
    std::unique_ptr<hs_server> s(new hs_server);
    s->ctx = ctx;
    s->mode = mode;
    hipError_t e = hipMalloc(&s->arena_mem, arena_bytes);
    if (e == hipErrorOutOfMemory) {
        hs::set_error(HS_ERR_NOMEM, "server arena allocation");
        return HS_ERR_NOMEM;
    }
    if (e != hipSuccess) return hs::hip_fail(e, "hipMalloc");
    s->sched.reset(new hs::serve::Scheduler(n_slots, arena_bytes));
    s->streams.resize(n_slots, nullptr);
    for (int i = 0; i < n_slots; ++i) {
        e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipStreamDestroy(s->streams[j]);
            (void)hipFree(s->arena_mem);
            return hs::hip_fail(e, "hipStreamCreateWithFlags");
        }
    }
    s->epoch = Clock::now();
    *out = s.release();
    return HS_OK;
}

int hs_server_submit(hs_server *s, const hs_request *req) {
    if (!s) return -1;
    if (!req || req->N_G < 1 || !req->A_host || !req->B_host || req->ld < req->N_G) return -2;
    const size_t bytes = footprint(s->ctx->plan, req->N_G, s->mode);
    if (!s->sched->fits_ever(bytes)) {
        hs::set_error(HS_ERR_NOMEM, "request footprint exceeds the server arena");
        return HS_ERR_NOMEM;
    }
    Live *l = new Live;
    l->req = *req;
    l->id = req->id;
    l->bytes = bytes;
    l->epoch = s->epoch;
    s->sched->submit(l, s->now());
    return HS_OK;
}

int hs_server_set_admission(hs_server *s, int policy, int max_bypass) {
    if (!s) return -1;
    if (policy != HS_ADMIT_FIFO && policy != HS_ADMIT_BYPASS) return -2;
    if (max_bypass < 0) return -3;
    s->sched->set_policy(policy, max_bypass);
    return HS_OK;
}

int hs_server_progress(hs_server *s) {
    if (!s) return -1;
    return s->sched->progress([s](hs::serve::Request *r) { return launch(s, static_cast<Live *>(r)); },
                              s->now());
}

int hs_server_pop(hs_server *s, hs_result *out) {
    if (!s || !out) return -1;
    Live *l = static_cast<Live *>(s->sched->pop());
    if (!l) return 0;
    out->id = l->req.id;
    out->N_G = l->req.N_G;
    out->status = l->status;
    out->H = out->S = nullptr;
    if (l->slot >= 0) {
        const Placement d = place(s, l);
        out->H = d.H;
        out->S = d.S;
    }
    out->t_submit = l->t_submit;
    out->t_admit = l->t_admit;
    out->t_done = l->t_done.load();
    return 1;
}

int hs_server_release(hs_server *s, int64_t id) {
    if (!s) return -1;
    hs::serve::Request *r = s->sched->release(id);
    if (!r) return -2;
    delete r;
    return HS_OK;
}

int hs_server_pending(const hs_server *s) { return s ? s->sched->pending() : 0; }

size_t hs_server_used_bytes(const hs_server *s) { return s ? s->sched->used() : 0; }

double hs_server_now(const hs_server *s) { return s ? s->now() : 0.0; }

void hs_server_destroy(hs_server *s) {
    if (!s) return;
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    s->sched->for_each([](hs::serve::Request *r) { delete r; });
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    delete s;
}

}  // extern "C"
