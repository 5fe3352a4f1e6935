// The diffusion cartogram as a flow-based projection (SI Appendix, section
// 2, the diffusion choice of f_mn), for comparison with the linear
// equalisation of the main method: the fields rho(t), J(t) change with t, so
// every attempt of the integrator first rebuilds them at its five distinct
// stage times (one batched set of inverse transforms), then advances all
// points through the six stages, then decides on the device.  An attempt is
// a fixed sequence of launches that reads its step and stage times from a
// device control block, so it is captured once as a graph and replayed; the
// host reads one word per chunk of attempts to learn when t_end is reached.
#include <cmath>

#include "ffb_internal.h"

using namespace ffbi;

namespace {

constexpr int kChunk = 8;   // attempts enqueued between two host checks

hipError_t make_ws(ffb_ctx *ctx, diff_ws **out)
{
    if (ctx->diff) {
        *out = ctx->diff;
        return hipSuccess;
    }
    diff_ws *w = new diff_ws();
    ctx->diff = w;          // diff_free releases whatever was allocated
    w->use_graph = ctx->diff_graph != 0;
    w->plane = (int64_t)ctx->lx * ctx->ly;
    w->fplane = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    hipError_t e = hipMalloc(&w->spec, sizeof(float) * w->plane);
    if (e == hipSuccess) e = hipMalloc(&w->q, sizeof(float) * 3 * kDiffSlots * w->plane);
    if (e == hipSuccess) e = hipMalloc(&w->r, sizeof(float) * 3 * kDiffSlots * w->plane);
    if (e == hipSuccess) e = hipMalloc(&w->fields, sizeof(float4) * kDiffSlots * w->fplane);
    if (e == hipSuccess) e = hipMalloc(&w->ctl, sizeof(diff_ctl));
    if (e == hipSuccess) e = hipMalloc(&w->part, sizeof(float) * kDiffMaxBlocks);
    if (e == hipSuccess) e = hipHostMalloc(&w->done_host, sizeof(int32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&w->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        diff_free(ctx);
        return e;
    }
    *out = w;
    return hipSuccess;
}

hipError_t enqueue_attempt(ffb_ctx *ctx, diff_ws *w, int64_t n)
{
    hipError_t e = launch_diff_fields(ctx, w, kDiffSlots);
    if (e == hipSuccess) e = launch_diff_points(ctx, w, n);
    if (e == hipSuccess) e = launch_diff_control(ctx, w, n, 0);
    return e;
}

// The attempt graph for n points and the current state buffers.
hipError_t ensure_graph(ffb_ctx *ctx, diff_ws *w, int64_t n)
{
    if (w->exec && w->exec_n == n && w->exec_st == ctx->st[0] && w->exec_st1 == ctx->st[1] &&
        w->exec_kv == ctx->kv[0] && w->exec_kv1 == ctx->kv[1])
        return hipSuccess;
    if (w->exec) {
        (void)hipGraphExecDestroy(w->exec);
        w->exec = nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(w->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e2 = enqueue_attempt(ctx, w, n);
    e = hipStreamEndCapture(w->stream, &g);
    if (e2 != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e2 != hipSuccess ? e2 : e;
    }
    e = hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        w->exec = nullptr;
        return e;
    }
    w->exec_n = n;
    w->exec_st = ctx->st[0];
    w->exec_st1 = ctx->st[1];
    w->exec_kv = ctx->kv[0];
    w->exec_kv1 = ctx->kv[1];
    return hipSuccess;
}

int check_common(ffb_ctx *ctx, const double *rho, float sigma, const char *what)
{
    if (!rho) return fail(ctx, FFB_E_INVALID, "%s: NULL density", what);
    if (!(sigma >= 0.f) || !std::isfinite(sigma))
        return fail(ctx, FFB_E_INVALID, "%s: blur width must be finite and >= 0", what);
    return FFB_OK;
}

}  // namespace

namespace ffbi {
void diff_free(ffb_ctx *ctx)
{
    diff_ws *w = ctx->diff;
    if (!w) return;
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    if (w->exec) (void)hipGraphExecDestroy(w->exec);
    void *ptrs[] = {w->spec, w->q, w->r, w->fields, w->ctl, w->part};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (w->done_host) (void)hipHostFree(w->done_host);
    if (w->ev_in) (void)hipEventDestroy(w->ev_in);
    if (w->ev_out) (void)hipEventDestroy(w->ev_out);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
    ctx->diff = nullptr;
}
}  // namespace ffbi

extern "C" {

int ffb_diffusion_fields(ffb_ctx *ctx, const double *rho, float sigma, double t, float *fields)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_common(ctx, rho, sigma, "ffb_diffusion_fields");
    if (st) return st;
    if (!fields) return fail(ctx, FFB_E_INVALID, "%s: NULL fields", "ffb_diffusion_fields");
    if (!(t >= 0.0) || !std::isfinite(t))
        return fail(ctx, FFB_E_INVALID, "%s: t must be finite and >= 0", "ffb_diffusion_fields");
    diff_ws *w = nullptr;
    hipError_t e = make_ws(ctx, &w);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_diffusion_fields buffers");
    diff_ctl init{};
    for (int z = 0; z < kDiffSlots; ++z) init.ts[z] = t;
    e = launch_diff_setup(ctx, w, init);
    if (e == hipSuccess) e = launch_diff_spectrum(ctx, rho, sigma, w->spec);
    if (e == hipSuccess) e = launch_diff_fields(ctx, w, 1);
    if (e == hipSuccess)
        e = hipMemcpyAsync(fields, w->fields, sizeof(float4) * w->fplane, hipMemcpyDeviceToDevice,
                           ctx->stream);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_diffusion_fields");
}

int ffb_diffusion(ffb_ctx *ctx, const double *rho, float sigma, double t_end, float *xy, int64_t n,
                  const ffb_integrate_opts *o, int32_t *stats, double *h_out, int32_t h_cap)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_common(ctx, rho, sigma, "ffb_diffusion");
    if (st) return st;
    if (!o || !stats || (n > 0 && !xy))
        return fail(ctx, FFB_E_INVALID, "%s: NULL argument", "ffb_diffusion");
    if (n < 0 || n > INT32_MAX - 4096)
        return fail(ctx, FFB_E_INVALID, "%s: n out of range", "ffb_diffusion");
    if (!(t_end > 0.0) || !std::isfinite(t_end))
        return fail(ctx, FFB_E_INVALID, "%s: t_end must be finite and > 0", "ffb_diffusion");
    st = check_controller(ctx, o, h_out, h_cap, "ffb_diffusion");
    if (st) return st;
    diff_ws *w = nullptr;
    hipError_t e = make_ws(ctx, &w);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_diffusion buffers");
    e = ensure_state_capacity(ctx, n);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_diffusion state buffers");

    diff_ctl init{};
    init.t = 0.0;
    init.h = o->h0;
    init.t_end = t_end;
    init.tol = o->tol;
    init.h0 = o->h0;
    init.safety = o->safety;
    init.fac_min = o->fac_min;
    init.fac_max = o->fac_max;
    init.h_min = o->h_min;
    init.replay_h = o->n_replay > 0 ? o->replay_h : nullptr;
    init.n_replay = o->n_replay;
    init.max_attempts = o->max_attempts;
    init.h_out = h_out;
    init.h_cap = h_cap;
    init.stats = stats;

    // the private stream follows the caller's, and the caller's follows it
    const hipStream_t user = ctx->stream;
    e = hipEventRecord(w->ev_in, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(w->stream, w->ev_in, 0);
    ctx->stream = w->stream;
    if (e == hipSuccess) e = launch_diff_setup(ctx, w, init);
    if (e == hipSuccess) e = launch_diff_spectrum(ctx, rho, sigma, w->spec);
    if (e == hipSuccess) e = launch_diff_fields(ctx, w, 1);      // t = 0 (stage times all 0)
    const int32_t *perm = nullptr;
    if (e == hipSuccess) perm = prepare_point_order(ctx, xy, n, &e);
    if (e == hipSuccess)
        e = launch_diff_init_points(ctx, w, reinterpret_cast<float2 *>(xy), n, perm);
    if (e == hipSuccess) e = launch_diff_control(ctx, w, n, 1);
    if (e == hipSuccess && w->use_graph) e = ensure_graph(ctx, w, n);
    // at most max_attempts attempts do work; the control block stops the rest
    const int64_t limit = (int64_t)o->max_attempts + kChunk;
    for (int64_t enq = 0; e == hipSuccess && enq < limit; enq += kChunk) {
        for (int k = 0; k < kChunk && e == hipSuccess; ++k)
            e = w->use_graph ? hipGraphLaunch(w->exec, w->stream) : enqueue_attempt(ctx, w, n);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->done_host, &w->ctl->done, sizeof(int32_t),
                               hipMemcpyDeviceToHost, w->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(w->stream);
        if (e == hipSuccess && *w->done_host) break;
    }
    if (e == hipSuccess) e = launch_diff_finish(ctx, w, reinterpret_cast<float2 *>(xy), n, perm);
    ctx->stream = user;
    hipError_t e2 = hipEventRecord(w->ev_out, w->stream);
    if (e2 == hipSuccess) e2 = hipStreamWaitEvent(user, w->ev_out, 0);
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_diffusion");
}

}  // extern "C"
