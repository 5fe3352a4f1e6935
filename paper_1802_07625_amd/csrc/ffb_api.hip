// C ABI of libffb: context management, host-side argument validation and
// the entry points declared in include/ffb.h.  Kernels live in k_*.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "ffb_internal.h"

namespace ffbi {

int fail(ffb_ctx *ctx, int code, const char *fmt, const char *detail)
{
    if (ctx) {
        char buf[512];
        snprintf(buf, sizeof buf, fmt, detail);
        ctx->last_error = buf;
    }
    return code;
}

int hip_fail(ffb_ctx *ctx, hipError_t e, const char *where)
{
    if (ctx) {
        ctx->last_error = std::string(where) + ": " + hipGetErrorString(e);
    }
    return e == hipErrorOutOfMemory ? FFB_E_NOMEM : FFB_E_DEVICE;
}

int check_controller(ffb_ctx *ctx, const ffb_integrate_opts *o, const double *h_out,
                     int32_t h_cap, const char *what)
{
    if (h_cap < 0 || (h_cap > 0 && !h_out))
        return fail(ctx, FFB_E_INVALID, "%s: bad h_out/h_cap", what);
    if (o->max_attempts <= 0 || o->max_attempts > (1 << 20))
        return fail(ctx, FFB_E_INVALID, "%s: max_attempts out of range", what);
    if (o->n_replay < 0 || (o->n_replay > 0 && !o->replay_h))
        return fail(ctx, FFB_E_INVALID, "%s: bad replay schedule", what);
    if (o->n_replay == 0) {
        if (!(o->tol > 0.0) || !(o->h0 > 0.0) || !(o->safety > 0.0) || !(o->fac_min > 0.0) ||
            !(o->fac_min <= 1.0) || !(o->fac_max >= 1.0) || !(o->h_min >= 0.0) ||
            !isfinite(o->tol) || !isfinite(o->h0) || !isfinite(o->fac_max))
            return fail(ctx, FFB_E_INVALID, "%s: bad controller constants", what);
    }
    return FFB_OK;
}

hipError_t ensure_state_capacity(ffb_ctx *ctx, int64_t n)
{
    if (n <= ctx->st_cap) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = grow(&ctx->st[b], ctx->st_cap, n);
        if (e == hipSuccess) e = grow(&ctx->kv[b], ctx->st_cap, n);
    }
    ctx->st_cap = e == hipSuccess ? n : 0;
    return e;
}

// FFB_OPT_POINT_ORDER = 1 sorts when both hold: at least kOrderMinPoints
// points (below that the sort's fixed cost, five short launches, outweighs
// the cheaper lookups) and packed fields larger than kOrderMinFieldBytes,
// twice the 4 MB L2 of one XCD.  Measured on MI355X: at 1024 x 1024 cells
// (16 MB of fields) the sort saves 0.5-1.3 us per RK attempt against
// ~45 us per call; at 1024 x 512 and 512 x 512 (whose XCD shares of the
// fields stay L2-resident in the caller's order) it saves nothing.
constexpr int64_t kOrderMinPoints = 65536;
constexpr int64_t kOrderMinFieldBytes = (int64_t)8 << 20;

bool use_point_order(const ffb_ctx *ctx, int64_t n)
{
    if (n <= 0 || ctx->ord_mode == 0) return false;
    if (ctx->ord_mode == 2) return true;
    return n >= kOrderMinPoints && 16 * (int64_t)ctx->lx * ctx->ly > kOrderMinFieldBytes;
}

int32_t *prepare_point_order(ffb_ctx *ctx, const float *xy, int64_t n, hipError_t *err)
{
    *err = hipSuccess;
    if (!use_point_order(ctx, n)) return nullptr;
    // any permutation of [0, n) gives the same results, so a kept order is
    // always valid; it is only as fast as the points are still close to
    // where they were when it was computed
    if (ctx->ord_mode == 3 && ctx->ord_xy == xy && ctx->ord_n == n && ctx->ord_cap >= n)
        return ctx->ord_perm;
    ctx->ord_xy = nullptr;
    ctx->ord_n = -1;
    *err = ensure_order_capacity(ctx, n);
    if (*err == hipSuccess) *err = launch_point_order(ctx, reinterpret_cast<const float2 *>(xy), n);
    if (*err != hipSuccess) return nullptr;
    if (ctx->ord_mode == 3) {
        ctx->ord_xy = xy;
        ctx->ord_n = n;
    }
    return ctx->ord_perm;
}

hipError_t ensure_order_capacity(ffb_ctx *ctx, int64_t n)
{
    hipError_t e = hipSuccess;
    if (!ctx->ord_count || !ctx->ord_offs || !ctx->ord_sums) {
        const int64_t cells = (int64_t)ctx->lx * ctx->ly + 1;
        e = grow(&ctx->ord_count, 0, cells);
        if (e == hipSuccess) e = grow(&ctx->ord_offs, 0, cells);
        if (e == hipSuccess) e = grow(&ctx->ord_sums, 0, (int64_t)scan_blocks(cells));
        if (e != hipSuccess) return e;
    }
    if (n > ctx->ord_cap) {
        e = grow(&ctx->ord_perm, ctx->ord_cap, n);
        if (e == hipSuccess) e = grow(&ctx->ord_rank, ctx->ord_cap, n);
        ctx->ord_cap = e == hipSuccess ? n : 0;
    }
    return e;
}

hipError_t grow_bytes(void **p, int64_t have, int64_t need)
{
    if (need <= have && *p) return hipSuccess;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        if (e != hipSuccess) return e;
    }
    return hipMalloc(p, (size_t)(need > 0 ? need : 1));
}

int check_geometry(ffb_ctx *ctx, const ffb_geometry *g)
{
    if (!g) return fail(ctx, FFB_E_INVALID, "geometry is NULL%s");
    if (g->n_vertices < 0 || g->n_rings < 0 || g->n_regions < 1 || g->n_entries < 0)
        return fail(ctx, FFB_E_INVALID, "negative geometry size or no region%s");
    if (g->n_rings == 0 && g->n_entries != 0)
        return fail(ctx, FFB_E_INVALID, "ring entries without rings%s");
    if (g->n_entries < 3 * (int64_t)g->n_rings)
        return fail(ctx, FFB_E_INVALID, "fewer than three entries per ring%s");
    if (g->n_entries > INT32_MAX) return fail(ctx, FFB_E_INVALID, "too many ring entries%s");
    if (g->n_vertices > INT32_MAX) return fail(ctx, FFB_E_INVALID, "too many vertices%s");
    if ((g->n_vertices > 0 && !g->xy) || !g->ring_offsets ||
        (g->n_entries > 0 && !g->ring_vidx) || (g->n_rings > 0 && !g->ring_region))
        return fail(ctx, FFB_E_INVALID, "geometry array is NULL%s");
    return FFB_OK;
}

hipError_t ensure_region_capacity(ffb_ctx *ctx, int32_t R)
{
    if (R <= ctx->w_cap) return hipSuccess;
    hipError_t e = grow(&ctx->w_region, ctx->w_cap, R);
    if (e == hipSuccess) e = grow(&ctx->lam_w, ctx->w_cap, R);
    ctx->w_cap = e == hipSuccess ? R : 0;
    return e;
}

hipError_t ensure_adjoint_capacity(ffb_ctx *ctx, int32_t cap, int64_t n)
{
    hipError_t e = hipSuccess;
    if (cap > ctx->adj_t_cap) {
        e = grow(&ctx->adj_t, ctx->adj_t_cap, cap);
        ctx->adj_t_cap = e == hipSuccess ? cap : 0;
    }
    const int64_t need = (int64_t)cap * (n > 0 ? n : 1);
    if (e == hipSuccess && need > ctx->adj_jac_cap) {
        e = grow(&ctx->adj_jac, ctx->adj_jac_cap, need);
        ctx->adj_jac_cap = e == hipSuccess ? need : 0;
    }
    return e;
}

}  // namespace ffbi

using namespace ffbi;

namespace {

bool pow2_in_range(int32_t n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

// exp(-2 pi i k / N), k < N/2 and exp(-i pi m / (2N)), m < N, in FP64: the
// tables as computed (tw64, tq64) and rounded to FP32 (tw, tq).
hipError_t upload_twiddles(float2 **tw, float2 **tq, double2 **tw64, double2 **tq64, int N)
{
    std::vector<float2> a(N / 2), b(N);
    std::vector<double2> a64(N / 2), b64(N);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < N / 2; ++k) {
        a64[k] = make_double2(cos(2 * pi * k / N), -sin(2 * pi * k / N));
        a[k] = make_float2((float)a64[k].x, (float)a64[k].y);
    }
    for (int m = 0; m < N; ++m) {
        b64[m] = make_double2(cos(pi * m / (2.0 * N)), -sin(pi * m / (2.0 * N)));
        b[m] = make_float2((float)b64[m].x, (float)b64[m].y);
    }
    hipError_t e = hipMalloc(reinterpret_cast<void **>(tw), sizeof(float2) * a.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(tq), sizeof(float2) * b.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(tw64), sizeof(double2) * a.size());
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(tq64), sizeof(double2) * b.size());
    if (e == hipSuccess)
        e = hipMemcpy(*tw, a.data(), sizeof(float2) * a.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(*tq, b.data(), sizeof(float2) * b.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(*tw64, a64.data(), sizeof(double2) * a64.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(*tq64, b64.data(), sizeof(double2) * b64.size(), hipMemcpyHostToDevice);
    return e;
}

void free_all(ffb_ctx *c)
{
    void *ptrs[] = {c->d_status, c->tw_x, c->tq_x, c->tw_y, c->tq_y, c->tw64_x, c->tq64_x,
                    c->tw64_y, c->tq64_y, c->t1, c->t2, c->t3, c->pa,
                    c->pb, c->pc, c->red, c->acc, c->w_region, c->st[0], c->st[1], c->kv[0],
                    c->kv[1], c->errslot, c->lam_w, c->adj_t, c->adj_jac, c->ord_perm,
                    c->ord_rank, c->ord_count, c->ord_offs, c->ord_sums};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    tape_free(c);
    diff_free(c);
    if (c->inv) {
        void *iv[] = {c->inv->count, c->inv->offs, c->inv->fill, c->inv->sums, c->inv->order,
                      c->inv->best, c->inv->big, c->inv->big_nb, c->inv->big_off,
                      c->inv->sums64, c->inv->n_big};
        for (void *p : iv)
            if (p) (void)hipFree(p);
        delete c->inv;
        c->inv = nullptr;
    }
}

int check_integrate(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy,
                    int64_t n, const ffb_integrate_opts *o, int32_t *stats, double *h_out,
                    int32_t h_cap)
{
    if (!ctx) return FFB_E_INVALID;
    if (!fields || !rho_bar || !o || !stats || (n > 0 && !xy))
        return fail(ctx, FFB_E_INVALID, "ffb_integrate: NULL argument%s");
    if (n < 0 || n > INT32_MAX - 4096)
        return fail(ctx, FFB_E_INVALID, "ffb_integrate: n out of range%s");
    return check_controller(ctx, o, h_out, h_cap, "ffb_integrate");
}

int run_integrate(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy, int64_t n,
                  const ffb_integrate_opts *o, int32_t *stats, double *h_out, int32_t h_cap,
                  const advect_tape *rec)
{
    hipError_t e = ensure_state_capacity(ctx, n);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_integrate state buffers");
    e = launch_fill_i32(stats, 4, 0, ctx->stream);
    if (e == hipSuccess && rec && rec->count) e = launch_fill_i32(rec->count, 1, 0, ctx->stream);
    const int32_t *perm = nullptr;
    if (e == hipSuccess) perm = prepare_point_order(ctx, xy, n, &e);
    if (e == hipSuccess)
        e = launch_advect(ctx, reinterpret_cast<const float4 *>(fields), rho_bar,
                          reinterpret_cast<float2 *>(xy), n, o, stats, h_out, h_cap, rec, perm);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_integrate launch");
}

}  // namespace

extern "C" {

int ffb_create(ffb_ctx **out, int32_t lx, int32_t ly, int64_t max_points, void *hip_stream)
{
    if (!out) return FFB_E_INVALID;
    *out = nullptr;
    if (!pow2_in_range(lx) || !pow2_in_range(ly) || max_points < 0) return FFB_E_INVALID;
    ffb_ctx *c = new ffb_ctx();
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->lx = lx;
    c->ly = ly;
    hipError_t e = hipGetDevice(&c->device);
    const int64_t plane = (int64_t)lx * ly;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->d_status), sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(int32_t));
    if (e == hipSuccess) e = upload_twiddles(&c->tw_x, &c->tq_x, &c->tw64_x, &c->tq64_x, lx);
    if (e == hipSuccess) e = upload_twiddles(&c->tw_y, &c->tq_y, &c->tw64_y, &c->tq64_y, ly);
    float **planes[] = {&c->t1, &c->t2, &c->t3, &c->pa, &c->pb, &c->pc};
    for (float **pl : planes)
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(pl), sizeof(double) * plane);
    if (e == hipSuccess) e = grow(&c->red, 0, kRedDoubles);
    c->red_cap = kRedDoubles;
    if (e == hipSuccess) e = grow(&c->acc, 0, (int64_t)ly * (lx + 1));
    if (e == hipSuccess) e = grow(&c->w_region, 0, 1024);
    if (e == hipSuccess) e = grow(&c->lam_w, 0, 1024);
    c->w_cap = 1024;
    if (e == hipSuccess) e = grow(&c->errslot, 0, 4096);   // advection sync words
    c->err_cap = 4096;
    if (e == hipSuccess && max_points > 0) {
        for (int b = 0; b < 2 && e == hipSuccess; ++b) {
            e = grow(&c->st[b], 0, max_points);
            if (e == hipSuccess) e = grow(&c->kv[b], 0, max_points);
        }
        c->st_cap = max_points;
    }
    if (e == hipSuccess) {
        int blocks = 0;
        if (advect_max_blocks(&blocks) != 0 || blocks <= 0) e = hipErrorInvalidValue;
        c->adv_blocks = blocks;
    }
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return e == hipErrorOutOfMemory ? FFB_E_NOMEM : FFB_E_DEVICE;
    }
    *out = c;
    return FFB_OK;
}

int ffb_destroy(ffb_ctx *ctx)
{
    if (!ctx) return FFB_E_INVALID;
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return FFB_OK;
}

int ffb_sync(ffb_ctx *ctx)
{
    if (!ctx) return FFB_E_INVALID;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    int32_t st = 0;
    e = hipMemcpy(&st, ctx->d_status, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "status read");
    return st;
}

int ffb_reset_status(ffb_ctx *ctx)
{
    if (!ctx) return FFB_E_INVALID;
    hipError_t e = launch_fill_i32(ctx->d_status, 1, 0, ctx->stream);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "reset status");
}

const char *ffb_last_error(const ffb_ctx *ctx)
{
    return ctx ? ctx->last_error.c_str() : "null context";
}

int ffb_set_option(ffb_ctx *ctx, int32_t option, int32_t value)
{
    if (!ctx) return FFB_E_INVALID;
    if (option == FFB_OPT_ADVECT_STATE) {
        if (value < 0 || value > 2) return fail(ctx, FFB_E_INVALID, "advect state mode out of range%s");
        ctx->adv_mode = value;
        return FFB_OK;
    }
    if (option == FFB_OPT_ADVECT_BLOCKS) {
        if (value < 0) return fail(ctx, FFB_E_INVALID, "negative workgroup cap%s");
        ctx->adv_cap = value;
        return FFB_OK;
    }
    if (option == FFB_OPT_POINT_ORDER) {
        if (value < 0 || value > 3) return fail(ctx, FFB_E_INVALID, "point order mode out of range%s");
        ctx->ord_mode = value;
        ctx->ord_xy = nullptr;                 // setting the option drops a kept order
        ctx->ord_n = -1;
        return FFB_OK;
    }
    if (option == FFB_OPT_DIFFUSION_GRAPH) {
        if (value < 0 || value > 1) return fail(ctx, FFB_E_INVALID, "graph flag must be 0 or 1%s");
        ctx->diff_graph = value;
        if (ctx->diff) ctx->diff->use_graph = value != 0;
        return FFB_OK;
    }
    return fail(ctx, FFB_E_INVALID, "unknown option%s");
}

int ffb_area_error(ffb_ctx *ctx, const ffb_geometry *g, const double *value, double *area,
                   double *err, double *max_abs_err)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_geometry(ctx, g);
    if (st) return st;
    if (!value || !area || !err || !max_abs_err)
        return fail(ctx, FFB_E_INVALID, "ffb_area_error: NULL output or value%s");
    float2 *snap = nullptr;
    st = tape_on_area(ctx, g, &snap);
    if (st) return st;
    hipError_t e = launch_area(ctx, g, value, area, err, max_abs_err, snap);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_area_error launch");
}

int ffb_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value, const double *area,
                double *rho, double *rho_pad)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_geometry(ctx, g);
    if (st) return st;
    if (!value || !area || !rho || !rho_pad)
        return fail(ctx, FFB_E_INVALID, "ffb_density: NULL argument%s");
    hipError_t e = ensure_region_capacity(ctx, g->n_regions);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_density workspace");
    density_snap snap;
    st = tape_on_density(ctx, g, value, area, &snap);
    if (st) return st;
    e = launch_density(ctx, g, value, area, rho, rho_pad, snap.w ? &snap : nullptr);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_density launch");
}

int ffb_flux(ffb_ctx *ctx, const double *rho, float sigma, float *fields, double *rho_bar)
{
    if (!ctx) return FFB_E_INVALID;
    if (!rho || !fields || !rho_bar) return fail(ctx, FFB_E_INVALID, "ffb_flux: NULL argument%s");
    if (!(sigma >= 0.0f) || !isfinite(sigma))
        return fail(ctx, FFB_E_INVALID, "ffb_flux: sigma must be finite and >= 0%s");
    flux_snap snap;
    int st = tape_on_flux(ctx, sigma, reinterpret_cast<const float4 *>(fields), rho_bar, &snap);
    if (st) return st;
    hipError_t e = launch_flux(ctx, rho, sigma, reinterpret_cast<float4 *>(fields), rho_bar,
                               snap.fields ? &snap : nullptr);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_flux launch");
}

int ffb_pack_fields(ffb_ctx *ctx, const float *jx, const float *jy, const float *rho_s,
                    float *fields)
{
    if (!ctx) return FFB_E_INVALID;
    if (!jx || !jy || !rho_s || !fields)
        return fail(ctx, FFB_E_INVALID, "ffb_pack_fields: NULL argument%s");
    hipError_t e = launch_pack_fields(ctx, jx, jy, rho_s, reinterpret_cast<float4 *>(fields));
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_pack_fields launch");
}

int ffb_integrate(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy, int64_t n,
                  const ffb_integrate_opts *o, int32_t *stats, double *h_out, int32_t h_cap)
{
    int st = check_integrate(ctx, fields, rho_bar, xy, n, o, stats, h_out, h_cap);
    if (st) return st;
    advect_tape rec{};
    bool record = false;
    st = tape_on_integrate(ctx, n, reinterpret_cast<const float4 *>(fields), rho_bar, &rec,
                           &record);
    if (st) return st;
    return run_integrate(ctx, fields, rho_bar, xy, n, o, stats, h_out, h_cap,
                         record ? &rec : nullptr);
}

int ffb_distortion(ffb_ctx *ctx, int32_t lx, int32_t ly, const float *nodes, double *stats,
                   float *e, float *e_tilde)
{
    if (!ctx) return FFB_E_INVALID;
    if (!nodes || !stats) return fail(ctx, FFB_E_INVALID, "ffb_distortion: NULL argument%s");
    if (lx < 2 || ly < 2 || (int64_t)lx * ly > ((int64_t)1 << 31))
        return fail(ctx, FFB_E_INVALID, "ffb_distortion: grid must be at least 2 x 2 nodes%s");
    hipError_t err = launch_distortion(ctx, lx, ly, reinterpret_cast<const float2 *>(nodes),
                                       stats, e, e_tilde);
    return err == hipSuccess ? FFB_OK : hip_fail(ctx, err, "ffb_distortion launch");
}

int ffb_inverse(ffb_ctx *ctx, int32_t lx, int32_t ly, const float *nodes, const float *queries,
                int64_t nq, int32_t *tri, double *pre)
{
    if (!ctx) return FFB_E_INVALID;
    if (!nodes || (nq > 0 && (!queries || !tri || !pre)))
        return fail(ctx, FFB_E_INVALID, "ffb_inverse: NULL argument%s");
    if (lx < 2 || ly < 2 || (int64_t)lx * ly > ((int64_t)1 << 26))
        return fail(ctx, FFB_E_INVALID, "ffb_inverse: grid must be 2 x 2 to 2^26 nodes%s");
    if (nq < 0 || nq > INT32_MAX - 1)
        return fail(ctx, FFB_E_INVALID, "ffb_inverse: query count out of range%s");
    if (!ctx->inv) ctx->inv = new inverse_ws();
    inverse_ws *w = ctx->inv;
    const int64_t bins = (int64_t)lx * ly;
    const int64_t sums = scan_blocks(bins + 1);
    const int64_t qn = nq > 0 ? nq : 1;
    hipError_t e = hipSuccess;
    if (bins > w->bins_cap) {
        e = grow(&w->count, w->bins_cap + 1, bins + 1);
        if (e == hipSuccess) e = grow(&w->offs, w->bins_cap + 1, bins + 1);
        if (e == hipSuccess) e = grow(&w->fill, w->bins_cap, bins);
        w->bins_cap = e == hipSuccess ? bins : 0;
    }
    if (e == hipSuccess && sums > w->sums_cap) {
        e = grow(&w->sums, w->sums_cap, sums);
        w->sums_cap = e == hipSuccess ? sums : 0;
    }
    if (e == hipSuccess && qn > w->q_cap) {
        e = grow(&w->order, w->q_cap, qn);
        if (e == hipSuccess) e = grow(&w->best, w->q_cap, qn);
        w->q_cap = e == hipSuccess ? qn : 0;
    }
    const int64_t ntri = 2 * (int64_t)(lx - 1) * (ly - 1);
    if (e == hipSuccess && ntri > w->tri_cap) {
        e = grow(&w->big, w->tri_cap, ntri);
        if (e == hipSuccess) e = grow(&w->big_nb, w->tri_cap + 1, ntri + 1);
        if (e == hipSuccess) e = grow(&w->big_off, w->tri_cap + 1, ntri + 1);
        if (e == hipSuccess)
            e = grow(&w->sums64, scan_blocks(w->tri_cap + 1),
                     scan_blocks(ntri + 1));
        if (e == hipSuccess && !w->n_big) e = grow(&w->n_big, 0, 1);
        w->tri_cap = e == hipSuccess ? ntri : 0;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_inverse workspace");
    e = launch_inverse(ctx, lx, ly, reinterpret_cast<const float2 *>(nodes),
                       reinterpret_cast<const float2 *>(queries), nq, tri,
                       reinterpret_cast<double2 *>(pre), w);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_inverse launch");
}

int ffb_integrate_record(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy,
                         int64_t n, const ffb_integrate_opts *o, int32_t *stats,
                         float *tape_states, int64_t tape_n, int32_t tape_cap, double *tape_h)
{
    int st = check_integrate(ctx, fields, rho_bar, xy, n, o, stats, nullptr, 0);
    if (st) return st;
    if (tape_n < 0 || tape_n > n || tape_cap < 1 || !tape_states || !tape_h)
        return fail(ctx, FFB_E_INVALID, "ffb_integrate_record: bad tape arguments%s");
    advect_tape rec{reinterpret_cast<float4 *>(tape_states), tape_n, tape_cap, tape_h, nullptr};
    return run_integrate(ctx, fields, rho_bar, xy, n, o, stats, nullptr, 0, &rec);
}

}  // extern "C"
