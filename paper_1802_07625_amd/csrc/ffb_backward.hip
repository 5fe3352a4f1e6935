// C ABI of the adjoints (reverse-mode gradients of the rounds with the
// accepted step sizes frozen) and the context tape that ffb_backward replays.
//
// A recorded round is the call sequence area -> density -> flux -> integrate
// on the same vertices; the tape keeps, per call, exactly what its adjoint
// needs (device copies made on the stream at the time of the call):
//   area      vertices;
//   density   vertices, value, area;
//   flux      sigma (the flux is linear in rho);
//   integrate fields, rho_bar, and the state of the vertices before every
//             accepted step with the step sizes.
// ffb_backward walks the records backwards: area adjoint of the closing area
// call, then per round integrate -> flux -> density -> area adjoints, with the
// area adjoint of a round applied at the area call that fed its density.
#include <math.h>
#include <stdio.h>

#include <cmath>
#include <string>
#include <vector>

#include "ffb_internal.h"

using namespace ffbi;

struct tape_rec {
    char kind = 0;                 // 'A'rea, 'D'ensity, 'F'lux, 'I'ntegrate
    ffb_geometry g{};              // A, D: ring arrays referenced; xy -> own copy
    float2 *xy = nullptr;          // A, D
    double *value = nullptr;       // D
    double *area = nullptr;        // D
    float sigma = 0.f;             // F
    float4 *fields = nullptr;      // I
    double *rho_bar = nullptr;     // I
    advect_tape at{};              // I: states, h, count owned by the record
};

struct ffb_tape {
    bool recording = false;
    int32_t max_steps = 0;
    std::vector<tape_rec> recs;
    // backward workspace
    double *lam_xy = nullptr;
    int64_t lam_xy_cap = 0;
    double *lam_area = nullptr;
    int64_t lam_area_cap = 0;
    float4 *lam_f = nullptr;
    double *lam_rb = nullptr;
    float *lam_rho = nullptr;
};

namespace {

void free_rec(tape_rec &r)
{
    void *ptrs[] = {r.xy, r.value, r.area, r.fields, r.rho_bar, r.at.states, r.at.h, r.at.count};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    r = tape_rec{};
}

void clear_records(ffb_tape *t)
{
    for (tape_rec &r : t->recs) free_rec(r);
    t->recs.clear();
}

bool recording(ffb_ctx *ctx) { return ctx->tape && ctx->tape->recording; }

template <typename T>
hipError_t alloc_copy(T **dst, const T *src, int64_t n, hipStream_t s)
{
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), sizeof(T) * (size_t)(n > 0 ? n : 1));
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpyAsync(*dst, src, sizeof(T) * (size_t)n, hipMemcpyDeviceToDevice, s);
}

int push(ffb_ctx *ctx, tape_rec &r, hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        free_rec(r);
        return hip_fail(ctx, e, what);
    }
    ctx->tape->recs.push_back(r);
    return FFB_OK;
}

// Number of vertices and regions of the recorded rounds (from the first record).
bool tape_sizes(const ffb_tape *t, int64_t *V, int32_t *R)
{
    for (const tape_rec &r : t->recs)
        if (r.kind == 'A' || r.kind == 'D') {
            *V = r.g.n_vertices;
            *R = r.g.n_regions;
            return true;
        }
    return false;
}

}  // namespace

int tape_on_area(ffb_ctx *ctx, const ffb_geometry *g)
{
    if (!recording(ctx)) return FFB_OK;
    tape_rec r;
    r.kind = 'A';
    r.g = *g;
    hipError_t e = alloc_copy(&r.xy, reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                              ctx->stream);
    r.g.xy = reinterpret_cast<const float *>(r.xy);
    return push(ctx, r, e, "tape (area)");
}

int tape_on_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value, const double *area)
{
    if (!recording(ctx)) return FFB_OK;
    tape_rec r;
    r.kind = 'D';
    r.g = *g;
    hipError_t e = alloc_copy(&r.xy, reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                              ctx->stream);
    r.g.xy = reinterpret_cast<const float *>(r.xy);
    if (e == hipSuccess) e = alloc_copy(&r.value, value, g->n_regions, ctx->stream);
    if (e == hipSuccess) e = alloc_copy(&r.area, area, g->n_regions, ctx->stream);
    return push(ctx, r, e, "tape (density)");
}

int tape_on_flux(ffb_ctx *ctx, float sigma)
{
    if (!recording(ctx)) return FFB_OK;
    tape_rec r;
    r.kind = 'F';
    r.sigma = sigma;
    return push(ctx, r, hipSuccess, "tape (flux)");
}

int tape_on_integrate(ffb_ctx *ctx, int64_t n, const float4 *fields, const double *rho_bar,
                      advect_tape *out, bool *record)
{
    *record = false;
    if (!recording(ctx)) return FFB_OK;
    ffb_tape *t = ctx->tape;
    int64_t V = 0;
    int32_t R = 0;
    if (!tape_sizes(t, &V, &R))
        return fail(ctx, FFB_E_INVALID, "tape: ffb_integrate recorded before any area or density call%s");
    if (n < V)
        return fail(ctx, FFB_E_INVALID, "tape: ffb_integrate must advect the recorded vertices first%s");
    tape_rec r;
    r.kind = 'I';
    const int64_t nf = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    hipError_t e = alloc_copy(&r.fields, fields, nf, ctx->stream);
    if (e == hipSuccess) e = alloc_copy(&r.rho_bar, rho_bar, 1, ctx->stream);
    r.at.n = V;
    r.at.cap = t->max_steps;
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&r.at.states),
                      sizeof(float4) * (size_t)(V > 0 ? V : 1) * (size_t)t->max_steps);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&r.at.h), sizeof(double) * (size_t)t->max_steps);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&r.at.count), sizeof(int32_t));
    const int st = push(ctx, r, e, "tape (integrate)");
    if (st == FFB_OK) {
        *out = r.at;
        *record = true;
    }
    return st;
}

void tape_free(ffb_ctx *ctx)
{
    ffb_tape *t = ctx->tape;
    if (!t) return;
    clear_records(t);
    void *ptrs[] = {t->lam_xy, t->lam_area, t->lam_f, t->lam_rb, t->lam_rho};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete t;
    ctx->tape = nullptr;
}

extern "C" {

int ffb_area_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *lam_area, double *lam_xy)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_geometry(ctx, g);
    if (st) return st;
    if (!lam_area || (g->n_vertices > 0 && !lam_xy))
        return fail(ctx, FFB_E_INVALID, "ffb_area_adj: NULL argument%s");
    hipError_t e = launch_area_adj(ctx, g, lam_area, lam_xy);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_area_adj launch");
}

int ffb_density_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *value, const double *area,
                    const float *lam_rho, double *lam_value, double *lam_area, double *lam_xy)
{
    if (!ctx) return FFB_E_INVALID;
    int st = check_geometry(ctx, g);
    if (st) return st;
    if (!value || !area || !lam_rho || !lam_value || !lam_area || (g->n_vertices > 0 && !lam_xy))
        return fail(ctx, FFB_E_INVALID, "ffb_density_adj: NULL argument%s");
    hipError_t e = ensure_region_capacity(ctx, g->n_regions);
    if (e == hipSuccess)
        e = launch_density_adj(ctx, g, value, area, lam_rho, lam_value, lam_area, lam_xy);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_density_adj launch");
}

int ffb_flux_adj(ffb_ctx *ctx, float sigma, const float *lam_fields, const double *lam_rho_bar,
                 float *lam_rho)
{
    if (!ctx) return FFB_E_INVALID;
    if (!lam_fields || !lam_rho_bar || !lam_rho)
        return fail(ctx, FFB_E_INVALID, "ffb_flux_adj: NULL argument%s");
    if (!(sigma >= 0.0f) || !std::isfinite(sigma))
        return fail(ctx, FFB_E_INVALID, "ffb_flux_adj: sigma must be finite and >= 0%s");
    hipError_t e = launch_flux_adj(ctx, sigma, reinterpret_cast<const float4 *>(lam_fields),
                                   lam_rho_bar, lam_rho);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_flux_adj launch");
}

int ffb_integrate_adj(ffb_ctx *ctx, const float *fields, const double *rho_bar,
                      const int32_t *stats, const float *tape_states, int64_t tape_n,
                      int32_t tape_cap, const double *tape_h, double *lam_xy, float *lam_fields,
                      double *lam_rho_bar)
{
    if (!ctx) return FFB_E_INVALID;
    if (!fields || !rho_bar || !stats || !tape_h || !lam_fields || !lam_rho_bar ||
        (tape_n > 0 && (!tape_states || !lam_xy)))
        return fail(ctx, FFB_E_INVALID, "ffb_integrate_adj: NULL argument%s");
    if (tape_n < 0 || tape_n > INT32_MAX - 4096 || tape_cap < 1)
        return fail(ctx, FFB_E_INVALID, "ffb_integrate_adj: bad tape size%s");
    advect_tape t{const_cast<float4 *>(reinterpret_cast<const float4 *>(tape_states)), tape_n,
                  tape_cap, const_cast<double *>(tape_h), const_cast<int32_t *>(stats)};
    hipError_t e = launch_advect_adj(ctx, reinterpret_cast<const float4 *>(fields), rho_bar, &t,
                                     lam_xy, reinterpret_cast<float4 *>(lam_fields), lam_rho_bar);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_integrate_adj launch");
}

int ffb_tape_begin(ffb_ctx *ctx, int32_t max_steps)
{
    if (!ctx) return FFB_E_INVALID;
    if (max_steps < 1 || max_steps > (1 << 20))
        return fail(ctx, FFB_E_INVALID, "ffb_tape_begin: max_steps out of range%s");
    if (!ctx->tape) ctx->tape = new ffb_tape();
    // records may still be read by queued work
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_tape_begin");
    clear_records(ctx->tape);
    ctx->tape->recording = true;
    ctx->tape->max_steps = max_steps;
    return FFB_OK;
}

int ffb_tape_end(ffb_ctx *ctx)
{
    if (!ctx) return FFB_E_INVALID;
    if (ctx->tape) ctx->tape->recording = false;
    return FFB_OK;
}

int ffb_tape_clear(ffb_ctx *ctx)
{
    if (!ctx) return FFB_E_INVALID;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_tape_clear");
    tape_free(ctx);
    return FFB_OK;
}

int ffb_backward(ffb_ctx *ctx, const double *dL_darea, double *dL_dvalue, double *dL_dxy0)
{
    if (!ctx) return FFB_E_INVALID;
    if (!dL_darea || !dL_dvalue) return fail(ctx, FFB_E_INVALID, "ffb_backward: NULL argument%s");
    ffb_tape *t = ctx->tape;
    if (!t || t->recs.empty())
        return fail(ctx, FFB_E_NO_TAPE, "ffb_backward: nothing recorded (call ffb_tape_begin)%s");
    t->recording = false;
    std::vector<tape_rec> &recs = t->recs;
    // the record sequence must be A+ (D F I A+)*
    std::string seq;
    for (const tape_rec &r : recs) seq += r.kind;
    {
        size_t k = 0;
        bool ok = k < seq.size() && seq[k] == 'A';
        while (ok && k < seq.size() && seq[k] == 'A') ++k;
        while (ok && k < seq.size()) {
            ok = seq.compare(k, 3, "DFI") == 0;
            k += 3;
            ok = ok && k < seq.size() && seq[k] == 'A';
            while (ok && k < seq.size() && seq[k] == 'A') ++k;
        }
        if (!ok)
            return fail(ctx, FFB_E_NO_TAPE,
                        "ffb_backward: tape is not area (density flux integrate area)* (got %s)",
                        seq.c_str());
    }
    int64_t V = 0;
    int32_t R = 0;
    tape_sizes(t, &V, &R);
    for (const tape_rec &r : recs) {
        if ((r.kind == 'A' || r.kind == 'D') && (r.g.n_vertices != V || r.g.n_regions != R))
            return fail(ctx, FFB_E_INVALID, "ffb_backward: rounds differ in vertices or regions%s");
    }
    hipStream_t s = ctx->stream;
    const int64_t nf = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    hipError_t e = hipSuccess;
    if (!t->lam_f) {
        e = hipMalloc(reinterpret_cast<void **>(&t->lam_f), sizeof(float4) * (size_t)nf);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&t->lam_rb), sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&t->lam_rho),
                          sizeof(float) * (size_t)ctx->lx * ctx->ly);
        if (e != hipSuccess) return hip_fail(ctx, e, "ffb_backward workspace");
    }
    if (2 * V > t->lam_xy_cap) {
        e = grow(&t->lam_xy, t->lam_xy_cap, 2 * V);
        t->lam_xy_cap = e == hipSuccess ? 2 * V : 0;
    }
    if (e == hipSuccess && R > t->lam_area_cap) {
        e = grow(&t->lam_area, t->lam_area_cap, R);
        t->lam_area_cap = e == hipSuccess ? R : 0;
    }
    if (e == hipSuccess) e = ensure_region_capacity(ctx, R);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_backward workspace");

    e = launch_fill_f64(t->lam_xy, 2 * V, 0.0, s);
    if (e == hipSuccess) e = launch_fill_f64(dL_dvalue, R, 0.0, s);
    if (e == hipSuccess) e = launch_area_adj(ctx, &recs.back().g, dL_darea, t->lam_xy);
    bool pending = false;           // an area adjoint from a density record waits
    for (int64_t k = (int64_t)recs.size() - 2; k >= 0 && e == hipSuccess; --k) {
        tape_rec &r = recs[k];
        switch (r.kind) {
        case 'I':
            e = launch_fill_f32(reinterpret_cast<float *>(t->lam_f), 4 * nf, 0.f, s);
            if (e == hipSuccess) e = launch_fill_f64(t->lam_rb, 1, 0.0, s);
            if (e == hipSuccess)
                e = launch_advect_adj(ctx, r.fields, r.rho_bar, &r.at, t->lam_xy, t->lam_f,
                                      t->lam_rb);
            break;
        case 'F':
            e = launch_flux_adj(ctx, r.sigma, t->lam_f, t->lam_rb, t->lam_rho);
            break;
        case 'D':
            e = launch_fill_f64(t->lam_area, R, 0.0, s);
            if (e == hipSuccess)
                e = launch_density_adj(ctx, &r.g, r.value, r.area, t->lam_rho, dL_dvalue,
                                       t->lam_area, t->lam_xy);
            pending = true;
            break;
        case 'A':
            if (pending) e = launch_area_adj(ctx, &r.g, t->lam_area, t->lam_xy);
            pending = false;
            break;
        }
    }
    if (e == hipSuccess && dL_dxy0 && V > 0)
        e = hipMemcpyAsync(dL_dxy0, t->lam_xy, sizeof(double) * 2 * (size_t)V,
                           hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_backward launch");
}

}  // extern "C"
