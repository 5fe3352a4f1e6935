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
    float2 *xy = nullptr;          // A, D: the ring vertices' positions
    double *value = nullptr;       // D
    double *area = nullptr;        // D
    double *w = nullptr;           // D: the weights w_r of the raster
    float sigma = 0.f;             // F
    float4 *fields = nullptr;      // F: the flux outputs; I: a copy if needed
    double *rho_bar = nullptr;     // F, I (as fields)
    const float4 *src_fields = nullptr;    // F: the caller's output buffers
    const double *src_rho_bar = nullptr;
    const float4 *fields_in = nullptr;     // I: what the integration read
    const double *rho_bar_in = nullptr;    //    (the flux record's or own copy)
    advect_tape at{};              // I: states, h, count owned by the record
    // allocated sizes (elements), so a later recording can reuse the buffers
    int64_t xy_cap = 0, r_cap = 0, st_cap = 0, h_cap = 0;
};

struct ffb_tape {
    bool recording = false;
    int32_t max_steps = 0;
    std::vector<tape_rec> recs;    // recs[0, used) is the current record
    size_t used = 0;
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
    void *ptrs[] = {r.xy,      r.value, r.area, r.w,         r.fields,
                    r.rho_bar, r.at.states, r.at.h, r.at.count};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    r = tape_rec{};
}

void clear_records(ffb_tape *t)
{
    for (tape_rec &r : t->recs) free_rec(r);
    t->recs.clear();
    t->used = 0;
}

bool recording(ffb_ctx *ctx) { return ctx->tape && ctx->tape->recording; }

// The next record slot: buffers of an earlier recording at the same position
// are kept (queued work that still reads them precedes, on the same stream,
// whatever overwrites them).
tape_rec &next_slot(ffb_tape *t, char kind)
{
    if (t->used == t->recs.size()) t->recs.emplace_back();
    tape_rec &r = t->recs[t->used];
    r.kind = kind;
    return r;
}

template <typename T>
hipError_t ensure(T **p, int64_t *cap, int64_t need)
{
    if (need <= *cap && *p) return hipSuccess;
    hipError_t e = grow(p, *cap, need);
    *cap = e == hipSuccess ? need : 0;
    return e;
}

template <typename T>
hipError_t copy_in(T **dst, int64_t *cap, const T *src, int64_t n, hipStream_t s)
{
    hipError_t e = ensure(dst, cap, n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpyAsync(*dst, src, sizeof(T) * (size_t)n, hipMemcpyDeviceToDevice, s);
}

int commit(ffb_ctx *ctx, hipError_t e, const char *what)
{
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    ++ctx->tape->used;
    return FFB_OK;
}

// Number of vertices and regions of the recorded rounds (from the first record).
bool tape_sizes(const ffb_tape *t, int64_t *V, int32_t *R)
{
    for (size_t k = 0; k < t->used; ++k) {
        const tape_rec &r = t->recs[k];
        if (r.kind == 'A' || r.kind == 'D') {
            *V = r.g.n_vertices;
            *R = r.g.n_regions;
            return true;
        }
    }
    return false;
}

}  // namespace

int tape_on_area(ffb_ctx *ctx, const ffb_geometry *g, float2 **xy_snap)
{
    *xy_snap = nullptr;
    if (!recording(ctx)) return FFB_OK;
    tape_rec &r = next_slot(ctx->tape, 'A');
    r.g = *g;
    hipError_t e = ensure(&r.xy, &r.xy_cap, g->n_vertices);
    r.g.xy = reinterpret_cast<const float *>(r.xy);
    if (e == hipSuccess) *xy_snap = r.xy;     // written by the area kernel
    return commit(ctx, e, "tape (area)");
}

int tape_on_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value, const double *area,
                    density_snap *snap)
{
    *snap = density_snap{};
    if (!recording(ctx)) return FFB_OK;
    (void)value;
    (void)area;
    tape_rec &r = next_slot(ctx->tape, 'D');
    r.g = *g;
    hipError_t e = ensure(&r.xy, &r.xy_cap, g->n_vertices);
    r.g.xy = reinterpret_cast<const float *>(r.xy);
    if (e == hipSuccess) {
        // value, area and w share one capacity
        const int64_t R = g->n_regions;
        int64_t rc = r.r_cap;
        e = ensure(&r.value, &rc, R);
        if (e == hipSuccess) {
            rc = r.r_cap;
            e = ensure(&r.area, &rc, R);
        }
        if (e == hipSuccess) {
            rc = r.r_cap;
            e = ensure(&r.w, &rc, R);
        }
        r.r_cap = e == hipSuccess ? rc : 0;
    }
    if (e == hipSuccess) *snap = density_snap{r.xy, r.value, r.area, r.w};
    return commit(ctx, e, "tape (density)");
}

int tape_on_flux(ffb_ctx *ctx, float sigma, const float4 *fields, const double *rho_bar,
                 flux_snap *snap)
{
    *snap = flux_snap{};
    if (!recording(ctx)) return FFB_OK;
    tape_rec &r = next_slot(ctx->tape, 'F');
    r.sigma = sigma;
    const int64_t nf = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    int64_t fcap = r.fields ? nf : 0, one = r.rho_bar ? 1 : 0;
    hipError_t e = ensure(&r.fields, &fcap, nf);
    if (e == hipSuccess) e = ensure(&r.rho_bar, &one, 1);
    r.src_fields = fields;
    r.src_rho_bar = rho_bar;
    if (e == hipSuccess) *snap = flux_snap{r.fields, r.rho_bar};
    return commit(ctx, e, "tape (flux)");
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
    // the integration of a round reads the fields and rho_bar that the
    // round's flux call wrote (the reverse pass assumes it): then the flux
    // record's copies serve, else the inputs are copied here
    const float4 *ff = nullptr;
    const double *fr = nullptr;
    if (t->used > 0) {
        const tape_rec &f = t->recs[t->used - 1];
        if (f.kind == 'F' && f.src_fields == fields && f.src_rho_bar == rho_bar) {
            ff = f.fields;
            fr = f.rho_bar;
        }
    }
    tape_rec &r = next_slot(t, 'I');
    const int64_t nf = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    int64_t fcap = r.fields ? nf : 0, one = r.rho_bar ? 1 : 0, cnt = r.at.count ? 1 : 0;
    hipError_t e = hipSuccess;
    if (ff) {
        r.fields_in = ff;
        r.rho_bar_in = fr;
    } else {
        e = copy_in(&r.fields, &fcap, fields, nf, ctx->stream);
        if (e == hipSuccess) e = copy_in(&r.rho_bar, &one, rho_bar, 1, ctx->stream);
        r.fields_in = r.fields;
        r.rho_bar_in = r.rho_bar;
    }
    if (e == hipSuccess) e = ensure(&r.at.states, &r.st_cap, (V > 0 ? V : 1) * (int64_t)t->max_steps);
    if (e == hipSuccess) e = ensure(&r.at.h, &r.h_cap, (int64_t)t->max_steps);
    if (e == hipSuccess) e = ensure(&r.at.count, &cnt, 1);
    r.at.n = V;
    r.at.cap = t->max_steps;
    const int st = commit(ctx, e, "tape (integrate)");
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
    hipError_t e = ensure_adjoint_capacity(ctx, tape_cap, tape_n);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_integrate_adj workspace");
    e = launch_advect_adj(ctx, reinterpret_cast<const float4 *>(fields), rho_bar, &t,
                                     lam_xy, reinterpret_cast<float4 *>(lam_fields), lam_rho_bar);
    return e == hipSuccess ? FFB_OK : hip_fail(ctx, e, "ffb_integrate_adj launch");
}

int ffb_tape_begin(ffb_ctx *ctx, int32_t max_steps)
{
    if (!ctx) return FFB_E_INVALID;
    if (max_steps < 1 || max_steps > (1 << 20))
        return fail(ctx, FFB_E_INVALID, "ffb_tape_begin: max_steps out of range%s");
    if (!ctx->tape) ctx->tape = new ffb_tape();
    ctx->tape->used = 0;          // buffers are kept and reused in stream order
    ++ctx->tape_gen;
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
    ++ctx->tape_gen;
    return FFB_OK;
}

int ffb_tape_generation(const ffb_ctx *ctx, int64_t *out)
{
    if (!ctx || !out) return FFB_E_INVALID;
    *out = ctx->tape_gen;
    return FFB_OK;
}

int ffb_tape_check(ffb_ctx *ctx, int64_t generation)
{
    if (!ctx) return FFB_E_INVALID;
    if (generation != ctx->tape_gen)
        return fail(ctx, FFB_E_NO_TAPE,
                    "ffb_tape_check: the record was replaced or cleared since it was begun%s");
    if (!ctx->tape || ctx->tape->used == 0)
        return fail(ctx, FFB_E_NO_TAPE, "ffb_tape_check: nothing recorded%s");
    return FFB_OK;
}

int ffb_backward(ffb_ctx *ctx, const double *dL_darea, double *dL_dvalue, double *dL_dxy0)
{
    if (!ctx) return FFB_E_INVALID;
    if (!dL_darea || !dL_dvalue) return fail(ctx, FFB_E_INVALID, "ffb_backward: NULL argument%s");
    ffb_tape *t = ctx->tape;
    if (!t || t->used == 0)
        return fail(ctx, FFB_E_NO_TAPE, "ffb_backward: nothing recorded (call ffb_tape_begin)%s");
    t->recording = false;
    std::vector<tape_rec> &recs = t->recs;
    const int64_t used = (int64_t)t->used;
    // the record sequence must be A+ (D F I A+)*
    std::string seq;
    for (int64_t k = 0; k < used; ++k) seq += recs[k].kind;
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
    for (int64_t k = 0; k < used; ++k) {
        const tape_rec &r = recs[k];
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
    if (e == hipSuccess) e = ensure_adjoint_capacity(ctx, t->max_steps, V);
    if (e != hipSuccess) return hip_fail(ctx, e, "ffb_backward workspace");

    {
        zero_spans z{};
        z.p[0] = t->lam_xy;
        z.words[0] = 4 * V;
        z.p[1] = dL_dvalue;
        z.words[1] = 2 * (int64_t)R;
        e = launch_zero_spans(z, s);
    }
    if (e == hipSuccess) e = launch_area_adj(ctx, &recs[used - 1].g, dL_darea, t->lam_xy);
    bool pending = false;           // an area adjoint from a density record waits
    bool cleared = false;           // the next density record's accumulators are zero
    bool suffixed = false;          // ... and its row suffix sums are computed
    for (int64_t k = used - 2; k >= 0 && e == hipSuccess; --k) {
        tape_rec &r = recs[k];
        switch (r.kind) {
        case 'I': {
            // this round's accumulators (the field and rho_bar adjoints, and
            // those of the density record that follows) are zeroed by the
            // integration adjoint's first launch
            zero_spans z{};
            z.p[0] = t->lam_f;
            z.words[0] = 4 * nf;
            z.p[1] = t->lam_rb;
            z.words[1] = 2;
            z.p[2] = t->lam_area;
            z.words[2] = 2 * (int64_t)R;
            z.p[3] = density_adj_total(ctx);
            z.words[3] = 2;
            z.p[4] = ctx->lam_w;
            z.words[4] = 2 * (int64_t)R;
            e = launch_advect_adj(ctx, r.fields_in, r.rho_bar_in, &r.at, t->lam_xy, t->lam_f,
                                  t->lam_rb, &z);
            cleared = e == hipSuccess;
            break;
        }
        case 'F':
            // with the density accumulators zeroed, the flux adjoint's last
            // pass also leaves the row suffix sums the density adjoint reads
            e = launch_flux_adj(ctx, r.sigma, t->lam_f, t->lam_rb, t->lam_rho,
                                cleared ? ctx->acc : nullptr,
                                cleared ? density_adj_total(ctx) : nullptr);
            suffixed = cleared && e == hipSuccess;
            break;
        case 'D': {
            // the area record before it (whose areas the density read) takes
            // lam_area in the same call
            const tape_rec *a = k > 0 && recs[k - 1].kind == 'A' ? &recs[k - 1] : nullptr;
            if (!cleared) e = launch_fill_f64(t->lam_area, R, 0.0, s);
            if (e == hipSuccess)
                e = launch_density_adj(ctx, &r.g, r.value, r.area, t->lam_rho, dL_dvalue,
                                       t->lam_area, t->lam_xy, cleared, suffixed, r.w,
                                       a ? &a->g : nullptr);
            cleared = false;
            suffixed = false;
            pending = a == nullptr;
            break;
        }
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
