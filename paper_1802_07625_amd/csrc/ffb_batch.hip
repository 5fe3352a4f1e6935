// C ABI of batched runs: many independent maps of different grid sizes
// iterated together, each map with its own rounds, blur schedule, step
// control and stopping rule.  One iteration of every still-active map is a
// fixed sequence of launches (densities, transforms, integration, areas and
// loop state); it is captured once in a hipGraph and replayed until no map
// is active, with one 4-byte read per iteration.  The integration runs one
// workgroup per map (no inter-workgroup waits, so the graph needs no
// cooperative launch).  The autotuner times the launch shapes on the batch
// itself: the workgroup size of the transform passes per grid size and of
// the integration.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ffb_internal.h"

using namespace ffbi;

namespace {

constexpr int kMaxClasses = kBatchMaxClasses;   // distinct transform lengths in one batch
constexpr int kFftChoices[] = {64, 128, 256, 512};
constexpr int kAdvectChoices[] = {256, 512, 1024};

template <typename T>
hipError_t upload(T **d, const std::vector<T> &h)
{
    hipError_t e = hipMalloc(reinterpret_cast<void **>(d), sizeof(T) * std::max<size_t>(1, h.size()));
    if (e != hipSuccess || h.empty()) return e;
    return hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
}

template <typename T>
hipError_t alloc(T **d, int64_t n)
{
    return hipMalloc(reinterpret_cast<void **>(d), sizeof(T) * (size_t)std::max<int64_t>(1, n));
}

}  // namespace

struct ffb_batch {
    hipStream_t user_stream = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the transform classes' streams (cs.s[0] = stream) and their events
    class_streams cs{};
    std::string last_error;
    int32_t M = 0;
    std::vector<int32_t> lx, ly;
    int64_t P = 0, plane_total = 0, field_total = 0, acc_total = 0;
    ffb_geometry g{};
    float *xy = nullptr;
    const double *value = nullptr;

    // per-map device arrays
    int32_t *d_lx = nullptr, *d_ly = nullptr, *d_region_off = nullptr, *d_ring_map = nullptr;
    int32_t *d_entry_ring = nullptr;
    int64_t *d_plane_off = nullptr, *d_field_off = nullptr, *d_acc_off = nullptr,
            *d_point_off = nullptr, *d_nvert = nullptr;
    int32_t *d_active = nullptr, *d_round = nullptr, *d_rounds_done = nullptr, *d_order = nullptr,
            *d_stats = nullptr, *d_n_active = nullptr, *d_status = nullptr;
    double *d_max_err = nullptr;
    // launch tables, rows and columns grouped by transform-length class
    int2 *d_rows = nullptr, *d_cols = nullptr;
    int32_t n_rows = 0, n_cols = 0;
    int n_classes = 0;
    int32_t class_n[kMaxClasses];                  // transform length of each class
    int32_t row_beg[kMaxClasses + 1], col_beg[kMaxClasses + 1];
    // workspace
    // density grids and transform planes (FP64)
    double *t1 = nullptr, *pa = nullptr, *pb = nullptr, *pc = nullptr;
    float4 *fields = nullptr;
    double *acc = nullptr, *w_region = nullptr, *rho_pad = nullptr, *rho_bar = nullptr,
           *area = nullptr, *err = nullptr;
    float4 *st0 = nullptr, *st1 = nullptr;
    float2 *kv0 = nullptr, *kv1 = nullptr, *scratch_xy = nullptr;
    double2 *tw1024 = nullptr, *tq1024 = nullptr;
    int32_t *h_n_active = nullptr;                 // pinned host word
    // launch shapes
    int fft_threads[kMaxClasses];
    int advect_threads = 1024;
    bool tuned = false;
    // captured iteration
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ffb_batch_opts graph_opts{};
    bool graph_valid = false;
};

namespace {

int bfail(ffb_batch *b, int code, const std::string &msg)
{
    if (b) b->last_error = msg;
    return code;
}

int bhip(ffb_batch *b, hipError_t e, const char *where)
{
    if (b) b->last_error = std::string(where) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? FFB_E_NOMEM : FFB_E_DEVICE;
}

void free_batch(ffb_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void *ptrs[] = {b->d_lx, b->d_ly, b->d_region_off, b->d_ring_map, b->d_entry_ring, b->d_plane_off,
                    b->d_field_off, b->d_acc_off, b->d_point_off, b->d_nvert, b->d_active,
                    b->d_round, b->d_rounds_done, b->d_order, b->d_stats, b->d_n_active,
                    b->d_status, b->d_max_err, b->d_rows, b->d_cols,
                    b->t1, b->pa, b->pb, b->pc,
                    b->fields, b->acc, b->w_region, b->rho_pad, b->rho_bar, b->area, b->err,
                    b->st0, b->st1, b->kv0, b->kv1, b->scratch_xy, b->tw1024, b->tq1024};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->h_n_active) (void)hipHostFree(b->h_n_active);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cs.fork) (void)hipEventDestroy(b->cs.fork);
    for (int c = 1; c < kMaxClasses; ++c) {
        if (b->cs.join[c]) (void)hipEventDestroy(b->cs.join[c]);
        if (b->cs.s[c]) (void)hipStreamDestroy(b->cs.s[c]);
    }
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

batch_view view_of(const ffb_batch *b, const ffb_batch_opts &o)
{
    batch_view v;
    v.n_maps = b->M;
    v.lx = b->d_lx;
    v.ly = b->d_ly;
    v.plane_off = b->d_plane_off;
    v.field_off = b->d_field_off;
    v.acc_off = b->d_acc_off;
    v.point_off = b->d_point_off;
    v.n_vert = b->d_nvert;
    v.region_off = b->d_region_off;
    v.ring_map = b->d_ring_map;
    v.entry_ring = b->d_entry_ring;
    v.active = b->d_active;
    v.round = b->d_round;
    v.rounds_done = b->d_rounds_done;
    v.max_err = b->d_max_err;
    v.sigma0 = o.sigma0;
    v.stop_err = o.stop_err;
    v.max_rounds = o.max_rounds;
    return v;
}

batch_tables tables_of(const ffb_batch *b)
{
    batch_tables t;
    t.rows = b->d_rows;
    t.cols = b->d_cols;
    t.n_rows = b->n_rows;
    t.n_cols = b->n_cols;
    return t;
}

batch_fft_plan plan_of(const ffb_batch *b, const int *threads)
{
    batch_fft_plan p;
    p.n_classes = b->n_classes;
    for (int c = 0; c <= b->n_classes; ++c) {
        p.row_beg[c] = b->row_beg[c];
        p.col_beg[c] = b->col_beg[c];
    }
    for (int c = 0; c < b->n_classes; ++c) {
        p.threads[c] = threads[c];
        p.n[c] = b->class_n[c];
    }
    return p;
}

// The geometry of all maps over the points the batch advects.
ffb_geometry geom_of(const ffb_batch *b, const float *xy)
{
    ffb_geometry g = b->g;
    g.xy = xy;
    return g;
}

bool opts_equal(const ffb_batch_opts &a, const ffb_batch_opts &b)
{
    const ffb_integrate_opts &x = a.integrate, &y = b.integrate;
    return a.stop_err == b.stop_err && a.max_rounds == b.max_rounds && a.sigma0 == b.sigma0 &&
           x.tol == y.tol && x.h0 == y.h0 && x.safety == y.safety && x.fac_min == y.fac_min &&
           x.fac_max == y.fac_max && x.h_min == y.h_min && x.max_attempts == y.max_attempts;
}

int check_opts(ffb_batch *b, const ffb_batch_opts *o)
{
    if (!o) return bfail(b, FFB_E_INVALID, "batch: NULL options");
    const ffb_integrate_opts &i = o->integrate;
    if (!(o->stop_err > 0.0) || o->max_rounds < 1 || o->max_rounds > 1000 || !(o->sigma0 >= 0.0) ||
        !std::isfinite(o->sigma0))
        return bfail(b, FFB_E_INVALID, "batch: bad stop_err, max_rounds or sigma0");
    if (!(i.tol > 0.0) || !(i.h0 > 0.0) || !(i.safety > 0.0) || !(i.fac_min > 0.0) ||
        !(i.fac_min <= 1.0) || !(i.fac_max >= 1.0) || !(i.h_min >= 0.0) || i.max_attempts <= 0 ||
        i.max_attempts > (1 << 20) || !std::isfinite(i.tol) || !std::isfinite(i.h0))
        return bfail(b, FFB_E_INVALID, "batch: bad integration controller");
    return FFB_OK;
}

batch_advect_args advect_args(ffb_batch *b, const ffb_batch_opts &o, float *xy,
                              const int32_t *replay_off, const double *replay_h)
{
    batch_advect_args a;
    a.fields = b->fields;
    a.rho_bar = b->rho_bar;
    a.xy = reinterpret_cast<float2 *>(xy);
    a.st0 = b->st0;
    a.st1 = b->st1;
    a.kv0 = b->kv0;
    a.kv1 = b->kv1;
    a.stats = b->d_stats;
    a.order = b->d_order;
    a.replay_off = replay_off;
    a.replay_h = replay_h;
    a.tol = o.integrate.tol;
    a.h0 = o.integrate.h0;
    a.safety = o.integrate.safety;
    a.fac_min = o.integrate.fac_min;
    a.fac_max = o.integrate.fac_max;
    a.h_min = o.integrate.h_min;
    a.max_attempts = o.integrate.max_attempts;
    return a;
}

// Every map active at round 0, areas of the current points.
hipError_t enqueue_reset(ffb_batch *b)
{
    hipStream_t s = b->stream;
    hipError_t e = launch_fill_i32(b->d_active, b->M, 1, s);
    if (e == hipSuccess) e = launch_fill_i32(b->d_round, b->M, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(b->d_rounds_done, b->M, 0, s);
    if (e == hipSuccess) e = launch_fill_f64(b->d_max_err, b->M, 0.0, s);
    if (e == hipSuccess) e = launch_fill_i32(b->d_stats, 4 * (int64_t)b->M, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(b->d_n_active, 1, b->M, s);
    if (e == hipSuccess) {
        ffb_geometry g = geom_of(b, b->xy);
        e = launch_ring_areas(s, &g, b->area, b->d_status);
    }
    return e;
}

// One iteration of every active map (the sequence a graph captures).
hipError_t enqueue_step(ffb_batch *b, const ffb_batch_opts &o, float *xy,
                        const int32_t *replay_off, const double *replay_h)
{
    hipStream_t s = b->stream;
    const batch_view bv = view_of(b, o);
    const batch_tables bt = tables_of(b);
    ffb_geometry g = geom_of(b, xy);
    hipError_t e = launch_batch_density(s, bv, bt, &g, b->value, b->area, b->w_region, b->rho_pad,
                                        b->acc, b->acc_total, b->d_status);
    if (e == hipSuccess)
        e = launch_batch_flux(b->cs, bv, bt, plan_of(b, b->fft_threads), b->tw1024, b->tq1024, b->rho_pad,
                              b->acc, b->t1, b->pa, b->pb, b->pc, b->fields, b->rho_bar,
                              b->d_status);
    if (e == hipSuccess)
        e = launch_batch_advect(s, bv, advect_args(b, o, xy, replay_off, replay_h),
                                b->advect_threads, b->d_status);
    if (e == hipSuccess) e = launch_ring_areas(s, &g, b->area, b->d_status);
    if (e == hipSuccess)
        e = launch_batch_finalize(s, bv, b->value, b->area, b->err, b->d_n_active, b->d_status);
    return e;
}

// Order the batch's stream after the caller's and vice versa.
hipError_t enter(ffb_batch *b)
{
    hipError_t e = hipEventRecord(b->ev_in, b->user_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    return e;
}

hipError_t leave(ffb_batch *b)
{
    hipError_t e = hipEventRecord(b->ev_out, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user_stream, b->ev_out, 0);
    return e;
}

hipError_t drop_graph(ffb_batch *b)
{
    hipError_t e = hipSuccess;
    if (b->exec) e = hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
    return e;
}

hipError_t ensure_graph(ffb_batch *b, const ffb_batch_opts &o)
{
    if (b->graph_valid && opts_equal(b->graph_opts, o)) return hipSuccess;
    hipError_t e = drop_graph(b);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e2 = enqueue_step(b, o, b->xy, nullptr, nullptr);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (e2 != hipSuccess) return e2;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
    b->graph_opts = o;
    b->graph_valid = true;
    return hipSuccess;
}

int read_status(ffb_batch *b, int32_t *st)
{
    hipError_t e = hipMemcpyAsync(b->h_n_active, b->d_status, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(b, e, "batch status");
    *st = *b->h_n_active;
    return FFB_OK;
}

// Mean time of `fn` over `reps` runs on the batch stream (after one warm-up).
template <typename F>
float time_it(ffb_batch *b, F fn, int reps, hipError_t *err)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    *err = e;
    return ms / (float)reps;
}

}  // namespace

extern "C" {

int ffb_batch_create(ffb_batch **out, const ffb_batch_desc *d, void *hip_stream)
{
    if (!out) return FFB_E_INVALID;
    *out = nullptr;
    if (!d || d->n_maps < 1 || !d->lx || !d->ly || !d->point_offsets || !d->n_vertices ||
        !d->ring_offsets_map || !d->region_offsets || !d->points || !d->value)
        return FFB_E_INVALID;
    const int32_t M = d->n_maps;
    const ffb_geometry &g = d->geometry;
    if (g.n_rings < 1 || g.n_regions < 1 || !g.ring_offsets || !g.ring_vidx || !g.ring_region ||
        g.n_entries < 3 * (int64_t)g.n_rings || g.n_entries > INT32_MAX)
        return FFB_E_INVALID;
    if (d->point_offsets[0] != 0 || d->ring_offsets_map[0] != 0 || d->region_offsets[0] != 0 ||
        d->point_offsets[M] != g.n_vertices || d->ring_offsets_map[M] != g.n_rings ||
        d->region_offsets[M] != g.n_regions || g.n_vertices > INT32_MAX - 4096)
        return FFB_E_INVALID;
    std::vector<int32_t> widths;
    for (int32_t m = 0; m < M; ++m) {
        const int32_t lx = d->lx[m], ly = d->ly[m];
        auto pow2 = [](int32_t n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; };
        if (!pow2(lx) || !pow2(ly)) return FFB_E_INVALID;
        const int64_t np = d->point_offsets[m + 1] - d->point_offsets[m];
        if (np < 0 || d->n_vertices[m] < 0 || d->n_vertices[m] > np) return FFB_E_INVALID;
        if (d->ring_offsets_map[m + 1] <= d->ring_offsets_map[m] ||
            d->region_offsets[m + 1] <= d->region_offsets[m])
            return FFB_E_INVALID;
        // transform lengths: the rows of a map have length lx, its columns ly
        for (int32_t L : {lx, ly})
            if (std::find(widths.begin(), widths.end(), L) == widths.end()) widths.push_back(L);
    }
    if ((int)widths.size() > kMaxClasses) return FFB_E_INVALID;
    std::sort(widths.begin(), widths.end());

    ffb_batch *b = new ffb_batch();
    b->user_stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->M = M;
    b->g = g;
    b->P = g.n_vertices;
    b->xy = d->points;
    b->value = d->value;
    b->lx.assign(d->lx, d->lx + M);
    b->ly.assign(d->ly, d->ly + M);
    std::vector<int64_t> plane_off(M), field_off(M), acc_off(M), point_off(M + 1), nvert(M);
    std::vector<int32_t> region_off(M + 1), ring_map(g.n_rings), order(M);
    for (int32_t m = 0; m < M; ++m) {
        plane_off[m] = b->plane_total;
        field_off[m] = b->field_total;
        acc_off[m] = b->acc_total;
        b->plane_total += (int64_t)b->lx[m] * b->ly[m];
        b->field_total += (int64_t)(b->lx[m] + 2) * (b->ly[m] + 2);
        b->acc_total += (int64_t)b->ly[m] * (b->lx[m] + 1);
        nvert[m] = d->n_vertices[m];
        for (int32_t r = d->ring_offsets_map[m]; r < d->ring_offsets_map[m + 1]; ++r) ring_map[r] = m;
        order[m] = m;
    }
    for (int32_t m = 0; m <= M; ++m) {
        point_off[m] = d->point_offsets[m];
        region_off[m] = d->region_offsets[m];
    }
    // largest maps first, so that they start first
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return point_off[x + 1] - point_off[x] > point_off[y + 1] - point_off[y];
    });
    // launch tables: the rows of maps with lx = N and the columns of maps
    // with ly = N form class N
    std::vector<int2> rows, cols;
    b->n_classes = (int)widths.size();
    for (int c = 0; c < b->n_classes; ++c) {
        b->class_n[c] = widths[c];
        b->row_beg[c] = (int32_t)rows.size();
        b->col_beg[c] = (int32_t)cols.size();
        for (int32_t m = 0; m < M; ++m) {
            if (b->lx[m] == widths[c])
                for (int j = 0; j < b->ly[m]; j += 2) rows.push_back(make_int2(m, j));
            if (b->ly[m] == widths[c])
                for (int i = 0; i < b->lx[m]; i += 2) cols.push_back(make_int2(m, i));
        }
        // the column pass reads and writes consecutive pairs of one map
        // together (one workgroup takes consecutive entries), so the
        // entries stay in column order
        b->fft_threads[c] = 256;
    }
    b->row_beg[b->n_classes] = (int32_t)rows.size();
    b->col_beg[b->n_classes] = (int32_t)cols.size();
    b->n_rows = (int32_t)rows.size();
    b->n_cols = (int32_t)cols.size();

    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    // one stream per transform class beyond the first (default priority)
    b->cs.n = b->n_classes;
    b->cs.own = true;
    for (int32_t m = 0; m < b->M; ++m) b->cs.own = b->cs.own && b->lx[m] == b->ly[m];
    b->cs.s[0] = b->stream;
    if (e == hipSuccess && b->cs.n > 1)
        e = hipEventCreateWithFlags(&b->cs.fork, hipEventDisableTiming);
    for (int c = 1; c < b->cs.n && e == hipSuccess; ++c) {
        e = hipStreamCreateWithFlags(&b->cs.s[c], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->cs.join[c], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = upload(&b->d_lx, b->lx);
    if (e == hipSuccess) e = upload(&b->d_ly, b->ly);
    if (e == hipSuccess) e = upload(&b->d_plane_off, plane_off);
    if (e == hipSuccess) e = upload(&b->d_field_off, field_off);
    if (e == hipSuccess) e = upload(&b->d_acc_off, acc_off);
    if (e == hipSuccess) e = upload(&b->d_point_off, point_off);
    if (e == hipSuccess) e = upload(&b->d_nvert, nvert);
    if (e == hipSuccess) e = upload(&b->d_region_off, region_off);
    if (e == hipSuccess) e = upload(&b->d_ring_map, ring_map);
    if (e == hipSuccess) e = alloc(&b->d_entry_ring, g.n_entries > 0 ? g.n_entries : 1);
    if (e == hipSuccess)
        e = launch_entry_ring(b->stream, g.ring_offsets, g.n_rings, g.n_entries, b->d_entry_ring);
    if (e == hipSuccess) e = upload(&b->d_order, order);
    if (e == hipSuccess) e = upload(&b->d_rows, rows);
    if (e == hipSuccess) e = upload(&b->d_cols, cols);
    if (e == hipSuccess) e = alloc(&b->d_active, M);
    if (e == hipSuccess) e = alloc(&b->d_round, M);
    if (e == hipSuccess) e = alloc(&b->d_rounds_done, M);
    if (e == hipSuccess) e = alloc(&b->d_stats, 4 * (int64_t)M);
    if (e == hipSuccess) e = alloc(&b->d_n_active, 1);
    if (e == hipSuccess) e = alloc(&b->d_status, 1);
    if (e == hipSuccess) e = alloc(&b->d_max_err, M);
    double **planes[] = {&b->t1, &b->pa, &b->pb, &b->pc};
    for (double **pl : planes)
        if (e == hipSuccess) e = alloc(pl, b->plane_total);
    if (e == hipSuccess) e = alloc(&b->fields, b->field_total);
    if (e == hipSuccess) e = alloc(&b->acc, b->acc_total);
    if (e == hipSuccess) e = alloc(&b->w_region, g.n_regions);
    if (e == hipSuccess) e = alloc(&b->area, g.n_regions);
    if (e == hipSuccess) e = alloc(&b->err, g.n_regions);
    if (e == hipSuccess) e = alloc(&b->rho_pad, M);
    if (e == hipSuccess) e = alloc(&b->rho_bar, M);
    if (e == hipSuccess) e = alloc(&b->st0, b->P);
    if (e == hipSuccess) e = alloc(&b->st1, b->P);
    if (e == hipSuccess) e = alloc(&b->kv0, b->P);
    if (e == hipSuccess) e = alloc(&b->kv1, b->P);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&b->h_n_active), sizeof(int32_t));
    if (e == hipSuccess) {
        // twiddles of the longest transform; shorter ones read them at a stride
        const int N = 1024;
        std::vector<double2> tw(N / 2), tq(N);
        const double pi = 3.14159265358979323846;
        for (int k = 0; k < N / 2; ++k) tw[k] = make_double2(cos(2 * pi * k / N), -sin(2 * pi * k / N));
        for (int m = 0; m < N; ++m)
            tq[m] = make_double2(cos(pi * m / (2.0 * N)), -sin(pi * m / (2.0 * N)));
        e = upload(&b->tw1024, tw);
        if (e == hipSuccess) e = upload(&b->tq1024, tq);
    }
    if (e == hipSuccess) e = launch_fill_i32(b->d_status, 1, 0, b->stream);
    if (e == hipSuccess) e = enqueue_reset(b);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        free_batch(b);
        delete b;
        return e == hipErrorOutOfMemory ? FFB_E_NOMEM : FFB_E_DEVICE;
    }
    *out = b;
    return FFB_OK;
}

int ffb_batch_destroy(ffb_batch *b)
{
    if (!b) return FFB_E_INVALID;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
    delete b;
    return FFB_OK;
}

const char *ffb_batch_last_error(const ffb_batch *b)
{
    return b ? b->last_error.c_str() : "null batch";
}

int ffb_batch_set_shapes(ffb_batch *b, int32_t fft_threads, int32_t advect_threads)
{
    if (!b) return FFB_E_INVALID;
    const bool fft_ok = fft_threads == 0 ||
        std::find(std::begin(kFftChoices), std::end(kFftChoices), fft_threads) != std::end(kFftChoices);
    const bool adv_ok = advect_threads == 0 ||
        std::find(std::begin(kAdvectChoices), std::end(kAdvectChoices), advect_threads) !=
            std::end(kAdvectChoices);
    if (!fft_ok || !adv_ok) return bfail(b, FFB_E_INVALID, "batch: unsupported launch shape");
    if (fft_threads)
        for (int c = 0; c < b->n_classes; ++c) b->fft_threads[c] = fft_threads;
    if (advect_threads) b->advect_threads = advect_threads;
    b->graph_valid = false;
    return FFB_OK;
}

int ffb_batch_get_shapes(const ffb_batch *b, int32_t *n_classes, int32_t *widths,
                         int32_t *fft_threads, int32_t *advect_threads)
{
    if (!b) return FFB_E_INVALID;
    if (n_classes) *n_classes = b->n_classes;
    for (int c = 0; c < b->n_classes; ++c) {
        if (widths) widths[c] = b->class_n[c];
        if (fft_threads) fft_threads[c] = b->fft_threads[c];
    }
    if (advect_threads) *advect_threads = b->advect_threads;
    return FFB_OK;
}

int ffb_batch_reset(ffb_batch *b)
{
    if (!b) return FFB_E_INVALID;
    hipError_t e = enter(b);
    if (e == hipSuccess) e = enqueue_reset(b);
    if (e == hipSuccess) e = leave(b);
    return e == hipSuccess ? FFB_OK : bhip(b, e, "ffb_batch_reset");
}

int ffb_batch_step(ffb_batch *b, const ffb_batch_opts *o, const int32_t *replay_offsets,
                   const double *replay_h)
{
    if (!b) return FFB_E_INVALID;
    int st = check_opts(b, o);
    if (st) return st;
    if ((replay_offsets != nullptr) != (replay_h != nullptr))
        return bfail(b, FFB_E_INVALID, "batch: replay offsets and steps go together");
    hipError_t e = enter(b);
    if (e == hipSuccess) {
        if (o->use_graph && !replay_offsets) {
            e = ensure_graph(b, *o);
            if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
        } else {
            e = enqueue_step(b, *o, b->xy, replay_offsets, replay_h);
        }
    }
    if (e == hipSuccess) e = leave(b);
    return e == hipSuccess ? FFB_OK : bhip(b, e, "ffb_batch_step");
}

int ffb_batch_run(ffb_batch *b, const ffb_batch_opts *o, int32_t *iterations)
{
    if (!b) return FFB_E_INVALID;
    int st = check_opts(b, o);
    if (st) return st;
    hipError_t e = enter(b);
    if (e == hipSuccess) e = enqueue_reset(b);
    if (e == hipSuccess && o->use_graph) e = ensure_graph(b, *o);
    int32_t it = 0;
    while (e == hipSuccess && it < o->max_rounds) {
        e = o->use_graph ? hipGraphLaunch(b->exec, b->stream)
                         : enqueue_step(b, *o, b->xy, nullptr, nullptr);
        ++it;
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->h_n_active, b->d_n_active, sizeof(int32_t),
                               hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e == hipSuccess && *b->h_n_active == 0) break;
    }
    if (iterations) *iterations = it;
    if (e == hipSuccess) e = leave(b);
    if (e != hipSuccess) return bhip(b, e, "ffb_batch_run");
    int32_t status = 0;
    st = read_status(b, &status);
    return st ? st : status;
}

int ffb_batch_results(ffb_batch *b, int32_t *rounds, double *max_err, int32_t *stats,
                      double *area)
{
    if (!b) return FFB_E_INVALID;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && rounds)
        e = hipMemcpy(rounds, b->d_rounds_done, sizeof(int32_t) * b->M, hipMemcpyDeviceToHost);
    if (e == hipSuccess && max_err)
        e = hipMemcpy(max_err, b->d_max_err, sizeof(double) * b->M, hipMemcpyDeviceToHost);
    if (e == hipSuccess && stats)
        e = hipMemcpy(stats, b->d_stats, sizeof(int32_t) * 4 * b->M, hipMemcpyDeviceToHost);
    if (e == hipSuccess && area)
        e = hipMemcpy(area, b->area, sizeof(double) * b->g.n_regions, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) return bhip(b, e, "ffb_batch_results");
    int32_t status = 0;
    int st = read_status(b, &status);
    return st ? st : status;
}

int ffb_batch_autotune(ffb_batch *b, const ffb_batch_opts *o)
{
    if (!b) return FFB_E_INVALID;
    int st = check_opts(b, o);
    if (st) return st;
    hipError_t e = enter(b);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && !b->scratch_xy) e = alloc(&b->scratch_xy, b->P);
    // fields of round 0 from the current points
    const batch_view bv0 = view_of(b, *o);
    ffb_geometry g = geom_of(b, b->xy);
    if (e == hipSuccess) e = enqueue_reset(b);
    if (e == hipSuccess)
        e = launch_batch_density(b->stream, bv0, tables_of(b), &g, b->value, b->area, b->w_region,
                                 b->rho_pad, b->acc, b->acc_total, b->d_status);
    // transform passes: one class at a time, the others fixed
    for (int c = 0; c < b->n_classes && e == hipSuccess; ++c) {
        float best = 1e30f;
        int best_t = b->fft_threads[c];
        for (int t : kFftChoices) {
            if (t < b->class_n[c] / 8) continue;    // runs as N / 8 lanes anyway
            int threads[kMaxClasses];
            std::copy(b->fft_threads, b->fft_threads + b->n_classes, threads);
            threads[c] = t;
            const batch_fft_plan plan = plan_of(b, threads);
            float ms = time_it(b, [&]() {
                return launch_batch_flux(b->cs, bv0, tables_of(b), plan, b->tw1024, b->tq1024,
                                         b->rho_pad, b->acc, b->t1, b->pa, b->pb, b->pc,
                                         b->fields, b->rho_bar, b->d_status);
            }, 3, &e);
            if (e == hipSuccess && ms < best) {
                best = ms;
                best_t = t;
            }
        }
        b->fft_threads[c] = best_t;
    }
    // integration: on a scratch copy of the points
    float best = 1e30f;
    int best_t = b->advect_threads;
    for (int t : kAdvectChoices) {
        if (e != hipSuccess) break;
        float ms = time_it(b, [&]() {
            hipError_t x = hipMemcpyAsync(b->scratch_xy, b->xy, sizeof(float2) * b->P,
                                          hipMemcpyDeviceToDevice, b->stream);
            if (x == hipSuccess)
                x = launch_batch_advect(b->stream, bv0,
                                        advect_args(b, *o, reinterpret_cast<float *>(b->scratch_xy),
                                                    nullptr, nullptr),
                                        t, b->d_status);
            return x;
        }, 2, &e);
        if (e == hipSuccess && ms < best) {
            best = ms;
            best_t = t;
        }
    }
    b->advect_threads = best_t;
    b->tuned = true;
    b->graph_valid = false;
    if (e == hipSuccess) e = enqueue_reset(b);
    if (e == hipSuccess) e = leave(b);
    if (e != hipSuccess) return bhip(b, e, "ffb_batch_autotune");
    int32_t status = 0;
    st = read_status(b, &status);
    return st ? st : status;
}

}  // extern "C"
