// Internal declarations shared by the HIP translation units of libffb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ffb.h"

// Context: stream, sizes, sticky device status and the device workspace.
// FP64 reduction workspace per context: block partials of the sums and
// maxima (largest user: 5 statistics x 2048 blocks of the distortion pass).
constexpr int kRedDoubles = 5 * 2048;

struct ffb_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int32_t lx = 0, ly = 0;
    std::string last_error;

    int32_t *d_status = nullptr;   // sticky device status word

    // transform workspace
    float2 *tw_x = nullptr, *tq_x = nullptr;   // FFT and DCT twiddles for length lx
    float2 *tw_y = nullptr, *tq_y = nullptr;   // ... for length ly
    double2 *tw64_x = nullptr, *tq64_x = nullptr;   // the same tables in FP64 (flux)
    double2 *tw64_y = nullptr, *tq64_y = nullptr;
    // [lx*ly] scratch planes, sized for FP64 (the flux); FP32 users take
    // the first half
    float *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
    float *pa = nullptr, *pb = nullptr, *pc = nullptr;
    double *red = nullptr;                     // reduction partials (kRedDoubles)
    int32_t red_cap = 0;

    // raster workspace
    double *acc = nullptr;                     // [ly][lx+1] coverage deltas
    double *w_region = nullptr;                // [cap] d_r - rho_pad
    double *lam_w = nullptr;                   // [cap] adjoint of w_r
    int32_t w_cap = 0;

    // integrator workspace
    float4 *st[2] = {nullptr, nullptr};        // (hi.x, hi.y, lo.x, lo.y) per point
    float2 *kv[2] = {nullptr, nullptr};        // first stage velocity (FSAL)
    int64_t st_cap = 0;
    uint32_t *errslot = nullptr;               // advection grid-sync words
    int32_t err_cap = 0;
    int adv_blocks = 0;                        // co-resident blocks of the advection kernel
    int adv_mode = 1;                          // advection state placement (FFB_OPT_ADVECT_STATE)
    int adv_cap = 0;                           // cap on advection workgroups, 0 = none

    // spatial point order of the integration (FFB_OPT_POINT_ORDER)
    int ord_mode = 1;
    int32_t *ord_perm = nullptr;               // [n] point index of each sorted slot
    int32_t *ord_rank = nullptr;               // [n] rank of a point within its cell
    int64_t ord_cap = 0;
    int32_t *ord_count = nullptr;              // [lx*ly + 1] points per cell
    int32_t *ord_offs = nullptr;               // [lx*ly + 1] their exclusive scan
    int32_t *ord_sums = nullptr;               // [scan workgroups of lx*ly + 1]
    const void *ord_xy = nullptr;              // mode 3: points and count the saved
    int64_t ord_n = -1;                        // order was computed for

    struct ffb_tape *tape = nullptr;           // recording for ffb_backward
    int64_t tape_gen = 0;                      // bumped by ffb_tape_begin and ffb_tape_clear
    struct diff_ws *diff = nullptr;            // diffusion-variant buffers (on first use)
    int diff_graph = 1;                        // FFB_OPT_DIFFUSION_GRAPH
    struct inverse_ws *inv = nullptr;          // inverse-map workspace (on first use)
    double *adj_t = nullptr;                   // [cap] step start times (adjoint)
    int64_t adj_t_cap = 0;
    float4 *adj_jac = nullptr;                 // [cap][n] step Jacobians (adjoint)
    int64_t adj_jac_cap = 0;
};

// ------------------------------------------------------------ host helpers
namespace ffbi {
// Record `fmt` (with one %s for detail) as the context's last error; returns code.
int fail(ffb_ctx *ctx, int code, const char *fmt, const char *detail = "");
// Record a HIP failure; returns FFB_E_NOMEM or FFB_E_DEVICE.
int hip_fail(ffb_ctx *ctx, hipError_t e, const char *where);
// Host-side checks of a geometry struct (sizes and NULL arrays).
int check_geometry(ffb_ctx *ctx, const ffb_geometry *g);
// Reallocate *p to at least `need` bytes (contents not kept) if `have` is short.
hipError_t grow_bytes(void **p, int64_t have, int64_t need);
template <typename T>
hipError_t grow(T **p, int64_t have, int64_t need)
{
    return grow_bytes(reinterpret_cast<void **>(p), have * (int64_t)sizeof(T),
                      need * (int64_t)sizeof(T));
}
// Per-region workspace (w_region, lam_w) for at least R regions.
hipError_t ensure_region_capacity(ffb_ctx *ctx, int32_t R);
// Integration adjoint workspace for `cap` steps of n points.
hipError_t ensure_adjoint_capacity(ffb_ctx *ctx, int32_t cap, int64_t n);
// Double-buffered integrator state (st, kv) for at least n points.
hipError_t ensure_state_capacity(ffb_ctx *ctx, int64_t n);
// Whether an integration of n points visits them sorted by start cell
// (FFB_OPT_POINT_ORDER), and the sort's buffers for n points.
bool use_point_order(const ffb_ctx *ctx, int64_t n);
hipError_t ensure_order_capacity(ffb_ctx *ctx, int64_t n);
// The visiting order of an integration of the n points at xy, enqueued on
// the context's stream: nullptr (the caller's order) or ctx->ord_perm, sorted
// afresh or, in mode 3, kept from the last sort of the same xy and n.
int32_t *prepare_point_order(ffb_ctx *ctx, const float *xy, int64_t n, hipError_t *err);
// Controller options, step record and replay schedule of an integration.
int check_controller(ffb_ctx *ctx, const ffb_integrate_opts *o, const double *h_out,
                     int32_t h_cap, const char *what);
// Release the diffusion-variant buffers of a context (if any).
void diff_free(ffb_ctx *ctx);
}  // namespace ffbi

// Context tape (recording for ffb_backward).  Each hook returns FFB_OK when
// the context is not recording.  The records' copies of the call's inputs
// (and of the flux outputs) are written by the call's own kernels into the
// buffers a hook hands out, so recording adds no launch; a buffer left null
// means nothing to write.
//   area:    xy of every ring vertex (the area kernel's reads);
//   density: xy of every ring vertex, value, area and the weights w_r;
//   flux:    the fields and rho_bar (what the integration of the round reads).
struct density_snap {
    float2 *xy = nullptr;
    double *value = nullptr, *area = nullptr, *w = nullptr;
};
struct flux_snap {
    float4 *fields = nullptr;
    double *rho_bar = nullptr;
};
int tape_on_area(ffb_ctx *ctx, const ffb_geometry *g, float2 **xy_snap);
int tape_on_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                    const double *area, density_snap *snap);
int tape_on_flux(ffb_ctx *ctx, float sigma, const float4 *fields, const double *rho_bar,
                 flux_snap *snap);
// Sets *record and fills *out with the record's buffers when recording.
int tape_on_integrate(ffb_ctx *ctx, int64_t n, const float4 *fields, const double *rho_bar,
                      struct advect_tape *out, bool *record);
void tape_free(ffb_ctx *ctx);

// ---------------------------------------------------------------- launches
// Every launcher enqueues on ctx->stream and returns hipSuccess or the
// launch error.  Arguments are validated by the C-ABI layer beforehand.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// Exclusive prefix sums of n values (out must not alias a); `sums` holds
// scan_blocks(n) values.
int scan_blocks(int64_t n);
hipError_t launch_scan_i32(const int32_t *a, int32_t *out, int64_t n, int32_t *sums,
                           hipStream_t s);
hipError_t launch_scan_i64(const int64_t *a, int64_t *out, int64_t n, int64_t *sums,
                           hipStream_t s);
// Sorted-slot order of n points by their start cell into ctx->ord_perm
// (workspace ensured by the caller).
hipError_t launch_point_order(ffb_ctx *ctx, const float2 *xy, int64_t n);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
// Several buffers zeroed by one launch: span q is words[q] 4-byte words at p[q]
// (unused spans: words 0).
constexpr int kZeroSpans = 6;
struct zero_spans {
    void *p[kZeroSpans];
    int64_t words[kZeroSpans];
};
hipError_t launch_zero_spans(const zero_spans &z, hipStream_t s);

hipError_t launch_area(const ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                       double *area, double *err, double *max_abs_err,
                       float2 *xy_snap = nullptr);

// With `snap`, the weights go to snap->w (and the raster reads them there).
hipError_t launch_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                          const double *area, double *rho, double *rho_pad,
                          const density_snap *snap = nullptr);

// Transform workspace of one flux call (FP64): twiddle tables of both
// lengths, six [lx*ly] planes and kRedDoubles reduction partials.
struct flux_ws {
    double2 *tw_x, *tq_x, *tw_y, *tq_y;
    double *t1, *pa, *pb, *pc;          // [ly][lx] planes: row DCTs, column-pass outputs
    double *red;
};
hipError_t launch_flux_ws(hipStream_t s, int lx, int ly, const flux_ws &w, const double *rho,
                          float sigma, float4 *fields, double *rho_bar, int32_t *status,
                          const flux_snap *snap = nullptr);
// FP64 twiddle tables of length N on the device (tw: N/2 entries, tq: N).
hipError_t launch_twiddles(hipStream_t s, int N, double2 *tw, double2 *tq);
hipError_t launch_flux(ffb_ctx *ctx, const double *rho, float sigma, float4 *fields,
                       double *rho_bar, const flux_snap *snap = nullptr);
hipError_t launch_pack_fields(ffb_ctx *ctx, const float *jx, const float *jy,
                              const float *rho_s, float4 *fields);

hipError_t launch_density_weights(ffb_ctx *ctx, int32_t R, const double *value,
                                  const double *area, double *rho_pad);

// Where ffb_integrate records what its adjoint needs (all device memory).
struct advect_tape {
    float4 *states;       // [cap][n] (hi.x, hi.y, lo.x, lo.y) before each accepted step
    int64_t n;            // recorded points: the first n of the integration
    int32_t cap;          // steps the record holds
    double *h;            // [cap] accepted step sizes
    int32_t *count;       // [1] accepted steps of the integration
};

hipError_t launch_distortion(ffb_ctx *ctx, int lx, int ly, const float2 *nodes, double *stats,
                             float *e, float *e_tilde);

int advect_max_blocks(int *out);
hipError_t launch_advect(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                         float2 *xy, int64_t n, const ffb_integrate_opts *o,
                         int32_t *stats, double *h_out, int32_t h_cap, const advect_tape *tape,
                         const int32_t *perm);

// Adjoints.  lam_fields has the ghosted layout of the fields, [(ly+2)(lx+2)]
// float4 (J_x, J_y, rho_s, unused); lam_xy is [n][2] FP64.
hipError_t launch_area_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *lam_area,
                           double *lam_xy);
// `cleared`: the caller has already zeroed the context's density-adjoint
// accumulators (density_adj_scratch) on the stream.
// `suffixed`: the row suffix sums of lam_rho are in ctx->acc and their total
// in density_adj_total (from launch_flux_adj; implies `cleared`).  `w`
// (optional): the forward's weights w_r, else they are recomputed from value
// and area.  `area_g` (optional): also the area adjoint of that geometry
// with the lam_area just formed (lam_area zero before the call when
// `cleared`), fused into the last launch when the regions are few.
hipError_t launch_density_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                              const double *area, const float *lam_rho, double *lam_value,
                              double *lam_area, double *lam_xy, bool cleared = false,
                              bool suffixed = false, const double *w = nullptr,
                              const ffb_geometry *area_g = nullptr);
// The context's accumulators that launch_density_adj starts from zero: the
// sum of lam_rho (one double) and the per-region coverage sums (R doubles).
inline double *density_adj_total(ffb_ctx *ctx) { return ctx->red + 513; }
// With `suf` (optional): also the row suffix sums of lam_rho, rows of lx + 1
// doubles, and their total added to *total (which the caller zeroed).
hipError_t launch_flux_adj(ffb_ctx *ctx, float sigma, const float4 *lam_fields,
                           const double *lam_rho_bar, float *lam_rho, double *suf = nullptr,
                           double *total = nullptr);
// `clear` (optional): spans zeroed on the stream before any adjoint is added
// (by the launch that also sums the step start times).
hipError_t launch_advect_adj(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                             const advect_tape *tape, double *lam_xy, float4 *lam_fields,
                             double *lam_rho_bar, const zero_spans *clear = nullptr);

// ---------------------------------------------------------------- inverse
// Workspace of the inverse of the piecewise-linear T (grown on demand).
struct inverse_ws {
    int32_t *count = nullptr, *offs = nullptr;   // [bins + 1]
    int32_t *fill = nullptr;                     // [bins]
    int32_t *sums = nullptr;                     // [scan workgroups]
    int32_t *order = nullptr, *best = nullptr;   // [queries]
    int32_t *big = nullptr;                      // [triangles] list of large image boxes
    int64_t *big_nb = nullptr, *big_off = nullptr;  // [triangles + 1] their bin counts, scanned
    int64_t *sums64 = nullptr;                   // [scan workgroups of triangles + 1]
    int32_t *n_big = nullptr;                    // [1]
    int64_t bins_cap = 0, q_cap = 0, sums_cap = 0, tri_cap = 0;
};
hipError_t launch_inverse(ffb_ctx *ctx, int lx, int ly, const float2 *nodes, const float2 *q,
                          int64_t nq, int32_t *tri, double2 *pre, inverse_ws *w);

// ---------------------------------------------------------------- diffusion
// Control block of a diffusion integration (device memory).  The attempt's
// kernels read the step and the stage times from it; the control kernel
// takes the accept/reject decision and arms the next attempt.  Every kernel
// of an attempt returns at once when `done` is set, so surplus replays of
// the attempt graph do nothing.
constexpr int kDiffSlots = 5;        // distinct stage times of an attempt
struct diff_ctl {
    double t, h, h_att, t_end;
    double ts[kDiffSlots];           // stage times t + c_s h of the armed attempt
    double tol, h0, safety, fac_min, fac_max, h_min;
    const double *replay_h;
    double *h_out;
    int32_t *stats;                  // [4] accepted, rejected, attempts, status
    int32_t n_replay, max_attempts, h_cap;
    int32_t acc, rej, attempts, cur, done, last_rejected, final_step, status;
};

// Device buffers of the diffusion path of one context.
struct diff_ws {
    int64_t plane = 0;               // lx * ly
    int64_t fplane = 0;              // (lx + 2) * (ly + 2)
    float *spec = nullptr;           // [lx][ly] blurred coefficients (m-major)
    float *q = nullptr;              // [3][kDiffSlots][lx][ly] column-pass output
    float *r = nullptr;              // [3][kDiffSlots][ly][lx] transposed
    float4 *fields = nullptr;        // [kDiffSlots][(ly+2)(lx+2)] fields per stage time
    diff_ctl *ctl = nullptr;
    float *part = nullptr;           // [kDiffMaxBlocks] error maxima per workgroup
    int32_t *done_host = nullptr;    // pinned host copy of ctl->done
    hipStream_t stream = nullptr;    // private stream (capturable), ordered with the caller's
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the captured attempt and what it was captured for
    hipGraphExec_t exec = nullptr;
    int64_t exec_n = -1;
    const void *exec_st = nullptr, *exec_st1 = nullptr, *exec_kv = nullptr, *exec_kv1 = nullptr;
    bool use_graph = true;
};
constexpr int kDiffMaxBlocks = 2048;

// Blurred cosine coefficients of rho (Eq. 7 and the blur), m-major, into spec.
hipError_t launch_diff_spectrum(ffb_ctx *ctx, const double *rho, float sigma, float *spec);
// Fields at the first `slots` stage times of ctl (slots <= kDiffSlots).
hipError_t launch_diff_fields(ffb_ctx *ctx, diff_ws *w, int slots);
// Initial state (hi = xy, lo = 0) and first-stage velocity at t = 0 (slot 0).
// perm (optional): slot k of the state holds point perm[k]
hipError_t launch_diff_init_points(ffb_ctx *ctx, diff_ws *w, const float2 *xy, int64_t n,
                                   const int32_t *perm);
// One attempt's point pass and its control step.
hipError_t launch_diff_points(ffb_ctx *ctx, diff_ws *w, int64_t n);
hipError_t launch_diff_control(ffb_ctx *ctx, diff_ws *w, int64_t n, int arm_only);
// Positions out of the current state buffer (if the integration succeeded).
hipError_t launch_diff_finish(ffb_ctx *ctx, diff_ws *w, float2 *xy, int64_t n,
                              const int32_t *perm);
// Copy `init` into the device control block (a kernel, so graph-safe).
hipError_t launch_diff_setup(ffb_ctx *ctx, diff_ws *w, const diff_ctl &init);

// ---------------------------------------------------------------- batches
// Device view of a batch of maps, passed by value to the batched kernels.
// Map m owns grid planes at plane_off[m] ([ly][lx] doubles), fields at
// field_off[m] ([(ly+2)][(lx+2)] float4), coverage deltas at acc_off[m]
// ([ly][lx+1] doubles), points [point_off[m], point_off[m+1]) of which the
// first n_vert[m] are its vertices, and regions [region_off[m],
// region_off[m+1]).  Rings and regions use global indices.
struct batch_view {
    int32_t n_maps;
    const int32_t *lx, *ly;
    const int64_t *plane_off, *field_off, *acc_off, *point_off, *n_vert;
    const int32_t *region_off;
    const int32_t *ring_map;       // [G] map of each ring
    const int32_t *entry_ring;     // [E] ring of each ring entry (fixed per batch)
    int32_t *active;               // [M] 1 while the map iterates
    int32_t *round;                // [M] 0-based round index of the next iteration
    int32_t *rounds_done;          // [M] rounds taken when the map stopped
    double *max_err;               // [M] max |e_r| after the last iteration
    double sigma0;                 // blur of round k = sigma0 * 2^-k
    double stop_err;               // stop when max |e_r| < stop_err
    int32_t max_rounds;
};

// Launch tables: entry k of a table names (map, index) for block k.
struct batch_tables {
    const int2 *rows;              // (map, j0) for every even row j0 of every map
    const int2 *cols;              // (map, m0) for every even column m0
    int32_t n_rows, n_cols;
};

// Batched launchers (k_area.hip, k_raster.hip, k_flux.hip, k_advect.hip).
hipError_t launch_ring_areas(hipStream_t s, const ffb_geometry *g, double *area, int32_t *status);
hipError_t launch_batch_finalize(hipStream_t s, const batch_view &bv, const double *value,
                                 const double *area, double *err, int32_t *n_active,
                                 int32_t *status);
// Ring of every ring entry, entry_ring[k] = g for off[g] <= k < off[g + 1].
hipError_t launch_entry_ring(hipStream_t s, const int32_t *off, int32_t G, int64_t E,
                             int32_t *entry_ring);
// Coverage deltas of every active map into acc (rows of lx + 1); the row
// prefix sums that turn them into densities are the first pass of
// launch_batch_flux.
hipError_t launch_batch_density(hipStream_t s, const batch_view &bv, const batch_tables &bt,
                                const ffb_geometry *g, const double *value, const double *area,
                                double *w_region, double *rho_pad, double *acc, int64_t acc_total,
                                int32_t *status);
// Row and column tables are sorted by grid width; class c owns entries
// [row_beg[c], row_beg[c+1]) and [col_beg[c], col_beg[c+1]) and its passes
// run with threads[c] lanes per workgroup.
constexpr int kBatchMaxClasses = 8;
struct batch_fft_plan {
    int n_classes;
    int32_t row_beg[kBatchMaxClasses + 1], col_beg[kBatchMaxClasses + 1];
    int threads[kBatchMaxClasses];
    int n[kBatchMaxClasses];           // transform length of each class
};
// Streams of a batch's transform classes: class c's passes run on s[c]; s[0]
// is the batch stream, on which the transforms start and end (an event fork
// before and a join after, so that a graph captured from s[0] holds the
// classes' launches as parallel branches).  With `own` (every map square,
// so a class's passes read only its own maps' earlier passes) each class
// runs its passes back to back; otherwise the classes are joined after
// every pass.  n <= 1: s[0] only.
struct class_streams {
    int n;
    bool own;
    hipStream_t s[kBatchMaxClasses];
    hipEvent_t fork;
    hipEvent_t join[kBatchMaxClasses];
};
hipError_t launch_batch_flux(const class_streams &cs, const batch_view &bv, const batch_tables &bt,
                             const batch_fft_plan &plan, const double2 *tw1024,
                             const double2 *tq1024, const double *rho_pad, double *acc,
                             double *t1, double *pa, double *pb, double *pc,
                             float4 *fields, double *rho_bar, int32_t *status);
struct batch_advect_args {
    const float4 *fields;
    const double *rho_bar;         // [M]
    float2 *xy;
    float4 *st0, *st1;
    float2 *kv0, *kv1;
    int32_t *stats;                // [M][4]
    const int32_t *order;          // [M] map of block b (largest first)
    const int32_t *replay_off;     // [M + 1] or NULL
    const double *replay_h;
    double tol, h0, safety, fac_min, fac_max, h_min;
    int32_t max_attempts;
};
hipError_t launch_batch_advect(hipStream_t s, const batch_view &bv, const batch_advect_args &a,
                               int threads, int32_t *status);

// ---------------------------------------------------------------- device
// Record the first error code in the sticky status word.
__device__ inline void set_status(int32_t *status, int32_t code)
{
    atomicCAS(status, 0, code);
}

// Ring of ring entry k: the largest g in [0, G) with off[g] <= k (binary
// search over off[0..G]; the caller checks off[g] <= k < off[g + 1]).
// Kernels with one entry per lane first copy off[0..G] to LDS when it fits
// (kStagedRingOffsets ints): each step of the search is then an LDS read
// instead of a dependent global load.
constexpr int kStagedRingOffsets = 4096;

__device__ inline int32_t ring_search(const int32_t *off, int32_t G, int64_t k)
{
    int32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

// Copies off[0..G] to s_off when it fits; every thread of the workgroup
// calls it (it passes a barrier).  Returns whether s_off holds the offsets.
__device__ inline bool stage_ring_offsets(const int32_t *__restrict__ off, int32_t G,
                                          int32_t *s_off)
{
    if (G + 1 > kStagedRingOffsets) return false;
    for (int i = threadIdx.x; i <= G; i += blockDim.x) s_off[i] = off[i];
    __syncthreads();
    return true;
}
