/*
 * ffb.h -- C ABI of the MI355X (gfx950) implementation of one iteration of
 * the fast flow-based cartogram method (Gastner, Seguy & More, "Fast
 * flow-based algorithm for creating density-equalizing map projections").
 *
 * One iteration ("round") of the method:
 *   1. ffb_area_error  -- region areas and relative area errors (the stopping
 *                         rule of the benchmarking section: stop when the
 *                         largest relative area error is below 1 %);
 *   2. ffb_density     -- region densities value/area painted onto the
 *                         lx x ly grid with exact cell coverage, the space
 *                         outside the map at the mean density;
 *   3. ffb_flux        -- Gaussian blur, the cosine coefficients of Eq. 7 and
 *                         the flux series of the SI Appendix (section 2) for
 *                         linear equalisation, evaluated on the grid nodes;
 *   4. ffb_integrate   -- every point advected from t = 0 to t = 1 with
 *                         v = J / rho_t (Eq. 4-6), bilinear interpolation
 *                         between grid nodes and adaptive Dormand-Prince 5(4)
 *                         steps shared by all points (main text, section
 *                         "Flow-based cartogram with linear equalization");
 *   5. ffb_area_error  -- again, on the advected polygons.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE memory unless marked (host).  The caller owns every
 *    buffer it passes and keeps it alive until the stream has passed the
 *    work; the library never frees caller memory.
 *  - Every call only enqueues work on the context's HIP stream and returns.
 *    Host-detectable argument errors return a non-zero status before any
 *    launch (ffb_last_error has the detail).  Errors found on the device
 *    (non-finite or out-of-box coordinates, non-positive densities, step
 *    underflow, malformed rings) set a sticky status word that ffb_sync
 *    returns; later kernels of the same context see it and do nothing.
 *  - Grids are row-major with x fastest: cell (i, j) = [i, i+1] x [j, j+1]
 *    is element j * lx + i; its node (centre) is (i + 1/2, j + 1/2).
 *  - lx and ly are powers of two in [8, 1024].  Coordinates live in the box
 *    [0, lx] x [0, ly] whose edges reflect the flow.
 *  - Precision: FP32 fields and positions; FP64 for area sums, the
 *    density grid, the transforms of ffb_flux (the fields are rounded to
 *    FP32 once, at the end), the padding density, the mean density rho_bar
 *    and the step controller.  The density grid is FP64 because rounding it
 *    to FP32 (a relative change of 6e-8 per cell) already moves the most
 *    sensitive trajectories of a 1024 x 1024 map with a 700:1 density
 *    range by up to 5e-4 grid units.
 *  - One context per stream; a context is not thread-safe.
 *
 * Gradients (not part of the paper's method): the adjoint calls at the end
 * of this header differentiate the rounds above in reverse mode, for a
 * scalar loss of the final region areas, with the integration's accepted
 * step sizes frozen.
 */
#ifndef FFB_H
#define FFB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffb_ctx ffb_ctx;

enum {
    FFB_OK = 0,
    FFB_E_INVALID = 1,          /* bad argument, malformed rings            */
    FFB_E_NOMEM = 2,            /* device allocation failed                 */
    FFB_E_DEVICE = 3,           /* HIP runtime or launch failure            */
    FFB_E_NONPOSITIVE = 4,      /* value, area or blurred density <= 0      */
    FFB_E_DOMAIN = 5,           /* polygon vertex outside the box           */
    FFB_E_STEP_UNDERFLOW = 6,   /* adaptive step fell below h_min           */
    FFB_E_NONFINITE = 7,        /* NaN or Inf in coordinates or velocities  */
    FFB_E_NO_TAPE = 8,          /* backward without a complete record       */
    FFB_E_MAX_ATTEMPTS = 9,     /* integration used up max_attempts         */
    FFB_E_TOO_LARGE = 10        /* size beyond a fixed workspace's maximum  */
};

/* Polygon geometry in CSR-ring form over unique vertices (a region is one or
 * more rings; counter-clockwise rings add area, clockwise rings are holes).
 * The struct itself is host memory; its arrays are device memory. */
typedef struct {
    int64_t n_vertices;          /* V                                         */
    const float *xy;             /* [V][2] vertex coordinates (box units)     */
    int32_t n_rings;             /* G                                         */
    const int32_t *ring_offsets; /* [G + 1], ring g is entries [off[g], off[g+1]) */
    const int32_t *ring_vidx;    /* [E] vertex index of each ring entry       */
    const int32_t *ring_region;  /* [G] region of each ring, in [0, R)        */
    int32_t n_regions;           /* R                                         */
    int64_t n_entries;           /* E = ring_offsets[G] (passed by the host)  */
} ffb_geometry;

/* Controller of the adaptive integration (host struct).  The paper only says
 * that a predictor-corrector method adapts the next step; these constants
 * are the caller's choice.  An attempt of size h has error estimate
 * err = max over points and components |h sum_s (b_s - b*_s) k_s| (grid
 * units); it is accepted iff err <= tol; then h *= clamp(safety *
 * (err/tol)^(-1/5), fac_min, fac_max), with no growth right after a
 * rejection; a rejection multiplies h by max(fac_min, safety *
 * (err/tol)^(-1/5)).  The last step is clipped to end exactly at t = 1. */
typedef struct {
    double tol;            /* > 0, e.g. 1e-3                                   */
    double h0;             /* first attempted step, e.g. 1e-2                  */
    double safety;         /* e.g. 0.9                                         */
    double fac_min;        /* e.g. 0.2                                         */
    double fac_max;        /* e.g. 5                                           */
    double h_min;          /* step underflow threshold, e.g. 1e-7              */
    int32_t max_attempts;  /* attempts allowed before FFB_E_MAX_ATTEMPTS       */
    int32_t n_replay;      /* > 0: take exactly these accepted steps (below)   */
    const double *replay_h;/* device [n_replay] step sizes summing to 1, or NULL */
} ffb_integrate_opts;

/* Create a context bound to `hip_stream` (a hipStream_t, NULL = default
 * stream) for an lx x ly grid.  `max_points` sizes the integrator's state
 * buffers (they grow on demand later; growth allocates).  *out (host)
 * receives the context.  Returns FFB_E_INVALID for bad sizes. */
int ffb_create(ffb_ctx **out, int32_t lx, int32_t ly, int64_t max_points, void *hip_stream);

/* Free the context and its device workspace (waits for its stream). */
int ffb_destroy(ffb_ctx *ctx);

/* Wait for the stream; return the sticky device status (FFB_OK if none). */
int ffb_sync(ffb_ctx *ctx);

/* Clear the sticky device status (enqueued on the stream). */
int ffb_reset_status(ffb_ctx *ctx);

/* Human-readable detail of the last host-side failure (host string owned by
 * the context; valid until the next call on it). */
const char *ffb_last_error(const ffb_ctx *ctx);

/* Implementation options of a context (host call, takes effect for later
 * calls).  They change where work happens, never what is computed beyond
 * FP32 rounding.
 *   FFB_OPT_ADVECT_STATE: where ffb_integrate keeps each point's state
 *     0 = device memory (any number of points);
 *     1 = LDS, first-stage velocity carried between steps (default);
 *     2 = LDS, first-stage velocity recomputed each step.
 *     Modes 1 and 2 apply when one workgroup's share of points fits in LDS
 *     (about 2.5 M points on 256 CUs); otherwise mode 0 runs.
 *   FFB_OPT_ADVECT_BLOCKS: cap on the persistent workgroups of
 *     ffb_integrate (0 = one per CU, the default).
 *   FFB_OPT_DIFFUSION_GRAPH: ffb_diffusion replays one captured graph per
 *     attempt (1, default) or launches each attempt's kernels (0).
 *   FFB_OPT_POINT_ORDER: order in which ffb_integrate, the recording
 *     forward and ffb_diffusion visit the points; results are the same bits
 *     in every mode, only the cost of the field lookups changes.
 *     0 = the caller's order;
 *     1 = sorted by the grid cell each point starts in when n >= 65536
 *         and the packed fields exceed 8 MB (lx * ly > 2^19; default; the
 *         sort is five short launches on the call's stream, ~45 us at
 *         1024 x 1024 with 2 M points);
 *     2 = sorted for every n > 0;
 *     3 = as 1, but a call with the same xy pointer and n as the call that
 *         last sorted reuses that order instead of sorting again (for
 *         loops of rounds over one point array, whose points move smoothly;
 *         any order gives the same results, a kept one may only be slower).
 *         Setting the option (any value) drops a kept order.
 *     The sort keeps n int32 slots and 2 (lx*ly + 1) int32 cell tables in
 *     the context.
 * Returns FFB_E_INVALID for an unknown option or value. */
enum { FFB_OPT_ADVECT_STATE = 1, FFB_OPT_ADVECT_BLOCKS = 2, FFB_OPT_DIFFUSION_GRAPH = 3,
       FFB_OPT_POINT_ORDER = 4 };
int ffb_set_option(ffb_ctx *ctx, int32_t option, int32_t value);

/* Areas and relative area errors (benchmarking section, stopping rule).
 *   area[r]  (out, [R]) = sum over the rings of region r of the shoelace sum
 *            1/2 sum_k (x_k y_{k+1} - x_{k+1} y_k), FP64 sums of products of
 *            the FP32 coordinates;
 *   err[r]   (out, [R]) = area_r / T_r - 1 with T_r = value_r sum(area)/sum(value);
 *   max_abs_err (out, [1]) = max_r |err[r]|.
 * value[r] (in, [R]) is the region's statistic, > 0 (else FFB_E_NONPOSITIVE
 * on the device).  Malformed rings (offsets out of range, fewer than three
 * entries, vertex or region index out of range) give FFB_E_INVALID on the
 * device; NaN/Inf coordinates give FFB_E_NONFINITE. */
int ffb_area_error(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                   double *area, double *err, double *max_abs_err);

/* Density grid (section on previous all-coordinates methods: region density
 * = statistic / area; benchmarking section: the box around the map holds the
 * mean density).  With d_r = value_r / area_r and
 * rho_pad = sum(value) / sum(area),
 *   rho[j][i] = rho_pad + sum_r (d_r - rho_pad) * |cell(i,j) ∩ region_r|
 * (exact signed coverage of each cell).  area is ffb_area_error's output for
 * the same vertices.  rho (out) is [ly][lx] FP64, rho_pad (out) [1] FP64.
 * Vertices outside [0,lx] x [0,ly] give FFB_E_DOMAIN on the device. */
int ffb_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                const double *area, double *rho, double *rho_pad);

/* Blur and flux (Eq. 7; SI Appendix section 2, flux of linear equalisation).
 * From rho [ly][lx] (in, FP64), with FP64 transforms:
 *   rt_mn  = 4 S_mn / ((1+delta_m0)(1+delta_n0)),
 *            S_mn = sum_ij rho_ij cos(pi m (i+1/2)/lx) cos(pi n (j+1/2)/ly);
 *   rts_mn = rt_mn exp(-pi^2 sigma^2 (m^2/lx^2 + n^2/ly^2) / 2)   (sigma >= 0,
 *            grid cells: the Gaussian blur applied before integration);
 *   rho_s  = (1/(lx ly)) sum_mn rts_mn cos cos;
 *   J_x    = (ly/pi) sum_{m>=1} m/(m^2 ly^2 + n^2 lx^2) rts_mn sin cos;
 *   J_y    = (lx/pi) sum_{n>=1} n/(m^2 ly^2 + n^2 lx^2) rts_mn cos sin;
 * on the nodes, written as fields (out) = float4 [(ly+2)][(lx+2)] holding
 * (J_x, J_y, rho_s, 0) with a one-node ghost border: node (i, j) is element
 * (j+1)(lx+2) + (i+1); ghost nodes hold the series' values at the mirrored
 * cell centres (J_x odd and J_y even across x edges, J_x even and J_y odd
 * across y edges, rho_s even).  rho_bar (out, [1], FP64) = mean of rho.
 * min rho_s <= 0 gives FFB_E_NONPOSITIVE on the device. */
int ffb_flux(ffb_ctx *ctx, const double *rho, float sigma, float *fields, double *rho_bar);

/* ffb_flux for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and output as ffb_flux, with no context.  lx, ly: powers
 * of two in [8, 512] (FFB_E_TOO_LARGE above 512, FFB_E_INVALID otherwise);
 * rho (in, [ly][lx] FP64), fields (out, ghosted layout as ffb_flux),
 * rho_bar (out, [1] FP64), status (in/out, [1] int32, device): a sticky
 * status word the call sets to FFB_E_NONPOSITIVE if min rho_s <= 0 (the
 * caller clears it); hip_stream: the stream to enqueue on (the current
 * device must be the stream's).  The transform workspace (about 8.4 MB) is
 * a fixed device array of the library, one per device, looked up on the
 * first call on a device; the call allocates nothing.  Calls that overlap
 * on one device (several streams or host threads) race on that array.
 * Returns FFB_E_INVALID for NULL pointers, bad sizes or sigma, and
 * FFB_E_DEVICE for a launch failure. */
int ffb_flux_noalloc(int32_t lx, int32_t ly, const double *rho, float sigma, float *fields,
                     double *rho_bar, int32_t *status, void *hip_stream);

/* Pack node arrays jx, jy, rho_s ([ly][lx] each, in) into the ghosted
 * float4 field layout of ffb_flux (out, [(ly+2)][(lx+2)][4]). */
int ffb_pack_fields(ffb_ctx *ctx, const float *jx, const float *jy, const float *rho_s,
                    float *fields);

/* Advect n points xy ([n][2], in/out, FP32) from t = 0 to t = 1 through
 * v(r, t) = J(r) / ((1 - t) rho_s(r) + t rho_bar) (Eq. 4-6), with node
 * velocities interpolated bilinearly (lookups clamped to the box, ghost
 * nodes from `fields`) and Dormand-Prince 5(4) steps shared by all points.
 * fields and rho_bar are ffb_flux outputs (or ffb_pack_fields + a caller
 * value).  During the call positions are carried as compensated FP32 pairs;
 * the result is rounded to FP32.  opts (host) is read at the call.
 * stats (out, [4] int32): accepted, rejected, attempts, final status.
 * h_out (out, [h_cap] FP64, may be NULL): the accepted step sizes in order.
 * The whole integration is one persistent launch: step control happens on
 * the device, with no host round trip per step. */
int ffb_integrate(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy,
                  int64_t n, const ffb_integrate_opts *opts, int32_t *stats,
                  double *h_out, int32_t h_cap);

/* ------------------------------------------------------- diffusion variant
 * The diffusion cartogram written as a flow-based projection (SI Appendix,
 * section 2, the diffusion choice of f_mn), the comparison method of the
 * paper: with the blurred coefficients rts_mn of ffb_flux and
 *   f_mn(t) = exp(-(m^2/lx^2 + n^2/ly^2) t),
 *   rho(t)  = (1/(lx ly)) sum_mn rts_mn f_mn(t) cos(m pi x/lx) cos(n pi y/ly),
 *   J_x(t)  = (1/(lx ly)) sum (m / (pi lx)) rts_mn f_mn(t) sin(...) cos(...),
 *   J_y(t)  = (1/(lx ly)) sum (n / (pi ly)) rts_mn f_mn(t) cos(...) sin(...),
 * the points move with v = J(t) / rho(t) (bilinear between the nodes, as
 * ffb_integrate).  Unlike the main method the fields depend on t, so they
 * are rebuilt at every stage time, and the flow runs to t = infinity,
 * approximated by a cut-off t_end.
 *
 * ffb_diffusion_fields: fields (out, ghosted layout as ffb_flux) at time t
 * (>= 0) for the raster density rho (in, [ly][lx] FP64) blurred by sigma
 * (FP32 transforms).  Enqueue-only. */
int ffb_diffusion_fields(ffb_ctx *ctx, const double *rho, float sigma, double t, float *fields);

/* ffb_diffusion: advect xy (in/out, [n][2] FP32) from t = 0 to t_end (> 0)
 * with the same controller as ffb_integrate (opts; a replayed schedule must
 * sum to t_end), stats (out, [4]: accepted, rejected, attempts, status) and
 * h_out (out, [h_cap] accepted steps, may be NULL with h_cap = 0).  Per
 * attempt the fields at the five distinct stage times are rebuilt in one
 * batched set of transforms, then every point takes the six stages.  The
 * call returns when the integration has ended: it waits for its work once
 * per few attempts (the number of attempts is decided on the device).  Host
 * argument errors return FFB_E_INVALID before any launch; device errors
 * (non-positive rho(t), non-finite steps, step underflow, too many
 * attempts) land in stats[3] and the sticky status, and leave xy as it was. */
int ffb_diffusion(ffb_ctx *ctx, const double *rho, float sigma, double t_end, float *xy, int64_t n,
                  const ffb_integrate_opts *opts, int32_t *stats, double *h_out, int32_t h_cap);

/* Angular distortion of the cartogram (main text, section "Measures of
 * distortion"; SI Appendix section 3).  nodes (in, device, [ly][lx][2] FP32)
 * are the images of the cell centres (i + 1/2, j + 1/2) of an lx x ly grid
 * (any sizes >= 2, independent of the context's transform sizes; the context
 * gives the stream and the reduction workspace) in row-major order, e.g. the
 * grid nodes after the rounds.  On each of the (lx-1)(ly-1) unit squares
 * between four neighbouring nodes, grad T is the Jacobian of the bilinear
 * interpolant of the node images at the square's centre; its singular values
 * a >= b (the semi-axes of the Tissot ellipse) give e = ln(a/b) and
 * e~ = 2 arcsin((a-b)/(a+b)).  stats (out, [5] FP64) = e_a (mean of e over the
 * squares, all of unit area on the input map), e_inf (max), e~_a, e~_inf and
 * the number of squares with det(grad T) <= 0 (folded).  e and e_tilde (out,
 * [(ly-1)][(lx-1)] FP32, each may be NULL) receive the per-square values.
 * FP64 arithmetic on the FP32 positions.  Returns FFB_E_INVALID for NULL
 * nodes or stats, or a grid below 2 x 2 nodes; all outputs device memory,
 * written in stream order. */
int ffb_distortion(ffb_ctx *ctx, int32_t lx, int32_t ly, const float *nodes, double *stats,
                   float *e, float *e_tilde);

/* Inverse of the piecewise-linear approximation of T (Conclusion: the
 * graticule of the inverse transformation, obtained by approximating T as
 * piecewise linear and inverting it).  nodes (in, device, [ly][lx][2] FP32):
 * images of the cell centres (i + 1/2, j + 1/2) of an lx x ly grid (any
 * sizes >= 2 up to 2^26 nodes; the context lends its stream and a workspace
 * grown on demand).  Each cell c = j (lx-1) + i is split along its
 * (i,j)-(i+1,j+1) diagonal into triangles 2c = (i,j),(i+1,j),(i+1,j+1) and
 * 2c+1 = (i,j),(i+1,j+1),(i,j+1), on which T is affine.  For each of the nq
 * queries (in, [nq][2] FP32, points on the cartogram) tri (out, [nq] int32)
 * receives the lowest-numbered triangle whose image contains it (edges
 * included; -1 if none; image triangles of zero area contain nothing) and
 * pre (out, [nq][2] FP64) the preimage, the original point mapped to the
 * query (NaN if none).  Containment signs are plain FP64 on the FP32
 * inputs.  Returns FFB_E_INVALID for NULL pointers or bad sizes. */
int ffb_inverse(ffb_ctx *ctx, int32_t lx, int32_t ly, const float *nodes, const float *queries,
                int64_t nq, int32_t *tri, double *pre);

/* ------------------------------------------------------------------ adjoints
 * Reverse-mode derivatives of the calls above, for a scalar L of the final
 * region areas.  The accepted step sizes of each integration are frozen at
 * the forward pass's values (the step-size controller is not
 * differentiated); otherwise each adjoint is the exact transpose of its
 * forward map up to FP32 rounding (bilinear lookups and cell coverage are
 * piecewise smooth; the derivative taken is the one of the piece the
 * forward pass evaluated).  Arguments marked (+=) accumulate into the
 * caller's buffer; (out) ones are overwritten.  Enqueue-only, like the
 * forward calls; the same status rules apply. */

/* Adjoint of the areas of ffb_area_error: with lam_area (in, [R] FP64),
 * lam_xy (+=, [V][2] FP64) += sum_r lam_area_r d area_r / d xy, where over
 * the ring entries k of region r d area_r/d x_k = (y_{k+1} - y_{k-1}) / 2 and
 * d area_r/d y_k = (x_{k-1} - x_{k+1}) / 2. */
int ffb_area_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *lam_area, double *lam_xy);

/* Adjoint of ffb_density for lam_rho = dL/drho (in, [ly][lx] FP32), at the
 * same g, value and area as the forward call:
 *   lam_value (+=, [R] FP64), lam_area (+=, [R] FP64) through d_r and
 *   rho_pad, and lam_xy (+=, [V][2] FP64): moving a ring edge p0 -> p1 (a
 *   counter-clockwise ring) changes the coverage integral of lam_rho over
 *   its region by the edge integral of lam_rho times the normal speed, so
 *   d/dp0 = (d_r - rho_pad) (dy, -dx) int lam (1 - s) ds and
 *   d/dp1 = (d_r - rho_pad) (dy, -dx) int lam s ds, s in [0, 1]. */
int ffb_density_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                    const double *area, const float *lam_rho, double *lam_value,
                    double *lam_area, double *lam_xy);

/* Adjoint of ffb_flux (linear in rho): lam_fields (in) has the ghosted
 * layout of ffb_flux's fields and holds dL/dJ_x, dL/dJ_y, dL/drho_s (the
 * fourth component is ignored; ghost entries count for the node they mirror,
 * with the parity sign of the component); lam_rho_bar (in, [1] FP64) is
 * dL/drho_bar.  lam_rho (out, [ly][lx] FP32) = dL/drho: the transposed
 * sine/cosine transforms, the same blur and Eq. 7 factors, and the 2D
 * DCT-III. */
int ffb_flux_adj(ffb_ctx *ctx, float sigma, const float *lam_fields, const double *lam_rho_bar,
                 float *lam_rho);

/* ffb_integrate that also records what ffb_integrate_adj needs: before
 * each accepted step, the state of the first tape_n points (tape_n <= n) as
 * (hi.x, hi.y, lo.x, lo.y) compensated FP32 pairs, tape_states (out,
 * [tape_cap][tape_n][4] FP32), and the step, tape_h (out, [tape_cap] FP64).
 * stats[0] (the accepted steps) sizes the record; more than tape_cap
 * accepted steps make ffb_integrate_adj fail with FFB_E_NO_TAPE. */
int ffb_integrate_record(ffb_ctx *ctx, const float *fields, const double *rho_bar, float *xy,
                         int64_t n, const ffb_integrate_opts *opts, int32_t *stats,
                         float *tape_states, int64_t tape_n, int32_t tape_cap, double *tape_h);

/* Adjoint of a recorded integration (steps frozen).  fields, rho_bar, stats
 * and the tape are those of the ffb_integrate_record call.  lam_xy (in/out,
 * [tape_n][2] FP64): dL/d(positions at t = 1) on entry, dL/d(positions at
 * t = 0) after.  lam_fields (+=, ghosted field layout, FP32: J_x, J_y,
 * rho_s, unused) and lam_rho_bar (+=, [1] FP64) receive the field
 * adjoints.  Each step's six stages are recomputed from its record. */
int ffb_integrate_adj(ffb_ctx *ctx, const float *fields, const double *rho_bar,
                      const int32_t *stats, const float *tape_states, int64_t tape_n,
                      int32_t tape_cap, const double *tape_h, double *lam_xy, float *lam_fields,
                      double *lam_rho_bar);

/* Context tape (host calls).  ffb_tape_begin drops any previous record
 * (its device buffers are reused in stream order, so no wait is needed) and
 * starts recording: every later ffb_area_error,
 * ffb_density, ffb_flux and ffb_integrate call appends what its adjoint
 * needs to the context (device copies of the ring vertices' positions,
 * values, areas, the density weights, fields and rho_bar, written on the
 * stream by the call's own kernels, so callers may reuse those buffers; the
 * geometry's ring arrays are referenced and must stay alive).  The reverse
 * pass differentiates each integration through the flux call before it:
 * when ffb_integrate reads the buffers that flux call wrote, the flux's
 * record serves (the fields as the flux produced them); other buffers are
 * copied when ffb_integrate is called.
 * ffb_integrate records the state of the first V points (the recorded
 * geometry's vertices, which must come first in its xy) before each
 * accepted step, for at most max_steps steps per call.  Memory per round:
 * about 16 max_steps V + 16 (lx+2)(ly+2) + 40 V bytes.
 * ffb_tape_end stops recording (the record stays); ffb_tape_clear frees it. */
int ffb_tape_begin(ffb_ctx *ctx, int32_t max_steps);
int ffb_tape_end(ffb_ctx *ctx);
int ffb_tape_clear(ffb_ctx *ctx);

/* Generation of the context's record: a counter that ffb_tape_begin and
 * ffb_tape_clear increase.  A caller that keeps a handle to one recording
 * (e.g. an autograd graph) reads it right after ffb_tape_begin and later
 * asks ffb_tape_check whether that recording is still the context's:
 * FFB_OK if it is and is not empty, FFB_E_NO_TAPE (with ffb_last_error
 * detail) if another ffb_tape_begin or ffb_tape_clear came in between or
 * nothing was recorded.  out is host memory. */
int ffb_tape_generation(const ffb_ctx *ctx, int64_t *out);
int ffb_tape_check(ffb_ctx *ctx, int64_t generation);

/* Reverse pass over the context's record, which must read
 *   area+ (density flux integrate area+)*
 * (one or more ffb_area_error calls, then rounds on the same vertices and
 * regions; each density call uses the areas of the area call before it).
 * dL_darea (in, [R] FP64): dL/d(areas of the last recorded ffb_area_error).
 * dL_dvalue (out, [R] FP64): dL/dvalue through the densities of every
 * recorded round (a direct dependence of L on value is the caller's to add).
 * dL_dxy0 (out, [V][2] FP64, may be NULL): dL/d(vertices of the first
 * record).  Stops recording.  A malformed record gives FFB_E_NO_TAPE; a
 * round with more accepted steps than max_steps gives FFB_E_NO_TAPE on the
 * device. */
int ffb_backward(ffb_ctx *ctx, const double *dL_darea, double *dL_dvalue, double *dL_dxy0);

/* ------------------------------------------------------------------ batches
 * Many independent maps -- each with its own box and grid (lx[m] x ly[m]),
 * vertices, rings, regions and statistics -- iterated together: every round
 * of every map (areas, density, flux, integration, areas and errors, as
 * above) runs inside one pass of batched launches, and each map keeps its
 * own round counter (blur sigma0 * 2^-k in round k), its own adaptive step
 * control and its own stopping rule (max |e_r| < stop_err, or max_rounds).
 * Host-side descriptors are copied at creation; device arrays are
 * referenced and must stay alive.  The batch runs on a stream of its own,
 * ordered after the caller's stream at each call and before it at each
 * return.  Device-side errors set the batch's sticky status. */
typedef struct ffb_batch ffb_batch;

typedef struct {
    int32_t n_maps;
    const int32_t *lx, *ly;           /* (host) [n_maps] grid sizes, powers of two in [8, 1024];
                                         at most 8 distinct lx in one batch */
    const int64_t *point_offsets;     /* (host) [n_maps + 1]: map m advects points
                                         [point_offsets[m], point_offsets[m+1])           */
    const int64_t *n_vertices;        /* (host) [n_maps]: the first n_vertices[m] of them
                                         are its polygon vertices                           */
    const int32_t *ring_offsets_map;  /* (host) [n_maps + 1]: map m owns rings [.., ..)    */
    const int32_t *region_offsets;    /* (host) [n_maps + 1]: map m owns regions [.., ..)  */
    ffb_geometry geometry;            /* all maps: n_vertices = total points, ring_vidx are
                                         global point indices (into the owning map's range),
                                         ring_region global region ids; xy is ignored      */
    float *points;                    /* device [total points][2], in/out, advected in place */
    const double *value;              /* device [total regions] statistics, > 0             */
} ffb_batch_desc;

typedef struct {
    double stop_err;                  /* stop a map once max |e_r| < stop_err (e.g. 0.01) */
    int32_t max_rounds;               /* ... or after this many rounds                     */
    double sigma0;                    /* blur of round k = sigma0 * 2^-k cells (e.g. 4)    */
    ffb_integrate_opts integrate;     /* step controller of every integration (its
                                         n_replay / replay_h are ignored)                  */
    int32_t use_graph;                /* 1: capture one iteration in a HIP graph and replay it */
} ffb_batch_opts;

/* Create a batch (allocates its workspace; computes the initial areas and
 * sets every map active at round 0).  hip_stream is the caller's stream. */
int ffb_batch_create(ffb_batch **out, const ffb_batch_desc *d, void *hip_stream);
int ffb_batch_destroy(ffb_batch *b);
const char *ffb_batch_last_error(const ffb_batch *b);

/* Launch shapes: the workgroup size of the transform passes (64, 128, 256
 * or 512; 0 = keep) for every transform-length class (the rows of maps
 * with lx = N and the columns of maps with ly = N) -- a workgroup holds
 * size / (N / 8) row or column pairs of length N, and at least one -- and of
 * the integration (256, 512 or 1024; 0 = keep).  Results do not depend on
 * them. */
int ffb_batch_set_shapes(ffb_batch *b, int32_t fft_threads, int32_t advect_threads);
/* (host outs) number of transform-length classes, their lengths N, transform
 * workgroup size per class, integration workgroup size. */
int ffb_batch_get_shapes(const ffb_batch *b, int32_t *n_classes, int32_t *widths,
                         int32_t *fft_threads, int32_t *advect_threads);
/* Time the candidate shapes on this batch (round-0 inputs, points left
 * unchanged) and keep the fastest: per class for the transforms, one for
 * the integration.  Waits for the device; resets the loop state. */
int ffb_batch_autotune(ffb_batch *b, const ffb_batch_opts *opts);

/* Every map active at round 0; areas from the current points (enqueued). */
int ffb_batch_reset(ffb_batch *b);
/* One round of every active map (enqueued).  replay_offsets (device
 * [n_maps + 1]) and replay_h (device) optionally give each map's accepted
 * steps, map m using replay_h[replay_offsets[m] .. replay_offsets[m+1]);
 * with them the step is issued directly, without the graph. */
int ffb_batch_step(ffb_batch *b, const ffb_batch_opts *opts, const int32_t *replay_offsets,
                   const double *replay_h);
/* Reset, then rounds until no map is active (one 4-byte device read per
 * round); *iterations (host) receives the rounds issued.  Waits; returns the
 * sticky status. */
int ffb_batch_run(ffb_batch *b, const ffb_batch_opts *opts, int32_t *iterations);
/* Waits, then copies per-map results: rounds (host [n_maps]) taken when the
 * map stopped (0 while still active), max_err (host [n_maps]) after its
 * last round, stats (host [n_maps][4]) of its last integration, area
 * (device [total regions]) the last areas; any may be NULL.  Returns the
 * sticky status. */
int ffb_batch_results(ffb_batch *b, int32_t *rounds, double *max_err, int32_t *stats,
                      double *area);

#ifdef __cplusplus
}
#endif

#endif /* FFB_H */
