// Density grid with exact cell coverage.
//
// The paper models the population density as piecewise constant per region
// (density = statistic / area) and fills the box around the map with the
// mean density.  Here rho_ij = rho_pad + sum_r (d_r - rho_pad) * |cell ∩ r|.
//
// Coverage is accumulated edge by edge.  For a counter-clockwise polygon the
// indicator at height y is the number of downward edges minus upward edges
// crossed to the left of x, so the coverage of cell (i, j) is
//   sum_edges  integral_{y in edge ∩ row j} clamp(i + 1 - x_edge(y), 0, 1) (-dy).
// Split at every grid line, each edge piece lies in one cell (k, j); with
// D = -dy of the piece and xm the mean x along it, the piece adds
// D (k + 1 - xm) to cell k and D to every cell right of it.  So
// acc[j][k] += D (k + 1 - xm) and acc[j][k + 1] += D (xm - k), and a prefix
// sum along each row yields the coverage.  Pieces are weighted by
// d_r - rho_pad before accumulation (linearity), so one grid serves all
// regions.  The walk runs in FP64 and the deltas go to an FP64 grid with
// hardware FP64 atomics: cell values stay mass-exact for density contrasts
// of 1e3 (FP32 deltas would lose ~1e-4 relative there).
#include "ffb_internal.h"

namespace {

constexpr int kPrepThreads = 1024;
constexpr int kEdgeThreads = 256;
constexpr int kScanThreads = 256;

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
__device__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (w == 0) {
        r = (l < NT / 64) ? lds[l] : 0.0;
        r = wave_sum(r);
        if (l == 0) lds[NT / 64] = r;
    }
    __syncthreads();
    r = lds[NT / 64];
    __syncthreads();
    return r;
}

// rho_pad = sum(value) / sum(area); w_r = value_r / area_r - rho_pad.
// Optional copies of value and area (snap_v, snap_a).
__global__ __launch_bounds__(kPrepThreads) void k_density_prep(
    const double *__restrict__ value, const double *__restrict__ area, int32_t R,
    double *__restrict__ w, double *__restrict__ rho_pad, int32_t *status,
    double *__restrict__ snap_v, double *__restrict__ snap_a)
{
    __shared__ double lds[kPrepThreads / 64 + 1];
    double sa = 0.0, sv = 0.0;
    int bad = 0;
    for (int32_t r = threadIdx.x; r < R; r += kPrepThreads) {
        const double a = area[r], v = value[r];
        bad |= !(a > 0.0) || !(v > 0.0);
        sa += a;
        sv += v;
    }
    sa = block_sum<kPrepThreads>(sa, lds);
    sv = block_sum<kPrepThreads>(sv, lds);
    const double pad = sv / sa;
    for (int32_t r = threadIdx.x; r < R; r += kPrepThreads) {
        const double a = area[r], v = value[r];
        w[r] = v / a - pad;
        if (snap_v) {
            snap_v[r] = v;
            snap_a[r] = a;
        }
    }
    if (bad) set_status(status, FFB_E_NONPOSITIVE);
    if (threadIdx.x == 0) *rho_pad = pad;
}

// Number of integer lines strictly between a and b, and the first of them in
// the direction of travel.
__device__ inline int32_t lines_between(double a, double b, double *first, double *stepdir)
{
    if (b > a) {
        const double f = floor(a) + 1.0, l = ceil(b) - 1.0;
        *first = f;
        *stepdir = 1.0;
        return l >= f ? (int32_t)(l - f) + 1 : 0;
    }
    if (b < a) {
        const double f = ceil(a) - 1.0, l = floor(b) + 1.0;
        *first = f;
        *stepdir = -1.0;
        return f >= l ? (int32_t)(f - l) + 1 : 0;
    }
    *first = 0.0;
    *stepdir = 0.0;
    return 0;
}

// Lanes of a wave hold consecutive edges of a ring, so runs of lanes deposit
// into the same cell.  A segmented sum over each run of equal keys (a run
// starts where the key differs from the previous lane's) leaves one pair of
// atomic adds per run instead of one per edge.  Every lane of the wave must
// call this; key < 0 means no keyed deposit.
__device__ inline void run_add(double *__restrict__ acc, int64_t key, double va, double vb)
{
    const int lane = threadIdx.x & 63;
    const int64_t prev = __shfl_up(key, 1, 64);
    int seg = (lane == 0 || prev != key) ? 1 : 0;   // a run head lies in (lane - span, lane]
    for (int o = 1; o < 64; o <<= 1) {
        const double ta = __shfl_up(va, o, 64), tb = __shfl_up(vb, o, 64);
        const int ts = __shfl_up(seg, o, 64);
        if (lane >= o) {
            if (!seg) {
                va += ta;
                vb += tb;
            }
            seg |= ts;
        }
    }
    const int64_t next = __shfl_down(key, 1, 64);
    if (key >= 0 && (lane == 63 || next != key)) {
        unsafeAtomicAdd(acc + key, va);
        unsafeAtomicAdd(acc + key + 1, vb);
    }
}

// The pieces of the wave's edges (one edge per lane, `have` false for none)
// one piece per lane and round: the pieces are cut at the grid lines in
// order of the edge parameter, each becomes a keyed pair of deltas for its
// cell, and run_add merges the lanes' pairs of each round (consecutive edges
// of a ring mostly have their k-th pieces in the same cells).  Every lane of
// the wave runs the same number of rounds (the wave's largest piece count).
__device__ inline void edge_pieces(double *__restrict__ acc, int64_t base, int32_t lx, int32_t ly,
                                   double wt, double x0, double y0, double x1, double y1,
                                   bool have)
{
    have = have && y0 != y1;                    // horizontal edges add nothing
    const double dx = x1 - x0, dy = y1 - y0;
    double fx = 0.0, sx = 0.0, fy = 0.0, sy = 0.0;
    const int32_t nx = have ? lines_between(x0, x1, &fx, &sx) : 0;
    const int32_t ny = have ? lines_between(y0, y1, &fy, &sy) : 0;
    int32_t ix = 0, iy = 0;
    double xa = x0, ya = y0;
    bool done = !have;
    while (__any(!done)) {
        int64_t key = -1;
        double va = 0.0, vb = 0.0;
        if (!done) {
            double xb, yb;
            if (ix < nx || iy < ny) {
                const double X = fx + sx * ix, Y = fy + sy * iy;
                const double tx = (ix < nx) ? (X - x0) / dx : 2.0;
                const double ty = (iy < ny) ? (Y - y0) / dy : 2.0;
                if (tx < ty) {
                    xb = X;
                    yb = y0 + tx * dy;
                    ++ix;
                } else if (ty < tx) {
                    xb = x0 + ty * dx;
                    yb = Y;
                    ++iy;
                } else {
                    xb = X;
                    yb = Y;
                    ++ix;
                    ++iy;
                }
            } else {
                xb = x1;
                yb = y1;
                done = true;
            }
            const double D = ya - yb;
            if (D != 0.0) {
                const double xm = 0.5 * (xa + xb);
                int32_t k = (int32_t)floor(xm), j = (int32_t)floor(0.5 * (ya + yb));
                k = min(max(k, 0), lx - 1);
                j = min(max(j, 0), ly - 1);
                key = base + (int64_t)j * (lx + 1) + k;
                va = wt * D * ((double)(k + 1) - xm);
                vb = wt * D * (xm - (double)k);
            }
            xa = xb;
            ya = yb;
        }
        run_add(acc, key, va, vb);
    }
}

// Ring entry k of the CSR rings: its ring g, region r and edge endpoints
// (x0, y0) -> (x1, y1) in FP64.  Malformed rings, indices out of range,
// non-finite vertices and vertices outside [0, lx] x [0, ly] set the status
// word and return false.  lx and ly come from the caller, or (batches,
// lx = ly = 0) from the map that owns the ring through `map_of`.
struct EdgeOf {
    int32_t g, r, i0;
    double x0, y0, x1, y1;
};

template <typename MapOf>
__device__ inline bool edge_of(int64_t k, const float2 *__restrict__ xy, int64_t nv,
                               const int32_t *__restrict__ off, const int32_t *__restrict__ vidx,
                               const int32_t *__restrict__ region, int32_t G, int32_t R,
                               int64_t E, MapOf map_of, int32_t *status, EdgeOf &ed,
                               const int32_t *__restrict__ entry_ring = nullptr,
                               const int32_t *s_off = nullptr, bool staged = false)
{
    // ring of entry k: from the table if there is one (checked below like
    // the search's result), else the largest g with off[g] <= k, searched in
    // the LDS copy of the offsets if the workgroup made one
    int32_t g;
    int64_t b, e;
    if (entry_ring) {
        g = entry_ring[k];
        if (g < 0 || g >= G) {
            set_status(status, FFB_E_INVALID);
            return false;
        }
        b = off[g];
        e = off[g + 1];
    } else if (staged) {
        g = ring_search(s_off, G, k);
        b = s_off[g];
        e = s_off[g + 1];
    } else {
        g = ring_search(off, G, k);
        b = off[g];
        e = off[g + 1];
    }
    if (!(b <= k && k < e) || e - b < 3 || e > E) {
        set_status(status, FFB_E_INVALID);
        return false;
    }
    int32_t lx, ly;
    if (!map_of(g, lx, ly)) return false;
    const int32_t r = region[g];
    const int32_t i0 = vidx[k], i1 = vidx[(k + 1 == e) ? b : k + 1];
    if (r < 0 || r >= R || i0 < 0 || i0 >= nv || i1 < 0 || i1 >= nv) {
        set_status(status, FFB_E_INVALID);
        return false;
    }
    const float2 p = xy[i0], q = xy[i1];
    if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(q.x) || !isfinite(q.y)) {
        set_status(status, FFB_E_NONFINITE);
        return false;
    }
    if (p.x < 0.0f || p.x > lx || p.y < 0.0f || p.y > ly || q.x < 0.0f || q.x > lx ||
        q.y < 0.0f || q.y > ly) {
        set_status(status, FFB_E_DOMAIN);
        return false;
    }
    ed.g = g;
    ed.r = r;
    ed.i0 = i0;
    ed.x0 = p.x;
    ed.y0 = p.y;
    ed.x1 = q.x;
    ed.y1 = q.y;
    return true;
}

__global__ __launch_bounds__(kEdgeThreads) void k_raster_edges(
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G,
    int32_t R, int64_t E, const double *__restrict__ w, int32_t lx, int32_t ly,
    double *__restrict__ acc, int32_t *status, float2 *__restrict__ snap)
{
    __shared__ int32_t s_off[kStagedRingOffsets];
    const bool staged = stage_ring_offsets(off, G, s_off);
    const int64_t k = blockIdx.x * (int64_t)kEdgeThreads + threadIdx.x;
    EdgeOf ed{};
    auto one_map = [&](int32_t, int32_t &mx, int32_t &my) {
        mx = lx;
        my = ly;
        return true;
    };
    // no early return: every lane of the wave takes part in the merged adds
    const bool have = k < E && edge_of(k, xy, nv, off, vidx, region, G, R, E, one_map, status,
                                       ed, nullptr, s_off, staged);
    // optional copy of the edge's start vertex (every ring vertex starts one)
    if (have && snap) snap[ed.i0] = make_float2((float)ed.x0, (float)ed.y0);
    edge_pieces(acc, 0, lx, ly, have ? w[ed.r] : 0.0, ed.x0, ed.y0, ed.x1, ed.y1, have);
}

// rho[j][i] = rho_pad + inclusive prefix sum of acc[j][0..i] (FP64, stored
// in FP64), one row per workgroup, contiguous chunks per lane.
__global__ __launch_bounds__(kScanThreads) void k_raster_scan(
    const double *__restrict__ acc, int32_t lx, const double *__restrict__ rho_pad,
    double *__restrict__ rho)
{
    __shared__ double part[kScanThreads];
    const int32_t j = blockIdx.x;
    const double *row = acc + (int64_t)j * (lx + 1);
    const int32_t chunk = (lx + kScanThreads - 1) / kScanThreads;
    const int32_t beg = threadIdx.x * chunk;
    const int32_t end = min(beg + chunk, lx);
    double s = 0.0;
    for (int32_t i = beg; i < end; ++i) s += row[i];
    part[threadIdx.x] = s;
    __syncthreads();
    // exclusive scan of the chunk sums (Hillis-Steele in LDS, fixed order)
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const double v = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0.0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    double run = part[threadIdx.x] - s + *rho_pad;
    double *out = rho + (int64_t)j * lx;
    for (int32_t i = beg; i < end; ++i) {
        run += row[i];
        out[i] = run;
    }
}

// ------------------------------------------------------------- batched
// One workgroup per map: its rho_pad and w_r (maps that stopped are skipped).
__global__ __launch_bounds__(kPrepThreads) void kb_density_prep(
    batch_view bv, const double *__restrict__ value, const double *__restrict__ area,
    double *__restrict__ w, double *__restrict__ rho_pad, int32_t *status)
{
    __shared__ double lds[kPrepThreads / 64 + 1];
    const int m = blockIdx.x;
    if (!bv.active[m]) return;
    const int32_t r0 = bv.region_off[m], r1 = bv.region_off[m + 1];
    double sa = 0.0, sv = 0.0;
    int bad = 0;
    for (int32_t r = r0 + threadIdx.x; r < r1; r += kPrepThreads) {
        const double a = area[r], v = value[r];
        bad |= !(a > 0.0) || !(v > 0.0);
        sa += a;
        sv += v;
    }
    sa = block_sum<kPrepThreads>(sa, lds);
    sv = block_sum<kPrepThreads>(sv, lds);
    const double pad = sv / sa;
    for (int32_t r = r0 + threadIdx.x; r < r1; r += kPrepThreads) w[r] = value[r] / area[r] - pad;
    if (bad) set_status(status, FFB_E_NONPOSITIVE);
    if (threadIdx.x == 0) rho_pad[m] = pad;
}

// One lane per ring entry of every map (global ring and vertex indices); the
// deltas go to the map's coverage grid.
__global__ __launch_bounds__(kEdgeThreads) void kb_raster_edges(
    batch_view bv, const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G, int32_t R,
    int64_t E, const double *__restrict__ w, double *__restrict__ acc, int32_t *status)
{
    const int64_t k = blockIdx.x * (int64_t)kEdgeThreads + threadIdx.x;
    EdgeOf ed{};
    int32_t m = -1;
    // the map of the ring; rings of maps that have stopped deposit nothing
    auto map_of = [&](int32_t g, int32_t &mx, int32_t &my) {
        m = bv.ring_map[g];
        if (m < 0 || m >= bv.n_maps) {
            set_status(status, FFB_E_INVALID);
            return false;
        }
        if (!bv.active[m]) return false;
        mx = bv.lx[m];
        my = bv.ly[m];
        return true;
    };
    // no early return: every lane of the wave takes part in the merged adds
    const bool have = k < E && edge_of(k, xy, nv, off, vidx, region, G, R, E, map_of, status,
                                       ed, bv.entry_ring);
    edge_pieces(acc, have ? bv.acc_off[m] : 0, have ? bv.lx[m] : 1, have ? bv.ly[m] : 1,
                have ? w[ed.r] : 0.0, ed.x0, ed.y0, ed.x1, ed.y1, have);
}

// One lane per ring entry: the ring whose offsets bracket it (rings with
// offsets out of order leave -1, which the raster reports as malformed).
__global__ __launch_bounds__(256) void k_entry_ring(const int32_t *__restrict__ off, int32_t G,
                                                    int64_t E, int32_t *__restrict__ entry_ring)
{
    const int64_t k = blockIdx.x * 256ll + threadIdx.x;
    if (k >= E) return;
    int32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    entry_ring[k] = (G > 0 && off[lo] <= k && k < off[lo + 1]) ? lo : -1;
}

}  // namespace

hipError_t launch_density_weights(ffb_ctx *ctx, int32_t R, const double *value,
                                  const double *area, double *rho_pad)
{
    hipLaunchKernelGGL(k_density_prep, dim3(1), dim3(kPrepThreads), 0, ctx->stream, value, area,
                       R, ctx->w_region, rho_pad, ctx->d_status, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                          const double *area, double *rho, double *rho_pad,
                          const density_snap *snap)
{
    hipStream_t s = ctx->stream;
    double *w = snap ? snap->w : ctx->w_region;
    hipLaunchKernelGGL(k_density_prep, dim3(1), dim3(kPrepThreads), 0, s, value, area,
                       g->n_regions, w, rho_pad, ctx->d_status, snap ? snap->value : nullptr,
                       snap ? snap->area : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_fill_f64(ctx->acc, (int64_t)ctx->ly * (ctx->lx + 1), 0.0, s);
    if (e != hipSuccess) return e;
    if (g->n_entries > 0) {
        const int64_t blocks = (g->n_entries + kEdgeThreads - 1) / kEdgeThreads;
        hipLaunchKernelGGL(k_raster_edges, dim3((unsigned)blocks), dim3(kEdgeThreads), 0, s,
                           reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                           g->ring_offsets, g->ring_vidx, g->ring_region, g->n_rings,
                           g->n_regions, g->n_entries, w, ctx->lx, ctx->ly, ctx->acc,
                           ctx->d_status, snap ? snap->xy : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_raster_scan, dim3(ctx->ly), dim3(kScanThreads), 0, s, ctx->acc,
                       ctx->lx, rho_pad, rho);
    return hipGetLastError();
}

hipError_t launch_batch_density(hipStream_t s, const batch_view &bv, const batch_tables &bt,
                                const ffb_geometry *g, const double *value, const double *area,
                                double *w_region, double *rho_pad, double *acc, int64_t acc_total,
                                int32_t *status)
{
    hipLaunchKernelGGL(kb_density_prep, dim3(bv.n_maps), dim3(kPrepThreads), 0, s, bv, value,
                       area, w_region, rho_pad, status);
    hipError_t e = launch_fill_f64(acc, acc_total, 0.0, s);
    if (e != hipSuccess) return e;
    if (g->n_entries > 0) {
        const int64_t blocks = (g->n_entries + kEdgeThreads - 1) / kEdgeThreads;
        hipLaunchKernelGGL(kb_raster_edges, dim3((unsigned)blocks), dim3(kEdgeThreads), 0, s, bv,
                           reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                           g->ring_offsets, g->ring_vidx, g->ring_region, g->n_rings,
                           g->n_regions, g->n_entries, w_region, acc, status);
    }
    (void)bt;                                  // the prefix sums are the flux's first pass
    return hipGetLastError();
}

hipError_t launch_entry_ring(hipStream_t s, const int32_t *off, int32_t G, int64_t E,
                             int32_t *entry_ring)
{
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_entry_ring, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, off, G,
                       E, entry_ring);
    return hipGetLastError();
}
