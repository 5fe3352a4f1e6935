// Adjoints (vector-Jacobian products) of the area, density and integration
// steps, for gradients of functions of the final region areas with respect to
// the region statistics.  The flux adjoint lives beside the forward
// transforms in k_flux.hip.
//
// Area:      A_r = 1/2 sum_k (x_k y_{k+1} - x_{k+1} y_k)
//            dA_r/dx_k = (y_{k+1} - y_{k-1}) / 2,  dA_r/dy_k = (x_{k-1} - x_{k+1}) / 2.
// Density:   rho = rho_pad + sum_r w_r cov_r(X),  w_r = value_r / A_r - rho_pad,
//            rho_pad = sum(value) / sum(A).
//            sum_c lam_c cov_r(c) is the integral of the piecewise-constant lam over
//            region r; moving an edge endpoint changes it by the boundary
//            integral of lam times the normal speed: for an edge p0 -> p1 of a
//            counter-clockwise ring, d/dp0 = n I0 and d/dp1 = n I1 with
//            n = (dy, -dx) (outward normal times length), I0 = int lam (1 - s) ds,
//            I1 = int lam s ds over the edge parameter s in [0, 1].
// Integration (fixed accepted steps, Dormand-Prince 5(4), stages 1..6 build the
//            order-5 solution): with stage inputs Y_s, k_s = f(Y_s, t_s) and
//            X' = X + h sum_s b_s k_s, the adjoint of one step is
//            kbar_s = h b_s lam' + h sum_{j > s} a_js Ybar_j,  Ybar_s = (df/dY)^T kbar_s,
//            lam = lam' + sum_s Ybar_s,
//            and each stage adds (df/dfields)^T kbar_s to the field adjoints.
//            Stages are recomputed from the checkpointed state of the step.
//            The position adjoint is only 2D per point, so the steps are
//            split into three passes that each run over all (point, step)
//            pairs or all points: the 2 x 2 Jacobian of every step (forward
//            mode), a cheap per-point scan lam_k = M_k^T lam_{k+1}, and the
//            field adjoints of every step given lam_{k+1} -- parallel over
//            steps, instead of one long dependent chain per point.
#include <algorithm>

#include "ffb_internal.h"

namespace {

constexpr int kThreads = 256;

// ------------------------------------------------------------------ area
__global__ __launch_bounds__(kThreads) void k_area_adj(
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G, int32_t R,
    int64_t E, const double *__restrict__ lam_area, double *__restrict__ lam_xy,
    int32_t *status)
{
    __shared__ int32_t s_off[kStagedRingOffsets];
    const bool staged = stage_ring_offsets(off, G, s_off);
    const int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (k >= E) return;
    int32_t lo;
    int64_t b, e;
    if (staged) {
        lo = ring_search(s_off, G, k);
        b = s_off[lo];
        e = s_off[lo + 1];
    } else {
        lo = ring_search(off, G, k);
        b = off[lo];
        e = off[lo + 1];
    }
    if (!(b <= k && k < e) || e - b < 3 || e > E) { set_status(status, FFB_E_INVALID); return; }
    const int32_t r = region[lo];
    const int32_t ic = vidx[k];
    const int32_t ip = vidx[(k == b) ? e - 1 : k - 1];
    const int32_t in = vidx[(k + 1 == e) ? b : k + 1];
    if (r < 0 || r >= R || ic < 0 || ic >= nv || ip < 0 || ip >= nv || in < 0 || in >= nv) {
        set_status(status, FFB_E_INVALID);
        return;
    }
    const float2 pp = xy[ip], pn = xy[in];
    const double l = lam_area[r];
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)ic], 0.5 * l * ((double)pn.y - (double)pp.y));
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)ic + 1], 0.5 * l * ((double)pp.x - (double)pn.x));
}

// --------------------------------------------------------------- density
// Suffix sums along rows: suf[j][k] = sum_{i >= k} lam[j][i], k in [0, lx]
// (suf[j][lx] = 0), and the total sum of lam (for rho_pad).
__global__ __launch_bounds__(kThreads) void k_row_suffix(const float *__restrict__ lam,
                                                         int32_t lx,
                                                         double *__restrict__ suf,
                                                         double *__restrict__ total)
{
    __shared__ double part[kThreads];
    const int32_t j = blockIdx.x;
    const float *row = lam + (int64_t)j * lx;
    double *out = suf + (int64_t)j * (lx + 1);
    const int32_t chunk = (lx + kThreads - 1) / kThreads;
    // lanes own contiguous chunks in reverse order: lane 0 the last chunk
    const int32_t end = lx - (int32_t)threadIdx.x * chunk;
    const int32_t beg = max(0, end - chunk);
    double s = 0.0;
    for (int32_t i = beg; i < end; ++i) s += row[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const double v = (threadIdx.x >= (unsigned)o) ? part[threadIdx.x - o] : 0.0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    double run = part[threadIdx.x] - s;             // sum of the chunks to the right
    for (int32_t i = end - 1; i >= beg; --i) {
        run += row[i];
        out[i] = run;
    }
    if (threadIdx.x == 0) {
        out[lx] = 0.0;
        unsafeAtomicAdd(total, part[kThreads - 1]);
    }
}

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

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One edge: its contribution to sum_c lam_c cov_r(c) (through the coverage
// deltas of the forward raster and the row suffix sums) and the geometric
// derivatives of that sum with respect to both endpoints.  A wavefront
// usually covers 64 entries of one ring, i.e. one region: then its coverage
// sums are reduced in registers and added with one atomic (thousands of
// edges share each region's word).  Every lane stays active to the end.
__global__ __launch_bounds__(kThreads) void k_raster_adj(
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G,
    int32_t R, int64_t E, const double *__restrict__ w, const float *__restrict__ lam,
    const double *__restrict__ suf, int32_t lx, int32_t ly, double *__restrict__ lam_w,
    double *__restrict__ lam_xy, int32_t *status)
{
    __shared__ int32_t s_off[kStagedRingOffsets];
    const bool staged = stage_ring_offsets(off, G, s_off);
    const int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    int32_t r = -1, i0 = 0, i1 = 0;
    double x0 = 0.0, y0 = 0.0, x1 = 0.0, y1 = 0.0;
    if (k < E) {
        int32_t lo;
        int64_t b, e;
        if (staged) {
            lo = ring_search(s_off, G, k);
            b = s_off[lo];
            e = s_off[lo + 1];
        } else {
            lo = ring_search(off, G, k);
            b = off[lo];
            e = off[lo + 1];
        }
        if (!(b <= k && k < e) || e - b < 3 || e > E) {
            set_status(status, FFB_E_INVALID);
        } else {
            const int32_t rr = region[lo];
            i0 = vidx[k];
            i1 = vidx[(k + 1 == e) ? b : k + 1];
            if (rr < 0 || rr >= R || i0 < 0 || i0 >= nv || i1 < 0 || i1 >= nv) {
                set_status(status, FFB_E_INVALID);
            } else {
                const float2 p = xy[i0], q = xy[i1];
                x0 = p.x; y0 = p.y; x1 = q.x; y1 = q.y;
                if (!(x0 >= 0.0 && x0 <= lx && y0 >= 0.0 && y0 <= ly && x1 >= 0.0 && x1 <= lx &&
                      y1 >= 0.0 && y1 <= ly))
                    set_status(status, FFB_E_DOMAIN);
                else
                    r = rr;
            }
        }
    }
    double cov = 0.0, I0 = 0.0, I1 = 0.0;
    const double dx = x1 - x0, dy = y1 - y0;
    if (r >= 0) {
        double fx, sx, fy, sy;
        const int32_t nx = lines_between(x0, x1, &fx, &sx);
        const int32_t ny = lines_between(y0, y1, &fy, &sy);
        int32_t ix = 0, iy = 0;
        double sa = 0.0, xa = x0, ya = y0;
        for (;;) {
            double sb, xb, yb;
            const bool last = !(ix < nx || iy < ny);
            if (last) {
                sb = 1.0;
                xb = x1;
                yb = y1;
            } else {
                const double X = fx + sx * ix, Y = fy + sy * iy;
                const double tx = (ix < nx) ? (X - x0) / dx : 2.0;
                const double ty = (iy < ny) ? (Y - y0) / dy : 2.0;
                if (tx < ty) {
                    sb = tx; xb = X; yb = y0 + tx * dy; ++ix;
                } else if (ty < tx) {
                    sb = ty; xb = x0 + ty * dx; yb = Y; ++iy;
                } else {
                    sb = tx; xb = X; yb = Y; ++ix; ++iy;
                }
            }
            // the piece [sa, sb] lies in cell (kc, jc)
            const double xm = 0.5 * (xa + xb);
            int32_t kc = (int32_t)floor(xm), jc = (int32_t)floor(0.5 * (ya + yb));
            kc = min(max(kc, 0), lx - 1);
            jc = min(max(jc, 0), ly - 1);
            const double D = ya - yb;
            if (D != 0.0) {
                const double *srow = suf + (int64_t)jc * (lx + 1);
                cov += D * ((double)(kc + 1) - xm) * srow[kc] + D * (xm - (double)kc) * srow[kc + 1];
            }
            const double lc = lam[(int64_t)jc * lx + kc];
            I0 += lc * ((sb - sa) - 0.5 * (sb * sb - sa * sa));
            I1 += lc * 0.5 * (sb * sb - sa * sa);
            sa = sb; xa = xb; ya = yb;
            if (last) break;
        }
    }
    // outward normal times length of a counter-clockwise edge: (dy, -dx);
    // the end vertex of lane l's edge is usually the start vertex of lane
    // l + 1's (consecutive entries of one ring): such pairs are summed in
    // registers and added with one atomic per coordinate
    const double wr = r >= 0 ? w[r] : 0.0;
    double ax = wr * dy * I0, ay = -wr * dx * I0;       // to vertex i0
    const double bx = wr * dy * I1, by = -wr * dx * I1; // to vertex i1
    const int32_t v0 = r >= 0 ? i0 : -1, v1 = r >= 0 ? i1 : -2;
    const int lane = threadIdx.x & 63;
    const double pbx = __shfl_up(bx, 1, 64), pby = __shfl_up(by, 1, 64);
    const int32_t pv1 = __shfl_up(v1, 1, 64), nv0 = __shfl_down(v0, 1, 64);
    if (lane > 0 && pv1 == v0) {
        ax += pbx;
        ay += pby;
    }
    const bool handed_on = lane < 63 && nv0 == v1;
    if (r >= 0) {
        unsafeAtomicAdd(&lam_xy[2 * (int64_t)i0], ax);
        unsafeAtomicAdd(&lam_xy[2 * (int64_t)i0 + 1], ay);
        if (!handed_on) {
            unsafeAtomicAdd(&lam_xy[2 * (int64_t)i1], bx);
            unsafeAtomicAdd(&lam_xy[2 * (int64_t)i1 + 1], by);
        }
    }
    // region sums of the coverage term
    int32_t rlo = r >= 0 ? r : INT32_MAX, rhi = r;
    for (int o = 32; o > 0; o >>= 1) {
        rlo = min(rlo, __shfl_xor(rlo, o, 64));
        rhi = max(rhi, __shfl_xor(rhi, o, 64));
    }
    if (rlo == rhi) {
        const double s = wave_sum(cov);
        if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(&lam_w[rhi], s);
    } else if (r >= 0) {
        unsafeAtomicAdd(&lam_w[r], cov);
    }
}

// Per region: w_r = value_r / A_r - rho_pad, rho_pad = sum(value) / sum(A).
//   lam_value_r += lam_w_r / A_r + lam_pad / sum(A)
//   lam_area_r  += -lam_w_r value_r / A_r^2 - lam_pad sum(value) / sum(A)^2
// with lam_pad = (sum of lam over all cells) - sum_r lam_w_r.
__global__ __launch_bounds__(1024) void k_density_chain(
    const double *__restrict__ value, const double *__restrict__ area, int32_t R,
    const double *__restrict__ lam_w, const double *__restrict__ lam_total,
    double *__restrict__ lam_value, double *__restrict__ lam_area)
{
    __shared__ double lds[3][1024];
    double sa = 0.0, sv = 0.0, sw = 0.0;
    for (int32_t r = threadIdx.x; r < R; r += 1024) {
        sa += area[r];
        sv += value[r];
        sw += lam_w[r];
    }
    lds[0][threadIdx.x] = sa;
    lds[1][threadIdx.x] = sv;
    lds[2][threadIdx.x] = sw;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            for (int q = 0; q < 3; ++q) lds[q][threadIdx.x] += lds[q][threadIdx.x + o];
        __syncthreads();
    }
    const double SA = lds[0][0], SV = lds[1][0];
    const double lam_pad = *lam_total - lds[2][0];
    for (int32_t r = threadIdx.x; r < R; r += 1024) {
        const double a = area[r];
        lam_value[r] += lam_w[r] / a + lam_pad / SA;
        lam_area[r] += -lam_w[r] * value[r] / (a * a) - lam_pad * SV / (SA * SA);
    }
}


// The density chain and the area adjoint that follows it in one launch, for
// few regions (every workgroup sums the R values itself, in the same order,
// so all arrive at the same sums): lam_area_r of the density record
// (starting from zero) is formed where the area adjoint needs it;
// workgroup 0 also stores lam_value and lam_area.
constexpr int kChainAreaMaxRegions = 1024;

__global__ __launch_bounds__(kThreads) void k_density_chain_area(
    const double *__restrict__ value, const double *__restrict__ area, int32_t R,
    const double *__restrict__ lam_w, const double *__restrict__ lam_total,
    double *__restrict__ lam_value, double *__restrict__ lam_area,
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G, int64_t E,
    double *__restrict__ lam_xy, int32_t *status)
{
    __shared__ int32_t s_off[kStagedRingOffsets];
    __shared__ double part[3][kThreads / 64];
    double sa = 0.0, sv = 0.0, sw = 0.0;
    for (int32_t r = threadIdx.x; r < R; r += kThreads) {
        sa += area[r];
        sv += value[r];
        sw += lam_w[r];
    }
    for (int o = 32; o > 0; o >>= 1) {
        sa += __shfl_xor(sa, o, 64);
        sv += __shfl_xor(sv, o, 64);
        sw += __shfl_xor(sw, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = sa;
        part[1][threadIdx.x >> 6] = sv;
        part[2][threadIdx.x >> 6] = sw;
    }
    __syncthreads();
    double SA = 0.0, SV = 0.0, SW = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) {
        SA += part[0][w];
        SV += part[1][w];
        SW += part[2][w];
    }
    const double lam_pad = *lam_total - SW;
    if (blockIdx.x == 0)
        for (int32_t r = threadIdx.x; r < R; r += kThreads) {
            const double a = area[r];
            lam_value[r] += lam_w[r] / a + lam_pad / SA;
            lam_area[r] += -lam_w[r] * value[r] / (a * a) - lam_pad * SV / (SA * SA);
        }
    const bool staged = stage_ring_offsets(off, G, s_off);
    const int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (k >= E) return;
    int32_t lo;
    int64_t b, e;
    if (staged) {
        lo = ring_search(s_off, G, k);
        b = s_off[lo];
        e = s_off[lo + 1];
    } else {
        lo = ring_search(off, G, k);
        b = off[lo];
        e = off[lo + 1];
    }
    if (!(b <= k && k < e) || e - b < 3 || e > E) { set_status(status, FFB_E_INVALID); return; }
    const int32_t r = region[lo];
    const int32_t ic = vidx[k];
    const int32_t ip = vidx[(k == b) ? e - 1 : k - 1];
    const int32_t in = vidx[(k + 1 == e) ? b : k + 1];
    if (r < 0 || r >= R || ic < 0 || ic >= nv || ip < 0 || ip >= nv || in < 0 || in >= nv) {
        set_status(status, FFB_E_INVALID);
        return;
    }
    const float2 pp = xy[ip], pn = xy[in];
    const double a = area[r];
    const double l = -lam_w[r] * value[r] / (a * a) - lam_pad * SV / (SA * SA);
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)ic], 0.5 * l * ((double)pn.y - (double)pp.y));
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)ic + 1], 0.5 * l * ((double)pp.x - (double)pn.x));
}

// ------------------------------------------------------------ integration
__constant__ double kC[6] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0};
__constant__ float kA[6][5] = {
    {0, 0, 0, 0, 0},
    {(float)(1.0 / 5), 0, 0, 0, 0},
    {(float)(3.0 / 40), (float)(9.0 / 40), 0, 0, 0},
    {(float)(44.0 / 45), (float)(-56.0 / 15), (float)(32.0 / 9), 0, 0},
    {(float)(19372.0 / 6561), (float)(-25360.0 / 2187), (float)(64448.0 / 6561),
     (float)(-212.0 / 729), 0},
    {(float)(9017.0 / 3168), (float)(-355.0 / 33), (float)(46732.0 / 5247), (float)(49.0 / 176),
     (float)(-5103.0 / 18656)}};
__constant__ float kB[6] = {(float)(35.0 / 384), 0.f, (float)(500.0 / 1113),
                            (float)(125.0 / 192), (float)(-2187.0 / 6784), (float)(11.0 / 84)};

constexpr int kChunk = 4;          // consecutive steps of one point per work item

// Lookup of one stage position: the cell of the ghosted field layout (key =
// (j + 1) pitch + (i + 1) of its lower-left node), the bilinear fractions,
// and whether the position lies strictly inside the box along x / y (where
// the clamped lookup has a derivative).
struct Stage {
    int ci, cj;           // lower-left node of the cell in the ghosted frame (i + 1, j + 1)
    float a, b;
    bool fx, fy;
};

__device__ inline Stage lookup(float qx, float qy, int lx, int ly)
{
    Stage L;
    L.fx = qx > 0.f && qx < (float)lx;
    L.fy = qy > 0.f && qy < (float)ly;
    qx = fminf(fmaxf(qx, 0.f), (float)lx);
    qy = fminf(fmaxf(qy, 0.f), (float)ly);
    const float u = qx - 0.5f, v = qy - 0.5f;
    const int i = min(max((int)floorf(u), -1), lx - 1);
    const int j = min(max((int)floorf(v), -1), ly - 1);
    L.a = u - (float)i;
    L.b = v - (float)j;
    L.ci = i + 1;
    L.cj = j + 1;
    return L;
}

// Field records (J_x, J_y, rho_s) of the four nodes of the last cell used.
struct Cell {
    int key;
    float3 c[4];          // nodes 00, 10, 01, 11
};

__device__ inline void load_cell(const float4 *__restrict__ f, int pitch, int key, Cell &cc)
{
    if (key == cc.key) return;
    cc.key = key;
    const int idx[4] = {key, key + 1, key + pitch, key + pitch + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = f[idx[q]];
        cc.c[q] = make_float3(v.x, v.y, v.z);
    }
}

// Node velocities of the cached cell at one stage time and their reciprocal
// densities; the bilinear value and its derivatives in the cell fractions.
struct Local {
    float vx[4], vy[4], r[4];
    float kx, ky;                      // v at (a, b)
    float xa, xb, ya, yb;              // dvx/da, dvx/db, dvy/da, dvy/db
};

__device__ inline void local_velocity(const Cell &cc, float omt, float tb, float a, float b,
                                      Local &o)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o.r[q] = __builtin_amdgcn_rcpf(fmaf(cc.c[q].z, omt, tb));
        o.vx[q] = cc.c[q].x * o.r[q];
        o.vy[q] = cc.c[q].y * o.r[q];
    }
    const float x0 = fmaf(a, o.vx[1] - o.vx[0], o.vx[0]), x1 = fmaf(a, o.vx[3] - o.vx[2], o.vx[2]);
    const float y0 = fmaf(a, o.vy[1] - o.vy[0], o.vy[0]), y1 = fmaf(a, o.vy[3] - o.vy[2], o.vy[2]);
    o.kx = fmaf(b, x1 - x0, x0);
    o.ky = fmaf(b, y1 - y0, y0);
    o.xa = (1.f - b) * (o.vx[1] - o.vx[0]) + b * (o.vx[3] - o.vx[2]);
    o.ya = (1.f - b) * (o.vy[1] - o.vy[0]) + b * (o.vy[3] - o.vy[2]);
    o.xb = x1 - x0;
    o.yb = y1 - y0;
}

// Field adjoints are summed in three levels.  (1) Each lane keeps two cell
// accumulators in registers (the stages of a point walk through few cells,
// and near a cell boundary they alternate between two); a third cell pushes
// the older accumulator out.  (2) Pushed sums go with LDS atomics to a
// window of kWin x kWin nodes (ghosted frame) private to the wavefront and
// placed around the cells of its 64 consecutive vertices; the window has
// kCopies copies, lane l using copy l mod kCopies, so that neighbouring
// vertices (which share nodes) do not collide on one LDS address.  (3) At
// the end of a tile the copies are summed and every touched node is added to
// the global adjoint with one atomic.  Cells outside the window go to the
// global adjoint directly.
constexpr int kWin = 18;
constexpr int kCopies = 4;
constexpr int kWinFloats = 3 * kWin * kWin;
constexpr int kWaveFloats = kCopies * kWinFloats;

// The wavefront's accepted node region, in window coordinates
// [x0, x1) x [y0, y1) (inside the window); the end-of-tile pass visits
// exactly this region.
struct Region {
    int wx0, wy0;         // window origin in the ghosted node frame
    int x0, x1, y0, y1;
};

struct CellAcc {
    int ci, cj;           // lower-left node (ghosted frame), ci < 0 = empty
    float3 g[4];
};

__device__ inline void push(float4 *__restrict__ lam, int pitch, float *cw, const Region &R,
                            const CellAcc &ac)
{
    if (ac.ci < 0) return;
    const int wx = ac.ci - R.wx0, wy = ac.cj - R.wy0;
    if (wx >= R.x0 && wy >= R.y0 && wx + 1 < R.x1 && wy + 1 < R.y1) {
        const int b = wy * kWin + wx;
        const int idx[4] = {b, b + 1, b + kWin, b + kWin + 1};
        // workgroup-scoped adds: they stay LDS atomics (with the same scope
        // as the global ones below, the compiler may merge the two branches'
        // last add into one flat atomic, which every later wait for a field
        // load then has to wait for as well)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float *d = cw + 3 * idx[q];
            __hip_atomic_fetch_add(d, ac.g[q].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(d + 1, ac.g[q].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(d + 2, ac.g[q].z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    } else {
        const int key = ac.cj * pitch + ac.ci;
        const int idx[4] = {key, key + 1, key + pitch, key + pitch + 1};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float *d = reinterpret_cast<float *>(lam + idx[q]);
            unsafeAtomicAdd(d, ac.g[q].x);
            unsafeAtomicAdd(d + 1, ac.g[q].y);
            unsafeAtomicAdd(d + 2, ac.g[q].z);
        }
    }
}

struct AdjParams {
    const float4 *fields;
    int lx, ly, pitch;
    const double *rho_bar;
    int n;
    const float4 *tape;        // [cap][n] state before each accepted step
    const double *h;           // [cap]
    const int32_t *count;      // accepted steps
    int cap;
    double *tstart;            // [cap] start time of each step (workspace)
    float4 *jac;               // [cap][n] step Jacobians, then lam after each step (workspace)
    double *lam_xy;            // [n][2] in: dL/dX(t=1), out: dL/dX(t=0)
    float4 *lam_f;             // ghosted field adjoints (accumulated)
    double *lam_rb;            // rho_bar adjoint (accumulated)
    int32_t *status;
};

__device__ inline bool adj_ok(const AdjParams &p, int &S)
{
    if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    S = *p.count;
    return S >= 0 && S <= p.cap;
}

// Start times of the steps, summed in the order the integration summed them,
// and the record check (block 0, thread 0); every block also takes part in
// zeroing the spans `z` (accumulators the caller wants cleared first).
__global__ __launch_bounds__(256) void k_adj_times(AdjParams p, zero_spans z)
{
    for (int q = 0; q < kZeroSpans; ++q) {
        uint32_t *w = static_cast<uint32_t *>(z.p[q]);
        for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < z.words[q];
             i += (int64_t)gridDim.x * 256)
            w[i] = 0u;
    }
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int S = *p.count;
    if (S < 0 || S > p.cap) {
        set_status(p.status, FFB_E_NO_TAPE);
        return;
    }
    double t = 0.0;
    for (int k = 0; k < S; ++k) {
        p.tstart[k] = t;
        t += p.h[k];
    }
}

// Work tiles: `chunk` consecutive steps of kThreads consecutive points.
// `spread` deals the tile's points to the wavefronts round-robin, so that
// the lanes of one wavefront hold every (kThreads/64)-th vertex of a chain:
// fewer lanes of one atomic instruction then share a grid node.
__device__ inline void tile_of(int tile, int n_pt_tiles, int chunk, int &step0, int &i,
                               bool spread)
{
    const int st = tile / n_pt_tiles;
    step0 = st * chunk;
    const int t = (int)threadIdx.x;
    const int r = spread ? (t & 63) * (kThreads / 64) + (t >> 6) : t;
    i = (tile - st * n_pt_tiles) * kThreads + r;
}

// Steps per tile: kChunk, halved while a record of few steps would give
// fewer tiles than a quarter of the grid's workgroups (at most two of them
// are resident per CU), so that short rounds still spread over the chip.
__device__ inline int chunk_for(int S, int n_pt_tiles)
{
    int c = kChunk;
    while (c > 1 && (int64_t)((S + c - 1) / c) * n_pt_tiles < (int64_t)gridDim.x / 4) c >>= 1;
    return c;
}

// The six stages of step k of a point: lookups, velocities K_s and their
// derivatives in the position (Jv_s, masked where the lookup is clamped).
// Forward mode gives the step's Jacobian M = dX_{k+1}/dX_k:
//   T_s = I + h sum_{q<s} a_sq dK_q,  dK_s = Jv_s T_s,  M = I + h sum_s b_s dK_s.
__global__ __launch_bounds__(kThreads) void k_adj_jacobian(AdjParams p)
{
    int S;
    if (!adj_ok(p, S)) return;
    const double rho_bar = *p.rho_bar;
    const int n_pt_tiles = (p.n + kThreads - 1) / kThreads;
    const int chunk = chunk_for(S, n_pt_tiles);
    const int n_tiles = ((S + chunk - 1) / chunk) * n_pt_tiles;
    Cell cc;
    cc.key = -1;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        int step0, i;
        tile_of(tile, n_pt_tiles, chunk, step0, i, false);
        if (i >= p.n) continue;
        const int step1 = min(S, step0 + chunk);
        // the tile's recorded states, all loads in flight at once
        float4 qs[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
            qs[u] = step0 + u < step1 ? p.tape[(int64_t)(step0 + u) * p.n + i]
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
        for (int k = step0; k < step1; ++k) {
            const double h = p.h[k], t0 = p.tstart[k];
            const float hf = (float)h;
            const float4 st = qs[0];
#pragma unroll
            for (int u = 0; u + 1 < kChunk; ++u) qs[u] = qs[u + 1];
            float Kx[6], Ky[6];
            float D[6][4];                     // dK_s, row-major 2 x 2
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                float dx = 0.f, dy = 0.f;
                float T0 = 1.f, T1 = 0.f, T2 = 0.f, T3 = 1.f;
#pragma unroll
                for (int q = 0; q < s; ++q) {
                    const float c = hf * kA[s][q];
                    dx = fmaf(c, Kx[q], dx);
                    dy = fmaf(c, Ky[q], dy);
                    T0 = fmaf(c, D[q][0], T0);
                    T1 = fmaf(c, D[q][1], T1);
                    T2 = fmaf(c, D[q][2], T2);
                    T3 = fmaf(c, D[q][3], T3);
                }
                const Stage L = lookup(st.x + (st.z + dx), st.y + (st.w + dy), p.lx, p.ly);
                load_cell(p.fields, p.pitch, L.cj * p.pitch + L.ci, cc);
                const double ts = t0 + kC[s] * h;
                Local o;
                local_velocity(cc, (float)(1.0 - ts), (float)(ts * rho_bar), L.a, L.b, o);
                Kx[s] = o.kx;
                Ky[s] = o.ky;
                const float j00 = L.fx ? o.xa : 0.f, j01 = L.fy ? o.xb : 0.f;
                const float j10 = L.fx ? o.ya : 0.f, j11 = L.fy ? o.yb : 0.f;
                D[s][0] = j00 * T0 + j01 * T2;
                D[s][1] = j00 * T1 + j01 * T3;
                D[s][2] = j10 * T0 + j11 * T2;
                D[s][3] = j10 * T1 + j11 * T3;
            }
            float M0 = 1.f, M1 = 0.f, M2 = 0.f, M3 = 1.f;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const float c = hf * kB[s];
                M0 = fmaf(c, D[s][0], M0);
                M1 = fmaf(c, D[s][1], M1);
                M2 = fmaf(c, D[s][2], M2);
                M3 = fmaf(c, D[s][3], M3);
            }
            p.jac[(int64_t)k * p.n + i] = make_float4(M0, M1, M2, M3);
        }
    }
}

// Position adjoints through the steps, per point: lam_k = M_k^T lam_{k+1};
// lam_{k+1} is stored over M_k for the field pass.
__global__ __launch_bounds__(kThreads) void k_adj_scan(AdjParams p)
{
    int S;
    if (!adj_ok(p, S)) return;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= p.n) return;
    float lx_ = (float)p.lam_xy[2 * (int64_t)i], ly_ = (float)p.lam_xy[2 * (int64_t)i + 1];
    int k = S - 1;
    // groups of four steps: the four loads do not depend on lam
    for (; k >= 3; k -= 4) {
        float4 M[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) M[u] = p.jac[(int64_t)(k - u) * p.n + i];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            p.jac[(int64_t)(k - u) * p.n + i] = make_float4(lx_, ly_, 0.f, 0.f);
            const float nx = fmaf(M[u].x, lx_, M[u].z * ly_);
            const float ny = fmaf(M[u].y, lx_, M[u].w * ly_);
            lx_ = nx;
            ly_ = ny;
        }
    }
    for (; k >= 0; --k) {
        const float4 M = p.jac[(int64_t)k * p.n + i];
        p.jac[(int64_t)k * p.n + i] = make_float4(lx_, ly_, 0.f, 0.f);
        const float nx = fmaf(M.x, lx_, M.z * ly_);
        const float ny = fmaf(M.y, lx_, M.w * ly_);
        lx_ = nx;
        ly_ = ny;
    }
    p.lam_xy[2 * (int64_t)i] = lx_;
    p.lam_xy[2 * (int64_t)i + 1] = ly_;
}

// Field adjoints of every (point, step): with lam' = dL/dX_{k+1}, the reverse
// sweep over the recomputed stages gives
//   kbar_s = h b_s lam' + h sum_{j > s} a_js Ybar_j,  Ybar_s = Jv_s^T kbar_s,
// and (v = J / rt, rt = (1 - t) rho_s + t rho_bar) each stage adds, at its
// four nodes with bilinear weight w, w kbar / rt to the J adjoints,
// -w (1 - t) (kbar . J) / rt^2 to rho_s and -w t (kbar . J) / rt^2 to rho_bar.
// The steps of a tile are taken last to first, so that each point's stages
// run monotonically backwards in time and its cell changes only where its
// path crosses a cell edge.
__global__ __launch_bounds__(kThreads) void k_adj_fields(AdjParams p)
{
    __shared__ double s_rb[kThreads / 64];
    __shared__ float win[(kThreads / 64) * kWaveFloats];
    int S;
    if (!adj_ok(p, S)) return;
    const double rho_bar = *p.rho_bar;
    const int n_pt_tiles = (p.n + kThreads - 1) / kThreads;
    const int chunk = chunk_for(S, n_pt_tiles);
    const int n_tiles = ((S + chunk - 1) / chunk) * n_pt_tiles;
    const int lane = threadIdx.x & 63;
    float *wwin = win + (threadIdx.x >> 6) * kWaveFloats;      // this wavefront's copies
    float *cw = wwin + (lane % kCopies) * kWinFloats;           // this lane's copy
    double lrb = 0.0;
    Cell cc;
    cc.key = -1;
    for (int k = lane; k < kWaveFloats; k += 64) wwin[k] = 0.f;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        int step0, i;
        tile_of(tile, n_pt_tiles, chunk, step0, i, false);
        const bool live = i < p.n;
        const int step1 = min(S, step0 + chunk);
        // the tile's recorded states and position adjoints, all loads in
        // flight at once; q[u] belongs to step step1 - 1 - u (last first)
        float4 qs[kChunk], ql[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int k = step1 - 1 - u;
            if (live && k >= step0) {
                qs[u] = p.tape[(int64_t)k * p.n + i];
                ql[u] = p.jac[(int64_t)k * p.n + i];
            } else {
                qs[u] = ql[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        // window: the box of the cells of the wavefront's recorded states
        int bx0 = INT32_MAX, by0 = INT32_MAX, bx1 = INT32_MIN, by1 = INT32_MIN;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            if (!live || step1 - 1 - u < step0) continue;
            const int cx = (int)fminf(fmaxf(qs[u].x + 0.5f, 0.f), (float)(p.lx + 1));
            const int cy = (int)fminf(fmaxf(qs[u].y + 0.5f, 0.f), (float)(p.ly + 1));
            bx0 = min(bx0, cx);
            bx1 = max(bx1, cx);
            by0 = min(by0, cy);
            by1 = max(by1, cy);
        }
        for (int o = 32; o > 0; o >>= 1) {
            bx0 = min(bx0, __shfl_xor(bx0, o, 64));
            by0 = min(by0, __shfl_xor(by0, o, 64));
            bx1 = max(bx1, __shfl_xor(bx1, o, 64));
            by1 = max(by1, __shfl_xor(by1, o, 64));
        }
        if (bx0 > bx1 || by0 > by1) bx0 = bx1 = by0 = by1 = 0;
        // a box too wide for the window (the wavefront's points lie on two
        // rings, or far apart on one) centres the window on the cell of
        // lane 32, which lies with the larger part of a wavefront split in
        // two, instead of on the box's middle, which may lie between them
        int ax = -1, ay = -1;
        if (live && step1 > step0) {
            ax = (int)fminf(fmaxf(qs[0].x + 0.5f, 0.f), (float)(p.lx + 1));
            ay = (int)fminf(fmaxf(qs[0].y + 0.5f, 0.f), (float)(p.ly + 1));
        }
        ax = __shfl(ax, 32, 64);
        ay = __shfl(ay, 32, 64);
        Region R;
        R.wx0 = bx0 - 1;
        R.wy0 = by0 - 1;
        if (bx1 - bx0 + 3 > kWin) R.wx0 = (ax >= 0 ? ax : (bx0 + bx1) / 2) - kWin / 2;
        if (by1 - by0 + 3 > kWin) R.wy0 = (ay >= 0 ? ay : (by0 + by1) / 2) - kWin / 2;
        R.wx0 = max(0, min(R.wx0, p.lx + 2 - kWin));
        R.wy0 = max(0, min(R.wy0, p.ly + 2 - kWin));
        R.x0 = 0;
        R.y0 = 0;
        R.x1 = min(kWin, p.lx + 2 - R.wx0);
        R.y1 = min(kWin, p.ly + 2 - R.wy0);

        CellAcc A, B;
        A.ci = B.ci = -1;
        A.cj = B.cj = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) A.g[q] = B.g[q] = make_float3(0.f, 0.f, 0.f);
        for (int k = step1 - 1; k >= step0 && live; --k) {
            const double h = p.h[k], t0 = p.tstart[k];
            const float hf = (float)h;
            const float4 st = qs[0], lam = ql[0];
#pragma unroll
            for (int u = 0; u + 1 < kChunk; ++u) {
                qs[u] = qs[u + 1];
                ql[u] = ql[u + 1];
            }
            float omt[6], tb[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const double ts = t0 + kC[s] * h;
                omt[s] = (float)(1.0 - ts);
                tb[s] = (float)(ts * rho_bar);
            }
            Stage L[6];
            float Kx[6], Ky[6];
            Local o5;                      // the last stage's, reused first below
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                float dx = 0.f, dy = 0.f;
#pragma unroll
                for (int q = 0; q < s; ++q) {
                    dx = fmaf(hf * kA[s][q], Kx[q], dx);
                    dy = fmaf(hf * kA[s][q], Ky[q], dy);
                }
                L[s] = lookup(st.x + (st.z + dx), st.y + (st.w + dy), p.lx, p.ly);
                load_cell(p.fields, p.pitch, L[s].cj * p.pitch + L[s].ci, cc);
                Local o;
                local_velocity(cc, omt[s], tb[s], L[s].a, L[s].b, o);
                Kx[s] = o.kx;
                Ky[s] = o.ky;
                if (s == 5) o5 = o;
            }
            float Ybx[6], Yby[6];
#pragma unroll
            for (int s = 5; s >= 0; --s) {
                float kbx = hf * kB[s] * lam.x, kby = hf * kB[s] * lam.y;
#pragma unroll
                for (int j = s + 1; j < 6; ++j) {
                    kbx = fmaf(hf * kA[j][s], Ybx[j], kbx);
                    kby = fmaf(hf * kA[j][s], Yby[j], kby);
                }
                const Stage &Ls = L[s];
                Local o;
                if (s == 5) {
                    o = o5;
                } else {
                    load_cell(p.fields, p.pitch, Ls.cj * p.pitch + Ls.ci, cc);
                    local_velocity(cc, omt[s], tb[s], Ls.a, Ls.b, o);
                }
                Ybx[s] = Ls.fx ? kbx * o.xa + kby * o.ya : 0.f;
                Yby[s] = Ls.fy ? kbx * o.xb + kby * o.yb : 0.f;
                const bool inA = Ls.ci == A.ci && Ls.cj == A.cj;
                const bool inB = Ls.ci == B.ci && Ls.cj == B.cj;
                if (!inA && !inB) {
                    // a third cell: push the older sum, A becomes B
                    push(p.lam_f, p.pitch, cw, R, B);
                    B = A;
                    A.ci = Ls.ci;
                    A.cj = Ls.cj;
#pragma unroll
                    for (int q = 0; q < 4; ++q) A.g[q] = make_float3(0.f, 0.f, 0.f);
                }
                const float ma = (inA || !inB) ? 1.f : 0.f, mb = 1.f - ma;
                const float a = Ls.a, b = Ls.b;
                const float w[4] = {(1.f - a) * (1.f - b), a * (1.f - b), (1.f - a) * b, a * b};
                float rb = 0.f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float gq = w[q] * o.r[q];
                    const float dot = kbx * o.vx[q] + kby * o.vy[q];     // (kbar . J) / rt
                    const float gx = kbx * gq, gy = kby * gq, gz = -dot * gq * omt[s];
                    A.g[q].x = fmaf(ma, gx, A.g[q].x);
                    A.g[q].y = fmaf(ma, gy, A.g[q].y);
                    A.g[q].z = fmaf(ma, gz, A.g[q].z);
                    B.g[q].x = fmaf(mb, gx, B.g[q].x);
                    B.g[q].y = fmaf(mb, gy, B.g[q].y);
                    B.g[q].z = fmaf(mb, gz, B.g[q].z);
                    rb = fmaf(-dot, gq, rb);
                }
                lrb += (double)rb * (t0 + kC[s] * h);
            }
        }
        if (live) {
            push(p.lam_f, p.pitch, cw, R, A);
            push(p.lam_f, p.pitch, cw, R, B);
        }
        __syncthreads();
        // the wavefront's window: sum the copies, add each touched node once,
        // clear for the next tile
        const int uw = R.x1 - R.x0, uh = R.y1 - R.y0;
        for (int k = lane; k < uw * uh; k += 64) {
            const int ry = k / uw;
            const int wy = R.y0 + ry, wx = R.x0 + (k - ry * uw);
            const int e = 3 * (wy * kWin + wx);
            float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
            for (int c = 0; c < kCopies; ++c) {
                float *w = wwin + c * kWinFloats + e;
                gx += w[0];
                gy += w[1];
                gz += w[2];
                w[0] = 0.f;
                w[1] = 0.f;
                w[2] = 0.f;
            }
            if (gx == 0.f && gy == 0.f && gz == 0.f) continue;
            float *d = reinterpret_cast<float *>(p.lam_f + (int64_t)(R.wy0 + wy) * p.pitch + (R.wx0 + wx));
            unsafeAtomicAdd(d, gx);
            unsafeAtomicAdd(d + 1, gy);
            unsafeAtomicAdd(d + 2, gz);
        }
        __syncthreads();
    }
    // workgroup sum of the rho_bar adjoint, one atomic per workgroup
    for (int o = 32; o > 0; o >>= 1) lrb += __shfl_xor(lrb, o, 64);
    if ((threadIdx.x & 63) == 0) s_rb[threadIdx.x >> 6] = lrb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) sum += s_rb[w];
        unsafeAtomicAdd(p.lam_rb, sum);
    }
}

}  // namespace

hipError_t launch_area_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *lam_area,
                           double *lam_xy)
{
    if (g->n_entries == 0) return hipSuccess;
    const int64_t blocks = (g->n_entries + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_area_adj, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream,
                       reinterpret_cast<const float2 *>(g->xy), g->n_vertices, g->ring_offsets,
                       g->ring_vidx, g->ring_region, g->n_rings, g->n_regions, g->n_entries,
                       lam_area, lam_xy, ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_density_adj(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                              const double *area, const float *lam_rho, double *lam_value,
                              double *lam_area, double *lam_xy, bool cleared, bool suffixed,
                              const double *w, const ffb_geometry *area_g)
{
    hipStream_t s = ctx->stream;
    double *total = density_adj_total(ctx);
    hipError_t e = hipSuccess;
    if (!w) {
        // w_r of the forward, recomputed from value and area
        e = launch_density_weights(ctx, g->n_regions, value, area, ctx->red + 512);
        if (e != hipSuccess) return e;
        w = ctx->w_region;
    }
    if (!cleared) {
        e = launch_fill_f64(total, 1, 0.0, s);
        if (e != hipSuccess) return e;
        e = launch_fill_f64(ctx->lam_w, g->n_regions, 0.0, s);
        if (e != hipSuccess) return e;
    }
    if (!suffixed)
        hipLaunchKernelGGL(k_row_suffix, dim3(ctx->ly), dim3(kThreads), 0, s, lam_rho, ctx->lx,
                           ctx->acc, total);
    if (g->n_entries > 0) {
        const int64_t blocks = (g->n_entries + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_raster_adj, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                           g->ring_offsets, g->ring_vidx, g->ring_region, g->n_rings,
                           g->n_regions, g->n_entries, w, lam_rho, ctx->acc, ctx->lx,
                           ctx->ly, ctx->lam_w, lam_xy, ctx->d_status);
    }
    if (area_g && cleared && g->n_regions <= kChainAreaMaxRegions &&
        area_g->n_regions == g->n_regions && area_g->n_entries > 0) {
        const int64_t blocks = (area_g->n_entries + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_density_chain_area, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           value, area, g->n_regions, ctx->lam_w, total, lam_value, lam_area,
                           reinterpret_cast<const float2 *>(area_g->xy), area_g->n_vertices,
                           area_g->ring_offsets, area_g->ring_vidx, area_g->ring_region,
                           area_g->n_rings, area_g->n_entries, lam_xy, ctx->d_status);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_density_chain, dim3(1), dim3(1024), 0, s, value, area, g->n_regions,
                       ctx->lam_w, total, lam_value, lam_area);
    e = hipGetLastError();
    if (e == hipSuccess && area_g) e = launch_area_adj(ctx, area_g, lam_area, lam_xy);
    return e;
}

hipError_t launch_advect_adj(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                             const advect_tape *tape, double *lam_xy, float4 *lam_fields,
                             double *lam_rho_bar, const zero_spans *clear)
{
    if (tape->n == 0) return clear ? launch_zero_spans(*clear, ctx->stream) : hipSuccess;
    if (ctx->adj_t_cap < tape->cap || ctx->adj_jac_cap < (int64_t)tape->cap * tape->n)
        return hipErrorInvalidValue;
    AdjParams p;
    p.fields = fields;
    p.lx = ctx->lx;
    p.ly = ctx->ly;
    p.pitch = ctx->lx + 2;
    p.rho_bar = rho_bar;
    p.n = (int)tape->n;
    p.tape = tape->states;
    p.h = tape->h;
    p.count = tape->count;
    p.cap = tape->cap;
    p.tstart = ctx->adj_t;
    p.jac = ctx->adj_jac;
    p.lam_xy = lam_xy;
    p.lam_f = lam_fields;
    p.lam_rb = lam_rho_bar;
    p.status = ctx->d_status;
    hipStream_t s = ctx->stream;
    const int64_t pt_tiles = (tape->n + kThreads - 1) / kThreads;
    const int64_t max_tiles = ((tape->cap + kChunk - 1) / kChunk) * pt_tiles;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(max_tiles, 8 * (int64_t)cus));
    zero_spans z{};
    int64_t most = 0;
    if (clear) {
        z = *clear;
        for (int q = 0; q < kZeroSpans; ++q) most = std::max<int64_t>(most, z.words[q]);
    }
    const int64_t zb = std::min<int64_t>(4096, std::max<int64_t>(1, (most + 255) / 256));
    hipLaunchKernelGGL(k_adj_times, dim3((unsigned)zb), dim3(256), 0, s, p, z);
    hipLaunchKernelGGL(k_adj_jacobian, dim3((unsigned)grid), dim3(kThreads), 0, s, p);
    hipLaunchKernelGGL(k_adj_scan, dim3((unsigned)pt_tiles), dim3(kThreads), 0, s, p);
    hipLaunchKernelGGL(k_adj_fields, dim3((unsigned)grid), dim3(kThreads), 0, s, p);
    return hipGetLastError();
}
