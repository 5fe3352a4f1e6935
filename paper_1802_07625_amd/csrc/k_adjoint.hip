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
    const int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (k >= E) return;
    int32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    const int64_t b = off[lo], e = off[lo + 1];
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

// One edge: its contribution to sum_c lam_c cov_r(c) (through the coverage
// deltas of the forward raster and the row suffix sums) and the geometric
// derivatives of that sum with respect to both endpoints.
__global__ __launch_bounds__(kThreads) void k_raster_adj(
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t G,
    int32_t R, int64_t E, const double *__restrict__ w, const float *__restrict__ lam,
    const double *__restrict__ suf, int32_t lx, int32_t ly, double *__restrict__ lam_w,
    double *__restrict__ lam_xy, int32_t *status)
{
    const int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (k >= E) return;
    int32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    const int64_t b = off[lo], e = off[lo + 1];
    if (!(b <= k && k < e) || e - b < 3 || e > E) { set_status(status, FFB_E_INVALID); return; }
    const int32_t r = region[lo];
    const int32_t i0 = vidx[k], i1 = vidx[(k + 1 == e) ? b : k + 1];
    if (r < 0 || r >= R || i0 < 0 || i0 >= nv || i1 < 0 || i1 >= nv) {
        set_status(status, FFB_E_INVALID);
        return;
    }
    const float2 p = xy[i0], q = xy[i1];
    const double x0 = p.x, y0 = p.y, x1 = q.x, y1 = q.y;
    if (!(x0 >= 0.0 && x0 <= lx && y0 >= 0.0 && y0 <= ly && x1 >= 0.0 && x1 <= lx &&
          y1 >= 0.0 && y1 <= ly)) {
        set_status(status, FFB_E_DOMAIN);
        return;
    }
    const double dx = x1 - x0, dy = y1 - y0;
    double fx, sx, fy, sy;
    const int32_t nx = lines_between(x0, x1, &fx, &sx);
    const int32_t ny = lines_between(y0, y1, &fy, &sy);
    int32_t ix = 0, iy = 0;
    double sa = 0.0, xa = x0, ya = y0;
    double cov = 0.0, I0 = 0.0, I1 = 0.0;
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
    const double wr = w[r];
    unsafeAtomicAdd(&lam_w[r], cov);
    // outward normal times length of a counter-clockwise edge: (dy, -dx)
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)i0], wr * dy * I0);
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)i0 + 1], -wr * dx * I0);
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)i1], wr * dy * I1);
    unsafeAtomicAdd(&lam_xy[2 * (int64_t)i1 + 1], -wr * dx * I1);
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

// Lookup of one stage position: the cell of the ghosted field layout (key =
// (j + 1) pitch + (i + 1) of its lower-left node), the bilinear fractions,
// and whether the position lies strictly inside the box along x / y (where
// the clamped lookup has a derivative).
struct Stage {
    int key;
    float a, b;
    bool fx, fy;
};

__device__ inline Stage lookup(float qx, float qy, int lx, int ly, int pitch)
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
    L.key = (j + 1) * pitch + (i + 1);
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

// Field adjoints of one cell, summed over consecutive stage evaluations that
// use it and scattered with atomics when the cell changes.
struct CellAcc {
    int key;
    float3 g[4];
};

__device__ inline void flush(float4 *__restrict__ lam, int pitch, CellAcc &ac)
{
    if (ac.key < 0) return;
    const int idx[4] = {ac.key, ac.key + 1, ac.key + pitch, ac.key + pitch + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float *d = reinterpret_cast<float *>(lam + idx[q]);
        unsafeAtomicAdd(d, ac.g[q].x);
        unsafeAtomicAdd(d + 1, ac.g[q].y);
        unsafeAtomicAdd(d + 2, ac.g[q].z);
        ac.g[q] = make_float3(0.f, 0.f, 0.f);
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
    double *lam_xy;            // [n][2] in: dL/dX(t=1), out: dL/dX(t=0)
    float4 *lam_f;             // ghosted field adjoints (accumulated)
    double *lam_rb;            // rho_bar adjoint (accumulated)
    int32_t *status;
};

// One lane per recorded point, steps in reverse.  Per step the six stages are
// recomputed from the recorded state (lookups only), then swept in reverse:
// kbar_s, the position adjoint of the stage and the field adjoints at its
// four nodes (v = J / rt with rt = (1 - t) rho_s + t rho_bar, so
// dv/dJ = 1/rt, dv/drho_s = -(1 - t) J/rt^2, dv/drho_bar = -t J/rt^2).
__global__ __launch_bounds__(kThreads) void k_advect_adj(AdjParams p)
{
    __shared__ double s_rb[kThreads / 64];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const int S = *p.count;
    if (S > p.cap || S < 0) {
        if (i == 0) set_status(p.status, FFB_E_NO_TAPE);
        return;
    }
    const double rho_bar = *p.rho_bar;
    const bool live = i < p.n;
    float lx_ = 0.f, ly_ = 0.f;
    if (live) {
        lx_ = (float)p.lam_xy[2 * (int64_t)i];
        ly_ = (float)p.lam_xy[2 * (int64_t)i + 1];
    }
    double lrb = 0.0;
    Cell cc;
    cc.key = -1;
    CellAcc ac;
    ac.key = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) ac.g[q] = make_float3(0.f, 0.f, 0.f);
    // start time of the last step; earlier ones by subtracting the steps
    double tn = 0.0;
    for (int s = 0; s < S - 1; ++s) tn += p.h[s];
    for (int n = S - 1; n >= 0 && live; --n) {
        const double h = p.h[n];
        if (n < S - 1) tn -= h;
        const float4 st = p.tape[(int64_t)n * p.n + i];
        const float hf = (float)h;
        float omt[6], tb[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const double ts = tn + kC[s] * h;
            omt[s] = (float)(1.0 - ts);
            tb[s] = (float)(ts * rho_bar);
        }
        // forward: the stage lookups and velocities
        Stage L[6];
        float Kx[6], Ky[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            float dx = 0.f, dy = 0.f;
#pragma unroll
            for (int q = 0; q < s; ++q) {
                dx = fmaf(hf * kA[s][q], Kx[q], dx);
                dy = fmaf(hf * kA[s][q], Ky[q], dy);
            }
            L[s] = lookup(st.x + (st.z + dx), st.y + (st.w + dy), p.lx, p.ly, p.pitch);
            load_cell(p.fields, p.pitch, L[s].key, cc);
            float vx[4], vy[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float r = 1.f / fmaf(cc.c[q].z, omt[s], tb[s]);
                vx[q] = cc.c[q].x * r;
                vy[q] = cc.c[q].y * r;
            }
            const float a = L[s].a, b = L[s].b;
            const float x0 = fmaf(a, vx[1] - vx[0], vx[0]), x1 = fmaf(a, vx[3] - vx[2], vx[2]);
            const float y0 = fmaf(a, vy[1] - vy[0], vy[0]), y1 = fmaf(a, vy[3] - vy[2], vy[2]);
            Kx[s] = fmaf(b, x1 - x0, x0);
            Ky[s] = fmaf(b, y1 - y0, y0);
        }
        // reverse sweep
        float Ybx[6], Yby[6];
        float sumx = 0.f, sumy = 0.f;
#pragma unroll
        for (int s = 5; s >= 0; --s) {
            float kbx = hf * kB[s] * lx_, kby = hf * kB[s] * ly_;
#pragma unroll
            for (int j = s + 1; j < 6; ++j) {
                kbx = fmaf(hf * kA[j][s], Ybx[j], kbx);
                kby = fmaf(hf * kA[j][s], Yby[j], kby);
            }
            const Stage &Ls = L[s];
            load_cell(p.fields, p.pitch, Ls.key, cc);
            float vx[4], vy[4], r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                r[q] = 1.f / fmaf(cc.c[q].z, omt[s], tb[s]);
                vx[q] = cc.c[q].x * r[q];
                vy[q] = cc.c[q].y * r[q];
            }
            const float a = Ls.a, b = Ls.b;
            const float dvx_da = (1.f - b) * (vx[1] - vx[0]) + b * (vx[3] - vx[2]);
            const float dvy_da = (1.f - b) * (vy[1] - vy[0]) + b * (vy[3] - vy[2]);
            const float dvx_db = (1.f - a) * (vx[2] - vx[0]) + a * (vx[3] - vx[1]);
            const float dvy_db = (1.f - a) * (vy[2] - vy[0]) + a * (vy[3] - vy[1]);
            Ybx[s] = Ls.fx ? kbx * dvx_da + kby * dvy_da : 0.f;
            Yby[s] = Ls.fy ? kbx * dvx_db + kby * dvy_db : 0.f;
            sumx += Ybx[s];
            sumy += Yby[s];
            if (Ls.key != ac.key) {
                flush(p.lam_f, p.pitch, ac);
                ac.key = Ls.key;
            }
            const float w[4] = {(1.f - a) * (1.f - b), a * (1.f - b), (1.f - a) * b, a * b};
            const double ts = tn + kC[s] * h;
            float rb = 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float g = w[q] * r[q];
                const float dot = kbx * vx[q] + kby * vy[q];     // (kbar . J) / rt
                ac.g[q].x = fmaf(kbx, g, ac.g[q].x);
                ac.g[q].y = fmaf(kby, g, ac.g[q].y);
                ac.g[q].z = fmaf(-dot * g, omt[s], ac.g[q].z);
                rb = fmaf(-dot, g, rb);
            }
            lrb += (double)rb * ts;
        }
        lx_ += sumx;
        ly_ += sumy;
    }
    if (live) {
        flush(p.lam_f, p.pitch, ac);
        p.lam_xy[2 * (int64_t)i] = lx_;
        p.lam_xy[2 * (int64_t)i + 1] = ly_;
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
                              double *lam_area, double *lam_xy)
{
    hipStream_t s = ctx->stream;
    // w_r and rho_pad of the forward, recomputed from value and area
    double *pad = ctx->red + 512, *total = ctx->red + 513;
    hipError_t e = launch_density_weights(ctx, g->n_regions, value, area, pad);
    if (e != hipSuccess) return e;
    e = launch_fill_f64(total, 1, 0.0, s);
    if (e != hipSuccess) return e;
    e = launch_fill_f64(ctx->lam_w, g->n_regions, 0.0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_suffix, dim3(ctx->ly), dim3(kThreads), 0, s, lam_rho, ctx->lx,
                       ctx->acc, total);
    if (g->n_entries > 0) {
        const int64_t blocks = (g->n_entries + kThreads - 1) / kThreads;
        hipLaunchKernelGGL(k_raster_adj, dim3((unsigned)blocks), dim3(kThreads), 0, s,
                           reinterpret_cast<const float2 *>(g->xy), g->n_vertices,
                           g->ring_offsets, g->ring_vidx, g->ring_region, g->n_rings,
                           g->n_regions, g->n_entries, ctx->w_region, lam_rho, ctx->acc, ctx->lx,
                           ctx->ly, ctx->lam_w, lam_xy, ctx->d_status);
    }
    hipLaunchKernelGGL(k_density_chain, dim3(1), dim3(1024), 0, s, value, area, g->n_regions,
                       ctx->lam_w, total, lam_value, lam_area);
    return hipGetLastError();
}

hipError_t launch_advect_adj(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                             const advect_tape *tape, double *lam_xy, float4 *lam_fields,
                             double *lam_rho_bar)
{
    if (tape->n == 0) return hipSuccess;
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
    p.lam_xy = lam_xy;
    p.lam_f = lam_fields;
    p.lam_rb = lam_rho_bar;
    p.status = ctx->d_status;
    const int64_t blocks = (tape->n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_advect_adj, dim3((unsigned)blocks), dim3(kThreads), 0, ctx->stream, p);
    return hipGetLastError();
}
