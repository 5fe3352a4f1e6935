// Region areas and relative area errors (the stopping rule of the paper's
// benchmarking section: a maximum relative area error below 1 %).
//
// k_ring_area: one workgroup per ring (1024 lanes when rings average 2048
// entries or more, else 256).  Each lane forms FP64 shoelace terms
// x_k y_{k+1} - x_{k+1} y_k from FP32 coordinates (the products are exact in
// FP64), the block reduces them with wavefront shuffles and one FP64 atomic
// adds half the sum to the ring's region (regions with one ring are therefore
// deterministic: 0 + a = a).
// k_area_finalize: one workgroup; fixed-order FP64 reductions of sum(area)
// and sum(value), then e_r = area_r / (value_r sum(area)/sum(value)) - 1 and
// max |e_r|.
#include "ffb_internal.h"

namespace {

constexpr int kAreaThreads = 256;
constexpr int kFinThreads = 1024;

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f32(float *p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
hipError_t fill(void (*k)(T *, int64_t, T), T *p, int64_t n, T v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide FP64 sum in a fixed order; every thread gets the result.
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

template <int NT>
__global__ __launch_bounds__(NT) void k_ring_area(
    const float2 *__restrict__ xy, int64_t nv, const int32_t *__restrict__ off,
    const int32_t *__restrict__ vidx, const int32_t *__restrict__ region, int32_t n_regions,
    int64_t n_entries, double *__restrict__ area, int32_t *status, float2 *__restrict__ snap)
{
    __shared__ double lds[NT / 64 + 1];
    const int32_t g = blockIdx.x;
    const int64_t b = off[g], e = off[g + 1];
    const int32_t r = region[g];
    // uniform per block: malformed ring -> error, no memory touched
    if (b < 0 || e > n_entries || e - b < 3 || r < 0 || r >= n_regions) {
        if (threadIdx.x == 0) set_status(status, FFB_E_INVALID);
        return;
    }
    double s = 0.0;
    int bad = 0;
    for (int64_t k = b + threadIdx.x; k < e; k += NT) {
        const int64_t k1 = (k + 1 == e) ? b : k + 1;
        const int32_t i = vidx[k], j = vidx[k1];
        if (i < 0 || i >= nv || j < 0 || j >= nv) { bad |= 1; continue; }
        const float2 p = xy[i], q = xy[j];
        if (snap) snap[i] = p;                   // every ring vertex starts one entry
        if (!isfinite(p.x) || !isfinite(p.y)) { bad |= 2; continue; }
        s += (double)p.x * (double)q.y - (double)q.x * (double)p.y;
    }
    if (bad & 1) set_status(status, FFB_E_INVALID);
    else if (bad & 2) set_status(status, FFB_E_NONFINITE);
    s = block_sum<NT>(s, lds);
    if (threadIdx.x == 0) atomicAdd(&area[r], 0.5 * s);
}

// One workgroup per ring; long rings (detailed borders) get 1024 lanes so
// that each lane takes only a few entries.
hipError_t launch_ring_area_kernel(hipStream_t s, const ffb_geometry *g, double *area,
                                   int32_t *status, float2 *snap)
{
    const float2 *xy = reinterpret_cast<const float2 *>(g->xy);
    if (g->n_entries >= (int64_t)2048 * g->n_rings)
        hipLaunchKernelGGL(k_ring_area<1024>, dim3(g->n_rings), dim3(1024), 0, s, xy,
                           g->n_vertices, g->ring_offsets, g->ring_vidx, g->ring_region,
                           g->n_regions, g->n_entries, area, status, snap);
    else
        hipLaunchKernelGGL(k_ring_area<kAreaThreads>, dim3(g->n_rings), dim3(kAreaThreads), 0,
                           s, xy, g->n_vertices, g->ring_offsets, g->ring_vidx, g->ring_region,
                           g->n_regions, g->n_entries, area, status, snap);
    return hipGetLastError();
}

__global__ __launch_bounds__(kFinThreads) void k_area_finalize(
    const double *__restrict__ value, const double *__restrict__ area, int32_t R,
    double *__restrict__ err, double *__restrict__ max_abs_err, int32_t *status)
{
    __shared__ double lds[kFinThreads / 64 + 1];
    double sa = 0.0, sv = 0.0;
    int bad = 0;
    for (int32_t r = threadIdx.x; r < R; r += kFinThreads) {
        sa += area[r];
        const double v = value[r];
        bad |= !(v > 0.0);
        sv += v;
    }
    sa = block_sum<kFinThreads>(sa, lds);
    sv = block_sum<kFinThreads>(sv, lds);
    if (bad) set_status(status, FFB_E_NONPOSITIVE);
    const double scale = sa / sv;
    double mxd = 0.0;
    int nan = 0;
    for (int32_t r = threadIdx.x; r < R; r += kFinThreads) {
        const double e = area[r] / (value[r] * scale) - 1.0;
        err[r] = e;
        const double a = fabs(e);
        if (isnan(a)) nan = 1;
        else if (a > mxd) mxd = a;
    }
    // block max in FP64 (order-free)
    for (int o = 32; o > 0; o >>= 1) {
        mxd = fmax(mxd, __shfl_xor(mxd, o, 64));
        nan |= __shfl_xor(nan, o, 64);
    }
    __shared__ double m_lds[kFinThreads / 64];
    __shared__ int n_lds[kFinThreads / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { m_lds[w] = mxd; n_lds[w] = nan; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        int anynan = 0;
        for (int i = 0; i < kFinThreads / 64; ++i) { m = fmax(m, m_lds[i]); anynan |= n_lds[i]; }
        *max_abs_err = anynan ? (double)NAN : m;
    }
}

// Batched end of an iteration, one workgroup per map: sums over the map's
// regions, e_r = A_r / T_r - 1, max |e_r|, and the map's loop state (stop
// below the threshold or at the round cap, else one more round).  Maps that
// already stopped keep their state.
__global__ __launch_bounds__(kFinThreads) void kb_finalize(batch_view bv,
                                                           const double *__restrict__ value,
                                                           const double *__restrict__ area,
                                                           double *__restrict__ err,
                                                           int32_t *status)
{
    __shared__ double lds[kFinThreads / 64 + 1];
    const int m = blockIdx.x;
    const int32_t r0 = bv.region_off[m], r1 = bv.region_off[m + 1];
    const bool was_active = bv.active[m] != 0;
    double sa = 0.0, sv = 0.0;
    for (int32_t r = r0 + threadIdx.x; r < r1; r += kFinThreads) {
        sa += area[r];
        sv += value[r];
    }
    sa = block_sum<kFinThreads>(sa, lds);
    sv = block_sum<kFinThreads>(sv, lds);
    const double scale = sa / sv;
    double mxd = 0.0;
    int nan = 0;
    for (int32_t r = r0 + threadIdx.x; r < r1; r += kFinThreads) {
        const double e = area[r] / (value[r] * scale) - 1.0;
        err[r] = e;
        const double a = fabs(e);
        if (isnan(a)) nan = 1;
        else if (a > mxd) mxd = a;
    }
    for (int o = 32; o > 0; o >>= 1) {
        mxd = fmax(mxd, __shfl_xor(mxd, o, 64));
        nan |= __shfl_xor(nan, o, 64);
    }
    __shared__ double m_lds[kFinThreads / 64];
    __shared__ int n_lds[kFinThreads / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) { m_lds[w] = mxd; n_lds[w] = nan; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = 0.0;
        int anynan = 0;
        for (int i = 0; i < kFinThreads / 64; ++i) { mx = fmax(mx, m_lds[i]); anynan |= n_lds[i]; }
        if (anynan) {
            mx = (double)NAN;
            set_status(status, FFB_E_NONFINITE);
        }
        if (was_active) {
            bv.max_err[m] = mx;
            const int32_t k = bv.round[m] + 1;           // rounds taken so far
            if (mx < bv.stop_err || k >= bv.max_rounds || anynan) {
                bv.active[m] = 0;
                bv.rounds_done[m] = k;
            } else {
                bv.round[m] = k;
            }
        }
    }
}

// Zero up to kZeroSpans device spans (4-byte words each) in one launch.
__global__ __launch_bounds__(256) void k_zero_spans(zero_spans z)
{
    for (int q = 0; q < kZeroSpans; ++q) {
        uint32_t *p = static_cast<uint32_t *>(z.p[q]);
        const int64_t n = z.words[q];
        for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
            p[i] = 0u;
    }
}

// Number of maps still iterating.
__global__ __launch_bounds__(256) void kb_count_active(const int32_t *__restrict__ active, int n,
                                                       int32_t *__restrict__ out)
{
    __shared__ int lds[256];
    int c = 0;
    for (int i = threadIdx.x; i < n; i += 256) c += active[i] != 0;
    lds[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = lds[0];
}

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    return fill<int32_t>(k_fill_i32, p, n, v, s);
}
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    return fill<uint32_t>(k_fill_u32, p, n, v, s);
}
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s)
{
    return fill<float>(k_fill_f32, p, n, v, s);
}
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    return fill<double>(k_fill_f64, p, n, v, s);
}
hipError_t launch_zero_spans(const zero_spans &z, hipStream_t s)
{
    int64_t most = 0;
    for (int q = 0; q < kZeroSpans; ++q) most = z.words[q] > most ? z.words[q] : most;
    if (most == 0) return hipSuccess;
    int64_t blocks = (most + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_spans, dim3((unsigned)blocks), dim3(256), 0, s, z);
    return hipGetLastError();
}

hipError_t launch_area(const ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                       double *area, double *err, double *max_abs_err, float2 *xy_snap)
{
    hipError_t e = launch_fill_f64(area, g->n_regions, 0.0, ctx->stream);
    if (e != hipSuccess) return e;
    if (g->n_rings > 0) {
        e = launch_ring_area_kernel(ctx->stream, g, area, ctx->d_status, xy_snap);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_area_finalize, dim3(1), dim3(kFinThreads), 0, ctx->stream, value,
                       area, g->n_regions, err, max_abs_err, ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_ring_areas(hipStream_t s, const ffb_geometry *g, double *area, int32_t *status)
{
    hipError_t e = launch_fill_f64(area, g->n_regions, 0.0, s);
    if (e != hipSuccess || g->n_rings == 0) return e;
    return launch_ring_area_kernel(s, g, area, status, nullptr);
}

hipError_t launch_batch_finalize(hipStream_t s, const batch_view &bv, const double *value,
                                 const double *area, double *err, int32_t *n_active,
                                 int32_t *status)
{
    hipLaunchKernelGGL(kb_finalize, dim3(bv.n_maps), dim3(kFinThreads), 0, s, bv, value, area,
                       err, status);
    hipLaunchKernelGGL(kb_count_active, dim3(1), dim3(256), 0, s, bv.active, bv.n_maps, n_active);
    return hipGetLastError();
}
