// Angular distortion of the map T given by the advected grid nodes (main
// text, section "Measures of distortion"; SI Appendix section 3, Tissot
// ellipses and angular-distortion metrics).
//
// On every unit square between four neighbouring nodes (images of cell
// centres (i+1/2, j+1/2) ... (i+3/2, j+3/2)), T is the bilinear interpolant
// of the node images and grad T at the square's centre is the mean of the two
// opposite-edge differences in each direction.  For grad T = [[p, q], [r, s]]
// the semi-axes of the Tissot ellipse are its singular values
//   a, b = Q +- R,  Q = |(p + s, r - q)| / 2,  R = |(p - s, r + q)| / 2,
// and the local distortion errors are e = ln(a / b) and
// e~ = 2 arcsin((a - b) / (a + b)).  The global measures average e and e~
// over the squares (all of unit area on the input map) and take their maxima;
// squares with det(grad T) <= 0 (folded) are counted.
//
// One lane per square, FP64 arithmetic on the FP32 node positions (their
// differences are exact in FP64), fixed-order FP64 reductions.
#include <algorithm>

#include "ffb_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;
static_assert(5 * kMaxBlocks <= kRedDoubles, "partials fit the reduction workspace");

// p s - q r with both products rounded (no fused multiply-add), so that the
// sign that counts a square as folded is the one plain FP64 arithmetic gives.
__device__ __forceinline__ double det_no_fma(double p, double s, double q, double r)
{
#pragma clang fp contract(off)
    return p * s - q * r;
}

// Maximum that propagates NaN (a square whose Jacobian vanishes has an
// undefined e), as the mean does.
__device__ __forceinline__ double max_nan(double a, double b) { return (a != a || a > b) ? a : b; }

// Tree over the workgroup's lanes: sums in slots 0, 1, 4; maxima in 2, 3.
__device__ void reduce5(double (*lds)[kThreads], const double v[5])
{
    for (int c = 0; c < 5; ++c) lds[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            lds[0][threadIdx.x] += lds[0][threadIdx.x + o];
            lds[1][threadIdx.x] += lds[1][threadIdx.x + o];
            lds[2][threadIdx.x] = max_nan(lds[2][threadIdx.x], lds[2][threadIdx.x + o]);
            lds[3][threadIdx.x] = max_nan(lds[3][threadIdx.x], lds[3][threadIdx.x + o]);
            lds[4][threadIdx.x] += lds[4][threadIdx.x + o];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_distortion(const float2 *__restrict__ nodes, int lx,
                                                         int ly, float *__restrict__ e_out,
                                                         float *__restrict__ et_out,
                                                         double *__restrict__ part)
{
    __shared__ double lds[5][kThreads];
    const int w = lx - 1;
    const int64_t n = (int64_t)w * (ly - 1);
    double se = 0.0, set = 0.0, me = 0.0, met = 0.0, folded = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * kThreads) {
        const int j = (int)(k / w), i = (int)(k - (int64_t)j * w);
        const float2 a00 = nodes[(int64_t)j * lx + i], a10 = nodes[(int64_t)j * lx + i + 1];
        const float2 a01 = nodes[(int64_t)(j + 1) * lx + i];
        const float2 a11 = nodes[(int64_t)(j + 1) * lx + i + 1];
        const double p = 0.5 * (((double)a10.x - a00.x) + ((double)a11.x - a01.x));   // dTx/dx
        const double r = 0.5 * (((double)a10.y - a00.y) + ((double)a11.y - a01.y));   // dTy/dx
        const double q = 0.5 * (((double)a01.x - a00.x) + ((double)a11.x - a10.x));   // dTx/dy
        const double s = 0.5 * (((double)a01.y - a00.y) + ((double)a11.y - a10.y));   // dTy/dy
        const double Q = 0.5 * hypot(p + s, r - q), R = 0.5 * hypot(p - s, r + q);
        const double ma = Q + R, mb = fabs(Q - R);
        const double e = log(ma / mb);
        const double et = 2.0 * asin((ma - mb) / (ma + mb));
        if (e_out) e_out[k] = (float)e;
        if (et_out) et_out[k] = (float)et;
        se += e;
        set += et;
        me = max_nan(me, e);
        met = max_nan(met, et);
        folded += (det_no_fma(p, s, q, r) <= 0.0) ? 1.0 : 0.0;
    }
    const double v[5] = {se, set, me, met, folded};
    reduce5(lds, v);
    if (threadIdx.x < 5) part[threadIdx.x * kMaxBlocks + blockIdx.x] = lds[threadIdx.x][0];
}

// Fixed-order combination of the block partials: lane t folds blocks
// t, t + 256, ... in order, then a tree over the lanes.
__global__ __launch_bounds__(kThreads) void k_distortion_final(const double *__restrict__ part,
                                                               int nb, int64_t n,
                                                               double *__restrict__ stats)
{
    __shared__ double lds[5][kThreads];
    double se = 0.0, set = 0.0, me = 0.0, met = 0.0, folded = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) {
        se += part[b];
        set += part[kMaxBlocks + b];
        me = max_nan(me, part[2 * kMaxBlocks + b]);
        met = max_nan(met, part[3 * kMaxBlocks + b]);
        folded += part[4 * kMaxBlocks + b];
    }
    const double v[5] = {se, set, me, met, folded};
    reduce5(lds, v);
    if (threadIdx.x == 0) {
        stats[0] = lds[0][0] / (double)n;
        stats[1] = lds[2][0];
        stats[2] = lds[1][0] / (double)n;
        stats[3] = lds[3][0];
        stats[4] = lds[4][0];
    }
}

}  // namespace

hipError_t launch_distortion(ffb_ctx *ctx, int lx, int ly, const float2 *nodes, double *stats,
                             float *e, float *e_tilde)
{
    const int64_t n = (int64_t)(lx - 1) * (ly - 1);
    const int nb = (int)std::min<int64_t>(kMaxBlocks, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_distortion, dim3(nb), dim3(kThreads), 0, ctx->stream, nodes, lx, ly,
                       e, e_tilde, ctx->red);
    hipLaunchKernelGGL(k_distortion_final, dim3(1), dim3(kThreads), 0, ctx->stream, ctx->red, nb, n,
                       stats);
    return hipGetLastError();
}
