// Inverse of the piecewise-linear approximation of T (Conclusion: the
// graticule of the inverse transformation, computed by approximating T as
// piecewise linear and inverting that approximation).
//
// T is known at the nodes: nodes[j][i] is the image of the cell centre
// (i + 1/2, j + 1/2).  Cell c = j (lx - 1) + i between four nodes is split
// along its (i,j)-(i+1,j+1) diagonal into triangle 2c = (i,j), (i+1,j),
// (i+1,j+1) and triangle 2c + 1 = (i,j), (i+1,j+1), (i,j+1); on each T is
// affine.  A query's preimage is taken in the lowest-numbered triangle
// whose image contains it (edges included; a folded map may have several);
// triangles with a zero-area image contain nothing; no triangle gives -1
// and NaN.  Orientation signs are FP64 on the FP32 inputs without fused
// multiply-add, so the containment decisions are those of plain FP64.
//
// Work: queries are counting-sorted by the unit cell of the box they fall
// in (count, exclusive scan, scatter); each triangle visits the cells under
// its image's bounding box and claims the queries it contains with an
// atomic minimum of its index (order-independent); a last pass takes each
// query's barycentric weights in its triangle and forms the preimage.
#include <climits>

#include "ffb_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ inline double orient2(double ax, double ay, double bx, double by, double qx, double qy)
{
#pragma clang fp contract(off)
    const double u = (bx - ax) * (qy - ay);
    const double v = (by - ay) * (qx - ax);
    return u - v;
}

// Unit cell of the box [0, L) holding v, clamped (NaN goes to 0).
__device__ inline int bin_of(float v, int L)
{
    const float c = fminf(fmaxf(v, 0.0f), (float)L - 0.5f);
    return (int)floorf(c);
}

__device__ inline void corners(int64_t t, int lx, int &i0, int &j0, int &i1, int &j1, int &i2,
                               int &j2)
{
    const int64_t c = t >> 1;
    const int i = (int)(c % (lx - 1)), j = (int)(c / (lx - 1));
    i0 = i;
    j0 = j;
    if ((t & 1) == 0) {
        i1 = i + 1; j1 = j;
        i2 = i + 1; j2 = j + 1;
    } else {
        i1 = i + 1; j1 = j + 1;
        i2 = i;     j2 = j + 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_inv_count(const float2 *__restrict__ q, int64_t nq,
                                                        int lx, int ly, int32_t *__restrict__ count)
{
    for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < nq;
         k += (int64_t)gridDim.x * kThreads) {
        const float2 p = q[k];
        atomicAdd(&count[bin_of(p.y, ly) * lx + bin_of(p.x, lx)], 1);
    }
}

__global__ __launch_bounds__(kThreads) void k_inv_scatter(const float2 *__restrict__ q, int64_t nq,
                                                          int lx, int ly,
                                                          const int32_t *__restrict__ offs,
                                                          int32_t *__restrict__ fill,
                                                          int32_t *__restrict__ order)
{
    for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < nq;
         k += (int64_t)gridDim.x * kThreads) {
        const float2 p = q[k];
        const int b = bin_of(p.y, ly) * lx + bin_of(p.x, lx);
        order[offs[b] + atomicAdd(&fill[b], 1)] = (int32_t)k;
    }
}

// Claims of triangle t on the queries of bin b.
__device__ inline void claim_bin(int b, float2 A, float2 B, float2 C, double o, int32_t t,
                                 const float2 *__restrict__ q, const int32_t *__restrict__ offs,
                                 const int32_t *__restrict__ order, int32_t *__restrict__ best)
{
    for (int p = offs[b]; p < offs[b + 1]; ++p) {
        const int32_t k = order[p];
        const float2 s = q[k];
        const double d0 = orient2(B.x, B.y, C.x, C.y, s.x, s.y);
        const double d1 = orient2(C.x, C.y, A.x, A.y, s.x, s.y);
        const double d2 = orient2(A.x, A.y, B.x, B.y, s.x, s.y);
        const bool in = (o > 0.0) ? (d0 >= 0.0 && d1 >= 0.0 && d2 >= 0.0)
                                  : (d0 <= 0.0 && d1 <= 0.0 && d2 <= 0.0);
        if (in) atomicMin(&best[k], t);
    }
}

struct TriBox {
    float2 A, B, C;
    double o;
    int bx0, bx1, by0, by1;
};

__device__ inline TriBox tri_box(const float2 *__restrict__ nodes, int lx, int ly, int64_t t)
{
    int i0, j0, i1, j1, i2, j2;
    corners(t, lx, i0, j0, i1, j1, i2, j2);
    TriBox r;
    r.A = nodes[(int64_t)j0 * lx + i0];
    r.B = nodes[(int64_t)j1 * lx + i1];
    r.C = nodes[(int64_t)j2 * lx + i2];
    r.o = orient2(r.A.x, r.A.y, r.B.x, r.B.y, r.C.x, r.C.y);
    r.bx0 = bin_of(fminf(r.A.x, fminf(r.B.x, r.C.x)), lx);
    r.bx1 = bin_of(fmaxf(r.A.x, fmaxf(r.B.x, r.C.x)), lx);
    r.by0 = bin_of(fminf(r.A.y, fminf(r.B.y, r.C.y)), ly);
    r.by1 = bin_of(fmaxf(r.A.y, fmaxf(r.B.y, r.C.y)), ly);
    return r;
}

// One lane per triangle whose image box covers at most kSmallBins bins;
// larger ones (expanded regions, folded slivers) go to a list with their
// bin counts; after a scan of the counts, k_inv_claim_items gives one lane
// to each (listed triangle, bin) pair, so no lane walks hundreds of bins
// while its wave waits.
constexpr int kSmallBins = 8;

__global__ __launch_bounds__(kThreads) void k_inv_claim(const float2 *__restrict__ nodes, int lx,
                                                        int ly, const float2 *__restrict__ q,
                                                        const int32_t *__restrict__ offs,
                                                        const int32_t *__restrict__ order,
                                                        int32_t *__restrict__ best,
                                                        int32_t *__restrict__ big,
                                                        int64_t *__restrict__ big_nb,
                                                        int32_t *__restrict__ n_big)
{
    const int64_t ntri = 2 * (int64_t)(lx - 1) * (ly - 1);
    for (int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x; t < ntri;
         t += (int64_t)gridDim.x * kThreads) {
        const TriBox r = tri_box(nodes, lx, ly, t);
        if (r.o == 0.0 || r.o != r.o) continue;
        const int64_t nb = (int64_t)(r.bx1 - r.bx0 + 1) * (r.by1 - r.by0 + 1);
        if (nb > kSmallBins) {
            const int e = atomicAdd(n_big, 1);
            big[e] = (int32_t)t;
            big_nb[e] = nb;
            continue;
        }
        for (int by = r.by0; by <= r.by1; ++by)
            for (int bx = r.bx0; bx <= r.bx1; ++bx)
                claim_bin(by * lx + bx, r.A, r.B, r.C, r.o, (int32_t)t, q, offs, order, best);
    }
}

// One lane per (listed triangle, bin) pair: item u belongs to the listed
// triangle e with off[e] <= u < off[e + 1] (binary search), and is the
// (u - off[e])-th bin of its box in row-major order.
__global__ __launch_bounds__(kThreads) void k_inv_claim_items(const float2 *__restrict__ nodes,
                                                              int lx, int ly,
                                                              const float2 *__restrict__ q,
                                                              const int32_t *__restrict__ offs,
                                                              const int32_t *__restrict__ order,
                                                              int32_t *__restrict__ best,
                                                              const int32_t *__restrict__ big,
                                                              const int64_t *__restrict__ off,
                                                              const int32_t *__restrict__ n_big,
                                                              int64_t total_slot)
{
    const int nbig = *n_big;
    if (nbig == 0) return;
    const int64_t total = off[total_slot];
    for (int64_t u = blockIdx.x * (int64_t)kThreads + threadIdx.x; u < total;
         u += (int64_t)gridDim.x * kThreads) {
        int lo = 0, hi = nbig - 1;                 // largest e with off[e] <= u
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const int32_t t = big[lo];
        const TriBox r = tri_box(nodes, lx, ly, t);
        const int w = r.bx1 - r.bx0 + 1;
        const int64_t local = u - off[lo];
        if (local < 0 || local >= (int64_t)w * (r.by1 - r.by0 + 1)) continue;
        const int by = r.by0 + (int)(local / w), bx = r.bx0 + (int)(local % w);
        claim_bin(by * lx + bx, r.A, r.B, r.C, r.o, t, q, offs, order, best);
    }
}

__global__ __launch_bounds__(kThreads) void k_inv_resolve(const float2 *__restrict__ nodes, int lx,
                                                          const float2 *__restrict__ q, int64_t nq,
                                                          const int32_t *__restrict__ best,
                                                          int32_t *__restrict__ tri,
                                                          double2 *__restrict__ pre)
{
    for (int64_t k = blockIdx.x * (int64_t)kThreads + threadIdx.x; k < nq;
         k += (int64_t)gridDim.x * kThreads) {
        const int32_t t = best[k];
        if (t == INT_MAX) {
            tri[k] = -1;
            pre[k] = make_double2(__builtin_nan(""), __builtin_nan(""));
            continue;
        }
        int i0, j0, i1, j1, i2, j2;
        corners(t, lx, i0, j0, i1, j1, i2, j2);
        const float2 A = nodes[(int64_t)j0 * lx + i0], B = nodes[(int64_t)j1 * lx + i1],
                     C = nodes[(int64_t)j2 * lx + i2];
        const float2 s = q[k];
        const double o = orient2(A.x, A.y, B.x, B.y, C.x, C.y);
        const double l0 = orient2(B.x, B.y, C.x, C.y, s.x, s.y) / o;
        const double l1 = orient2(C.x, C.y, A.x, A.y, s.x, s.y) / o;
        const double l2 = orient2(A.x, A.y, B.x, B.y, s.x, s.y) / o;
        double px, py;
        {
#pragma clang fp contract(off)
            px = l0 * (i0 + 0.5);
            px += l1 * (i1 + 0.5);
            px += l2 * (i2 + 0.5);
            py = l0 * (j0 + 0.5);
            py += l1 * (j1 + 0.5);
            py += l2 * (j2 + 0.5);
        }
        tri[k] = t;
        pre[k] = make_double2(px, py);
    }
}

inline unsigned grid_for(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_inverse(ffb_ctx *ctx, int lx, int ly, const float2 *nodes, const float2 *q,
                          int64_t nq, int32_t *tri, double2 *pre, inverse_ws *w)
{
    hipStream_t s = ctx->stream;
    const int64_t nbins = (int64_t)lx * ly;
    const int64_t nscan = nbins + 1;             // the last entry receives the total
    hipError_t e = launch_fill_i32(w->count, nscan, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(w->fill, nbins, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(w->best, nq, INT_MAX, s);
    if (e != hipSuccess) return e;
    if (nq == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_inv_count, dim3(grid_for(nq)), dim3(kThreads), 0, s, q, nq, lx, ly,
                       w->count);
    e = launch_scan_i32(w->count, w->offs, nscan, w->sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_scatter, dim3(grid_for(nq)), dim3(kThreads), 0, s, q, nq, lx, ly,
                       w->offs, w->fill, w->order);
    const int64_t ntri = 2 * (int64_t)(lx - 1) * (ly - 1);
    e = launch_fill_i32(w->n_big, 1, 0, s);
    // bin counts of listed triangles; entries past the list stay zero
    if (e == hipSuccess)
        e = launch_fill_i32(reinterpret_cast<int32_t *>(w->big_nb), 2 * (ntri + 1), 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_claim, dim3(grid_for(ntri)), dim3(kThreads), 0, s, nodes, lx, ly, q,
                       w->offs, w->order, w->best, w->big, w->big_nb, w->n_big);
    e = launch_scan_i64(w->big_nb, w->big_off, ntri + 1, w->sums64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inv_claim_items, dim3(8192), dim3(kThreads), 0, s, nodes, lx, ly, q,
                       w->offs, w->order, w->best, w->big, w->big_off, w->n_big, ntri);
    hipLaunchKernelGGL(k_inv_resolve, dim3(grid_for(nq)), dim3(kThreads), 0, s, nodes, lx, q, nq,
                       w->best, tri, pre);
    return hipGetLastError();
}

