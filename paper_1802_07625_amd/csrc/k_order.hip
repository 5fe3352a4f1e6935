// Spatial order of the points of one integration.
//
// Every point's trajectory is independent of the others and the step
// control only takes a maximum over them, so the order in which the
// integrator visits the points changes no result bit.  It does change the
// cost: each stage looks up the four field records around the point, and
// when the lanes of a wave and the workgroups sharing an XCD's L2 work on
// nearby points those lookups hit in cache.  Points are counting-sorted by
// the grid cell they start in, cells numbered tile-major (8 x 8 tiles in
// row-major order, cells row-major inside a tile); points of one cell keep
// no particular order.
//
// Passes: a count per cell that also gives each point its rank among the
// points of its cell (one atomic per run of equal cells within a wave),
// an exclusive scan of the counts, and a scatter of the point indices.
#include "ffb_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 8;                      // lx and ly are powers of two >= 8

// Tile-major number of the cell holding p, clamped to the box (NaN goes to
// the first cell): a permutation of [0, lx * ly).
__device__ inline int cell_key(float2 p, int lx, int ly)
{
    const int cx = (int)fminf(fmaxf(p.x, 0.0f), (float)lx - 0.5f);
    const int cy = (int)fminf(fmaxf(p.y, 0.0f), (float)ly - 0.5f);
    const int tiles_x = lx / kTile;
    const int tile = (cy / kTile) * tiles_x + cx / kTile;
    return tile * (kTile * kTile) + (cy % kTile) * kTile + cx % kTile;
}

// Rank of each active lane's point among the points of its cell: the lanes
// of a wave with the same key in a row form a run whose first lane adds the
// run length to the cell's count; the others take the returned base plus
// their position in the run.  Inactive lanes (a suffix of the wave) carry
// key -1 and take part in no atomic.  Every lane of the wave must call it.
__device__ inline int32_t rank_in_cell(int32_t *count, int key)
{
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool start = lane == 0 || prev != key;
    const uint64_t starts = __ballot(start);
    const uint64_t upto = lane == 63 ? starts : starts & ((2ull << lane) - 1);
    const int first = 63 - __builtin_clzll(upto);        // lane 0 is always a start
    const uint64_t later = first == 63 ? 0ull : starts & ~((2ull << first) - 1);
    const int end = later ? __builtin_ctzll(later) : 64;
    int base = 0;
    if (key >= 0 && lane == first) base = atomicAdd(&count[key], end - first);
    base = __shfl(base, first, 64);
    return base + (lane - first);
}

__global__ __launch_bounds__(kThreads) void k_order_count(const float2 *__restrict__ xy,
                                                          int64_t n, int lx, int ly,
                                                          int32_t *__restrict__ count,
                                                          int32_t *__restrict__ rank)
{
    // the loop bound is uniform per workgroup, so whole waves call the rank
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t b = (int64_t)blockIdx.x * kThreads; b < n; b += stride) {
        const int64_t j = b + threadIdx.x;
        const bool active = j < n;
        const int key = active ? cell_key(xy[j], lx, ly) : -1;
        const int32_t r = rank_in_cell(count, key);
        if (active) rank[j] = r;
    }
}

__global__ __launch_bounds__(kThreads) void k_order_scatter(const float2 *__restrict__ xy,
                                                            int64_t n, int lx, int ly,
                                                            const int32_t *__restrict__ offs,
                                                            const int32_t *__restrict__ rank,
                                                            int32_t *__restrict__ perm)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += stride)
        perm[offs[cell_key(xy[j], lx, ly)] + rank[j]] = (int32_t)j;
}

unsigned grid_for(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_point_order(ffb_ctx *ctx, const float2 *xy, int64_t n)
{
    hipStream_t s = ctx->stream;
    const int64_t cells = (int64_t)ctx->lx * ctx->ly;
    hipError_t e = launch_fill_i32(ctx->ord_count, cells + 1, 0, s);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_order_count, dim3(grid_for(n)), dim3(kThreads), 0, s, xy, n, ctx->lx,
                       ctx->ly, ctx->ord_count, ctx->ord_rank);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_scan_i32(ctx->ord_count, ctx->ord_offs, cells + 1,
                                             ctx->ord_sums, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_order_scatter, dim3(grid_for(n)), dim3(kThreads), 0, s, xy, n, ctx->lx,
                       ctx->ly, ctx->ord_offs, ctx->ord_rank, ctx->ord_perm);
    return hipGetLastError();
}
