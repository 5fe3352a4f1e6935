// Exclusive prefix sums on the device (used by the counting sorts of the
// inverse map and of the point order).
#include "ffb_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 2048;            // elements per workgroup of the scan

// Exclusive scan of n values, three passes: per-workgroup sums, a scan of
// those in one workgroup, then the per-workgroup scans.
template <typename T>
__device__ T block_exclusive(T v, T *lds)
{
    // Hillis-Steele over kThreads lanes (each lane holds the sum of its items)
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const T x = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : T(0);
        __syncthreads();
        lds[threadIdx.x] += x;
        __syncthreads();
    }
    const T incl = lds[threadIdx.x];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_sums(const T *__restrict__ a, int64_t n,
                                                        T *__restrict__ sums)
{
    __shared__ T lds[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    T s = 0;
    for (int k = threadIdx.x; k < kScanItems; k += kThreads)
        if (base + k < n) s += a[base + k];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = lds[0];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_top(T *__restrict__ sums, int nb)
{
    __shared__ T lds[kThreads];
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nb; b0 += kThreads) {
        const T v = (b0 + (int)threadIdx.x < nb) ? sums[b0 + threadIdx.x] : T(0);
        const T ex = block_exclusive(v, lds);
        const T c = carry;
        if (b0 + (int)threadIdx.x < nb) sums[b0 + threadIdx.x] = c + ex;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry = c + ex + v;
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const T *__restrict__ a, int64_t n,
                                                         const T *__restrict__ sums,
                                                         T *__restrict__ out)
{
    __shared__ T lds[kThreads];
    constexpr int kPer = kScanItems / kThreads;  // consecutive items per lane
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kPer;
    T v[kPer];
    T s = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        v[r] = (base + r < n) ? a[base + r] : T(0);
        s += v[r];
    }
    T run = block_exclusive(s, lds) + sums[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        if (base + r < n) out[base + r] = run;
        run += v[r];
    }
}

template <typename T>
void scan_exclusive(const T *a, T *out, int64_t n, T *sums, hipStream_t s)
{
    const int nb = (int)((n + kScanItems - 1) / kScanItems);
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(nb), dim3(kThreads), 0, s, a, n, sums);
    hipLaunchKernelGGL(k_scan_top<T>, dim3(1), dim3(kThreads), 0, s, sums, nb);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3(nb), dim3(kThreads), 0, s, a, n, sums, out);
}

template <typename T>
hipError_t scan_launch(const T *a, T *out, int64_t n, T *sums, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    scan_exclusive<T>(a, out, n, sums, s);
    return hipGetLastError();
}

}  // namespace

int scan_blocks(int64_t n) { return (int)((n + kScanItems - 1) / kScanItems); }

hipError_t launch_scan_i32(const int32_t *a, int32_t *out, int64_t n, int32_t *sums,
                           hipStream_t s)
{
    return scan_launch<int32_t>(a, out, n, sums, s);
}

hipError_t launch_scan_i64(const int64_t *a, int64_t *out, int64_t n, int64_t *sums,
                           hipStream_t s)
{
    return scan_launch<int64_t>(a, out, n, sums, s);
}
