// ffb_flux_noalloc: the blur and flux of ffb_flux (Eq. 7; SI Appendix,
// section 2) for callers that cannot allocate device memory -- code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// The transform workspace (twiddle tables, four grid planes, reduction
// partials) is one file-scope device array, `scratch`, sized for grids up
// to kMaxSide x kMaxSide.  Each device holds its own copy; its address is
// looked up once per device (hipGetSymbolAddress, with that device
// current) on the first call there and kept.  Kernels only ever receive
// that address: the array's name is not a device address in host code.
//
// Every call on a device shares the device's array: calls that overlap on
// one device (two streams, two host threads) race on it.  Nothing in the
// array needs clearing between calls: each kernel of the flux pipeline
// writes every element it later reads.
#include <cmath>
#include <mutex>

#include "ffb_internal.h"

namespace {

constexpr int kMaxSide = 512;
constexpr int kMaxDevices = 64;
constexpr size_t kAlign = 256;

constexpr size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Layout of the array (byte offsets).
constexpr size_t kTwBytes = align_up(sizeof(double2) * (kMaxSide / 2));
constexpr size_t kTqBytes = align_up(sizeof(double2) * kMaxSide);
constexpr size_t kPlaneBytes = align_up(sizeof(double) * kMaxSide * kMaxSide);
constexpr size_t kRedBytes = align_up(sizeof(double) * kRedDoubles);
constexpr size_t kOffTwX = 0;
constexpr size_t kOffTqX = kOffTwX + kTwBytes;
constexpr size_t kOffTwY = kOffTqX + kTqBytes;
constexpr size_t kOffTqY = kOffTwY + kTwBytes;
constexpr size_t kOffPlanes = kOffTqY + kTqBytes;
constexpr size_t kOffRed = kOffPlanes + 4 * kPlaneBytes;
constexpr size_t kScratchBytes = kOffRed + kRedBytes;   // about 8.4 MB

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of the current device's array (looked up once per device).
hipError_t scratch_ptr(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_ptr[dev]);
    return hipSuccess;
}

bool side_ok(int n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

}  // namespace

extern "C" int ffb_flux_noalloc(int32_t lx, int32_t ly, const double *rho, float sigma,
                                float *fields, double *rho_bar, int32_t *status,
                                void *hip_stream)
{
    if (!rho || !fields || !rho_bar || !status) return FFB_E_INVALID;
    if (!side_ok(lx) || !side_ok(ly)) return FFB_E_INVALID;
    if (lx > kMaxSide || ly > kMaxSide) return FFB_E_TOO_LARGE;
    if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return FFB_E_INVALID;
    unsigned char *base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) return FFB_E_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    flux_ws w;
    w.tw_x = reinterpret_cast<double2 *>(base + kOffTwX);
    w.tq_x = reinterpret_cast<double2 *>(base + kOffTqX);
    w.tw_y = reinterpret_cast<double2 *>(base + kOffTwY);
    w.tq_y = reinterpret_cast<double2 *>(base + kOffTqY);
    double *pl[4];
    for (int k = 0; k < 4; ++k)
        pl[k] = reinterpret_cast<double *>(base + kOffPlanes + k * kPlaneBytes);
    w.t1 = pl[0];
    w.pa = pl[1];
    w.pb = pl[2];
    w.pc = pl[3];
    w.red = reinterpret_cast<double *>(base + kOffRed);
    e = launch_twiddles(s, lx, w.tw_x, w.tq_x);
    if (e == hipSuccess) e = launch_twiddles(s, ly, w.tw_y, w.tq_y);
    if (e == hipSuccess)
        e = launch_flux_ws(s, lx, ly, w, rho, sigma, reinterpret_cast<float4 *>(fields), rho_bar,
                           status);
    return e == hipSuccess ? FFB_OK : FFB_E_DEVICE;
}
