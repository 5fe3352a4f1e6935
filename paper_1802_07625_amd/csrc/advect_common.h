// Device helpers shared by the integrators: the Dormand-Prince tableau,
// the packed fields as a buffer resource, the compensated-position lookup
// and the bilinear velocity at a point (main text, section "Flow-based
// cartogram with linear equalization": velocities at grid points by basic
// arithmetic, interpolation between grid points).  Included by the
// translation units that advect points; everything has internal linkage.
#pragma once

#include "ffb_internal.h"

namespace {

constexpr int kXcds = 8;               // workgroups are dealt to 8 XCDs round-robin

// Dormand & Prince (1980) tableau: nodes in FP64 for the stage times.
__constant__ double kC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
// The same tableau in FP32 for the stage sums (used as instruction literals).
constexpr float A21 = (float)(1.0 / 5);
constexpr float A31 = (float)(3.0 / 40), A32 = (float)(9.0 / 40);
constexpr float A41 = (float)(44.0 / 45), A42 = (float)(-56.0 / 15), A43 = (float)(32.0 / 9);
constexpr float A51 = (float)(19372.0 / 6561), A52 = (float)(-25360.0 / 2187),
                A53 = (float)(64448.0 / 6561), A54 = (float)(-212.0 / 729);
constexpr float A61 = (float)(9017.0 / 3168), A62 = (float)(-355.0 / 33),
                A63 = (float)(46732.0 / 5247), A64 = (float)(49.0 / 176),
                A65 = (float)(-5103.0 / 18656);
constexpr float B1 = (float)(35.0 / 384), B3 = (float)(500.0 / 1113), B4 = (float)(125.0 / 192),
                B5 = (float)(-2187.0 / 6784), B6 = (float)(11.0 / 84);
// b - b* (order-5 minus order-4 weights)
constexpr float E1 = (float)(35.0 / 384 - 5179.0 / 57600),
                E3 = (float)(500.0 / 1113 - 7571.0 / 16695),
                E4 = (float)(125.0 / 192 - 393.0 / 640),
                E5 = (float)(-2187.0 / 6784 + 92097.0 / 339200),
                E6 = (float)(11.0 / 84 - 187.0 / 2100), E7 = (float)(-1.0 / 40);

// The packed fields as a buffer resource: gathers take a 32-bit byte offset
// (no 64-bit address arithmetic per load), the row step rides in the scalar
// offset, and the hardware returns zeros for any offset past the end.
struct Field {
    __amdgpu_buffer_rsrc_t rs;
    int lx, ly, pitch;
    uint32_t max_base;       // largest lower-left node index of a cell
    int row_bytes;           // 16 * pitch
};

__device__ inline Field make_field(const float4 *f, int lx, int ly)
{
    Field F;
    const int pitch = lx + 2;
    const uint32_t bytes = 16u * (uint32_t)pitch * (uint32_t)(ly + 2);
    // third dword 0x00020000: raw 32-bit dword access on gfx9-family chips
    F.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float4 *>(f), 0, (int)bytes, 0x00020000);
    F.lx = lx;
    F.ly = ly;
    F.pitch = pitch;
    F.max_base = (uint32_t)(ly * pitch + lx);
    F.row_bytes = 16 * pitch;
    return F;
}

// One coordinate of a point, prepared once per point and attempt:
// hi - 1/2 = ifl + fr with ifl integral, frl = fr + lo, and the bounds of the
// box in the same frame ([-1/2, L - 1/2] relative to ifl).
struct Axis {
    int ifl;
    float frl, lo_t, hi_t;
};

__device__ inline Axis make_axis(float hi, float lo, int L)
{
    Axis a;
    const float u = hi - 0.5f;          // exact for |hi| < 2^22
    const float fu = floorf(u);
    a.ifl = (int)fu;
    a.frl = (u - fu) + lo;
    a.lo_t = -0.5f - fu;                // exact: fu is integral
    a.hi_t = ((float)L - 0.5f) - fu;
    return a;
}

// Cell index and fraction of the lookup at hi + lo + d, clamped to the box:
// with t clamped to [lo_t, hi_t] the index is in [-1, L-1] for every finite
// position (ifl and floor(t) are exact integers); the caller clamps the
// combined node index once more, so that no input (NaN or Inf included) can
// reach outside the fields.
//
// floor(t) as an integer is one instruction (v_cvt_flr_i32_f32; the compiler
// emits a floor and a convert), and the fraction is v_fract_f32, which
// equals t - floor(t) except where that difference would round up to 1: it
// then returns the largest float below 1, so the fraction stays in [0, 1).
__device__ inline int floor_to_int(float t)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(t));
    return r;
}

__device__ inline void locate(const Axis &a, float d, int &idx, float &frac)
{
    float t = a.frl + d;
    t = __builtin_amdgcn_fmed3f(t, a.lo_t, a.hi_t);
    idx = a.ifl + floor_to_int(t);
    frac = __builtin_amdgcn_fractf(t);
}

// The four field records around the last looked-up cell of one point.  The
// stage positions of one attempt lie within a fraction of a cell of each
// other, so most stage evaluations find their cell here and issue no gather.
struct CellCache {
    int key;                  // (j + 1) * pitch + (i + 1) of the cached cell, -1 = none
    float3 c00, c10, c01, c11;
};

__device__ inline float3 ld3(const Field &F, uint32_t off, int soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(F.rs, (int)off, soff, 0);
    return make_float3(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]));
}

// h * v at hi + lo + d, for the stage factors omh = (1 - t) / h and
// tbh = t rho_bar / h:  h v = J / ((1 - t) rho_s + t rho_bar) * h.
__device__ inline float2 velocity(const Field &F, const Axis &ax, const Axis &ay, float dx,
                                  float dy, float omh, float tbh, CellCache &cc)
{
    int i, j;
    float a, b;
    locate(ax, dx, i, a);
    locate(ay, dy, j, b);
    const int base = (int)min(__umul24(j + 1, F.pitch) + (uint32_t)(i + 1), F.max_base);
    if (base != cc.key) {
        cc.key = base;
        const uint32_t off = 16u * (uint32_t)base;
        cc.c00 = ld3(F, off, 0);
        cc.c10 = ld3(F, off + 16u, 0);
        cc.c01 = ld3(F, off, F.row_bytes);
        cc.c11 = ld3(F, off + 16u, F.row_bytes);
    }
    const float r00 = __builtin_amdgcn_rcpf(fmaf(cc.c00.z, omh, tbh));
    const float r10 = __builtin_amdgcn_rcpf(fmaf(cc.c10.z, omh, tbh));
    const float r01 = __builtin_amdgcn_rcpf(fmaf(cc.c01.z, omh, tbh));
    const float r11 = __builtin_amdgcn_rcpf(fmaf(cc.c11.z, omh, tbh));
    const float x00 = cc.c00.x * r00, x10 = cc.c10.x * r10;
    const float x01 = cc.c01.x * r01, x11 = cc.c11.x * r11;
    const float y00 = cc.c00.y * r00, y10 = cc.c10.y * r10;
    const float y01 = cc.c01.y * r01, y11 = cc.c11.y * r11;
    // along x on both node rows, then along y (exact zeros on the box edges)
    const float xr0 = fmaf(a, x10 - x00, x00), xr1 = fmaf(a, x11 - x01, x01);
    const float yr0 = fmaf(a, y10 - y00, y00), yr1 = fmaf(a, y11 - y01, y01);
    return make_float2(fmaf(b, xr1 - xr0, xr0), fmaf(b, yr1 - yr0, yr0));
}

// h * v as velocity(), with the stage position given in the point's frame
// (tx = frl + offset, ty likewise, not yet clamped) and B the node index of
// the cell of the point's integer part (ghost offset included): the cell of
// a stage is B + floor(ty) pitch + floor(tx), clamped once more as an
// unsigned index so that no input reaches outside the fields.
__device__ inline float2 velocity_at(const Field &F, const Axis &ax, const Axis &ay, int B,
                                     float tx, float ty, float omh, float tbh, CellCache &cc)
{
    tx = __builtin_amdgcn_fmed3f(tx, ax.lo_t, ax.hi_t);
    ty = __builtin_amdgcn_fmed3f(ty, ay.lo_t, ay.hi_t);
    const int fx = floor_to_int(tx), fy = floor_to_int(ty);
    const float a = __builtin_amdgcn_fractf(tx), b = __builtin_amdgcn_fractf(ty);
    const int base = (int)min((uint32_t)(__mul24(fy, F.pitch) + (B + fx)), F.max_base);
    if (base != cc.key) {
        cc.key = base;
        const uint32_t off = 16u * (uint32_t)base;
        cc.c00 = ld3(F, off, 0);
        cc.c10 = ld3(F, off + 16u, 0);
        cc.c01 = ld3(F, off, F.row_bytes);
        cc.c11 = ld3(F, off + 16u, F.row_bytes);
    }
    const float r00 = __builtin_amdgcn_rcpf(fmaf(cc.c00.z, omh, tbh));
    const float r10 = __builtin_amdgcn_rcpf(fmaf(cc.c10.z, omh, tbh));
    const float r01 = __builtin_amdgcn_rcpf(fmaf(cc.c01.z, omh, tbh));
    const float r11 = __builtin_amdgcn_rcpf(fmaf(cc.c11.z, omh, tbh));
    const float x00 = cc.c00.x * r00, x10 = cc.c10.x * r10;
    const float x01 = cc.c01.x * r01, x11 = cc.c11.x * r11;
    const float y00 = cc.c00.y * r00, y10 = cc.c10.y * r10;
    const float y01 = cc.c01.y * r01, y11 = cc.c11.y * r11;
    const float xr0 = fmaf(a, x10 - x00, x00), xr1 = fmaf(a, x11 - x01, x01);
    const float yr0 = fmaf(a, y10 - y00, y00), yr1 = fmaf(a, y11 - y01, y01);
    return make_float2(fmaf(b, xr1 - xr0, xr0), fmaf(b, yr1 - yr0, yr0));
}

// Node index of the cell holding the point's integer part (ghost offset
// included), the base of velocity_at's cell arithmetic.
__device__ inline int cell_base(const Axis &ax, const Axis &ay, int pitch)
{
    return __mul24(ay.ifl, pitch) + ax.ifl + (pitch + 1);
}

// x^(-1/5) for x > 0, to a few ulp: a single-precision estimate refined by
// two Newton steps on y^-5 = x, y <- y (6 - x y^5) / 5, each of which about
// squares the relative error (1e-7, 1e-14, then rounding level).  The chain
// is a third as long as a double-precision pow, and it sits on the critical
// path between the grid-wide error maximum and the next attempt.  Inputs
// whose single-precision estimate could under- or overflow take pow.
__device__ inline double inv_fifth_root(double x)
{
    if (!(x >= 1e-30 && x <= 1e30)) return pow(x, -0.2);
    double y = (double)powf((float)x, -0.2f);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double y2 = y * y;
        y *= fma(-0.2, x * (y2 * y2 * y), 1.2);
    }
    return y;
}

// Step-size update of the adaptive controller (all integrators): after an
// accepted attempt the step grows or shrinks by safety * (err / tol)^(-1/5)
// within [fac_min, fac_max] (fac_max when err = 0) and does not grow right
// after a rejection; after a rejected attempt it shrinks by the same factor,
// at most down to fac_min.
__device__ inline double step_after_accept(double h, double err, double tol, double safety,
                                           double fac_min, double fac_max, bool last_rejected)
{
    double fac = (err == 0.0) ? fac_max : safety * inv_fifth_root(err / tol);
    fac = fmin(fmax(fac, fac_min), fac_max);
    if (last_rejected && fac > 1.0) fac = 1.0;
    return h * fac;
}

__device__ inline double step_after_reject(double h, double err, double tol, double safety,
                                           double fac_min)
{
    return h * fmax(fac_min, safety * inv_fifth_root(err / tol));
}

// A wave-uniform float kept in a scalar register.
__device__ inline float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Error-free sum: s + e == a + b exactly.
__device__ inline void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ inline float wave_max(float v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Maximum over the 64 lanes of a wave by data-parallel-primitive moves
// (register-to-register, no LDS round trip): shifts within each row of 16
// lanes leave every row's maximum in its lane 15, two row broadcasts carry
// them to lane 63.  Lanes a move has no source for read 0, the identity of
// an unsigned maximum.  Returns the maximum in every lane (read from lane 63).
__device__ inline uint32_t wave_max_bits(uint32_t v)
{
    const auto step = [](uint32_t x, uint32_t y) { return x > y ? x : y; };
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = step(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// The same for non-negative FP32 values (+inf included), whose bit patterns
// order as the values do.
__device__ inline float wave_max_bits_f(float v)
{
    return __uint_as_float(wave_max_bits(__float_as_uint(v)));
}

}  // namespace
