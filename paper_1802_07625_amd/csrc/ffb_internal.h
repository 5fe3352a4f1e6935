// Internal declarations shared by the HIP translation units of libffb.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ffb.h"

// Context: stream, sizes, sticky device status and the device workspace.
struct ffb_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    int32_t lx = 0, ly = 0;
    std::string last_error;

    int32_t *d_status = nullptr;   // sticky device status word

    // transform workspace
    float2 *tw_x = nullptr, *tq_x = nullptr;   // FFT and DCT twiddles for length lx
    float2 *tw_y = nullptr, *tq_y = nullptr;   // ... for length ly
    float *t1 = nullptr, *t2 = nullptr;        // [lx*ly] scratch planes
    float *pa = nullptr, *pb = nullptr, *pc = nullptr;
    double *red = nullptr;                     // reduction partials
    int32_t red_cap = 0;

    // raster workspace
    double *acc = nullptr;                     // [ly][lx+1] coverage deltas
    double *w_region = nullptr;                // [cap] d_r - rho_pad
    int32_t w_cap = 0;

    // integrator workspace
    float4 *st[2] = {nullptr, nullptr};        // (hi.x, hi.y, lo.x, lo.y) per point
    float2 *kv[2] = {nullptr, nullptr};        // first stage velocity (FSAL)
    int64_t st_cap = 0;
    uint32_t *errslot = nullptr;               // advection grid-sync words
    int32_t err_cap = 0;
    int adv_blocks = 0;                        // co-resident blocks of the advection kernel
    int adv_mode = 1;                          // advection state placement (FFB_OPT_ADVECT_STATE)
    int adv_cap = 0;                           // cap on advection workgroups, 0 = none
};

// ---------------------------------------------------------------- launches
// Every launcher enqueues on ctx->stream and returns hipSuccess or the
// launch error.  Arguments are validated by the C-ABI layer beforehand.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);

hipError_t launch_area(const ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                       double *area, double *err, double *max_abs_err);

hipError_t launch_density(ffb_ctx *ctx, const ffb_geometry *g, const double *value,
                          const double *area, float *rho, double *rho_pad);

hipError_t launch_flux(ffb_ctx *ctx, const float *rho, float sigma, float4 *fields,
                       double *rho_bar);
hipError_t launch_pack_fields(ffb_ctx *ctx, const float *jx, const float *jy,
                              const float *rho_s, float4 *fields);

int advect_max_blocks(int *out);
hipError_t launch_advect(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                         float2 *xy, int64_t n, const ffb_integrate_opts *o,
                         int32_t *stats, double *h_out, int32_t h_cap);

// ---------------------------------------------------------------- device
// Record the first error code in the sticky status word.
__device__ inline void set_status(int32_t *status, int32_t code)
{
    atomicCAS(status, 0, code);
}
