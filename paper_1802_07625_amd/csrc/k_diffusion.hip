// Point pass and step control of the diffusion-cartogram variant (SI
// Appendix, section 2, the diffusion choice of f_mn): the Dormand-Prince
// stages and compensated state of the main integrator, with fields that
// change with t -- each stage time has its own field set, rebuilt before the
// attempt -- and the accept/reject decision taken on the device by a small
// control kernel, so an attempt is a fixed launch sequence.
#include "advect_common.h"

namespace {

// The same Dormand-Prince stages and compensated state as k_advect, but each
// stage time has its own fields (rho(t), J(t) rebuilt at that time), so a
// stage looks up the fields of its slot and v = J / rho(t) there: the
// velocity helper with omh = 1 / h and tbh = 0 returns h v.  Stage times
// c = 1/5, 3/10, 4/5, 8/9 use slots 0-3; the last two stages (c = 1) share
// slot 4.  One launch per attempt; the control kernel decides.
constexpr int kDiffThreads = 256;

// Points of workgroup b: contiguous chunks, the chunks of one XCD adjacent
// (workgroups are dealt to the XCDs round-robin).
__device__ inline void diff_range(int b, int nb, int64_t n, int64_t &lo, int64_t &hi)
{
    const int per = nb / kXcds;                     // nb is a multiple of kXcds
    const int logical = (b % kXcds) * per + b / kXcds;
    const int64_t chunk = (n + nb - 1) / nb;
    lo = min(n, (int64_t)logical * chunk);
    hi = min(n, lo + chunk);
}

__global__ __launch_bounds__(kDiffThreads) void kd_init_points(const float4 *__restrict__ fields,
                                                               int lx, int ly,
                                                               const float2 *__restrict__ xy,
                                                               const int32_t *__restrict__ perm,
                                                               int64_t n, float4 *__restrict__ st0,
                                                               float2 *__restrict__ kv0,
                                                               const int32_t *status)
{
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const Field F = make_field(fields, lx, ly);
    for (int64_t i = blockIdx.x * (int64_t)kDiffThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDiffThreads) {
        const float2 y = xy[perm ? perm[i] : i];
        st0[i] = make_float4(y.x, y.y, 0.f, 0.f);
        CellCache cc;
        cc.key = -1;
        const Axis ax = make_axis(y.x, 0.f, lx), ay = make_axis(y.y, 0.f, ly);
        kv0[i] = velocity(F, ax, ay, 0.f, 0.f, 1.0f, 0.0f, cc);
    }
}

__global__ __launch_bounds__(kDiffThreads) void kd_points(const diff_ctl *__restrict__ ctl,
                                                          const float4 *__restrict__ fields,
                                                          int64_t fplane, int lx, int ly,
                                                          int64_t n, float4 *st0, float4 *st1,
                                                          float2 *kv0, float2 *kv1,
                                                          float *__restrict__ part)
{
    if (ctl->done) return;
    __shared__ float s_err[kDiffThreads / 64];
    const double h = ctl->h_att;
    const double rh = 1.0 / h;
    const float hf = uniform((float)h), rhf = uniform((float)rh);
    const int cur = ctl->cur;
    const float4 *stc = cur ? st1 : st0;
    const float2 *kvc = cur ? kv1 : kv0;
    float4 *stn = cur ? st0 : st1;
    float2 *kvn = cur ? kv0 : kv1;
    Field Fs[kDiffSlots];
#pragma unroll
    for (int z = 0; z < kDiffSlots; ++z) Fs[z] = make_field(fields + z * fplane, lx, ly);
    int64_t lo, hi;
    diff_range(blockIdx.x, gridDim.x, n, lo, hi);
    float emax = 0.0f;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kDiffThreads) {
        const float4 s0 = stc[i];
        const Axis ax = make_axis(s0.x, s0.z, lx), ay = make_axis(s0.y, s0.w, ly);
        const float2 k1 = kvc[i];
        const float2 q1 = make_float2(hf * k1.x, hf * k1.y);
        CellCache cc;
        float dx, dy;
        cc.key = -1;
        dx = A21 * q1.x;
        dy = A21 * q1.y;
        const float2 q2 = velocity(Fs[0], ax, ay, dx, dy, rhf, 0.f, cc);
        cc.key = -1;
        dx = fmaf(A32, q2.x, A31 * q1.x);
        dy = fmaf(A32, q2.y, A31 * q1.y);
        const float2 q3 = velocity(Fs[1], ax, ay, dx, dy, rhf, 0.f, cc);
        cc.key = -1;
        dx = fmaf(A43, q3.x, fmaf(A42, q2.x, A41 * q1.x));
        dy = fmaf(A43, q3.y, fmaf(A42, q2.y, A41 * q1.y));
        const float2 q4 = velocity(Fs[2], ax, ay, dx, dy, rhf, 0.f, cc);
        cc.key = -1;
        dx = fmaf(A54, q4.x, fmaf(A53, q3.x, fmaf(A52, q2.x, A51 * q1.x)));
        dy = fmaf(A54, q4.y, fmaf(A53, q3.y, fmaf(A52, q2.y, A51 * q1.y)));
        const float2 q5 = velocity(Fs[3], ax, ay, dx, dy, rhf, 0.f, cc);
        cc.key = -1;
        dx = fmaf(A65, q5.x, fmaf(A64, q4.x, fmaf(A63, q3.x, fmaf(A62, q2.x, A61 * q1.x))));
        dy = fmaf(A65, q5.y, fmaf(A64, q4.y, fmaf(A63, q3.y, fmaf(A62, q2.y, A61 * q1.y))));
        const float2 q6 = velocity(Fs[4], ax, ay, dx, dy, rhf, 0.f, cc);
        const float ix = fmaf(B6, q6.x, fmaf(B5, q5.x, fmaf(B4, q4.x, fmaf(B3, q3.x, B1 * q1.x))));
        const float iy = fmaf(B6, q6.y, fmaf(B5, q5.y, fmaf(B4, q4.y, fmaf(B3, q3.y, B1 * q1.y))));
        // last stage: same time as the sixth, same fields (the cache stays valid)
        const float2 q7 = velocity(Fs[4], ax, ay, ix, iy, rhf, 0.f, cc);
        const float ex = fmaf(E7, q7.x, fmaf(E6, q6.x, fmaf(E5, q5.x, fmaf(E4, q4.x,
                              fmaf(E3, q3.x, E1 * q1.x)))));
        const float ey = fmaf(E7, q7.y, fmaf(E6, q6.y, fmaf(E5, q5.y, fmaf(E4, q4.y,
                              fmaf(E3, q3.y, E1 * q1.y)))));
        float sx, ex2, sy, ey2;
        two_sum(s0.x, ix, sx, ex2);
        two_sum(s0.y, iy, sy, ey2);
        stn[i] = make_float4(sx, sy, s0.z + ex2, s0.w + ey2);
        const float poison = (ex + ey) + (sx + sy);
        const float e = __builtin_isfinite(poison) ? fmaxf(fabsf(ex), fabsf(ey))
                                                  : __builtin_inff();
        emax = fmaxf(emax, e);
        kvn[i] = make_float2(q7.x * rhf, q7.y * rhf);
    }
    emax = wave_max(emax);
    if ((threadIdx.x & 63) == 0) s_err[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = s_err[0];
#pragma unroll
        for (int w = 1; w < kDiffThreads / 64; ++w) m = fmaxf(m, s_err[w]);
        part[blockIdx.x] = m;
    }
}

// Arm the attempt at (t, h): clip the last step to t_end, or take the next
// replayed step, and write the stage times.
__device__ inline void diff_arm(diff_ctl *c)
{
    double h;
    int fin;
    if (c->n_replay > 0) {
        h = c->replay_h[c->acc];
        fin = c->acc == c->n_replay - 1;
    } else {
        h = c->h;
        fin = h >= c->t_end - c->t;
        if (fin) h = c->t_end - c->t;
    }
    c->h_att = h;
    c->final_step = fin;
    c->ts[0] = c->t + h * (1.0 / 5);
    c->ts[1] = c->t + h * (3.0 / 10);
    c->ts[2] = c->t + h * (4.0 / 5);
    c->ts[3] = c->t + h * (8.0 / 9);
    c->ts[4] = c->t + h;
}

__device__ inline void diff_stop(diff_ctl *c, int32_t code, int32_t *status)
{
    c->status = code;
    c->done = 1;
    if (code) set_status(status, code);
}

// The grid maximum of the attempt's errors (all lanes; the maximum does not
// depend on the order), then on one lane the decision, the step update (the
// controller of k_advect, with t_end in place of 1) and the next attempt's
// stage times.  arm_only: start of the integration.
constexpr int kControlThreads = 256;
__global__ __launch_bounds__(kControlThreads) void kd_control(diff_ctl *c,
                                                              const float *__restrict__ part,
                                                              int nb, int arm_only,
                                                              int32_t *status)
{
    if (c->done) return;
    __shared__ float s_max[kControlThreads / 64];
    float v = 0.0f;
    if (!arm_only)
        for (int b = threadIdx.x; b < nb; b += kControlThreads) v = fmaxf(v, part[b]);
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int32_t st = __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (st != 0) {
        diff_stop(c, st, status);
    } else if (arm_only) {
        if (c->max_attempts <= 0) diff_stop(c, FFB_E_MAX_ATTEMPTS, status);
        else diff_arm(c);
    } else {
        float gm = s_max[0];
#pragma unroll
        for (int w = 1; w < kControlThreads / 64; ++w) gm = fmaxf(gm, s_max[w]);
        const double err = (double)gm;
        const double h = c->h_att;
        c->attempts += 1;
        const bool replay = c->n_replay > 0;
        if (!(err < __builtin_huge_val())) {
            diff_stop(c, FFB_E_NONFINITE, status);
        } else {
            if (replay || err <= c->tol) {
                c->cur ^= 1;
                if (c->h_out && c->acc < c->h_cap) c->h_out[c->acc] = h;
                c->acc += 1;
                c->t = c->final_step ? c->t_end : c->t + h;
                if (!replay) {
                    c->h = step_after_accept(h, err, c->tol, c->safety, c->fac_min, c->fac_max,
                                             c->last_rejected != 0);
                    c->last_rejected = 0;
                }
            } else {
                c->rej += 1;
                c->h = step_after_reject(h, err, c->tol, c->safety, c->fac_min);
                c->last_rejected = 1;
            }
            if (c->t >= c->t_end) {
                diff_stop(c, 0, status);
            } else if (!replay && c->h < c->h_min) {
                diff_stop(c, FFB_E_STEP_UNDERFLOW, status);
            } else if (c->attempts >= c->max_attempts || (replay && c->acc >= c->n_replay)) {
                diff_stop(c, FFB_E_MAX_ATTEMPTS, status);
            } else {
                diff_arm(c);
            }
        }
    }
    c->stats[0] = c->acc;
    c->stats[1] = c->rej;
    c->stats[2] = c->attempts;
    c->stats[3] = c->status;
}

__global__ __launch_bounds__(kDiffThreads) void kd_finish(const diff_ctl *__restrict__ c,
                                                          const float4 *st0, const float4 *st1,
                                                          float2 *__restrict__ xy,
                                                          const int32_t *__restrict__ perm,
                                                          int64_t n)
{
    if (c->status != 0 || !c->done) return;
    const float4 *s = c->cur ? st1 : st0;
    for (int64_t i = blockIdx.x * (int64_t)kDiffThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kDiffThreads) {
        const float4 q = s[i];
        xy[perm ? perm[i] : i] = make_float2(q.x + q.z, q.y + q.w);
    }
}

__global__ void kd_setup(diff_ctl *c, diff_ctl init)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = init;
}

inline int diff_blocks(int64_t n)
{
    int64_t nb = (n + 4 * kDiffThreads - 1) / (4 * kDiffThreads);     // ~4 points per lane
    nb = (nb + kXcds - 1) / kXcds * kXcds;
    if (nb < kXcds) nb = kXcds;
    if (nb > kDiffMaxBlocks) nb = kDiffMaxBlocks;
    return (int)nb;
}

}  // namespace

hipError_t launch_diff_setup(ffb_ctx *ctx, diff_ws *w, const diff_ctl &init)
{
    hipLaunchKernelGGL(kd_setup, dim3(1), dim3(64), 0, ctx->stream, w->ctl, init);
    return hipGetLastError();
}

hipError_t launch_diff_init_points(ffb_ctx *ctx, diff_ws *w, const float2 *xy, int64_t n,
                                   const int32_t *perm)
{
    if (n == 0) return hipSuccess;
    int64_t nb = (n + kDiffThreads - 1) / kDiffThreads;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(kd_init_points, dim3((unsigned)nb), dim3(kDiffThreads), 0, ctx->stream,
                       w->fields, ctx->lx, ctx->ly, xy, perm, n, ctx->st[0], ctx->kv[0],
                       ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_diff_points(ffb_ctx *ctx, diff_ws *w, int64_t n)
{
    const int nb = diff_blocks(n);
    hipLaunchKernelGGL(kd_points, dim3(nb), dim3(kDiffThreads), 0, ctx->stream, w->ctl, w->fields,
                       w->fplane, ctx->lx, ctx->ly, n, ctx->st[0], ctx->st[1], ctx->kv[0],
                       ctx->kv[1], w->part);
    return hipGetLastError();
}

hipError_t launch_diff_control(ffb_ctx *ctx, diff_ws *w, int64_t n, int arm_only)
{
    hipLaunchKernelGGL(kd_control, dim3(1), dim3(kControlThreads), 0, ctx->stream, w->ctl,
                       w->part, diff_blocks(n), arm_only, ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_diff_finish(ffb_ctx *ctx, diff_ws *w, float2 *xy, int64_t n,
                              const int32_t *perm)
{
    if (n == 0) return hipSuccess;
    int64_t nb = (n + kDiffThreads - 1) / kDiffThreads;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(kd_finish, dim3((unsigned)nb), dim3(kDiffThreads), 0, ctx->stream, w->ctl,
                       ctx->st[0], ctx->st[1], xy, perm, n);
    return hipGetLastError();
}

