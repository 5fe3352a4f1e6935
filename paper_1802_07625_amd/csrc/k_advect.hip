// Advection of every point from t = 0 to t = 1 (main text, section
// "Flow-based cartogram with linear equalization": velocities at grid points
// by basic arithmetic, interpolation between grid points, an adaptive
// predictor-corrector method whose steps advance all integrands together).
//
// Velocity: v(r, t) = J(r) / ((1 - t) rho_s(r) + t rho_bar)  (Eq. 4-6), formed
// at the four grid nodes around r and interpolated bilinearly (first along x
// on both node rows, then along y).  Lookups are clamped to the box; ghost
// nodes come from the field layout, so v . n = 0 exactly on the box edges.
//
// Integrator: Dormand-Prince 5(4) with first-same-as-last stages, one step
// size for all points.  The whole integration is ONE cooperative launch:
//   * each lane owns a fixed set of points (see Slots below), so a point's state
//     (compensated position hi + lo and its FSAL stage velocity) is private
//     to one lane; the position lives in LDS (or, for too many points, in a
//     double-buffered device array), the FSAL velocity in a double-buffered
//     device array;
//   * per attempt every lane evaluates the six new stages of its points,
//     stores the candidate state (keeping the previous one for a rejection)
//     and takes the max error;
//   * each workgroup stores its max in a tagged per-attempt slot and reads
//     all slots (the grid barrier and the grid-wide max in one); every
//     workgroup then takes the same accept/reject decision and step update
//     in FP64, so no second barrier and no host round trip are needed;
//   * the points may be visited in any order (a permutation from the caller
//     of the launch): no result depends on it;
//   * the barrier has a bounded wait, so every wave exits even if something
//     goes wrong (the status word then says FFB_E_DEVICE).
//
// Positions are compensated pairs hi + lo (an error-free sum adds each
// accepted increment).  A lookup at hi + lo + d splits off the integer part
// of hi - 1/2 once per point and attempt and forms the fraction from
// (hi - 1/2 - floor) + lo + d, so the bilinear weights keep ~1e-7 cells of
// precision at L = 1024; clamping to the box is one med3 on that fraction.
#include "advect_common.h"

namespace {

constexpr int kThreads = 1024;          // one workgroup per CU
constexpr int kSegments = 2;           // contiguous point segments per XCD
constexpr uint32_t kSpinLimit = 1u << 22;

// Synchronisation words, cleared before each launch: two banks (by attempt
// parity) of one 64-bit slot per workgroup holding (attempt + 1) << 32 | the
// workgroup's error maximum (FP32 bits).

struct Params {
    const float4 *fields;
    int lx, ly, pitch;
    const double *rho_bar;
    float2 *xy;
    int n;                  // < 2^31 (checked by the caller)
    float4 *st0, *st1;
    float2 *kv0, *kv1;
    uint64_t *sync;         // 2 banks x gridDim.x tagged slots
    int32_t *status;
    int32_t *stats;         // [4] accepted, rejected, attempts, status
    double *h_out;
    int32_t h_cap;
    double tol, h0, safety, fac_min, fac_max, h_min;
    int32_t max_attempts;
    int32_t n_replay;
    const double *replay_h;
    // optional visiting order: slot k of the launch integrates point perm[k]
    // (state, carried velocity and the point ranges are per slot)
    const int32_t *perm;
    // optional record for the adjoint: the state of the first tape_n points
    // before every accepted step, [tape_cap][tape_n], the accepted steps and
    // their count
    float4 *tape;
    int tape_n, tape_cap;
    double *tape_h;
    int32_t *tape_count;
};

// Slots of a workgroup.  Slots are cut into kXcds * kSegments equal
// segments; segment s belongs to XCD s mod kXcds, so each XCD (whose L2 is
// private) works on kSegments contiguous runs of slots -- with the points
// sorted by cell, two bands of the box; with the caller's [vertices | grid
// nodes] order, one run of each.  The valid slots of an XCD's runs are dealt
// to its workgroups in chunks of kChunk, round robin: the cost of a point
// depends on where it is, and each workgroup then samples the XCD's whole
// share (with contiguous per-workgroup ranges the slowest workgroup ran
// 10-15 % behind the mean, and every attempt waits for it).  A wave still
// takes kChunk consecutive slots per pass.  (Spreading each XCD's share
// over four or eight bands, to even out the XCDs too, and finding a chunk's
// start with scalar arithmetic both measured slower.)
constexpr int kChunk = 64;

struct Slots {
    int base0, va, base1;   // share slot j: base0 + j for j < va, else base1 + (j - va)
    int first, stride;      // this workgroup's chunks: first, first + stride, ...
    int npts;               // slots of this workgroup

    // the slot of this workgroup's k-th point
    __device__ int slot(int k) const
    {
        const int j = (first + stride * (k / kChunk)) * kChunk + k % kChunk;
        return j < va ? base0 + j : base1 + (j - va);
    }
};

__device__ inline Slots slots_of(int b, int nb, int n)
{
    const int nx = nb < kXcds ? nb : kXcds;
    const int x = b % nx, rank = b / nx;
    const int size = nb / nx + (x < nb % nx ? 1 : 0);
    const int seg = (n + nx * kSegments - 1) / (nx * kSegments);
    Slots s;
    s.base0 = x * seg;
    s.base1 = (nx + x) * seg;
    s.va = max(0, min(seg, n - s.base0));
    const int vb = max(0, min(seg, n - s.base1));
    const int total = s.va + vb;                             // valid slots of the share
    const int nch = (total + kChunk - 1) / kChunk;
    s.first = rank;
    s.stride = size;
    // chunks rank, rank + size, ... below nch; only the last one may be short
    const int q = rank < nch ? (nch - 1 - rank) / size + 1 : 0;
    s.npts = q * kChunk;
    if (q > 0 && (nch - 1 - rank) % size == 0) s.npts -= nch * kChunk - total;
    return s;
}

// Grid-wide maximum of the workgroups' values for attempt n; it doubles as
// the grid barrier of the attempt.  Each workgroup stores one tagged 64-bit
// slot; wave 0 of every workgroup then scans all slots of the attempt's bank
// (one relaxed load per lane per 64 workgroups, the loads of one scan issued
// together, four at a time) until every tag is current.
// No read-modify-write atomic and no cache-maintaining fence is involved, so
// the cost does not grow with contention on one address.  Banks alternate
// by attempt parity: a workgroup can only overwrite a bank two attempts
// later, after every workgroup has stored the slot of the attempt between,
// i.e. after every workgroup has finished scanning this one.  Returns false
// if the bounded wait ran out.
__device__ bool grid_max(uint64_t *sync, int n, float m, int32_t *status, float &out)
{
    __shared__ int ok;
    __shared__ float res;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int nb = gridDim.x;
        uint64_t *bank = sync + (size_t)(n & 1) * nb;
        const uint32_t tag = (uint32_t)(n + 1);
        if (lane == 0)
            __hip_atomic_store(&bank[blockIdx.x], ((uint64_t)tag << 32) | __float_as_uint(m),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0, mx = 0;
        int good = 1;
        for (;;) {
            bool done = true;
            uint32_t v = 0;
            for (int r0 = lane; r0 < nb; r0 += 4 * 64) {
                uint64_t w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // past the last slot a lane reads the last one again
                    const int r = r0 + 64 * j < nb ? r0 + 64 * j : nb - 1;
                    w[j] = __hip_atomic_load(&bank[r], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if ((uint32_t)(w[j] >> 32) != tag) done = false;
                    const uint32_t x = (uint32_t)w[j];
                    v = v > x ? v : x;
                }
            }
            if (__all(done)) {
                mx = wave_max_bits(v);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                good = 0;
                if (lane == 0) set_status(status, FFB_E_DEVICE);
                break;
            }
            if ((spins & 255u) == 0 &&
                __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    FFB_E_DEVICE) {
                good = 0;
                break;
            }
        }
        if (lane == 0) {
            res = __uint_as_float(mx);
            ok = good;
        }
    }
    __syncthreads();
    // res and ok are written again only after the next attempt's workgroup
    // barrier, which every wave reaches after reading them here
    out = res;
    return ok != 0;
}

// Where a point's state lives during one launch.
enum StateMode {
    kGlobalState = 0,   // (hi, lo) and the FSAL velocity double-buffered in HBM
    kLdsState = 1,      // (hi, lo) in LDS, FSAL velocity double-buffered in HBM
    kLdsRecompute = 2,  // (hi, lo) in LDS, first-stage velocity recomputed
};

// The six new stages of one attempt for one point, from q1 = h k1.  Stage
// positions are formed in the point's frame with the in-cell fraction folded
// into the stage sums.  Returns the order-5 increment (ix, iy), q7 = h k7
// and the error estimate (ex, ey).
__device__ inline void dp_stages(const Field &F, const Axis &ax, const Axis &ay, int B, float2 q1,
                                 const float *omh, const float *tbh, CellCache &cc, float &ix,
                                 float &iy, float2 &q7, float &ex, float &ey)
{
    const float fx = ax.frl, fy = ay.frl;
    const float2 q2 = velocity_at(F, ax, ay, B, fmaf(A21, q1.x, fx), fmaf(A21, q1.y, fy), omh[1],
                                  tbh[1], cc);
    const float2 q3 = velocity_at(F, ax, ay, B, fmaf(A32, q2.x, fmaf(A31, q1.x, fx)),
                                  fmaf(A32, q2.y, fmaf(A31, q1.y, fy)), omh[2], tbh[2], cc);
    const float2 q4 = velocity_at(
        F, ax, ay, B, fmaf(A43, q3.x, fmaf(A42, q2.x, fmaf(A41, q1.x, fx))),
        fmaf(A43, q3.y, fmaf(A42, q2.y, fmaf(A41, q1.y, fy))), omh[3], tbh[3], cc);
    const float2 q5 = velocity_at(
        F, ax, ay, B, fmaf(A54, q4.x, fmaf(A53, q3.x, fmaf(A52, q2.x, fmaf(A51, q1.x, fx)))),
        fmaf(A54, q4.y, fmaf(A53, q3.y, fmaf(A52, q2.y, fmaf(A51, q1.y, fy)))), omh[4], tbh[4],
        cc);
    const float2 q6 = velocity_at(
        F, ax, ay, B,
        fmaf(A65, q5.x, fmaf(A64, q4.x, fmaf(A63, q3.x, fmaf(A62, q2.x, fmaf(A61, q1.x, fx))))),
        fmaf(A65, q5.y, fmaf(A64, q4.y, fmaf(A63, q3.y, fmaf(A62, q2.y, fmaf(A61, q1.y, fy))))),
        omh[5], tbh[5], cc);
    // order-5 increment (weights of the last stage row; the k2 weight is 0)
    ix = fmaf(B6, q6.x, fmaf(B5, q5.x, fmaf(B4, q4.x, fmaf(B3, q3.x, B1 * q1.x))));
    iy = fmaf(B6, q6.y, fmaf(B5, q5.y, fmaf(B4, q4.y, fmaf(B3, q3.y, B1 * q1.y))));
    q7 = velocity_at(F, ax, ay, B, fx + ix, fy + iy, omh[6], tbh[6], cc);
    ex = fmaf(E7, q7.x, fmaf(E6, q6.x, fmaf(E5, q5.x, fmaf(E4, q4.x, fmaf(E3, q3.x, E1 * q1.x)))));
    ey = fmaf(E7, q7.y, fmaf(E6, q6.y, fmaf(E5, q5.y, fmaf(E4, q4.y, fmaf(E3, q3.y, E1 * q1.y)))));
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_advect(Params p)
{
    extern __shared__ float4 lds_state[];      // LDS modes: one slot per owned point
    __shared__ float s_err[kThreads / 64];
    // a status set by an earlier call (e.g. non-positive density) stops the
    // integration before any point is touched; the value is uniform.
    if (__hip_atomic_load(p.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;

    const double rho_bar = *p.rho_bar;
    const Field F = make_field(p.fields, p.lx, p.ly);
    const Slots sl = slots_of(blockIdx.x, gridDim.x, p.n);
    const int npts = sl.npts;
    const bool replay = p.n_replay > 0;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    float4 *bak = p.st0;                       // LDS modes: state before the attempt

    // initial state: hi = xy, lo = 0 (and the FSAL velocity at t = 0)
    for (int k = threadIdx.x; k < npts; k += kThreads) {
        const int i = sl.slot(k);
        const float2 y = p.xy[p.perm ? p.perm[i] : i];
        const float4 s0 = make_float4(y.x, y.y, 0.f, 0.f);
        if (MODE == kGlobalState) p.st0[i] = s0;
        else lds_state[k] = s0;
        if (MODE != kLdsRecompute) {
            CellCache cc;
            cc.key = -1;
            const Axis ax = make_axis(y.x, 0.f, p.lx), ay = make_axis(y.y, 0.f, p.ly);
            p.kv0[i] = velocity_at(F, ax, ay, cell_base(ax, ay, p.pitch), ax.frl, ay.frl, 1.0f,
                                   0.0f, cc);
        }
    }

    double t = 0.0, h = replay ? p.replay_h[0] : p.h0;
    int last_rejected = 0, acc = 0, rej = 0, attempt = 0, cur = 0;
    int32_t final_status = 0;

    while (t < 1.0) {
        if (attempt >= p.max_attempts || (replay && acc >= p.n_replay)) {
            final_status = FFB_E_MAX_ATTEMPTS;
            break;
        }
        bool final_step;
        if (replay) {
            h = p.replay_h[acc];
            final_step = acc == p.n_replay - 1;
        } else {
            final_step = h >= 1.0 - t;
            if (final_step) h = 1.0 - t;
        }
        // per-attempt uniforms: the step, its inverse and the time factors of
        // each stage divided by h (so lookups return h * v); the tableau
        // itself enters as instruction literals
        const double rh = 1.0 / h;
        const float hf = uniform((float)h), rhf = uniform((float)rh);
        float omh[7], tbh[7];
#pragma unroll
        for (int s = 0; s < 7; ++s) {
            const double ts = t + kC[s] * h;
            omh[s] = uniform((float)((1.0 - ts) * rh));
            tbh[s] = uniform((float)(ts * rho_bar * rh));
        }
        const float4 *stc = cur ? p.st1 : p.st0;
        const float2 *kvc = cur ? p.kv1 : p.kv0;
        float4 *stn = cur ? p.st0 : p.st1;
        float2 *kvn = cur ? p.kv0 : p.kv1;

        float emax = 0.0f;
        // a rejected attempt leaves the state unchanged, so the retry writes
        // the same record again
        float4 *rec = (p.tape && acc < p.tape_cap) ? p.tape + (int64_t)acc * p.tape_n : nullptr;
        for (int k = threadIdx.x; k < npts; k += kThreads) {
            const int i = sl.slot(k);
            const float4 s0 = MODE == kGlobalState ? stc[i] : lds_state[k];
            if (rec) {
                const int g = p.perm ? p.perm[i] : i;
                if (g < p.tape_n) rec[g] = s0;
            }
            const float hx = s0.x, hy = s0.y, lx = s0.z, ly = s0.w;
            const Axis ax = make_axis(hx, lx, p.lx), ay = make_axis(hy, ly, p.ly);
            const int B = cell_base(ax, ay, p.pitch);
            CellCache cc;
            cc.key = -1;
            // stage velocities scaled by the step: q_s = h k_s
            float2 q1;
            if (MODE == kLdsRecompute) {
                q1 = velocity_at(F, ax, ay, B, ax.frl, ay.frl, omh[0], tbh[0], cc);
            } else {
                const float2 k1 = kvc[i];
                q1 = make_float2(hf * k1.x, hf * k1.y);
            }
            float ix, iy, ex, ey;
            float2 q7;
            dp_stages(F, ax, ay, B, q1, omh, tbh, cc, ix, iy, q7, ex, ey);
            // candidate state: hi + increment split error-free, the rounding
            // error added to lo (whose own rounding stays ~1e-12 cells)
            float sx, ex2, sy, ey2;
            two_sum(hx, ix, sx, ex2);
            two_sum(hy, iy, sy, ey2);
            const float4 cand = make_float4(sx, sy, lx + ex2, ly + ey2);
            // a NaN or Inf in the error estimate or in the new position
            // poisons the maximum (fmaxf alone would drop a NaN)
            const float poison = (ex + ey) + (sx + sy);
            const float e = __builtin_isfinite(poison) ? fmaxf(fabsf(ex), fabsf(ey))
                                                      : __builtin_inff();
            emax = fmaxf(emax, e);
            if (MODE == kGlobalState) {
                stn[i] = cand;
            } else {
                bak[i] = s0;
                lds_state[k] = cand;
            }
            if (MODE != kLdsRecompute) kvn[i] = make_float2(q7.x * rhf, q7.y * rhf);
        }
        // workgroup max, then the grid-wide max (one barrier per attempt)
        emax = wave_max_bits_f(emax);
        if ((threadIdx.x & 63) == 0) s_err[threadIdx.x >> 6] = emax;
        __syncthreads();
        float m = s_err[0];
#pragma unroll
        for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, s_err[w]);
        float gmax;
        if (!grid_max(p.sync, attempt, m, p.status, gmax)) {
            final_status = FFB_E_DEVICE;
            break;
        }
        const double err = (double)gmax;
        ++attempt;
        if (!(err < __builtin_huge_val())) {
            final_status = FFB_E_NONFINITE;
            break;
        }
        if (replay || err <= p.tol) {
            cur ^= 1;
            if (lead && acc < p.h_cap && p.h_out) p.h_out[acc] = h;
            if (lead && acc < p.tape_cap && p.tape_h) p.tape_h[acc] = h;
            ++acc;
            t = final_step ? 1.0 : t + h;
            if (!replay) {
                h = step_after_accept(h, err, p.tol, p.safety, p.fac_min, p.fac_max,
                                      last_rejected);
                last_rejected = 0;
            }
        } else {
            ++rej;
            h = step_after_reject(h, err, p.tol, p.safety, p.fac_min);
            last_rejected = 1;
            if (MODE != kGlobalState) {
                // undo the attempt: every lane restores its own points
                for (int k = threadIdx.x; k < npts; k += kThreads) {
                    const int i = sl.slot(k);
                    lds_state[k] = bak[i];
                }
            }
        }
        if (!replay && t < 1.0 && h < p.h_min) {
            final_status = FFB_E_STEP_UNDERFLOW;
            break;
        }
    }

    if (final_status == 0) {
        const float4 *stc = cur ? p.st1 : p.st0;
        for (int k = threadIdx.x; k < npts; k += kThreads) {
            const int i = sl.slot(k);
            const float4 s = MODE == kGlobalState ? stc[i] : lds_state[k];
            p.xy[p.perm ? p.perm[i] : i] = make_float2(s.x + s.z, s.y + s.w);
        }
    }
    if (lead) {
        p.stats[0] = acc;
        p.stats[1] = rej;
        p.stats[2] = attempt;
        p.stats[3] = final_status;
        if (p.tape_count) *p.tape_count = acc;
        if (final_status) set_status(p.status, final_status);
    }
}

// LDS bytes a workgroup needs for its point slots (the largest chunk of the
// span mapping), or -1 if they exceed the per-workgroup LDS.
inline int64_t lds_bytes_for(int nb, int64_t n)
{
    const int64_t nx = nb < kXcds ? nb : kXcds;
    const int64_t seg = (n + nx * kSegments - 1) / (nx * kSegments);
    const int64_t nch = (seg * kSegments + kChunk - 1) / kChunk;   // chunks of the largest share
    const int64_t size_min = nb / nx;
    return (nch + size_min - 1) / size_min * kChunk * (int64_t)sizeof(float4);
}

// ------------------------------------------------------------- batched
// Many maps, one workgroup per map (largest maps first): the same stages,
// controller and compensated state as k_advect, with the error maximum
// reduced over the workgroup only.  No workgroup waits for another, so the
// launch needs no co-residency and can be captured in a graph.  State and
// first-stage velocities live in HBM, double-buffered per point.
template <int NT>
__global__ __launch_bounds__(NT) void kb_advect(batch_view bv, batch_advect_args a,
                                                int32_t *status)
{
    __shared__ float s_err[2][NT / 64];
    const int m = a.order[blockIdx.x];
    if (!bv.active[m]) return;
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    const double rho_bar = a.rho_bar[m];
    const int lx = bv.lx[m], ly = bv.ly[m];
    const Field F = make_field(a.fields + bv.field_off[m], lx, ly);
    const int64_t p0 = bv.point_off[m];
    const int npts = (int)(bv.point_off[m + 1] - p0);
    const int n_replay = a.replay_off ? a.replay_off[m + 1] - a.replay_off[m] : 0;
    const double *replay_h = a.replay_off ? a.replay_h + a.replay_off[m] : nullptr;
    const bool replay = n_replay > 0;
    float4 *st0 = a.st0 + p0, *st1 = a.st1 + p0;
    float2 *kv0 = a.kv0 + p0, *kv1 = a.kv1 + p0;
    float2 *xy = a.xy + p0;

    for (int k = threadIdx.x; k < npts; k += NT) {
        const float2 y = xy[k];
        st0[k] = make_float4(y.x, y.y, 0.f, 0.f);
        CellCache cc;
        cc.key = -1;
        const Axis ax = make_axis(y.x, 0.f, lx), ay = make_axis(y.y, 0.f, ly);
        kv0[k] = velocity_at(F, ax, ay, cell_base(ax, ay, lx + 2), ax.frl, ay.frl, 1.0f, 0.0f,
                             cc);
    }

    double t = 0.0, h = replay ? replay_h[0] : a.h0;
    int last_rejected = 0, acc = 0, rej = 0, attempt = 0, cur = 0;
    int32_t final_status = 0;
    while (t < 1.0) {
        if (attempt >= a.max_attempts || (replay && acc >= n_replay)) {
            final_status = FFB_E_MAX_ATTEMPTS;
            break;
        }
        bool final_step;
        if (replay) {
            h = replay_h[acc];
            final_step = acc == n_replay - 1;
        } else {
            final_step = h >= 1.0 - t;
            if (final_step) h = 1.0 - t;
        }
        const double rh = 1.0 / h;
        const float hf = uniform((float)h), rhf = uniform((float)rh);
        float omh[7], tbh[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double ts = t + kC[q] * h;
            omh[q] = uniform((float)((1.0 - ts) * rh));
            tbh[q] = uniform((float)(ts * rho_bar * rh));
        }
        const float4 *stc = cur ? st1 : st0;
        const float2 *kvc = cur ? kv1 : kv0;
        float4 *stn = cur ? st0 : st1;
        float2 *kvn = cur ? kv0 : kv1;
        float emax = 0.0f;
        for (int k = threadIdx.x; k < npts; k += NT) {
            const float4 s0 = stc[k];
            const Axis ax = make_axis(s0.x, s0.z, lx), ay = make_axis(s0.y, s0.w, ly);
            CellCache cc;
            cc.key = -1;
            const float2 k1 = kvc[k];
            const float2 q1 = make_float2(hf * k1.x, hf * k1.y);
            float ix, iy, ex, ey;
            float2 q7;
            dp_stages(F, ax, ay, cell_base(ax, ay, lx + 2), q1, omh, tbh, cc, ix, iy, q7, ex, ey);
            float sx, ex2, sy, ey2;
            two_sum(s0.x, ix, sx, ex2);
            two_sum(s0.y, iy, sy, ey2);
            stn[k] = make_float4(sx, sy, s0.z + ex2, s0.w + ey2);
            const float poison = (ex + ey) + (sx + sy);
            const float e = __builtin_isfinite(poison) ? fmaxf(fabsf(ex), fabsf(ey))
                                                      : __builtin_inff();
            emax = fmaxf(emax, e);
            kvn[k] = make_float2(q7.x * rhf, q7.y * rhf);
        }
        // the banks alternate by attempt parity: a bank is written again two
        // attempts later, after a barrier every wave passes once it has read
        // this attempt's maxima, so one barrier per attempt suffices
        float *se = s_err[attempt & 1];
        emax = wave_max_bits_f(emax);
        if ((threadIdx.x & 63) == 0) se[threadIdx.x >> 6] = emax;
        __syncthreads();
        float gmax = se[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) gmax = fmaxf(gmax, se[w]);
        const double err = (double)gmax;
        ++attempt;
        if (!(err < __builtin_huge_val())) {
            final_status = FFB_E_NONFINITE;
            break;
        }
        if (replay || err <= a.tol) {
            cur ^= 1;
            ++acc;
            t = final_step ? 1.0 : t + h;
            if (!replay) {
                h = step_after_accept(h, err, a.tol, a.safety, a.fac_min, a.fac_max,
                                      last_rejected);
                last_rejected = 0;
            }
        } else {
            ++rej;
            h = step_after_reject(h, err, a.tol, a.safety, a.fac_min);
            last_rejected = 1;
        }
        if (!replay && t < 1.0 && h < a.h_min) {
            final_status = FFB_E_STEP_UNDERFLOW;
            break;
        }
    }
    if (final_status == 0) {
        const float4 *stc = cur ? st1 : st0;
        for (int k = threadIdx.x; k < npts; k += NT) {
            const float4 q = stc[k];
            xy[k] = make_float2(q.x + q.z, q.y + q.w);
        }
    }
    if (threadIdx.x == 0) {
        int32_t *st = a.stats + 4 * (int64_t)m;
        st[0] = acc;
        st[1] = rej;
        st[2] = attempt;
        st[3] = final_status;
        if (final_status) set_status(status, final_status);
    }
}

}  // namespace

int advect_max_blocks(int *out)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_advect<kGlobalState>, kThreads, 0) !=
        hipSuccess)
        return -1;
    *out = cus * per;
    return 0;
}

hipError_t launch_advect(ffb_ctx *ctx, const float4 *fields, const double *rho_bar,
                         float2 *xy, int64_t n, const ffb_integrate_opts *o, int32_t *stats,
                         double *h_out, int32_t h_cap, const advect_tape *tape,
                         const int32_t *perm)
{
    int64_t want = (n + kThreads - 1) / kThreads;
    if (want < 1) want = 1;
    int blocks = ctx->adv_blocks;
    if (ctx->adv_cap > 0 && ctx->adv_cap < blocks) blocks = ctx->adv_cap;
    if (want < blocks) blocks = (int)want;
    if (4 * blocks > ctx->err_cap) return hipErrorInvalidValue;
    // synchronisation slots, cleared by a kernel (graph-capture safe)
    hipError_t e = launch_fill_u32(ctx->errslot, 4 * (int64_t)blocks, 0u, ctx->stream);
    if (e != hipSuccess) return e;
    Params p;
    p.fields = fields;
    p.lx = ctx->lx;
    p.ly = ctx->ly;
    p.pitch = ctx->lx + 2;
    p.rho_bar = rho_bar;
    p.xy = xy;
    p.n = (int)n;
    p.st0 = ctx->st[0];
    p.st1 = ctx->st[1];
    p.kv0 = ctx->kv[0];
    p.kv1 = ctx->kv[1];
    p.sync = reinterpret_cast<uint64_t *>(ctx->errslot);
    p.status = ctx->d_status;
    p.stats = stats;
    p.h_out = h_out;
    p.h_cap = h_cap;
    p.tol = o->tol;
    p.h0 = o->h0;
    p.safety = o->safety;
    p.fac_min = o->fac_min;
    p.fac_max = o->fac_max;
    p.h_min = o->h_min;
    p.max_attempts = o->max_attempts;
    p.n_replay = o->n_replay;
    p.replay_h = o->replay_h;
    p.perm = perm;
    p.tape = tape ? tape->states : nullptr;
    p.tape_n = tape ? (int)tape->n : 0;
    p.tape_cap = tape ? tape->cap : 0;
    p.tape_h = tape ? tape->h : nullptr;
    p.tape_count = tape ? tape->count : nullptr;
    void *args[] = {&p};
    // keep the point state in LDS when one workgroup's share fits (one
    // workgroup per CU, 160 KB of LDS each on gfx950)
    const int64_t lds = lds_bytes_for(blocks, n);
    int dev = 0, lds_max = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t reserve = 1024;              // static LDS of the kernel
    if (ctx->adv_mode != kGlobalState && blocks <= cus && lds + reserve <= lds_max) {
        const void *k = ctx->adv_mode == kLdsState
                            ? reinterpret_cast<const void *>(k_advect<kLdsState>)
                            : reinterpret_cast<const void *>(k_advect<kLdsRecompute>);
        return hipLaunchCooperativeKernel(k, dim3(blocks), dim3(kThreads), args, (size_t)lds,
                                          ctx->stream);
    }
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_advect<kGlobalState>),
                                      dim3(blocks), dim3(kThreads), args, 0, ctx->stream);
}

hipError_t launch_batch_advect(hipStream_t s, const batch_view &bv, const batch_advect_args &a,
                               int threads, int32_t *status)
{
    const dim3 grid(bv.n_maps);
    switch (threads) {
    case 256:
        hipLaunchKernelGGL(kb_advect<256>, grid, dim3(256), 0, s, bv, a, status);
        break;
    case 512:
        hipLaunchKernelGGL(kb_advect<512>, grid, dim3(512), 0, s, bv, a, status);
        break;
    case 1024:
        hipLaunchKernelGGL(kb_advect<1024>, grid, dim3(1024), 0, s, bv, a, status);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
