// Blur and flux on the grid nodes: the cosine coefficients of Eq. 7 (the
// integral taken by the midpoint rule on cell centres, i.e. a 2D DCT-II),
// a Gaussian blur (diagonal in this basis), and the sine/cosine flux series
// of the SI Appendix (section 2) for linear equalisation, evaluated on the
// nodes with DCT-III / DST-III transforms.
//
// Pipeline (lx x ly grid, x fastest):
//   k_dct2_rows   rows j:      T1[j][m]  = sum_i rho[j][i] cos(pi m (i+1/2)/lx)
//   k_col_pass    columns m:   S[n][m]   = sum_j T1[j][m] cos(pi n (j+1/2)/ly)
//                              rts       = 4 S / ((1+d_m0)(1+d_n0)) * gauss(m, n)
//                              a[j][m]   = sum_n rts cos(pi n (j+1/2)/ly)
//                              b[j][m]   = sum_n wx(m,n) rts cos(...)
//                              c[j][m]   = sum_n wy(m,n) rts sin(pi n (j+1/2)/ly)
//   k_row_final   rows j:      rho_s = sum_m a cos / (lx ly), J_x = sum_m b sin,
//                              J_y = sum_m c cos  -> ghosted float4 fields
// with wx = (ly/pi) m/(m^2 ly^2 + n^2 lx^2), wy = (lx/pi) n/(...).
//
// Every 1D transform is a length-N complex FFT in LDS (radix-4 Stockham,
// twiddles staged in LDS) serving two real rows at once (one as the real,
// one as the imaginary part), with the even/odd reordering of Makhoul
// (1980) turning the real DCT-II/DCT-III into a plain FFT; the DST-III is a
// DCT-III of the index-reversed coefficients with alternating output signs.
#include <algorithm>

#include "ffb_internal.h"

namespace {

constexpr int kMaxN = 1024;

// Real and complex types of one precision: the single-map flux runs in FP64
// (double / double2), the batched, diffusion and adjoint transforms in FP32
// (float / float2).
template <typename R> struct cx_of;
template <> struct cx_of<float> { using T = float2; };
template <> struct cx_of<double> { using T = double2; };
template <typename R> using cx = typename cx_of<R>::T;

template <typename C> struct re_of;
template <> struct re_of<float2> { using T = float; };
template <> struct re_of<double2> { using T = double; };

template <typename C>
__device__ inline C mkc(typename re_of<C>::T x, typename re_of<C>::T y)
{
    C c;
    c.x = x;
    c.y = y;
    return c;
}

__device__ inline float rexp(float x) { return expf(x); }
__device__ inline double rexp(double x) { return exp(x); }

template <typename C>
__device__ inline C cmul(C a, C b)
{
    return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int ilog2(int n) { return 31 - __clz(n); }

// Stockham autosort FFT (unnormalised), decimation in time, radix 4 with one
// radix-2 pass first when log2 N is odd.  `a` holds the input; returns the
// buffer holding the output (a or b).  `tw` (LDS) = exp(-2 pi i k / N),
// k < N/2; the inverse uses the conjugates.
//
// Before a pass with sub-length Ls, a[p Ls + j] holds bin j of the length-Ls
// DFT of the decimated sequence x[p + r N/Ls].  A radix-4 pass combines the
// four sequences p = q + m N/(4 Ls), m = 0..3 (stored N/4 apart):
//   X[j + t Ls] = sum_m w_{4Ls}^{m j} w_4^{m t} x_m,  t = 0..3,
// written to b[q 4Ls + j + t Ls].  Half as many passes as radix 2, so half
// the LDS traffic and barriers.
template <typename C>
__device__ __forceinline__ C *fft_lds(C *a, C *b, int N, const C *tw, bool inverse)
{
    const int lgN = ilog2(N);
    const int half = N >> 1, quarter = N >> 2;
    int lgL = 0;
    if (lgN & 1) {
        // radix 2 with Ls = 1: every twiddle is 1
        __syncthreads();
        for (int bi = threadIdx.x; bi < half; bi += blockDim.x) {
            const C u = a[bi], v = a[bi + half];
            b[2 * bi] = mkc<C>(u.x + v.x, u.y + v.y);
            b[2 * bi + 1] = mkc<C>(u.x - v.x, u.y - v.y);
        }
        C *t = a;
        a = b;
        b = t;
        lgL = 1;
    }
    for (; lgL < lgN; lgL += 2) {
        const int Ls = 1 << lgL;
        const int sh = lgN - 2 - lgL;                 // log2 of N / (4 Ls)
        __syncthreads();
        for (int bi = threadIdx.x; bi < quarter; bi += blockDim.x) {
            const int j = bi & (Ls - 1);
            const int k = bi >> lgL;
            const int e1 = j << sh, e3 = 3 * e1;     // e1 < N/4, 2 e1 < N/2, e3 < 3N/4
            C w1 = tw[e1], w2 = tw[2 * e1];
            C w3 = e3 < half ? tw[e3] : tw[e3 - half];
            if (e3 >= half) w3 = mkc<C>(-w3.x, -w3.y);   // exp(-i pi) = -1
            if (inverse) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w3.y = -w3.y;
            }
            const C x0 = a[bi];
            const C x1 = cmul(a[bi + quarter], w1);
            const C x2 = cmul(a[bi + 2 * quarter], w2);
            const C x3 = cmul(a[bi + 3 * quarter], w3);
            const C a0 = mkc<C>(x0.x + x2.x, x0.y + x2.y);
            const C a1 = mkc<C>(x0.x - x2.x, x0.y - x2.y);
            const C b0 = mkc<C>(x1.x + x3.x, x1.y + x3.y);
            const C b1 = mkc<C>(x1.x - x3.x, x1.y - x3.y);
            // w_4 b1: -i b1 forward, +i b1 inverse
            const C rb = inverse ? mkc<C>(-b1.y, b1.x) : mkc<C>(b1.y, -b1.x);
            const int o = (k << (lgL + 2)) + j;
            b[o] = mkc<C>(a0.x + b0.x, a0.y + b0.y);
            b[o + Ls] = mkc<C>(a1.x + rb.x, a1.y + rb.y);
            b[o + 2 * Ls] = mkc<C>(a0.x - b0.x, a0.y - b0.y);
            b[o + 3 * Ls] = mkc<C>(a1.x - rb.x, a1.y - rb.y);
        }
        C *t = a;
        a = b;
        b = t;
    }
    __syncthreads();
    return a;
}

// `s`: stride into a table built for a longer transform (tables for length
// 1024 serve every power of two N <= 1024 with s = 1024 / N).
template <typename C>
__device__ inline void load_twiddles(C *tw_lds, const C *__restrict__ tw, int N, int s = 1)
{
    for (int k = threadIdx.x; k < (N >> 1); k += blockDim.x) tw_lds[k] = tw[k * s];
}

// Makhoul reordering position of input element i: v[i/2] for even i,
// v[N-1-(i-1)/2] for odd i.
__device__ inline int mk_pos(int i, int N) { return (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1); }

// From the FFT Z of a Makhoul-ordered pair (rows a + i b), the DCT-II pair
// (X_a[m], X_b[m]) (unnormalised: sum x_i cos(pi m (i+1/2)/N)).
template <typename C>
__device__ inline C dct2_bin(const C *Z, int m, int N, const C *__restrict__ tq, int qs)
{
    using R = typename re_of<C>::T;
    const C zm = Z[m];
    const C zc = Z[(N - m) & (N - 1)];
    // Va = (Zm + conj Zc)/2, Vb = (Zm - conj Zc)/(2i)
    const R h = R(0.5);
    const C va = mkc<C>(h * (zm.x + zc.x), h * (zm.y - zc.y));
    const C vb = mkc<C>(h * (zm.y + zc.y), -h * (zm.x - zc.x));
    const C q = tq[m * qs];      // exp(-i pi m / (2N))
    return mkc<C>(q.x * va.x - q.y * va.y, q.x * vb.x - q.y * vb.y);
}

// DCT-II of two rows held as (ra[i], rb[i]) pairs already placed in `a` in
// Makhoul order; leaves the pairs in `out`.
template <typename C>
__device__ __forceinline__ void dct2_pair(C *a, C *b, C *out, int N, const C *tw,
                                          const C *__restrict__ tq, int qs = 1)
{
    C *Z = fft_lds(a, b, N, tw, false);
    for (int m = threadIdx.x; m < N; m += blockDim.x) out[m] = dct2_bin(Z, m, N, tq, qs);
    __syncthreads();
}

// Build the inverse-transform input for a pair of DCT-III sums
//   y_i = sum_{m<N} c_m cos(pi m (i+1/2)/N)
// from coefficient pairs cpair(m) = (c_a[m], c_b[m]) into `a`:
//   X_0 = c_0, X_m = c_m / 2, W_m = exp(i pi m/(2N)) (X_m - i X_{N-m}), X_N = 0,
// and the pair is packed as W_a + i W_b.
template <typename C, typename F>
__device__ void dct3_input(C *a, int N, const C *__restrict__ tq, F cpair, int qs = 1)
{
    using R = typename re_of<C>::T;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        C xm = cpair(m);
        if (m) { xm.x *= R(0.5); xm.y *= R(0.5); }
        C xr = mkc<C>(R(0), R(0));
        if (m) { xr = cpair(N - m); xr.x *= R(0.5); xr.y *= R(0.5); }
        const C q = tq[m * qs];
        const R cr = q.x, ci = -q.y;          // exp(+i pi m/(2N))
        // Wa = (cr + i ci)(xm.x - i xr.x), Wb likewise with .y
        const R war = cr * xm.x + ci * xr.x, wai = ci * xm.x - cr * xr.x;
        const R wbr = cr * xm.y + ci * xr.y, wbi = ci * xm.y - cr * xr.y;
        a[m] = mkc<C>(war - wbi, wai + wbr);   // Wa + i Wb
    }
}

// After the inverse FFT of dct3_input, output y[i] of the pair:
// even i -> v[i/2], odd i -> v[N-1-(i-1)/2]; real part = row a, imag = row b.
template <typename C>
__device__ inline C dct3_output(const C *v, int i, int N) { return v[mk_pos(i, N)]; }

// ------------------------------------------------------------------ kernels
// DCT-II of rows r0, r0 + 1 of `in` [rows][N] (densities) into `out`
// (precision R; LDS: sa, sb of kMaxN and stw of kMaxN / 2 complex).
template <typename R, typename In>
__device__ __forceinline__ void dct2_rows_body(const In *__restrict__ in, R *__restrict__ out,
                                               int64_t r0, int N, const cx<R> *__restrict__ tw,
                                               const cx<R> *__restrict__ tq, int qs, cx<R> *sa,
                                               cx<R> *sb, cx<R> *stw)
{
    using C = cx<R>;
    load_twiddles(stw, tw, N, qs);
    const In *ra = in + r0 * N, *rb = ra + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x)
        sa[mk_pos(i, N)] = mkc<C>((R)ra[i], (R)rb[i]);
    // result pairs land in sa or sb; reuse the other as output staging
    C *Z = fft_lds(sa, sb, N, stw, false);
    C *o = (Z == sa) ? sb : sa;
    for (int m = threadIdx.x; m < N; m += blockDim.x) o[m] = dct2_bin(Z, m, N, tq, qs);
    __syncthreads();
    R *oa = out + r0 * N, *ob = oa + N;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        oa[m] = o[m].x;
        ob[m] = o[m].y;
    }
}

// Two rows per workgroup (FP64); with `rowsum` set, also the FP64 sum of the
// two input rows (in a fixed order), for the mean density.
__global__ __launch_bounds__(512) void k_dct2_rows(const double *__restrict__ in,
                                                   double *__restrict__ out, int N,
                                                   const double2 *__restrict__ tw,
                                                   const double2 *__restrict__ tq,
                                                   double *__restrict__ rowsum)
{
    __shared__ double2 sa[kMaxN], sb[kMaxN], stw[kMaxN / 2];
    __shared__ double ssum[512 / 64];
    if (rowsum) {
        const double *r = in + 2 * (int64_t)blockIdx.x * N;
        double v = 0.0;
        for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) v += r[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) ssum[threadIdx.x >> 6] = v;
    }
    dct2_rows_body<double, double>(in, out, 2 * (int64_t)blockIdx.x, N, tw, tq, 1, sa, sb, stw);
    if (rowsum && threadIdx.x == 0) {
        // dct2_rows_body passes workgroup barriers after the writes above
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += ssum[w];
        rowsum[blockIdx.x] = t;
    }
}

// Two rows per workgroup, FP32 transform of the FP64 densities (diffusion
// spectrum).
__global__ __launch_bounds__(512) void k_dct2_rows_f32(const double *__restrict__ in,
                                                       float *__restrict__ out, int N,
                                                       const float2 *__restrict__ tw,
                                                       const float2 *__restrict__ tq)
{
    __shared__ float2 sa[kMaxN], sb[kMaxN], stw[kMaxN / 2];
    dct2_rows_body<float, double>(in, out, 2 * (int64_t)blockIdx.x, N, tw, tq, 1, sa, sb, stw);
}

// One 32 x 32 tile (columns c0.., rows r0..) of in [R][C] -> out [C][R],
// through LDS; 256 threads.
template <typename T>
__device__ void transpose_tile(const T *__restrict__ in, T *__restrict__ out, int R, int C,
                               int c0, int r0, T (*tile)[33])
{
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        if (r < R && c < C) tile[k][tx] = in[(int64_t)r * C + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (r < R && c < C) out[(int64_t)c * R + r] = tile[tx][k];
    }
}

// 32 x 32 tiles through LDS; in [R][C] -> out [C][R]; z selects the plane.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ in0,
                                                   const T *__restrict__ in1,
                                                   const T *__restrict__ in2, T *__restrict__ out0,
                                                   T *__restrict__ out1, T *__restrict__ out2,
                                                   int R, int C)
{
    __shared__ T tile[32][33];
    const T *in = blockIdx.z == 0 ? in0 : (blockIdx.z == 1 ? in1 : in2);
    T *out = blockIdx.z == 0 ? out0 : (blockIdx.z == 1 ? out1 : out2);
    transpose_tile(in, out, R, C, blockIdx.x * 32, blockIdx.y * 32, tile);
}

// Column pass on columns m0, m1 = m0 + 1 of T1 [ly][lx] (precision R; LDS:
// sa, sb, coef of kMaxN and stw of kMaxN / 2 complex).  The pair is read and
// written in the row-major planes directly, one two-element access per row;
// the workgroups of the pairs that share a cache line run on one XCD (see
// col_pair), so the lines are fetched from HBM once.
template <typename R>
__device__ __forceinline__ void col_pass_body(const R *__restrict__ t1, int m0, int lx, int ly,
                                              float sigma, const cx<R> *__restrict__ tw,
                                              const cx<R> *__restrict__ tq, int qs,
                                              R *__restrict__ pa, R *__restrict__ pb,
                                              R *__restrict__ pc, cx<R> *sa, cx<R> *sb,
                                              cx<R> *coef, cx<R> *stw)
{
    using C = cx<R>;
    const int N = ly;
    const int64_t cs = lx / 2;                 // row stride in pairs
    load_twiddles(stw, tw, N, qs);
    const C *src = reinterpret_cast<const C *>(t1 + m0);
    for (int i = threadIdx.x; i < N; i += blockDim.x) sa[mk_pos(i, N)] = src[i * cs];
    dct2_pair(sa, sb, coef, N, stw, tq, qs);   // coef[n] = (S[n][m0], S[n][m1])

    // normalisation of Eq. 7 and the blur, separable in m and n
    const R PI = R(3.14159265358979323846);
    const R sg = (R)sigma;
    const R cgx = PI * PI * sg * sg / (R(2) * (R)lx * (R)lx);
    const R cgy = PI * PI * sg * sg / (R(2) * (R)ly * (R)ly);
    const R gx0 = rexp(-cgx * (R)m0 * (R)m0) * (m0 == 0 ? R(2) : R(4));
    const R gx1 = rexp(-cgx * (R)(m0 + 1) * (R)(m0 + 1)) * R(4);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const R gy = rexp(-cgy * (R)n * (R)n) * (n == 0 ? R(0.5) : R(1));
        const C s = coef[n];
        coef[n] = mkc<C>(s.x * gx0 * gy, s.y * gx1 * gy);
    }
    __syncthreads();

    const R flx = (R)lx, fly = (R)ly;
    const R inv_pi = R(0.318309886183790671537767526745);
    const R ma = (R)m0, mb = (R)(m0 + 1);

    // a: plain DCT-III of the coefficients
    dct3_input(sa, N, tq, [&](int n) { return coef[n]; }, qs);
    C *v = fft_lds(sa, sb, N, stw, true);
    C *oa = reinterpret_cast<C *>(pa + m0);
    for (int i = threadIdx.x; i < N; i += blockDim.x) oa[i * cs] = dct3_output(v, i, N);
    // b and c weigh the coefficients with
    //   wx(m, n) = (ly/pi) m / (m^2 ly^2 + n^2 lx^2),  wy(m, n) = (lx/pi) n / (...),
    // zero where the numerator vanishes: the coefficients are divided by the
    // common denominator once, in place, and each sum takes its numerator
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const R nl = (R)n * flx;
        const C c = coef[n];
        const R da = (ma * fly) * (ma * fly) + nl * nl, db = (mb * fly) * (mb * fly) + nl * nl;
        // the (m, n) = (0, 0) term has no flux (both numerators vanish)
        coef[n] = mkc<C>(da > R(0) ? c.x / da : R(0), c.y / db);
    }
    __syncthreads();
    // b: DCT-III of wx * coefficients
    const R kxa = fly * inv_pi * ma, kxb = fly * inv_pi * mb;
    dct3_input(sa, N, tq, [&](int n) {
        const C c = coef[n];
        return mkc<C>(kxa * c.x, kxb * c.y);
    }, qs);
    v = fft_lds(sa, sb, N, stw, true);
    C *ob = reinterpret_cast<C *>(pb + m0);
    for (int i = threadIdx.x; i < N; i += blockDim.x) ob[i * cs] = dct3_output(v, i, N);
    __syncthreads();
    // c: DST-III of wy * coefficients = (-1)^j DCT-III of the reversed sequence
    const R ky = flx * inv_pi;
    dct3_input(sa, N, tq, [&](int mm) {
        if (mm == 0) return mkc<C>(R(0), R(0));
        const int n = N - mm;
        const C c = coef[n];
        const R k = ky * (R)n;
        return mkc<C>(k * c.x, k * c.y);
    }, qs);
    v = fft_lds(sa, sb, N, stw, true);
    C *oc = reinterpret_cast<C *>(pc + m0);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const C y = dct3_output(v, i, N);
        const R s = (i & 1) ? R(-1) : R(1);
        oc[i * cs] = mkc<C>(s * y.x, s * y.y);
    }
}

// Column pair of workgroup b out of np pairs (FP64 pairs, 16 bytes): the
// eight pairs of one 128-byte line go to workgroups b, b + 8, ..., b + 56,
// which the dispatcher places on the same XCD one after another, so each
// line of the planes is fetched into that XCD's L2 once.  Any other count
// keeps the plain order.
__device__ __forceinline__ int col_pair(int b, int np)
{
    if (np % 64) return b;
    const int x = b & 7, s = b >> 3;
    return (((s >> 3) << 3) + x) * 8 + (s & 7);
}

__global__ __launch_bounds__(512) void k_col_pass(const double *__restrict__ t1, int lx, int ly,
                                                  float sigma, const double2 *__restrict__ tw,
                                                  const double2 *__restrict__ tq,
                                                  double *__restrict__ pa, double *__restrict__ pb,
                                                  double *__restrict__ pc)
{
    __shared__ double2 sa[kMaxN], sb[kMaxN], coef[kMaxN], stw[kMaxN / 2];
    const int m0 = 2 * col_pair(blockIdx.x, lx / 2);
    col_pass_body<double>(t1, m0, lx, ly, sigma, tw, tq, 1, pa, pb, pc, sa, sb, coef, stw);
}

// Row pass on rows j0, j1 = j0 + 1 of a, b, c [ly][lx] (precision R);
// writes the ghosted FP32 float4 fields (J_x, J_y, rho_s, 0), each value
// rounded once from R, to `fields` and, if not null, to `fields2` (LDS: sa,
// sb, rs, jx of kMaxN and stw of kMaxN / 2 complex).
template <typename R>
__device__ __forceinline__ void row_final_body(const R *__restrict__ pa, const R *__restrict__ pb,
                                               const R *__restrict__ pc, int j0, int lx, int ly,
                                               const cx<R> *__restrict__ tw,
                                               const cx<R> *__restrict__ tq, int qs,
                                               float4 *__restrict__ fields, int32_t *status,
                                               cx<R> *sa, cx<R> *sb, cx<R> *rs, cx<R> *jx,
                                               cx<R> *stw, float4 *__restrict__ fields2 = nullptr)
{
    using C = cx<R>;
    const int N = lx;
    load_twiddles(stw, tw, N, qs);
    const R norm = R(1) / ((R)lx * (R)ly);

    const R *a0 = pa + (int64_t)j0 * N, *a1 = a0 + N;
    dct3_input(sa, N, tq, [&](int m) { return mkc<C>(a0[m], a1[m]); }, qs);
    C *v = fft_lds(sa, sb, N, stw, true);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const C y = dct3_output(v, i, N);
        rs[i] = mkc<C>(y.x * norm, y.y * norm);
    }
    __syncthreads();
    const R *b0 = pb + (int64_t)j0 * N, *b1 = b0 + N;
    dct3_input(sa, N, tq, [&](int mm) {
        if (mm == 0) return mkc<C>(R(0), R(0));
        return mkc<C>(b0[N - mm], b1[N - mm]);
    }, qs);
    v = fft_lds(sa, sb, N, stw, true);
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const C y = dct3_output(v, i, N);
        const R s = (i & 1) ? R(-1) : R(1);
        jx[i] = mkc<C>(s * y.x, s * y.y);
    }
    __syncthreads();
    const R *c0 = pc + (int64_t)j0 * N, *c1 = c0 + N;
    dct3_input(sa, N, tq, [&](int m) { return mkc<C>(c0[m], c1[m]); }, qs);
    v = fft_lds(sa, sb, N, stw, true);

    const int P = lx + 2;
    int bad = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const C jy = dct3_output(v, i, N);
        const C r = rs[i], x = jx[i];
        const float4 f0 = make_float4((float)x.x, (float)jy.x, (float)r.x, 0.f);
        const float4 f1 = make_float4((float)x.y, (float)jy.y, (float)r.y, 0.f);
        bad |= !(f0.z > 0.f) || !(f1.z > 0.f);
        auto put = [&](float4 *__restrict__ out) {
            float4 *row0 = out + (int64_t)(j0 + 1) * P;
            float4 *row1 = row0 + P;
            row0[i + 1] = f0;
            row1[i + 1] = f1;
            // ghost columns: J_x odd across the x edges
            if (i == 0 || i == N - 1) {
                const int gi = (i == 0) ? 0 : N + 1;
                row0[gi] = make_float4(-f0.x, f0.y, f0.z, 0.f);
                row1[gi] = make_float4(-f1.x, f1.y, f1.z, 0.f);
            }
            // ghost rows: J_y odd across the y edges
            if (j0 == 0) {
                float4 *grow = out;
                grow[i + 1] = make_float4(f0.x, -f0.y, f0.z, 0.f);
                if (i == 0 || i == N - 1)
                    grow[(i == 0) ? 0 : N + 1] = make_float4(-f0.x, -f0.y, f0.z, 0.f);
            }
            if (j0 + 1 == ly - 1) {
                float4 *grow = out + (int64_t)(ly + 1) * P;
                grow[i + 1] = make_float4(f1.x, -f1.y, f1.z, 0.f);
                if (i == 0 || i == N - 1)
                    grow[(i == 0) ? 0 : N + 1] = make_float4(-f1.x, -f1.y, f1.z, 0.f);
            }
        };
        put(fields);
        if (fields2) put(fields2);
    }
    if (bad) set_status(status, FFB_E_NONPOSITIVE);
}

__global__ __launch_bounds__(512) void k_row_final(const double *__restrict__ pa,
                                                   const double *__restrict__ pb,
                                                   const double *__restrict__ pc, int lx, int ly,
                                                   const double2 *__restrict__ tw,
                                                   const double2 *__restrict__ tq,
                                                   float4 *__restrict__ fields, int32_t *status,
                                                   float4 *__restrict__ fields2)
{
    __shared__ double2 sa[kMaxN], sb[kMaxN], rs[kMaxN], jx[kMaxN], stw[kMaxN / 2];
    row_final_body<double>(pa, pb, pc, 2 * blockIdx.x, lx, ly, tw, tq, 1, fields, status, sa, sb,
                           rs, jx, stw, fields2);
}

// Pack caller node arrays into the ghosted layout (same ghost rule).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ jx,
                                              const float *__restrict__ jy,
                                              const float *__restrict__ rs, int lx, int ly,
                                              float4 *__restrict__ fields)
{
    const int P = lx + 2;
    const int64_t total = (int64_t)(lx + 2) * (ly + 2);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int pi = (int)(e % P), pj = (int)(e / P);
        int i = pi - 1, j = pj - 1;
        float sx = 1.f, sy = 1.f;
        if (i < 0) { i = 0; sx = -1.f; }
        if (i >= lx) { i = lx - 1; sx = -1.f; }
        if (j < 0) { j = 0; sy = -1.f; }
        if (j >= ly) { j = ly - 1; sy = -1.f; }
        const int64_t c = (int64_t)j * lx + i;
        fields[e] = make_float4(sx * jx[c], sy * jy[c], rs[c], 0.f);
    }
}

// Fixed-order FP64 sum of a float array: per-block partials then one block.

__global__ __launch_bounds__(256) void k_sum_final(const double *__restrict__ part, int np,
                                                   double scale, double *__restrict__ out,
                                                   int32_t *status, double *__restrict__ out2)
{
    __shared__ double lds[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = lds[0] * scale;
        *out = m;
        if (out2) *out2 = m;
        if (!(m > 0.0)) set_status(status, FFB_E_NONPOSITIVE);
    }
}

// ------------------------------------------------------------ adjoint
// The flux is linear in rho.  With S = C_y C_x rho (DCT-II sums), R = G o S
// (G: Eq. 7 factors times the blur), the forward gives
//   rho_s = C_x^T C_y^T R / (lx ly),  J_x = S_x^T C_y^T (W_x o R),
//   J_y = C_x^T S_y^T (W_y o R),      rho_bar = S_00 / (lx ly),
// so for adjoints (lr, lx_, ly_) of (rho_s, J_x, J_y) and lb of rho_bar
//   Rbar = C_y C_x lr / (lx ly) + W_x o (C_y S_x lx_) + W_y o (S_y C_x ly_),
//   Sbar = G o Rbar,  Sbar_00 += lb / (lx ly),  lam_rho = C_x^T C_y^T Sbar,
// where S_x lam = sum_i lam_i sin(pi m (i + 1/2) / lx) (a DST-II) is the
// DCT-II of (-1)^i lam_i read at index lx - m.

// DCT-II (rows a, b) of a pair of rows placed by `val(i)` in Makhoul order.
template <typename F>
__device__ void dct2_rows_pair(float2 *sa, float2 *sb, float2 *out, int N, const float2 *stw,
                               const float2 *__restrict__ tq, F val)
{
    for (int i = threadIdx.x; i < N; i += blockDim.x) sa[mk_pos(i, N)] = val(i);
    dct2_pair(sa, sb, out, N, stw, tq);
}

// Transpose of the ghost fill at node (i, j): the node's own entry of
// lam_fields plus every ghost entry that mirrors it, with the parity sign of
// its component (J_x odd across x edges, J_y odd across y edges, rho_s
// even).  Returns (J_x, J_y, rho_s) adjoints.
__device__ inline float3 fold_node(const float4 *__restrict__ lam, int lx, int ly, int i, int j)
{
    const int pitch = lx + 2;
    int ii[2] = {i, 0}, jj[2] = {j, 0};
    const float sxs[2] = {1.f, -1.f}, sys[2] = {1.f, -1.f};
    int ni = 1, nj = 1;
    if (i == 0) ii[ni++] = -1;
    else if (i == lx - 1) ii[ni++] = lx;
    if (j == 0) jj[nj++] = -1;
    else if (j == ly - 1) jj[nj++] = ly;
    float ax = 0.f, ay = 0.f, ar = 0.f;
    for (int q = 0; q < nj; ++q)
        for (int r = 0; r < ni; ++r) {
            const float4 v = lam[(int64_t)(jj[q] + 1) * pitch + (ii[r] + 1)];
            ax += sxs[r] * v.x;
            ay += sys[q] * v.y;
            ar += v.z;
        }
    return make_float3(ax, ay, ar);
}

// Row pass along x of the three node adjoints, folded from the ghosted
// layout (fold_node) as they are read (each workgroup owns rows j0, j0 + 1):
// rho_s -> DCT-II into pa, J_x -> DST-II into pb, J_y -> DCT-II into pc
// ([ly][lx] planes).
__global__ __launch_bounds__(512) void k_adj_rows(const float4 *__restrict__ lam, int lx, int ly,
                                                  const float2 *__restrict__ tw,
                                                  const float2 *__restrict__ tq,
                                                  float *__restrict__ pa, float *__restrict__ pb,
                                                  float *__restrict__ pc)
{
    __shared__ float2 sa[kMaxN], sb[kMaxN], o[kMaxN], stw[kMaxN / 2];
    __shared__ float3 fo[2][kMaxN];
    const int N = lx;
    load_twiddles(stw, tw, N);
    const int j0 = 2 * (int)blockIdx.x;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        fo[0][i] = fold_node(lam, lx, ly, i, j0);
        fo[1][i] = fold_node(lam, lx, ly, i, j0 + 1);
    }
    __syncthreads();
    float *a0 = pa + (int64_t)j0 * N, *a1 = a0 + N;
    float *b0 = pb + (int64_t)j0 * N, *b1 = b0 + N;
    float *c0 = pc + (int64_t)j0 * N, *c1 = c0 + N;
    dct2_rows_pair(sa, sb, o, N, stw, tq, [&](int i) { return make_float2(fo[0][i].z, fo[1][i].z); });
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        a0[m] = o[m].x;
        a1[m] = o[m].y;
    }
    dct2_rows_pair(sa, sb, o, N, stw, tq, [&](int i) {
        const float sg = (i & 1) ? -1.f : 1.f;
        return make_float2(sg * fo[0][i].x, sg * fo[1][i].x);
    });
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        const float2 v = m ? o[N - m] : make_float2(0.f, 0.f);
        b0[m] = v.x;
        b1[m] = v.y;
    }
    dct2_rows_pair(sa, sb, o, N, stw, tq, [&](int i) { return make_float2(fo[0][i].y, fo[1][i].y); });
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        c0[m] = o[m].x;
        c1[m] = o[m].y;
    }
}

// Column pass on columns m0, m0 + 1 of the row-pass outputs [ly][lx]
// (read and written row-major, one 8-byte access per row, as the forward's
// column pass): the transforms along y, the spectral weights, then the
// DCT-III along y into out [ly][lx].
__global__ __launch_bounds__(512) void k_adj_cols(const float *__restrict__ ta,
                                                  const float *__restrict__ tb,
                                                  const float *__restrict__ tc, int lx, int ly,
                                                  float sigma, const double *__restrict__ lam_rb,
                                                  const float2 *__restrict__ tw,
                                                  const float2 *__restrict__ tq,
                                                  float *__restrict__ out)
{
    __shared__ float2 sa[kMaxN], sb[kMaxN], A[kMaxN], B[kMaxN], stw[kMaxN / 2];
    const int N = ly;
    const int64_t cs = lx / 2;                  // row stride in pairs
    load_twiddles(stw, tw, N);
    const int m0 = 2 * col_pair(blockIdx.x, lx / 2);
    const float2 *pa_ = reinterpret_cast<const float2 *>(ta + m0);
    const float2 *pb_ = reinterpret_cast<const float2 *>(tb + m0);
    const float2 *pc_ = reinterpret_cast<const float2 *>(tc + m0);
    dct2_rows_pair(sa, sb, A, N, stw, tq, [&](int i) { return pa_[i * cs]; });
    dct2_rows_pair(sa, sb, B, N, stw, tq, [&](int i) { return pb_[i * cs]; });
    // C: DST-II along y, kept in the FFT scratch for the combination below
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float sg = (i & 1) ? -1.f : 1.f;
        const float2 c = pc_[i * cs];
        sa[mk_pos(i, N)] = make_float2(sg * c.x, sg * c.y);
    }
    float2 *Z = fft_lds(sa, sb, N, stw, false);
    float2 *C = (Z == sa) ? sb : sa;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        const float2 zm = Z[m];
        const float2 zc = Z[(N - m) & (N - 1)];
        const float2 va = make_float2(0.5f * (zm.x + zc.x), 0.5f * (zm.y - zc.y));
        const float2 vb = make_float2(0.5f * (zm.y + zc.y), -0.5f * (zm.x - zc.x));
        const float2 q = tq[m];
        C[m] = make_float2(q.x * va.x - q.y * va.y, q.x * vb.x - q.y * vb.y);
    }
    __syncthreads();
    // combine: Sbar = G o (A / (lx ly) + W_x B + W_y C), C read at index N - n
    const float PI_F = 3.14159265358979f;
    const float inv_pi = 0.318309886183790672f;
    const float flx = (float)lx, fly = (float)ly, norm = 1.0f / (flx * fly);
    const float cgx = PI_F * PI_F * sigma * sigma / (2.0f * flx * flx);
    const float cgy = PI_F * PI_F * sigma * sigma / (2.0f * fly * fly);
    const float gx0 = expf(-cgx * (float)m0 * (float)m0) * (m0 == 0 ? 2.0f : 4.0f);
    const float gx1 = expf(-cgx * (float)(m0 + 1) * (float)(m0 + 1)) * 4.0f;
    const float ma = (float)m0, mb = (float)(m0 + 1);
    const float lb = (float)(*lam_rb * (double)norm);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const float gy = expf(-cgy * (float)n * (float)n) * (n == 0 ? 0.5f : 1.0f);
        const float fn = (float)n;
        const float2 cv = n ? C[N - n] : make_float2(0.f, 0.f);
        const float da = (ma * fly) * (ma * fly) + (fn * flx) * (fn * flx);
        const float db = (mb * fly) * (mb * fly) + (fn * flx) * (fn * flx);
        const float wxa = m0 == 0 ? 0.f : fly * inv_pi * ma / da, wxb = fly * inv_pi * mb / db;
        const float wya = n == 0 ? 0.f : flx * inv_pi * fn / da;
        const float wyb = n == 0 ? 0.f : flx * inv_pi * fn / db;
        float ra = A[n].x * norm + wxa * B[n].x + wya * cv.x;
        float rb = A[n].y * norm + wxb * B[n].y + wyb * cv.y;
        ra *= gx0 * gy;
        rb *= gx1 * gy;
        if (m0 == 0 && n == 0) ra += lb;
        B[n] = make_float2(ra, rb);       // B is free now
    }
    __syncthreads();
    dct3_input(sa, N, tq, [&](int n) { return B[n]; });
    float2 *v = fft_lds(sa, sb, N, stw, true);
    float2 *o = reinterpret_cast<float2 *>(out + m0);
    for (int i = threadIdx.x; i < N; i += blockDim.x) o[i * cs] = dct3_output(v, i, N);
}

// Final row pass: DCT-III along x of the [ly][lx] plane.
// Suffix sums along a pair of rows held in LDS (u[i] = (row j0, row j0 + 1)
// at column i), in FP64: suf[j][k] = sum_{i >= k} row_j[i] for k in [0, N]
// (the last is 0), rows of N + 1; the sum of both rows is added to *total.
// Lanes own contiguous chunks in reverse order (lane 0 the last chunk), so
// an inclusive scan over the lanes gives each lane the sum to its right.
__device__ inline void row_pair_suffix(const float2 *u, int N, double *suf, double *total,
                                       double2 *part)
{
    const int T = blockDim.x, t = threadIdx.x;
    const int chunk = (N + T - 1) / T;
    const int end = max(0, N - t * chunk), beg = max(0, end - chunk);
    double sx = 0.0, sy = 0.0;
    for (int i = beg; i < end; ++i) {
        sx += u[i].x;
        sy += u[i].y;
    }
    part[t] = make_double2(sx, sy);
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {
        const double2 a = t >= o ? part[t - o] : make_double2(0.0, 0.0);
        __syncthreads();
        part[t].x += a.x;
        part[t].y += a.y;
        __syncthreads();
    }
    double rx = part[t].x - sx, ry = part[t].y - sy;
    double *q0 = suf, *q1 = suf + (N + 1);
    for (int i = end - 1; i >= beg; --i) {
        rx += u[i].x;
        ry += u[i].y;
        q0[i] = rx;
        q1[i] = ry;
    }
    if (t == 0) {
        q0[N] = 0.0;
        q1[N] = 0.0;
        unsafeAtomicAdd(total, part[T - 1].x + part[T - 1].y);
    }
}

// With `suf` (optional), also the row suffix sums of lam_rho that the
// density adjoint's boundary integrals read, and their total added to
// *total, from the values just stored.
__global__ __launch_bounds__(512) void k_adj_rows_final(const float *__restrict__ in, int lx,
                                                        const float2 *__restrict__ tw,
                                                        const float2 *__restrict__ tq,
                                                        float *__restrict__ lam_rho,
                                                        double *__restrict__ suf,
                                                        double *__restrict__ total)
{
    __shared__ float2 sa[kMaxN], sb[kMaxN], stw[kMaxN / 2];
    __shared__ double2 part[512];
    const int N = lx;
    load_twiddles(stw, tw, N);
    const int64_t j0 = 2 * (int64_t)blockIdx.x;
    const float *r0 = in + j0 * N, *r1 = r0 + N;
    dct3_input(sa, N, tq, [&](int m) { return make_float2(r0[m], r1[m]); });
    float2 *v = fft_lds(sa, sb, N, stw, true);
    float2 *u = v == sa ? sb : sa;               // free after the transform
    float *o0 = lam_rho + j0 * N, *o1 = o0 + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float2 y = dct3_output(v, i, N);
        o0[i] = y.x;
        o1[i] = y.y;
        u[i] = y;
    }
    if (!suf) return;
    __syncthreads();
    row_pair_suffix(u, N, suf + j0 * (N + 1), total, part);
}

// ------------------------------------------------------------- batched
// Transforms of many maps of different sizes (the grouped kernels below):
// every group reads its (map, index) from a launch table of its grid-size
// class, offsets its planes, and reads the length-1024 twiddle tables at
// stride 1024 / N.  Maps that stopped iterating are skipped.

// Mean density of every active map in FP64 from the row sums the raster
// scan left in the spare last slot of each accumulation row (fixed order).
__global__ __launch_bounds__(256) void kb_mean(batch_view bv, const double *__restrict__ acc,
                                               double *__restrict__ rho_bar, int32_t *status)
{
    __shared__ double lds[256];
    const int m = blockIdx.x;
    if (!bv.active[m]) return;
    const int lx = bv.lx[m], ly = bv.ly[m];
    const double *a = acc + bv.acc_off[m];
    double sum = 0.0;
    for (int j = threadIdx.x; j < ly; j += 256) sum += a[(int64_t)j * (lx + 1) + lx];
    lds[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = lds[0] / ((double)lx * (double)ly);
        rho_bar[m] = mean;
        if (!(mean > 0.0)) set_status(status, FFB_E_NONPOSITIVE);
    }
}

// ------------------------------------------------------- diffusion variant
// The diffusion choice of the SI Appendix (section 2): f_mn(t) =
// exp(-(m^2/lx^2 + n^2/ly^2) t) multiplies the blurred coefficients, and the
// flux coefficients become (m / (pi lx)) and (n / (pi ly)) times them, so
//   rho(t) = (1/(lx ly)) sum rts f cos cos,
//   J_x(t) = sum (m / (pi lx^2 ly)) rts f sin cos,
//   J_y(t) = sum (n / (pi lx ly^2)) rts f cos sin.
// The forward half (rows, transpose, columns with the Eq. 7 factor and the
// blur) runs once per round into spec; each stage time needs only the three
// inverse column transforms, a transpose and the row pass.

// Blurred coefficients of rows m0, m0 + 1 of T2 into spec [lx][ly].
__global__ __launch_bounds__(512) void kd_spectrum(const float *__restrict__ t2, int lx, int ly,
                                                   float sigma, const float2 *__restrict__ tw,
                                                   const float2 *__restrict__ tq,
                                                   float *__restrict__ spec)
{
    __shared__ float2 sa[kMaxN], sb[kMaxN], coef[kMaxN], stw[kMaxN / 2];
    const int m0 = 2 * blockIdx.x, N = ly;
    load_twiddles(stw, tw, N, 1);
    const float *ra = t2 + (int64_t)m0 * N, *rb = ra + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) sa[mk_pos(i, N)] = make_float2(ra[i], rb[i]);
    dct2_pair(sa, sb, coef, N, stw, tq, 1);
    const float PI_F = 3.14159265358979f;
    const float cgx = PI_F * PI_F * sigma * sigma / (2.0f * (float)lx * (float)lx);
    const float cgy = PI_F * PI_F * sigma * sigma / (2.0f * (float)ly * (float)ly);
    const float gx0 = expf(-cgx * (float)m0 * (float)m0) * (m0 == 0 ? 2.0f : 4.0f);
    const float gx1 = expf(-cgx * (float)(m0 + 1) * (float)(m0 + 1)) * 4.0f;
    float *o0 = spec + (int64_t)m0 * N, *o1 = o0 + N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const float gy = expf(-cgy * (float)n * (float)n) * (n == 0 ? 0.5f : 1.0f);
        const float2 c = coef[n];
        o0[n] = c.x * gx0 * gy;
        o1[n] = c.y * gx1 * gy;
    }
}

// Column pass at stage time slot blockIdx.y: rows m0, m0 + 1 of spec times
// f_mn(ts), then a (DCT-III), b (DCT-III, weight of m) and c (DST-III,
// weight of n) along y into q [3][slots][lx][ly].
__global__ __launch_bounds__(512) void kd_col(const diff_ctl *__restrict__ ctl,
                                              const float *__restrict__ spec, int lx, int ly,
                                              int slots, const float2 *__restrict__ tw,
                                              const float2 *__restrict__ tq, float *__restrict__ q)
{
    if (ctl->done) return;
    __shared__ float2 sa[kMaxN], sb[kMaxN], coef[kMaxN], stw[kMaxN / 2];
    const int m0 = 2 * blockIdx.x, z = blockIdx.y, N = ly;
    const double ts = ctl->ts[z];
    load_twiddles(stw, tw, N, 1);
    const double ix2 = 1.0 / ((double)lx * (double)lx), iy2 = 1.0 / ((double)ly * (double)ly);
    const float fx0 = expf((float)(-(double)m0 * m0 * ix2 * ts));
    const float fx1 = expf((float)(-(double)(m0 + 1) * (m0 + 1) * ix2 * ts));
    const float *s0 = spec + (int64_t)m0 * N, *s1 = s0 + N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const float fy = expf((float)(-(double)n * n * iy2 * ts));
        coef[n] = make_float2(s0[n] * fx0 * fy, s1[n] * fx1 * fy);
    }
    __syncthreads();
    const float inv_pi = 0.318309886183790672f;
    const float flx = (float)lx, fly = (float)ly;
    const float wb0 = (float)m0 * inv_pi / (flx * flx * fly);
    const float wb1 = (float)(m0 + 1) * inv_pi / (flx * flx * fly);
    const float wc = inv_pi / (flx * fly * fly);
    const int64_t plane = (int64_t)lx * ly;
    float *pa = q + (int64_t)z * plane, *pb = pa + (int64_t)slots * plane,
          *pc = pb + (int64_t)slots * plane;

    dct3_input(sa, N, tq, [&](int n) { return coef[n]; }, 1);
    float2 *v = fft_lds(sa, sb, N, stw, true);
    float *oa0 = pa + (int64_t)m0 * N, *oa1 = oa0 + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float2 y = dct3_output(v, i, N);
        oa0[i] = y.x;
        oa1[i] = y.y;
    }
    __syncthreads();
    dct3_input(sa, N, tq, [&](int n) {
        const float2 c = coef[n];
        return make_float2(wb0 * c.x, wb1 * c.y);
    }, 1);
    v = fft_lds(sa, sb, N, stw, true);
    float *ob0 = pb + (int64_t)m0 * N, *ob1 = ob0 + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float2 y = dct3_output(v, i, N);
        ob0[i] = y.x;
        ob1[i] = y.y;
    }
    __syncthreads();
    dct3_input(sa, N, tq, [&](int mm) {
        if (mm == 0) return make_float2(0.f, 0.f);
        const int n = N - mm;
        const float2 c = coef[n];
        const float w = wc * (float)n;
        return make_float2(w * c.x, w * c.y);
    }, 1);
    v = fft_lds(sa, sb, N, stw, true);
    float *oc0 = pc + (int64_t)m0 * N, *oc1 = oc0 + N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float2 y = dct3_output(v, i, N);
        const float sg = (i & 1) ? -1.0f : 1.0f;
        oc0[i] = sg * y.x;
        oc1[i] = sg * y.y;
    }
}

// Planes [R][C] -> [C][R]; plane blockIdx.z of `in`/`out`, `stride` apart.
__global__ __launch_bounds__(256) void kd_transpose(const diff_ctl *__restrict__ ctl,
                                                    const float *__restrict__ in,
                                                    float *__restrict__ out, int R, int C,
                                                    int slots, int64_t plane)
{
    if (ctl->done) return;
    __shared__ float tile[32][33];
    // plane index: kind * kDiffSlots + slot, for the first `slots` slots
    const int kind = blockIdx.z / slots, z = blockIdx.z % slots;
    const int64_t off = ((int64_t)kind * slots + z) * plane;
    transpose_tile(in + off, out + off, R, C, blockIdx.x * 32, blockIdx.y * 32, tile);
}

// Row pass at slot blockIdx.y: fields (J_x, J_y, rho(ts)) of that slot.
__global__ __launch_bounds__(512) void kd_row(const diff_ctl *__restrict__ ctl,
                                              const float *__restrict__ r, int lx, int ly,
                                              int slots, const float2 *__restrict__ tw,
                                              const float2 *__restrict__ tq,
                                              float4 *__restrict__ fields, int32_t *status)
{
    if (ctl->done) return;
    __shared__ float2 sa[kMaxN], sb[kMaxN], rs[kMaxN], jx[kMaxN], stw[kMaxN / 2];
    const int z = blockIdx.y;
    const int64_t plane = (int64_t)lx * ly;
    const float *pa = r + (int64_t)z * plane, *pb = pa + (int64_t)slots * plane,
                *pc = pb + (int64_t)slots * plane;
    row_final_body(pa, pb, pc, 2 * blockIdx.x, lx, ly, tw, tq, 1,
                   fields + (int64_t)z * (lx + 2) * (ly + 2), status, sa, sb, rs, jx, stw);
}

// The FP64 transform tables on the device (same definitions as the host
// tables of a context): tw[k] = exp(-2 pi i k / N), k < N/2, and
// tq[m] = exp(-i pi m / (2N)), m < N.
__global__ __launch_bounds__(256) void k_twiddles(int N, double2 *__restrict__ tw,
                                                  double2 *__restrict__ tq)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= N) return;
    double sn, cs;
    if (k < N / 2) {
        sincospi(2.0 * k / N, &sn, &cs);
        tw[k] = make_double2(cs, -sn);
    }
    sincospi(k / (2.0 * N), &sn, &cs);
    tq[k] = make_double2(cs, -sn);
}

inline int threads_for(int N)
{
    int t = N / 2;
    if (t < 64) t = 64;
    if (t > 512) t = 512;
    return t;
}

// ------------------------------------------------- grouped FP64 transforms
// The FP64 passes of the batched flux run many row or column pairs per
// workgroup: a group of G = N / 8 lanes owns one pair, holds eight
// complex values per lane in registers and runs the length-N FFT as radix-8
// Stockham passes (one radix-2 or radix-4 pass first when log2 N is not a
// multiple of 3), exchanging through its own LDS buffer in place.  A group
// of at most one wavefront needs no workgroup barrier (its lanes run in
// lockstep and the LDS serves a wavefront's accesses in order); at N = 1024
// a group spans two wavefronts and passes workgroup barriers.  The pre- and
// post-processing of the DCTs keeps each lane's bins in registers (a lane
// owns the index pairs (s, N - s)), so the only per-group LDS is the FFT
// buffer, with one spare slot per 16 elements so that the strided writes of
// the early passes spread over the banks.  (A single grid has too few pairs
// to fill the chip this way; the single-map flux keeps one pair per
// workgroup.)
// Workgroups of T lanes (64 to 512, at least G) hold P = T / G groups;
// their buffers take P * padded(N) = 8 T + T / 2 complex values.
template <int T> constexpr int grp_lds() { return 8 * T + T / 2; }

__device__ __forceinline__ int px(int i) { return i + (i >> 4); }
__device__ __forceinline__ int padded(int n) { return n + (n >> 4); }

struct Grp {
    int N, lgN, G, P, id, lane;
};

template <int T>
__device__ __forceinline__ Grp grp_of(int N)
{
    Grp g;
    g.N = N;
    g.lgN = ilog2(N);
    g.G = N >> 3;
    g.P = T / g.G;
    g.id = threadIdx.x >> (g.lgN - 3);
    g.lane = threadIdx.x & (g.G - 1);
    return g;
}

// Orders the LDS accesses of the group's lanes (uniform over the workgroup).
__device__ __forceinline__ void gsync(const Grp &g)
{
    if (g.G > 64) {
        __syncthreads();
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiplication by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 crot(double2 a)
{
    return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// Length-4 DFT in place (exponent sign by INV).
template <bool INV>
__device__ __forceinline__ void dft4(double2 &c0, double2 &c1, double2 &c2, double2 &c3)
{
    const double2 d0 = cadd(c0, c2), d1 = csub(c0, c2), d2 = cadd(c1, c3);
    const double2 d3 = crot<INV>(csub(c1, c3));
    c0 = cadd(d0, d2);
    c1 = cadd(d1, d3);
    c2 = csub(d0, d2);
    c3 = csub(d1, d3);
}

// Length-8 DFT in place: radix 2 over (m, m + 4), the twiddles w8^m, then two
// length-4 DFTs giving the even and the odd outputs.
template <bool INV>
__device__ __forceinline__ void dft8(double2 (&x)[8])
{
    const double r = 0.70710678118654752440084436210485;
    double2 a[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        a[m] = cadd(x[m], x[m + 4]);
        b[m] = csub(x[m], x[m + 4]);
    }
    // w8 = (1 - i)/sqrt 2 forward, (1 + i)/sqrt 2 inverse
    if (INV) {
        b[1] = make_double2(r * (b[1].x - b[1].y), r * (b[1].x + b[1].y));
        b[3] = make_double2(-r * (b[3].x + b[3].y), r * (b[3].x - b[3].y));
    } else {
        b[1] = make_double2(r * (b[1].x + b[1].y), r * (b[1].y - b[1].x));
        b[3] = make_double2(r * (b[3].y - b[3].x), -r * (b[3].x + b[3].y));
    }
    b[2] = crot<INV>(b[2]);
    dft4<INV>(a[0], a[1], a[2], a[3]);
    dft4<INV>(b[0], b[1], b[2], b[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        x[2 * t] = a[t];
        x[2 * t + 1] = b[t];
    }
}

// Unnormalised length-N FFT of the group's buffer a (padded, natural order
// in and out), exponent sign by INV.  tw (LDS) = exp(-2 pi i k / N), k < N/2.
template <bool INV>
__device__ void fft_grp(double2 *a, const double2 *tw, const Grp &g)
{
    const int N = g.N, G = g.G, lane = g.lane;
    const int r = g.lgN % 3;
    int lgL = 0;
    if (r == 1) {
        // radix 2, sub-length 1: N/2 butterflies, four per lane
        double2 x[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int bi = lane + u * G;
            x[2 * u] = a[px(bi)];
            x[2 * u + 1] = a[px(bi + (N >> 1))];
        }
        gsync(g);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int bi = lane + u * G;
            a[px(2 * bi)] = cadd(x[2 * u], x[2 * u + 1]);
            a[px(2 * bi + 1)] = csub(x[2 * u], x[2 * u + 1]);
        }
        gsync(g);
        lgL = 1;
    } else if (r == 2) {
        // radix 4, sub-length 1: N/4 butterflies, two per lane
        double2 x[8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int bi = lane + u * G;
#pragma unroll
            for (int m = 0; m < 4; ++m) x[4 * u + m] = a[px(bi + m * (N >> 2))];
        }
        gsync(g);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int bi = lane + u * G;
            dft4<INV>(x[4 * u], x[4 * u + 1], x[4 * u + 2], x[4 * u + 3]);
#pragma unroll
            for (int t = 0; t < 4; ++t) a[px(4 * bi + t)] = x[4 * u + t];
        }
        gsync(g);
        lgL = 2;
    }
    for (; lgL < g.lgN; lgL += 3) {
        // radix 8 with sub-length Ls: butterfly bi = lane combines the
        // eight sequences stored N/8 = G apart
        const int Ls = 1 << lgL;
        const int j = lane & (Ls - 1), k = lane >> lgL;
        double2 x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = a[px(lane + m * G)];
        if (lgL > 0) {
            // w^(m j), w = exp(-+2 pi i / (8 Ls)): w^j = tw[e1], e1 = j N / (8 Ls)
            const int e1 = j << (g.lgN - 3 - lgL);
            double2 w1 = tw[e1], w2 = tw[2 * e1], w4 = tw[4 * e1];
            if (INV) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w4.y = -w4.y;
            }
            const double2 w3 = cmul(w1, w2);
            x[1] = cmul(x[1], w1);
            x[2] = cmul(x[2], w2);
            x[3] = cmul(x[3], w3);
            x[4] = cmul(x[4], w4);
            x[5] = cmul(x[5], cmul(w4, w1));
            x[6] = cmul(x[6], cmul(w4, w2));
            x[7] = cmul(x[7], cmul(w4, w3));
        }
        dft8<INV>(x);
        gsync(g);
        const int o = (k << (lgL + 3)) + j;
#pragma unroll
        for (int t = 0; t < 8; ++t) a[px(o + t * Ls)] = x[t];
        gsync(g);
    }
}

__device__ __forceinline__ void load_tw_grp(double2 *stw, const double2 *__restrict__ tw, int N,
                                            int qs)
{
    for (int k = threadIdx.x; k < (N >> 1); k += blockDim.x) stw[k] = tw[k * qs];
    __syncthreads();
}

// Start of a batched grouped pass (length-1024 tables at stride 1024 / N):
// false if this lane's group has nothing to do and may leave -- a workgroup
// without live groups leaves before its barriers, a dead group of at most
// one wavefront after them (it passes no workgroup barrier later); a dead
// group of a 128-lane pair stays, gated, for the barriers.
__device__ __forceinline__ bool grp_enter(double2 *stw, const double2 *__restrict__ tw, int N,
                                          const Grp &g, bool live)
{
    if (!__syncthreads_or(live)) return false;
    load_tw_grp(stw, tw, N, kMaxN / N);
    return live || g.G > 64;
}

// DCT-II bin n of the pair from the FFT Z (padded) of its Makhoul-ordered
// input: (X_a[n], X_b[n]).
__device__ __forceinline__ double2 grp_dct2_bin(const double2 *Z, int n, int N, double2 q)
{
    const double2 zm = Z[px(n)], zc = Z[px((N - n) & (N - 1))];
    const double2 va = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y - zc.y));
    const double2 vb = make_double2(0.5 * (zm.y + zc.y), -0.5 * (zm.x - zc.x));
    return make_double2(q.x * va.x - q.y * va.y, q.x * vb.x - q.y * vb.y);
}

// Inverse-FFT input of a DCT-III pair at index m from the coefficient pairs
// xm = c[m] and xr = c[N - m] (xr unused for m = 0).
__device__ __forceinline__ double2 grp_dct3_in(int m, double2 xm, double2 xr, double2 q)
{
    if (m) {
        xm.x *= 0.5;
        xm.y *= 0.5;
        xr.x *= 0.5;
        xr.y *= 0.5;
    } else {
        xr = make_double2(0.0, 0.0);
    }
    const double cr = q.x, ci = -q.y;         // exp(+i pi m / (2N))
    const double war = cr * xm.x + ci * xr.x, wai = ci * xm.x - cr * xr.x;
    const double wbr = cr * xm.y + ci * xr.y, wbi = ci * xm.y - cr * xr.y;
    return make_double2(war - wbi, wai + wbr);
}

// 1 / d to full FP64 precision (hardware reciprocal, two Newton steps).
__device__ __forceinline__ double rcp64(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// Densities and row DCT of a row pair in one pass (batched maps): rho[j][i]
// = rho_pad + the inclusive prefix sum of the coverage deltas acc[j][0..i]
// (rows of N + 1; the spare slot receives the row's sum of rho, for the
// mean), in FP64, then the DCT-II of the two density rows into `out`.
// Lane l of the group holds elements 8 l .. 8 l + 7: a prefix within the
// lane, an exclusive scan of the lane totals over the group (butterflies
// within a wavefront, the lower wavefront's total through LDS for a
// 128-lane group), fixed order throughout.
__device__ void grp_scan_dct2_rows(double *__restrict__ acc, double pad, double *__restrict__ out,
                                   int64_t r0, const double2 *__restrict__ tq, int qs, double2 *a,
                                   const double2 *stw, double *part, const Grp &g, bool live)
{
    const int N = g.N, lane = g.lane;
    double *acc0 = acc + r0 * (N + 1), *acc1 = acc0 + (N + 1);
    double v0[8], v1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = 8 * lane + u;
        v0[u] = live ? acc0[i] : 0.0;
        v1[u] = live ? acc1[i] : 0.0;
    }
#pragma unroll
    for (int u = 1; u < 8; ++u) {
        v0[u] += v0[u - 1];
        v1[u] += v1[u - 1];
    }
    // inclusive scan of the lane totals over the group's lanes
    const int W = g.G < 64 ? g.G : 64;            // lanes of the group in this wavefront
    const int wl = threadIdx.x & (W - 1);
    double s0 = v0[7], s1 = v1[7];
    for (int o = 1; o < W; o <<= 1) {
        const double y0 = __shfl_up(s0, o, W), y1 = __shfl_up(s1, o, W);
        if (wl >= o) {
            s0 += y0;
            s1 += y1;
        }
    }
    double e0 = s0 - v0[7], e1 = s1 - v1[7];      // exclusive
    if (g.G > 64) {
        // the upper wavefront of the group adds the lower one's total
        if ((threadIdx.x & 63) == 63) {
            part[2 * (threadIdx.x >> 6)] = s0;
            part[2 * (threadIdx.x >> 6) + 1] = s1;
        }
        __syncthreads();
        if (lane >= 64) {
            const int w = (threadIdx.x >> 6) - 1;
            e0 += part[2 * w];
            e1 += part[2 * w + 1];
        }
    }
    double t0 = 0.0, t1 = 0.0;                    // row sums of rho
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = 8 * lane + u;
        const double r0v = pad + (e0 + v0[u]), r1v = pad + (e1 + v1[u]);
        t0 += r0v;
        t1 += r1v;
        a[px(mk_pos(i, N))] = make_double2(r0v, r1v);
    }
    for (int o = 1; o < W; o <<= 1) {
        t0 += __shfl_xor(t0, o, 64);
        t1 += __shfl_xor(t1, o, 64);
    }
    if (g.G > 64) {
        __syncthreads();                           // the exclusive totals are read
        if ((threadIdx.x & 63) == 0) {
            part[2 * (threadIdx.x >> 6)] = t0;
            part[2 * (threadIdx.x >> 6) + 1] = t1;
        }
        __syncthreads();
        const int w0 = 2 * g.id;
        t0 = part[2 * w0] + part[2 * (w0 + 1)];
        t1 = part[2 * w0 + 1] + part[2 * (w0 + 1) + 1];
    }
    if (live && lane == 0) {
        acc0[N] = t0;
        acc1[N] = t1;
    }
    gsync(g);
    fft_grp<false>(a, stw, g);
    double *oa = out + r0 * N, *ob = oa + N;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int n = lane + u * g.G;
        const double2 b = grp_dct2_bin(a, n, N, tq[n * qs]);
        if (live) {
            oa[n] = b.x;
            ob[n] = b.y;
        }
    }
}

// Column pass of a workgroup's P column pairs (entries P b .. P b + P - 1 of
// the class table, N = ly): the DCT-II along y, the normalisation and blur
// of Eq. 7, then the three DCT-III / DST-III sums of the flux series into
// a, b, c.  The pairs are read and written in the row-major planes by the
// whole workgroup at once: lane t takes pair t mod P of every (T / P)-th
// row, so consecutive pairs of one map share each access (64 bytes per row
// at N = 512, a full 128-byte line at N = 256).
struct ColEntry {
    const double2 *src;
    double2 *oa, *ob, *oc;
    int64_t cs;
    bool live;
};

__device__ __forceinline__ void col_load(const ColEntry &e, double2 *buf, int N, int lgP)
{
    const int P = 1 << lgP;
    for (int i = threadIdx.x >> lgP; i < N; i += blockDim.x / P)
        buf[px(mk_pos(i, N))] = e.live ? e.src[i * e.cs] : make_double2(0.0, 0.0);
}

template <int WHICH>
__device__ __forceinline__ void col_store(const ColEntry &e, const double2 *buf, int N, int lgP)
{
    const int P = 1 << lgP;
    if (!e.live) return;
    double2 *o = WHICH == 0 ? e.oa : (WHICH == 1 ? e.ob : e.oc);
    for (int i = threadIdx.x >> lgP; i < N; i += blockDim.x / P) {
        double2 y = buf[px(mk_pos(i, N))];
        if (WHICH == 2 && (i & 1)) y = make_double2(-y.x, -y.y);   // DST-III sign
        o[i * e.cs] = y;
    }
}

__device__ void grp_col_pass(int m0, int lx, float sigma, const double2 *__restrict__ tq, int qs,
                             double2 *a, const double2 *stw, const Grp &g, const ColEntry &mine,
                             double2 *mine_buf, int lgP)
{
    const int N = g.N, G = g.G, lane = g.lane;
    col_load(mine, mine_buf, N, lgP);
    __syncthreads();
    fft_grp<false>(a, stw, g);

    // Lane l owns the index pairs (n1, n2) = (s, N - s) of the slots
    // s = l + u G, u < 4 (slot 0: the self-paired 0 and N/2): the DCT-II
    // bins of both come from the same two FFT values, and the DCT-III inputs
    // of both from the same two coefficients, so the coefficients stay in
    // the lane's registers and no lane reads another's.
    const double PI = 3.14159265358979323846;
    const double sg = (double)sigma, flx = (double)lx, fly = (double)N;
    const double cgx = PI * PI * sg * sg / (2.0 * flx * flx);
    const double cgy = PI * PI * sg * sg / (2.0 * fly * fly);
    const double gx0 = exp(-cgx * (double)m0 * (double)m0) * (m0 == 0 ? 2.0 : 4.0);
    const double gx1 = exp(-cgx * (double)(m0 + 1) * (double)(m0 + 1)) * 4.0;
    // Gaussians exp(-cgy n^2) of n1 = l + u G (u up) and of N - l - u G
    // (u down, so that both recurrences multiply by factors <= 1)
    const double kap = exp(-2.0 * cgy * (double)G * (double)G);
    double f1 = exp(-cgy * (double)lane * (double)lane);
    double r1 = exp(-cgy * ((double)(2 * lane * G) + (double)G * (double)G));
    const double nb = (double)(N - lane - 3 * G);
    double f2 = exp(-cgy * nb * nb);
    double r2 = exp(-cgy * (2.0 * nb * (double)G + (double)G * (double)G));
    double g1[4], g2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        g1[u] = f1;
        f1 *= r1;
        r1 *= kap;
    }
#pragma unroll
    for (int u = 3; u >= 0; --u) {
        g2[u] = f2;
        f2 *= r2;
        r2 *= kap;
    }
    if (lane == 0) g2[0] = exp(-cgy * 0.25 * fly * fly);        // n2 = N/2
    auto bin = [&](double2 zm, double2 zc, int n) {
        const double2 q = tq[n * qs];
        const double2 va = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y - zc.y));
        const double2 vb = make_double2(0.5 * (zm.y + zc.y), -0.5 * (zm.x - zc.x));
        return make_double2(q.x * va.x - q.y * va.y, q.x * vb.x - q.y * vb.y);
    };
    double2 c1[4], c2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int sl = lane + u * G, n1 = sl, n2 = sl ? N - sl : N >> 1;
        const double2 A = a[px(n1)], B = a[px(n2)];
        const double2 b1 = bin(A, sl ? B : A, n1), b2 = bin(B, sl ? A : B, n2);
        const double y1 = n1 == 0 ? 0.5 * g1[u] : g1[u];
        c1[u] = make_double2(b1.x * gx0 * y1, b1.y * gx1 * y1);
        c2[u] = make_double2(b2.x * gx0 * g2[u], b2.y * gx1 * g2[u]);
    }
    // DCT-III inputs of both indices of every slot; K1, K2 map a slot's two
    // coefficients to the inputs' (xm, xr) pairs
    auto put_inputs = [&](auto K1, auto K2) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = lane + u * G, n1 = sl, n2 = sl ? N - sl : N >> 1;
            double2 xm1, xr1, xm2, xr2;
            K1(u, sl, xm1, xr1);
            K2(u, sl, xm2, xr2);
            a[px(n1)] = grp_dct3_in(n1, xm1, xr1, tq[n1 * qs]);
            a[px(n2)] = grp_dct3_in(n2, xm2, xr2, tq[n2 * qs]);
        }
        gsync(g);
    };

    // a: DCT-III of the coefficients
    put_inputs([&](int u, int sl, double2 &xm, double2 &xr) { xm = c1[u]; xr = sl ? c2[u] : c1[u]; },
               [&](int u, int sl, double2 &xm, double2 &xr) { xm = c2[u]; xr = sl ? c1[u] : c2[u]; });
    fft_grp<true>(a, stw, g);
    __syncthreads();
    col_store<0>(mine, mine_buf, N, lgP);
    __syncthreads();

    // b and c weigh the coefficients with
    //   wx(m, n) = (ly/pi) m / (m^2 ly^2 + n^2 lx^2),  wy(m, n) = (lx/pi) n / (...),
    // zero where the numerator vanishes; the coefficients are divided by the
    // common denominator once
    const double ma = (double)m0, mb = (double)(m0 + 1);
    const double inv_pi = 0.318309886183790671537767526745;
    const double ay = (ma * fly) * (ma * fly), by = (mb * fly) * (mb * fly);
    auto divide = [&](double2 c, int n) {
        const double dn = ((double)n * flx) * ((double)n * flx);
        // the (0, 0) term has no flux: both numerators vanish there
        return make_double2(ay + dn > 0.0 ? c.x * rcp64(ay + dn) : 0.0, c.y * rcp64(by + dn));
    };
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int sl = lane + u * G, n1 = sl, n2 = sl ? N - sl : N >> 1;
        c1[u] = divide(c1[u], n1);
        c2[u] = divide(c2[u], n2);
    }
    const double kxa = fly * inv_pi * ma, kxb = fly * inv_pi * mb;
    auto wxc = [&](double2 c) { return make_double2(kxa * c.x, kxb * c.y); };
    put_inputs(
        [&](int u, int sl, double2 &xm, double2 &xr) { xm = wxc(c1[u]); xr = wxc(sl ? c2[u] : c1[u]); },
        [&](int u, int sl, double2 &xm, double2 &xr) { xm = wxc(c2[u]); xr = wxc(sl ? c1[u] : c2[u]); });
    fft_grp<true>(a, stw, g);
    __syncthreads();
    col_store<1>(mine, mine_buf, N, lgP);
    __syncthreads();
    // c: DST-III of wy * coefficients = (-1)^j DCT-III of the reversed
    // sequence c'[m] = wy(N - m) c[N - m] (c'[0] = 0)
    const double ky = flx * inv_pi;
    auto wyc = [&](double2 c, int n) {
        const double k = ky * (double)n;
        return make_double2(k * c.x, k * c.y);
    };
    put_inputs(
        [&](int u, int sl, double2 &xm, double2 &xr) {
            // index n1 = s: c'[s] = wy(N - s) c[N - s], c'[N - s] = wy(s) c[s]
            xm = sl ? wyc(c2[u], N - sl) : make_double2(0.0, 0.0);
            xr = wyc(c1[u], sl);
        },
        [&](int u, int sl, double2 &xm, double2 &xr) {
            // index n2 = N - s: c'[N - s] = wy(s) c[s]; slot 0: n2 = N/2
            xm = sl ? wyc(c1[u], sl) : wyc(c2[u], N >> 1);
            xr = sl ? wyc(c2[u], N - sl) : wyc(c2[u], N >> 1);
        });
    fft_grp<true>(a, stw, g);
    __syncthreads();
    col_store<2>(mine, mine_buf, N, lgP);
}

// Row pass on rows j0, j0 + 1 of a, b, c [ly][lx] (N = lx): rho_s, J_x, J_y
// of the two rows, written as the ghosted FP32 float4 fields to `fields`
// and, if not null, `fields2`; rho_s and J_x wait in registers, each value
// rounded once to FP32.
__device__ void grp_row_final(const double *__restrict__ pa, const double *__restrict__ pb,
                              const double *__restrict__ pc, int j0, int ly,
                              const double2 *__restrict__ tq, int qs,
                              float4 *__restrict__ fields, float4 *__restrict__ fields2,
                              int32_t *status, double2 *a, const double2 *stw, const Grp &g,
                              bool live)
{
    const int N = g.N, G = g.G, lane = g.lane;
    const double norm = 1.0 / ((double)N * (double)ly);
    // each plane's row pair is staged in the buffer (one coalesced read per
    // element), then every lane takes its elements m and N - m from there
    auto stage = [&](const double *__restrict__ plane) {
        const double *r0 = plane + (int64_t)j0 * N, *r1 = r0 + N;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int m = lane + u * G;
            a[px(m)] = live ? make_double2(r0[m], r1[m]) : make_double2(0.0, 0.0);
        }
        gsync(g);
    };
    // DCT-III input from the staged pairs, in place: lane l takes the index
    // pairs (s, N - s) for the slots s = l + u G, u < 4 (slot 0: the
    // self-paired indices 0 and N/2), so it reads and writes only its own
    // elements.  REV: of the index-reversed sequence c'[m] = c[N - m]
    // (c'[0] = 0), for the DST-III.
    auto dct3_from_stage = [&](bool rev) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int sl = lane + u * G;
            const int m1 = sl, m2 = sl ? N - sl : N >> 1;
            const double2 A = a[px(m1)], B = a[px(m2)];
            const double2 h1 = sl ? B : A, h2 = sl ? A : B;      // partners' values
            a[px(m1)] = rev ? grp_dct3_in(m1, m1 ? h1 : make_double2(0.0, 0.0), A, tq[m1 * qs])
                            : grp_dct3_in(m1, A, h1, tq[m1 * qs]);
            a[px(m2)] = rev ? grp_dct3_in(m2, h2, B, tq[m2 * qs])
                            : grp_dct3_in(m2, B, h2, tq[m2 * qs]);
        }
        gsync(g);
    };
    float2 rs[8], jx[8];
    // rho_s: DCT-III of a
    stage(pa);
    dct3_from_stage(false);
    fft_grp<true>(a, stw, g);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double2 y = a[px(mk_pos(lane + u * G, N))];
        rs[u] = make_float2((float)(y.x * norm), (float)(y.y * norm));
    }
    gsync(g);
    // J_x: DST-III of b = (-1)^i DCT-III of b reversed
    stage(pb);
    dct3_from_stage(true);
    fft_grp<true>(a, stw, g);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = lane + u * G;
        const double2 y = a[px(mk_pos(i, N))];
        const double s = (i & 1) ? -1.0 : 1.0;
        jx[u] = make_float2((float)(s * y.x), (float)(s * y.y));
    }
    gsync(g);
    // J_y: DCT-III of c
    stage(pc);
    dct3_from_stage(false);
    fft_grp<true>(a, stw, g);
    const int P = N + 2;
    int bad = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = lane + u * G;
        const double2 y = a[px(mk_pos(i, N))];
        const float4 f0 = make_float4(jx[u].x, (float)y.x, rs[u].x, 0.f);
        const float4 f1 = make_float4(jx[u].y, (float)y.y, rs[u].y, 0.f);
        if (!live) continue;
        bad |= !(f0.z > 0.f) || !(f1.z > 0.f);
        auto put = [&](float4 *__restrict__ out) {
            float4 *row0 = out + (int64_t)(j0 + 1) * P;
            float4 *row1 = row0 + P;
            row0[i + 1] = f0;
            row1[i + 1] = f1;
            // ghost columns: J_x odd across the x edges
            if (i == 0 || i == N - 1) {
                const int gi = (i == 0) ? 0 : N + 1;
                row0[gi] = make_float4(-f0.x, f0.y, f0.z, 0.f);
                row1[gi] = make_float4(-f1.x, f1.y, f1.z, 0.f);
            }
            // ghost rows: J_y odd across the y edges
            if (j0 == 0) {
                out[i + 1] = make_float4(f0.x, -f0.y, f0.z, 0.f);
                if (i == 0 || i == N - 1)
                    out[(i == 0) ? 0 : N + 1] = make_float4(-f0.x, -f0.y, f0.z, 0.f);
            }
            if (j0 + 1 == ly - 1) {
                float4 *grow = out + (int64_t)(ly + 1) * P;
                grow[i + 1] = make_float4(f1.x, -f1.y, f1.z, 0.f);
                if (i == 0 || i == N - 1)
                    grow[(i == 0) ? 0 : N + 1] = make_float4(-f1.x, -f1.y, f1.z, 0.f);
            }
        };
        put(fields);
        if (fields2) put(fields2);
    }
    if (bad) set_status(status, FFB_E_NONPOSITIVE);
}

// Batched kernels: P table entries (map, first row or column of the pair)
// per workgroup, all of one grid-size class (length N).
template <int T>
__global__ __launch_bounds__(T) void kb_scan_dct2_g(batch_view bv, const int2 *__restrict__ rows,
                                                    int n, int N, double *__restrict__ acc,
                                                    const double *__restrict__ rho_pad,
                                                    double *__restrict__ out,
                                                    const double2 *__restrict__ tw,
                                                    const double2 *__restrict__ tq)
{
    __shared__ double2 buf[grp_lds<T>()], stw[kMaxN / 2];
    __shared__ double part[2 * (T / 64)];
    const Grp g = grp_of<T>(N);
    const int q = blockIdx.x * g.P + g.id;
    const int2 e = q < n ? rows[q] : make_int2(0, 0);
    const int m = e.x;
    const bool live = q < n && bv.active[m];
    if (!grp_enter(stw, tw, N, g, live)) return;
    grp_scan_dct2_rows(acc + bv.acc_off[m], rho_pad[m], out + bv.plane_off[m], live ? e.y : 0, tq,
                       kMaxN / N, buf + g.id * padded(N), stw, part, g, live);
}

template <int T>
__global__ __launch_bounds__(T) void kb_col_pass_g(batch_view bv,
                                                             const int2 *__restrict__ cols, int n,
                                                             int N, const double *__restrict__ t1,
                                                             const double2 *__restrict__ tw,
                                                             const double2 *__restrict__ tq,
                                                             double *__restrict__ pa,
                                                             double *__restrict__ pb,
                                                             double *__restrict__ pc)
{
    __shared__ double2 buf[grp_lds<T>()], stw[kMaxN / 2];
    const Grp g = grp_of<T>(N);
    const int lgP = ilog2(g.P);
    auto entry = [&](int p, int &m0, int &lx, float &sigma) {
        const int q = blockIdx.x * g.P + p;
        const int2 e = q < n ? cols[q] : make_int2(0, 0);
        const int m = e.x;
        ColEntry c;
        c.live = q < n && bv.active[m] && bv.ly[m] == N;
        const int64_t o = bv.plane_off[m];
        m0 = c.live ? e.y : 0;
        lx = bv.lx[m];
        sigma = (float)ldexp(bv.sigma0, -bv.round[m]);
        c.cs = lx / 2;
        c.src = reinterpret_cast<const double2 *>(t1 + o + m0);
        c.oa = reinterpret_cast<double2 *>(pa + o + m0);
        c.ob = reinterpret_cast<double2 *>(pb + o + m0);
        c.oc = reinterpret_cast<double2 *>(pc + o + m0);
        return c;
    };
    // this lane's group (transforms) and its pair of the block-wide accesses
    int m0, lx, m0c, lxc;
    float sigma, sgc;
    const ColEntry own = entry(g.id, m0, lx, sigma);
    const int pc_ = threadIdx.x & (g.P - 1);
    const ColEntry acc = entry(pc_, m0c, lxc, sgc);
    // leave only if no pair of the workgroup is live (barriers follow)
    if (!__syncthreads_or(own.live)) return;
    load_tw_grp(stw, tw, N, kMaxN / N);
    grp_col_pass(m0, lx, sigma, tq, kMaxN / N, buf + g.id * padded(N), stw, g, acc,
                 buf + pc_ * padded(N), lgP);
}

template <int T>
__global__ __launch_bounds__(T) void kb_row_final_g(
    batch_view bv, const int2 *__restrict__ rows, int n, int N, const double *__restrict__ pa,
    const double *__restrict__ pb, const double *__restrict__ pc, const double2 *__restrict__ tw,
    const double2 *__restrict__ tq, float4 *__restrict__ fields, int32_t *status)
{
    __shared__ double2 buf[grp_lds<T>()], stw[kMaxN / 2];
    const Grp g = grp_of<T>(N);
    const int q = blockIdx.x * g.P + g.id;
    const int2 e = q < n ? rows[q] : make_int2(0, 0);
    const int m = e.x;
    const bool live = q < n && bv.active[m];
    if (!grp_enter(stw, tw, N, g, live)) return;
    const int64_t o = bv.plane_off[m];
    grp_row_final(pa + o, pb + o, pc + o, live ? e.y : 0, bv.ly[m], tq, kMaxN / N,
                  fields + bv.field_off[m], nullptr, status, buf + g.id * padded(N), stw, g, live);
}

// Workgroups of T lanes for a grouped pass over n pairs of length N.
inline int grp_blocks(int n_pairs, int N, int T)
{
    const int P = T / (N / 8);
    return (n_pairs + P - 1) / P;
}

// Launches K<T> for a class with the requested workgroup size t (at least
// one group of N / 8 lanes).
template <template <int> class K, typename... A>
hipError_t launch_grp_class(int t, int n, int N, hipStream_t s, A... args)
{
    t = std::max(t, N / 8);
    switch (t) {
    case 64:
        return K<64>::go(dim3(grp_blocks(n, N, 64)), s, args...);
    case 128:
        return K<128>::go(dim3(grp_blocks(n, N, 128)), s, args...);
    case 256:
        return K<256>::go(dim3(grp_blocks(n, N, 256)), s, args...);
    case 512:
        return K<512>::go(dim3(grp_blocks(n, N, 512)), s, args...);
    default:
        return hipErrorInvalidValue;
    }
}
template <int T> struct RowsK {
    template <typename... A> static hipError_t go(dim3 grid, hipStream_t s, A... a)
    {
        hipLaunchKernelGGL(kb_scan_dct2_g<T>, grid, dim3(T), 0, s, a...);
        return hipGetLastError();
    }
};
template <int T> struct ColsK {
    template <typename... A> static hipError_t go(dim3 grid, hipStream_t s, A... a)
    {
        hipLaunchKernelGGL(kb_col_pass_g<T>, grid, dim3(T), 0, s, a...);
        return hipGetLastError();
    }
};
template <int T> struct FinalK {
    template <typename... A> static hipError_t go(dim3 grid, hipStream_t s, A... a)
    {
        hipLaunchKernelGGL(kb_row_final_g<T>, grid, dim3(T), 0, s, a...);
        return hipGetLastError();
    }
};

}  // namespace

hipError_t launch_flux_ws(hipStream_t s, int lx, int ly, const flux_ws &w, const double *rho,
                          float sigma, float4 *fields, double *rho_bar, int32_t *status,
                          const flux_snap *snap)
{
    const int64_t n = (int64_t)lx * ly;
    // row DCTs, with the FP64 sums of each row pair for the mean density
    hipLaunchKernelGGL(k_dct2_rows, dim3(ly / 2), dim3(threads_for(lx)), 0, s, rho, w.t1, lx,
                       w.tw_x, w.tq_x, w.red);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, w.red, ly / 2, 1.0 / (double)n,
                       rho_bar, status, snap ? snap->rho_bar : nullptr);
    hipLaunchKernelGGL(k_col_pass, dim3(lx / 2), dim3(threads_for(ly)), 0, s, w.t1, lx, ly,
                       sigma, w.tw_y, w.tq_y, w.pa, w.pb, w.pc);
    hipLaunchKernelGGL(k_row_final, dim3(ly / 2), dim3(threads_for(lx)), 0, s, w.pa, w.pb, w.pc,
                       lx, ly, w.tw_x, w.tq_x, fields, status, snap ? snap->fields : nullptr);
    return hipGetLastError();
}

hipError_t launch_flux(ffb_ctx *ctx, const double *rho, float sigma, float4 *fields,
                       double *rho_bar, const flux_snap *snap)
{
    // the context's planes are sized for FP64
    flux_ws w{ctx->tw64_x,
              ctx->tq64_x,
              ctx->tw64_y,
              ctx->tq64_y,
              reinterpret_cast<double *>(ctx->t1),
              reinterpret_cast<double *>(ctx->pa),
              reinterpret_cast<double *>(ctx->pb),
              reinterpret_cast<double *>(ctx->pc),
              ctx->red};
    return launch_flux_ws(ctx->stream, ctx->lx, ctx->ly, w, rho, sigma, fields, rho_bar,
                          ctx->d_status, snap);
}

hipError_t launch_twiddles(hipStream_t s, int N, double2 *tw, double2 *tq)
{
    hipLaunchKernelGGL(k_twiddles, dim3((N + 255) / 256), dim3(256), 0, s, N, tw, tq);
    return hipGetLastError();
}

hipError_t launch_pack_fields(ffb_ctx *ctx, const float *jx, const float *jy,
                              const float *rho_s, float4 *fields)
{
    const int64_t total = (int64_t)(ctx->lx + 2) * (ctx->ly + 2);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, jx, jy, rho_s,
                       ctx->lx, ctx->ly, fields);
    return hipGetLastError();
}

hipError_t launch_diff_spectrum(ffb_ctx *ctx, const double *rho, float sigma, float *spec)
{
    hipStream_t s = ctx->stream;
    const int lx = ctx->lx, ly = ctx->ly;
    hipLaunchKernelGGL(k_dct2_rows_f32, dim3(ly / 2), dim3(threads_for(lx)), 0, s, rho, ctx->t1,
                       lx, ctx->tw_x, ctx->tq_x);
    hipLaunchKernelGGL(k_transpose<float>, dim3((lx + 31) / 32, (ly + 31) / 32, 1), dim3(256), 0,
                       s, ctx->t1, ctx->t1, ctx->t1, ctx->t2, ctx->t2, ctx->t2, ly, lx);
    hipLaunchKernelGGL(kd_spectrum, dim3(lx / 2), dim3(threads_for(ly)), 0, s, ctx->t2, lx, ly,
                       sigma, ctx->tw_y, ctx->tq_y, spec);
    return hipGetLastError();
}

hipError_t launch_diff_fields(ffb_ctx *ctx, diff_ws *w, int slots)
{
    hipStream_t s = ctx->stream;
    const int lx = ctx->lx, ly = ctx->ly;
    hipLaunchKernelGGL(kd_col, dim3(lx / 2, slots), dim3(threads_for(ly)), 0, s, w->ctl, w->spec,
                       lx, ly, slots, ctx->tw_y, ctx->tq_y, w->q);
    // [lx][ly] -> [ly][lx], 3 * slots planes
    hipLaunchKernelGGL(kd_transpose, dim3((ly + 31) / 32, (lx + 31) / 32, 3 * slots), dim3(256),
                       0, s, w->ctl, w->q, w->r, lx, ly, slots, w->plane);
    hipLaunchKernelGGL(kd_row, dim3(ly / 2, slots), dim3(threads_for(lx)), 0, s, w->ctl, w->r,
                       lx, ly, slots, ctx->tw_x, ctx->tq_x, w->fields, ctx->d_status);
    return hipGetLastError();
}

hipError_t launch_flux_adj(ffb_ctx *ctx, float sigma, const float4 *lam_fields,
                           const double *lam_rho_bar, float *lam_rho, double *suf, double *total)
{
    hipStream_t s = ctx->stream;
    const int lx = ctx->lx, ly = ctx->ly;
    hipLaunchKernelGGL(k_adj_rows, dim3(ly / 2), dim3(threads_for(lx)), 0, s, lam_fields, lx, ly,
                       ctx->tw_x, ctx->tq_x, ctx->pa, ctx->pb, ctx->pc);
    hipLaunchKernelGGL(k_adj_cols, dim3(lx / 2), dim3(threads_for(ly)), 0, s, ctx->pa, ctx->pb,
                       ctx->pc, lx, ly, sigma, lam_rho_bar, ctx->tw_y, ctx->tq_y, ctx->t1);
    hipLaunchKernelGGL(k_adj_rows_final, dim3(ly / 2), dim3(threads_for(lx)), 0, s, ctx->t1, lx,
                       ctx->tw_x, ctx->tq_x, lam_rho, suf, total);
    return hipGetLastError();
}

// Fork the class streams off s[0] / join them back.
static hipError_t class_fork(const class_streams &cs)
{
    if (cs.n <= 1) return hipSuccess;
    hipError_t e = hipEventRecord(cs.fork, cs.s[0]);
    for (int c = 1; c < cs.n && e == hipSuccess; ++c) e = hipStreamWaitEvent(cs.s[c], cs.fork, 0);
    return e;
}

static hipError_t class_join(const class_streams &cs)
{
    hipError_t e = hipSuccess;
    for (int c = 1; c < cs.n && e == hipSuccess; ++c) {
        e = hipEventRecord(cs.join[c], cs.s[c]);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs.s[0], cs.join[c], 0);
    }
    return e;
}

hipError_t launch_batch_flux(const class_streams &cs, const batch_view &bv, const batch_tables &bt,
                             const batch_fft_plan &plan, const double2 *tw1024,
                             const double2 *tq1024, const double *rho_pad, double *acc,
                             double *t1, double *pa, double *pb, double *pc,
                             float4 *fields, double *rho_bar, int32_t *status)
{
    const auto on = [&](int c) { return cs.s[c < cs.n ? c : 0]; };
    hipError_t e = class_fork(cs);
    for (int c = 0; c < plan.n_classes && e == hipSuccess; ++c) {
        const int n = plan.row_beg[c + 1] - plan.row_beg[c], N = plan.n[c];
        if (n > 0)
            e = launch_grp_class<RowsK>(plan.threads[c], n, N, on(c), bv, bt.rows + plan.row_beg[c],
                                        n, N, acc, rho_pad, t1, tw1024, tq1024);
    }
    // with every map square, each class runs its three passes back to back
    // (its column and row passes read only its own maps' earlier passes) and
    // the mean density, which reads the first pass of every class and is
    // read by none of the passes, follows the final join; otherwise the
    // classes are joined after every pass
    if (e == hipSuccess && !cs.own) e = class_join(cs);
    // the mean density from the row sums the first pass left
    if (e == hipSuccess && !cs.own) {
        hipLaunchKernelGGL(kb_mean, dim3(bv.n_maps), dim3(256), 0, cs.s[0], bv, acc, rho_bar,
                           status);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !cs.own) e = class_fork(cs);
    for (int c = 0; c < plan.n_classes && e == hipSuccess; ++c) {
        const int n = plan.col_beg[c + 1] - plan.col_beg[c], N = plan.n[c];
        if (n > 0)
            e = launch_grp_class<ColsK>(plan.threads[c], n, N, on(c), bv, bt.cols + plan.col_beg[c],
                                        n, N, t1, tw1024, tq1024, pa, pb, pc);
    }
    if (e == hipSuccess && !cs.own) e = class_join(cs);
    if (e == hipSuccess && !cs.own) e = class_fork(cs);
    for (int c = 0; c < plan.n_classes && e == hipSuccess; ++c) {
        const int n = plan.row_beg[c + 1] - plan.row_beg[c], N = plan.n[c];
        if (n > 0)
            e = launch_grp_class<FinalK>(plan.threads[c], n, N, on(c), bv, bt.rows + plan.row_beg[c],
                                         n, N, pa, pb, pc, tw1024, tq1024, fields, status);
    }
    if (e == hipSuccess) e = class_join(cs);
    if (e == hipSuccess && cs.own) {
        hipLaunchKernelGGL(kb_mean, dim3(bv.n_maps), dim3(256), 0, cs.s[0], bv, acc, rho_bar,
                           status);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}
