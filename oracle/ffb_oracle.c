/*
 * ffb_oracle.c -- plain, slow, FP64 reference of one iteration of the fast
 * flow-based cartogram method (Gastner, Seguy & More, "Fast flow-based
 * algorithm for creating density-equalizing map projections").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP implementation, and the
 * product path never calls it.
 *
 * Every step follows the paper's definitions written out directly:
 *   - areas by the shoelace sum over polygon corners;
 *   - cell densities by exact polygon/cell clipping (Sutherland-Hodgman);
 *   - the cosine coefficients of Eq. 7 as direct separable sums (midpoint
 *     rule on the cell centres), no FFT;
 *   - the flux sums of the SI Appendix (section 2, the equations for J_x and
 *     J_y of linear equalisation) as direct separable sums;
 *   - the velocity v = J / rho_t with rho_t of Eq. 4, bilinear interpolation
 *     between grid points, and Dormand-Prince 5(4) integration to t = 1;
 *   - the diffusion variant of the SI Appendix (section 2) for comparison:
 *     fields rebuilt at every stage time, integration to a cut-off time.
 * Readings of points where the paper is silent are stated at each function.
 *
 * Parity of the integrator controller constants (tolerance, initial step,
 * safety factor, step-factor limits) is unpinned by the paper, which only
 * says that a predictor-corrector method adapts the next step size and that
 * a typical run takes about 100 steps.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes (same numeric meaning as the library's, defined here on
 * their own so that the two sides share no header) */
#define O_OK 0
#define O_E_INVALID 1
#define O_E_NOMEM 2
#define O_E_NONPOSITIVE 4
#define O_E_DOMAIN 5
#define O_E_STEP_UNDERFLOW 6
#define O_E_NONFINITE 7
#define O_E_MAX_ATTEMPTS 9

static const double PI = 3.14159265358979323846264338327950288;

int ffbo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Areas and area errors.
 * A region's area is the sum over its rings of the shoelace sum
 * 1/2 sum_k (x_k y_{k+1} - x_{k+1} y_k); counter-clockwise rings count
 * positive, clockwise rings (holes) negative.  The relative area error of
 * region r compares its current area A_r with its target share of the
 * current total, T_r = value_r * sum(A) / sum(value): e_r = A_r / T_r - 1
 * (main text, benchmarking section: the stopping rule of a maximum relative
 * area error below 1 %).
 * ---------------------------------------------------------------------- */
static double ring_area(const double *xy, const int32_t *vidx, int32_t n)
{
    double s = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        const double *p = xy + 2 * (int64_t)vidx[k];
        const double *q = xy + 2 * (int64_t)vidx[(k + 1) % n];
        s += p[0] * q[1] - q[0] * p[1];
    }
    return 0.5 * s;
}

static int check_geometry(int64_t nv, int32_t n_rings, const int32_t *ring_offsets,
                          const int32_t *ring_vidx, const int32_t *ring_region,
                          int32_t n_regions)
{
    if (nv < 0 || n_rings < 0 || n_regions <= 0) return O_E_INVALID;
    if (ring_offsets[0] != 0) return O_E_INVALID;
    for (int32_t r = 0; r < n_rings; ++r) {
        if (ring_offsets[r + 1] - ring_offsets[r] < 3) return O_E_INVALID;
        if (ring_region[r] < 0 || ring_region[r] >= n_regions) return O_E_INVALID;
    }
    int32_t ne = ring_offsets[n_rings];
    for (int32_t k = 0; k < ne; ++k)
        if (ring_vidx[k] < 0 || ring_vidx[k] >= nv) return O_E_INVALID;
    return O_OK;
}

int ffbo_region_areas(int64_t nv, const double *xy, int32_t n_rings,
                      const int32_t *ring_offsets, const int32_t *ring_vidx,
                      const int32_t *ring_region, int32_t n_regions, double *area)
{
    int st = check_geometry(nv, n_rings, ring_offsets, ring_vidx, ring_region, n_regions);
    if (st) return st;
    for (int64_t k = 0; k < 2 * nv; ++k)
        if (!isfinite(xy[k])) return O_E_NONFINITE;
    for (int32_t r = 0; r < n_regions; ++r) area[r] = 0.0;
    for (int32_t g = 0; g < n_rings; ++g) {
        int32_t b = ring_offsets[g], e = ring_offsets[g + 1];
        area[ring_region[g]] += ring_area(xy, ring_vidx + b, e - b);
    }
    return O_OK;
}

int ffbo_area_error(int32_t n_regions, const double *value, const double *area,
                    double *err, double *max_abs_err)
{
    double sa = 0.0, sv = 0.0;
    for (int32_t r = 0; r < n_regions; ++r) {
        if (!(value[r] > 0.0)) return O_E_NONPOSITIVE;
        sa += area[r];
        sv += value[r];
    }
    double mx = 0.0;
    for (int32_t r = 0; r < n_regions; ++r) {
        double target = value[r] * sa / sv;
        err[r] = area[r] / target - 1.0;
        if (fabs(err[r]) > mx || isnan(err[r])) mx = fabs(err[r]);
    }
    *max_abs_err = mx;
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Rasterisation.  The density is piecewise constant per region, d_r =
 * value_r / A_r (main text, section on previous all-coordinates methods),
 * and the space between the map and the box edges holds the mean density
 * (benchmarking section), read here as rho_pad = sum(value) / sum(A).  A
 * grid cell [i, i+1] x [j, j+1] gets the exact area-weighted average:
 *   rho0_ij = rho_pad + sum_r (d_r - rho_pad) * area(cell ∩ region_r).
 * The intersection is computed by clipping each ring against the cell's
 * four half-planes (first the row band, then the column) and taking the
 * signed shoelace area of the clipped polygon.
 * ---------------------------------------------------------------------- */
typedef struct { double *x, *y; int32_t n, cap; } poly_t;

static int poly_reserve(poly_t *p, int32_t cap)
{
    if (p->cap >= cap) return 0;
    double *nx = (double *)realloc(p->x, sizeof(double) * cap);
    if (!nx) return -1;
    p->x = nx;
    double *ny = (double *)realloc(p->y, sizeof(double) * cap);
    if (!ny) return -1;
    p->y = ny;
    p->cap = cap;
    return 0;
}

/* keep the part of `in` with s * (coord - c) <= 0, coord = x (axis 0) or y */
static int clip_half(const poly_t *in, poly_t *out, int axis, double c, double s)
{
    out->n = 0;
    if (poly_reserve(out, 2 * in->n + 4)) return -1;
    for (int32_t k = 0; k < in->n; ++k) {
        int32_t k1 = (k + 1) % in->n;
        double px = in->x[k], py = in->y[k], qx = in->x[k1], qy = in->y[k1];
        double fp = s * ((axis == 0 ? px : py) - c);
        double fq = s * ((axis == 0 ? qx : qy) - c);
        int pin = fp <= 0.0, qin = fq <= 0.0;
        if (pin) { out->x[out->n] = px; out->y[out->n] = py; out->n++; }
        if (pin != qin) {
            double w = fp / (fp - fq);
            double ix = px + w * (qx - px), iy = py + w * (qy - py);
            if (axis == 0) ix = c; else iy = c;
            out->x[out->n] = ix; out->y[out->n] = iy; out->n++;
        }
    }
    return 0;
}

/* Signed shoelace area of p, with the corners taken relative to (ox, oy):
 * the sum is unchanged by the translation, and with (ox, oy) the corner of
 * the clipped cell the products are of numbers below 1 instead of ~L, so
 * the rounding of the sum stays at FP64 level relative to the area. */
static double poly_area(const poly_t *p, double ox, double oy)
{
    double s = 0.0;
    for (int32_t k = 0; k < p->n; ++k) {
        int32_t k1 = (k + 1) % p->n;
        s += (p->x[k] - ox) * (p->y[k1] - oy) - (p->x[k1] - ox) * (p->y[k] - oy);
    }
    return 0.5 * s;
}

int ffbo_density(int32_t lx, int32_t ly, int64_t nv, const double *xy, int32_t n_rings,
                 const int32_t *ring_offsets, const int32_t *ring_vidx,
                 const int32_t *ring_region, int32_t n_regions, const double *value,
                 const double *area, double *rho, double *rho_pad_out)
{
    if (lx <= 0 || ly <= 0) return O_E_INVALID;
    int st = check_geometry(nv, n_rings, ring_offsets, ring_vidx, ring_region, n_regions);
    if (st) return st;
    for (int64_t k = 0; k < nv; ++k) {
        double x = xy[2 * k], y = xy[2 * k + 1];
        if (!isfinite(x) || !isfinite(y)) return O_E_NONFINITE;
        if (x < 0.0 || x > lx || y < 0.0 || y > ly) return O_E_DOMAIN;
    }
    double sa = 0.0, sv = 0.0;
    for (int32_t r = 0; r < n_regions; ++r) {
        if (!(value[r] > 0.0) || !(area[r] > 0.0)) return O_E_NONPOSITIVE;
        sa += area[r];
        sv += value[r];
    }
    const double rho_pad = sv / sa;
    double *w = (double *)malloc(sizeof(double) * n_regions);
    double *ymin = (double *)malloc(sizeof(double) * (n_rings + 1));
    double *ymax = (double *)malloc(sizeof(double) * (n_rings + 1));
    if (!w || !ymin || !ymax) { free(w); free(ymin); free(ymax); return O_E_NOMEM; }
    for (int32_t r = 0; r < n_regions; ++r) w[r] = value[r] / area[r] - rho_pad;
    for (int32_t g = 0; g < n_rings; ++g) {
        double lo = INFINITY, hi = -INFINITY;
        for (int32_t k = ring_offsets[g]; k < ring_offsets[g + 1]; ++k) {
            double y = xy[2 * (int64_t)ring_vidx[k] + 1];
            if (y < lo) lo = y;
            if (y > hi) hi = y;
        }
        ymin[g] = lo; ymax[g] = hi;
    }
    for (int64_t c = 0; c < (int64_t)lx * ly; ++c) rho[c] = rho_pad;

    int fail = 0;
#pragma omp parallel
    {
        poly_t ring = {0}, t1 = {0}, band = {0}, t2 = {0}, cell = {0};
#pragma omp for schedule(dynamic, 4)
        for (int32_t j = 0; j < ly; ++j) {
            for (int32_t g = 0; g < n_rings; ++g) {
                if (ymax[g] <= j || ymin[g] >= j + 1) continue;
                int32_t b = ring_offsets[g], n = ring_offsets[g + 1] - b;
                if (poly_reserve(&ring, n)) { fail = 1; continue; }
                for (int32_t k = 0; k < n; ++k) {
                    ring.x[k] = xy[2 * (int64_t)ring_vidx[b + k]];
                    ring.y[k] = xy[2 * (int64_t)ring_vidx[b + k] + 1];
                }
                ring.n = n;
                if (clip_half(&ring, &t1, 1, (double)j, -1.0)) { fail = 1; continue; }
                if (clip_half(&t1, &band, 1, (double)(j + 1), 1.0)) { fail = 1; continue; }
                if (band.n < 3) continue;
                double xlo = INFINITY, xhi = -INFINITY;
                for (int32_t k = 0; k < band.n; ++k) {
                    if (band.x[k] < xlo) xlo = band.x[k];
                    if (band.x[k] > xhi) xhi = band.x[k];
                }
                int32_t i0 = (int32_t)floor(xlo), i1 = (int32_t)ceil(xhi);
                if (i0 < 0) i0 = 0;
                if (i1 > lx) i1 = lx;
                for (int32_t i = i0; i < i1; ++i) {
                    if (clip_half(&band, &t2, 0, (double)i, -1.0)) { fail = 1; break; }
                    if (clip_half(&t2, &cell, 0, (double)(i + 1), 1.0)) { fail = 1; break; }
                    if (cell.n < 3) continue;
                    rho[(int64_t)j * lx + i] +=
                        w[ring_region[g]] * poly_area(&cell, (double)i, (double)j);
                }
            }
        }
        free(ring.x); free(ring.y); free(t1.x); free(t1.y); free(band.x); free(band.y);
        free(t2.x); free(t2.y); free(cell.x); free(cell.y);
    }
    free(w); free(ymin); free(ymax);
    if (fail) return O_E_NOMEM;
    *rho_pad_out = rho_pad;
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Cosine/sine tables.  cos(pi * m * (2i + 1) / (2L)) for integers m, i is
 * looked up as tab[(m * (2i + 1)) mod 4L] with tab[k] = cos(pi k / (2L)),
 * and the matching sine as tab[(m * (2i + 1) - L) mod 4L].
 * ---------------------------------------------------------------------- */
static double *make_table(int32_t L)
{
    double *tab = (double *)malloc(sizeof(double) * 4 * (size_t)L);
    if (!tab) return NULL;
    for (int32_t k = 0; k < 4 * L; ++k) tab[k] = cos(PI * (double)k / (2.0 * L));
    return tab;
}

static inline double tcos(const double *tab, int32_t L, int64_t m, int64_t i)
{
    int64_t k = (m * (2 * i + 1)) % (4 * (int64_t)L);
    return tab[k];
}

static inline double tsin(const double *tab, int32_t L, int64_t m, int64_t i)
{
    int64_t k = (m * (2 * i + 1) - L) % (4 * (int64_t)L);
    if (k < 0) k += 4 * (int64_t)L;
    return tab[k];
}

/* S_mn = sum_{i<lx} sum_{j<ly} rho_ij cos(pi m (i+1/2)/lx) cos(pi n (j+1/2)/ly),
 * stored as S[n * lx + m]: Eq. 7 with the integral taken by the midpoint
 * rule on the cell centres, before the 4 / ((1 + delta_m0)(1 + delta_n0))
 * factor.  Computed as two separable passes of direct sums. */
int ffbo_dct2(int32_t lx, int32_t ly, const double *rho, double *S)
{
    if (lx <= 0 || ly <= 0) return O_E_INVALID;
    double *tx = make_table(lx), *ty = make_table(ly);
    double *T = (double *)malloc(sizeof(double) * (size_t)lx * ly);
    if (!tx || !ty || !T) { free(tx); free(ty); free(T); return O_E_NOMEM; }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t m = 0; m < lx; ++m) {
            double s = 0.0;
            for (int32_t i = 0; i < lx; ++i) s += rho[(int64_t)j * lx + i] * tcos(tx, lx, m, i);
            T[(int64_t)j * lx + m] = s;
        }
#pragma omp parallel for schedule(static)
    for (int32_t n = 0; n < ly; ++n)
        for (int32_t m = 0; m < lx; ++m) {
            double s = 0.0;
            for (int32_t j = 0; j < ly; ++j) s += T[(int64_t)j * lx + m] * tcos(ty, ly, n, j);
            S[(int64_t)n * lx + m] = s;
        }
    free(tx); free(ty); free(T);
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Blur, flux and blurred density on the grid nodes (i + 1/2, j + 1/2).
 *
 *  rt_mn   = 4 S_mn / ((1 + delta_m0)(1 + delta_n0))                 (Eq. 7)
 *  rts_mn  = rt_mn * exp(-pi^2 sigma^2 (m^2/lx^2 + n^2/ly^2) / 2)
 *            (the Gaussian blur of the initial density, read as the heat
 *            kernel with the box's reflecting edges, which is diagonal in
 *            this cosine basis; sigma in grid units)
 *  rho_bar = rts_00 / (lx ly)                  (rt_00 = rho_bar lx ly, SI)
 *  rho_s   = (1/(lx ly)) sum_mn rts_mn cos cos        (SI backward series)
 *  J_x     = (ly/pi) sum_{m>=1,n>=0} m/(m^2 ly^2 + n^2 lx^2) rts_mn sin cos
 *  J_y     = (lx/pi) sum_{m>=0,n>=1} n/(m^2 ly^2 + n^2 lx^2) rts_mn cos sin
 *
 * Sign reading: the SI coefficients of the flux for linear equalisation are
 * positive multiples of rt_mn, and inserting them into the SI sine/cosine
 * series of J gives the "+" sign used here (the flux leaves dense regions,
 * div J = rho_0 - rho_bar, as the continuity equation with Eq. 4 demands);
 * the leading minus printed in Eq. 5-6 is taken as a typo.
 * The series are truncated at m < lx, n < ly.
 * ---------------------------------------------------------------------- */
/* Blurred coefficients rts[n][m] and rho_bar only (the forward half). */
int ffbo_coefficients(int32_t lx, int32_t ly, const double *rho, double sigma, double *coef,
                      double *rho_bar_out)
{
    if (lx <= 0 || ly <= 0 || !(sigma >= 0.0)) return O_E_INVALID;
    const int64_t N = (int64_t)lx * ly;
    for (int64_t c = 0; c < N; ++c)
        if (!isfinite(rho[c])) return O_E_NONFINITE;
    int st = ffbo_dct2(lx, ly, rho, coef);
    if (st) return st;
    for (int32_t n = 0; n < ly; ++n)
        for (int32_t m = 0; m < lx; ++m) {
            double f = 4.0 / ((m == 0 ? 2.0 : 1.0) * (n == 0 ? 2.0 : 1.0));
            double k2 = (double)m * m / ((double)lx * lx) + (double)n * n / ((double)ly * ly);
            coef[(int64_t)n * lx + m] *= f * exp(-PI * PI * sigma * sigma * k2 / 2.0);
        }
    *rho_bar_out = coef[0] / (double)N;
    return O_OK;
}

/* The three series at selected nodes (i[k], j[k]) by full double sums over
 * all coefficients: out[3k] = J_x, out[3k+1] = J_y, out[3k+2] = rho_s. */
int ffbo_flux_nodes(int32_t lx, int32_t ly, const double *coef, int64_t k, const int32_t *ii,
                    const int32_t *jj, double *out)
{
    if (lx <= 0 || ly <= 0 || k < 0) return O_E_INVALID;
    double *tx = make_table(lx), *ty = make_table(ly);
    if (!tx || !ty) { free(tx); free(ty); return O_E_NOMEM; }
    const double LX = lx, LY = ly;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < k; ++q) {
        const int32_t i = ii[q], j = jj[q];
        double a = 0.0, b = 0.0, c = 0.0;
        for (int32_t n = 0; n < ly; ++n) {
            const double cy = tcos(ty, ly, n, j), sy = tsin(ty, ly, n, j);
            for (int32_t m = 0; m < lx; ++m) {
                const double r = coef[(int64_t)n * lx + m];
                const double cx = tcos(tx, lx, m, i), sx = tsin(tx, lx, m, i);
                const double den = (double)m * m * LY * LY + (double)n * n * LX * LX;
                a += r * cx * cy;
                if (m > 0) b += (LY / PI) * ((double)m / den) * r * sx * cy;
                if (n > 0) c += (LX / PI) * ((double)n / den) * r * cx * sy;
            }
        }
        out[3 * q] = b;
        out[3 * q + 1] = c;
        out[3 * q + 2] = a / (LX * LY);
    }
    free(tx); free(ty);
    return O_OK;
}

int ffbo_flux(int32_t lx, int32_t ly, const double *rho, double sigma,
              double *rho_s, double *jx, double *jy, double *rho_bar_out, double *coef_out)
{
    if (lx <= 0 || ly <= 0 || !(sigma >= 0.0)) return O_E_INVALID;
    const int64_t N = (int64_t)lx * ly;
    double *S = (double *)malloc(sizeof(double) * N);
    double *A = (double *)malloc(sizeof(double) * N);
    double *B = (double *)malloc(sizeof(double) * N);
    double *C = (double *)malloc(sizeof(double) * N);
    double *tx = make_table(lx), *ty = make_table(ly);
    if (!S || !A || !B || !C || !tx || !ty) {
        free(S); free(A); free(B); free(C); free(tx); free(ty);
        return O_E_NOMEM;
    }
    double rho_bar = 0.0;
    int st = ffbo_coefficients(lx, ly, rho, sigma, S, &rho_bar);
    if (st) { free(S); free(A); free(B); free(C); free(tx); free(ty); return st; }
    if (coef_out) memcpy(coef_out, S, sizeof(double) * N);
    const double LX = lx, LY = ly;

    /* pass over n (y frequency) for each node row j and x frequency m */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t m = 0; m < lx; ++m) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t n = 0; n < ly; ++n) {
                double r = S[(int64_t)n * lx + m];
                double cy = tcos(ty, ly, n, j), sy = tsin(ty, ly, n, j);
                double den = (double)m * m * LY * LY + (double)n * n * LX * LX;
                a += r * cy;
                if (m > 0) b += (LY / PI) * ((double)m / den) * r * cy;
                if (n > 0) c += (LX / PI) * ((double)n / den) * r * sy;
            }
            A[(int64_t)j * lx + m] = a;
            B[(int64_t)j * lx + m] = b;
            C[(int64_t)j * lx + m] = c;
        }
    /* pass over m (x frequency) for each node (i, j) */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t i = 0; i < lx; ++i) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t m = 0; m < lx; ++m) {
                double cx = tcos(tx, lx, m, i), sx = tsin(tx, lx, m, i);
                a += A[(int64_t)j * lx + m] * cx;
                b += B[(int64_t)j * lx + m] * sx;
                c += C[(int64_t)j * lx + m] * cx;
            }
            rho_s[(int64_t)j * lx + i] = a / (double)N;
            jx[(int64_t)j * lx + i] = b;
            jy[(int64_t)j * lx + i] = c;
        }
    free(S); free(A); free(B); free(C); free(tx); free(ty);
    *rho_bar_out = rho_bar;
    double mn = INFINITY;
    for (int64_t c = 0; c < N; ++c) if (rho_s[c] < mn) mn = rho_s[c];
    if (!(mn > 0.0) || !(rho_bar > 0.0)) return O_E_NONPOSITIVE;
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Velocity at an arbitrary point (main text: v at each grid point by basic
 * arithmetic, then interpolation between grid points).
 * Node velocity: v_ij(t) = J_ij / ((1 - t) rho_s_ij + t rho_bar)   (Eq. 4-6).
 * Lookup at q clamped to the box: u = q_x - 1/2, i0 = floor(u), alpha =
 * u - i0 (same in y), bilinear in the four surrounding nodes.  Nodes outside
 * the grid (index -1 or L) take the values the sine/cosine series have at
 * the mirrored cell centres: v_x is odd and v_y even across the x edges,
 * v_x even and v_y odd across the y edges, so v . n = 0 on the box.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t lx, ly;
    const double *rho_s, *jx, *jy;
    double rho_bar;
} field_t;

static void node_velocity(const field_t *F, double t, int32_t i, int32_t j,
                          double *vx, double *vy)
{
    double sx = 1.0, sy = 1.0;
    if (i < 0) { i = 0; sx = -sx; }
    if (i >= F->lx) { i = F->lx - 1; sx = -sx; }
    if (j < 0) { j = 0; sy = -sy; }
    if (j >= F->ly) { j = F->ly - 1; sy = -sy; }
    int64_t c = (int64_t)j * F->lx + i;
    double rt = (1.0 - t) * F->rho_s[c] + t * F->rho_bar;
    *vx = sx * F->jx[c] / rt;
    *vy = sy * F->jy[c] / rt;
}

static void velocity_at(const field_t *F, double t, double qx, double qy,
                        double *vx, double *vy)
{
    if (qx < 0.0) qx = 0.0;
    if (qx > F->lx) qx = F->lx;
    if (qy < 0.0) qy = 0.0;
    if (qy > F->ly) qy = F->ly;
    double u = qx - 0.5, w = qy - 0.5;
    double fu = floor(u), fw = floor(w);
    int32_t i0 = (int32_t)fu, j0 = (int32_t)fw;
    double a = u - fu, b = w - fw;
    double x00, y00, x10, y10, x01, y01, x11, y11;
    node_velocity(F, t, i0, j0, &x00, &y00);
    node_velocity(F, t, i0 + 1, j0, &x10, &y10);
    node_velocity(F, t, i0, j0 + 1, &x01, &y01);
    node_velocity(F, t, i0 + 1, j0 + 1, &x11, &y11);
    /* interpolate along x on both node rows, then along y */
    *vx = (1 - b) * ((1 - a) * x00 + a * x10) + b * ((1 - a) * x01 + a * x11);
    *vy = (1 - b) * ((1 - a) * y00 + a * y10) + b * ((1 - a) * y01 + a * y11);
}

int ffbo_velocity(int32_t lx, int32_t ly, const double *rho_s, const double *jx,
                  const double *jy, double rho_bar, double t, int64_t n,
                  const double *q, double *v)
{
    if (lx <= 0 || ly <= 0 || n < 0) return O_E_INVALID;
    for (int64_t k = 0; k < 2 * n; ++k)
        if (!isfinite(q[k])) return O_E_NONFINITE;
    field_t F = {lx, ly, rho_s, jx, jy, rho_bar};
    for (int64_t p = 0; p < n; ++p)
        velocity_at(&F, t, q[2 * p], q[2 * p + 1], &v[2 * p], &v[2 * p + 1]);
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Time integration of dr/dt = v(r, t) from t = 0 to exactly t = 1 for all
 * points together (main text: an adaptive predictor-corrector method, with
 * the integrands of all grid points advanced in each step).  The method is
 * the embedded Runge-Kutta pair of Dormand and Prince (1980), order 5 with
 * an order-4 error estimate and first-same-as-last stages.  One step size
 * serves all points.  Controller (constants are arguments):
 *   err = max over points and both components of |h sum_s (b_s - b*_s) k_s|
 *   accept iff err <= tol;
 *   fac = safety * (err / tol)^(-1/5), limited to [fac_min, fac_max]
 *         (fac_max when err = 0), and to at most 1 on the attempt that
 *         follows a rejection;
 *   the step is clipped so that the last one ends exactly at t = 1;
 *   h < h_min before t = 1 is a step underflow.
 * Replay mode takes a given sequence of accepted steps and skips control.
 * ---------------------------------------------------------------------- */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192,
                               -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BS[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

void ffbo_tableau(double *c, double *a, double *b, double *bs)
{
    for (int s = 0; s < 7; ++s) {
        c[s] = DP_C[s];
        b[s] = DP_B[s];
        bs[s] = DP_BS[s];
        for (int q = 0; q < 6; ++q) a[s * 6 + q] = DP_A[s][q];
    }
}

/* Where the stage velocities come from: the field set to use at stage time
 * ts and the time argument that velocity_at takes with it.  For the fast
 * flow-based method the fields are fixed and rho_t carries the time; a
 * variant whose fields change with t returns fields already taken at ts. */
typedef struct field_source {
    const field_t *(*at)(struct field_source *self, double ts, double *tv, int *status);
} field_source;

typedef struct {
    field_source base;
    field_t F;
} fixed_source;

static const field_t *fixed_at(field_source *self, double ts, double *tv, int *status)
{
    (void)status;
    *tv = ts;
    return &((fixed_source *)self)->F;
}

/* One attempt of size h from (y, t) with k[0] = v(y, t) already known.
 * Writes the order-5 solution to ynew, its velocity to k[6], returns err
 * (INFINITY with *status set when a field evaluation fails). */
static double dp_attempt(field_source *src, int64_t n, const double *y, double t, double h,
                         double *k[7], double *ynew, int *status)
{
    for (int s = 1; s < 7; ++s) {
        double tv;
        const field_t *F = src->at(src, t + DP_C[s] * h, &tv, status);
        if (*status) return INFINITY;
        double *dst = (s == 6) ? ynew : NULL;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            double qx = y[2 * p], qy = y[2 * p + 1];
            for (int q = 0; q < s; ++q) {
                qx += h * DP_A[s][q] * k[q][2 * p];
                qy += h * DP_A[s][q] * k[q][2 * p + 1];
            }
            if (dst) { dst[2 * p] = qx; dst[2 * p + 1] = qy; }
            velocity_at(F, tv, qx, qy, &k[s][2 * p], &k[s][2 * p + 1]);
        }
    }
    double err = 0.0;
#pragma omp parallel for schedule(static) reduction(max : err)
    for (int64_t p = 0; p < n; ++p) {
        for (int d = 0; d < 2; ++d) {
            double e = 0.0;
            for (int s = 0; s < 7; ++s) e += (DP_B[s] - DP_BS[s]) * k[s][2 * p + d];
            e = fabs(h * e);
            if (!(e <= err)) err = isnan(e) ? INFINITY : e;
        }
    }
    return err;
}

/* The controller described above, from t = 0 to exactly t = t_end. */
static int dp_run(field_source *src, int64_t n, double *xy, double t_end, double tol, double h0,
                  double safety, double fac_min, double fac_max, double h_min,
                  int32_t max_attempts, const double *replay_h, int32_t n_replay,
                  int32_t *accepted_out, int32_t *rejected_out, double *h_out, int32_t h_cap)
{
    double *k[7];
    double *ynew = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
    int ok = ynew != NULL;
    for (int s = 0; s < 7; ++s) {
        k[s] = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
        ok = ok && k[s];
    }
    int st = O_OK;
    int32_t acc = 0, rej = 0;
    if (!ok) { st = O_E_NOMEM; goto done; }

    {
        double tv;
        const field_t *F0 = src->at(src, 0.0, &tv, &st);
        if (st) goto done;
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p)
            velocity_at(F0, tv, xy[2 * p], xy[2 * p + 1], &k[0][2 * p], &k[0][2 * p + 1]);
    }

    double t = 0.0;
    if (replay_h) {
        for (int32_t s = 0; s < n_replay; ++s) {
            double h = replay_h[s];
            double err = dp_attempt(src, n, xy, t, h, k, ynew, &st);
            if (st) break;
            if (!isfinite(err)) { st = O_E_NONFINITE; break; }
            memcpy(xy, ynew, sizeof(double) * 2 * (size_t)n);
            double *tmp = k[0]; k[0] = k[6]; k[6] = tmp;
            t = (s == n_replay - 1) ? t_end : t + h;
            if (h_out && acc < h_cap) h_out[acc] = h;
            acc++;
        }
        goto done;
    }

    double h = h0;
    int last_rejected = 0;
    int32_t attempts = 0;
    while (t < t_end) {
        if (attempts >= max_attempts) { st = O_E_MAX_ATTEMPTS; break; }
        int final_step = h >= t_end - t;
        if (final_step) h = t_end - t;
        double err = dp_attempt(src, n, xy, t, h, k, ynew, &st);
        attempts++;
        if (st) break;
        if (!isfinite(err)) { st = O_E_NONFINITE; break; }
        if (err <= tol) {
            memcpy(xy, ynew, sizeof(double) * 2 * (size_t)n);
            double *tmp = k[0]; k[0] = k[6]; k[6] = tmp;
            if (h_out && acc < h_cap) h_out[acc] = h;
            acc++;
            t = final_step ? t_end : t + h;
            double fac = (err == 0.0) ? fac_max : safety * pow(err / tol, -0.2);
            if (fac < fac_min) fac = fac_min;
            if (fac > fac_max) fac = fac_max;
            if (last_rejected && fac > 1.0) fac = 1.0;
            h *= fac;
            last_rejected = 0;
        } else {
            rej++;
            double fac = safety * pow(err / tol, -0.2);
            if (fac < fac_min) fac = fac_min;
            h *= fac;
            last_rejected = 1;
        }
        if (t < t_end && h < h_min) { st = O_E_STEP_UNDERFLOW; break; }
    }
done:
    free(ynew);
    for (int s = 0; s < 7; ++s) free(k[s]);
    if (accepted_out) *accepted_out = acc;
    if (rejected_out) *rejected_out = rej;
    return st;
}

int ffbo_integrate(int32_t lx, int32_t ly, const double *rho_s, const double *jx,
                   const double *jy, double rho_bar, int64_t n, double *xy,
                   double tol, double h0, double safety, double fac_min, double fac_max,
                   double h_min, int32_t max_attempts,
                   const double *replay_h, int32_t n_replay,
                   int32_t *accepted_out, int32_t *rejected_out,
                   double *h_out, int32_t h_cap)
{
    if (lx <= 0 || ly <= 0 || n < 0 || !(rho_bar > 0.0)) return O_E_INVALID;
    if (!replay_h && (!(tol > 0.0) || !(h0 > 0.0) || max_attempts <= 0)) return O_E_INVALID;
    for (int64_t k = 0; k < 2 * n; ++k)
        if (!isfinite(xy[k])) return O_E_NONFINITE;
    fixed_source src = {{fixed_at}, {lx, ly, rho_s, jx, jy, rho_bar}};
    return dp_run(&src.base, n, xy, 1.0, tol, h0, safety, fac_min, fac_max, h_min,
                  max_attempts, replay_h, n_replay, accepted_out, rejected_out, h_out, h_cap);
}

/* ------------------------------------------------------------------------
 * The diffusion cartogram as a flow-based projection (SI Appendix,
 * section 2, the diffusion choice of f_mn): with the same coefficients
 * rts_mn (Eq. 7 and the blur, as ffbo_coefficients),
 *
 *   f_mn(t) = exp(-(m^2/lx^2 + n^2/ly^2) t),
 *   rho(t)  = (1/(lx ly)) sum_mn rts_mn f_mn(t) cos(m pi x/lx) cos(n pi y/ly),
 *   J_x(t)  = (1/(lx ly)) sum_{m>=1,n>=0} (m / (pi lx)) rts_mn f_mn(t) sin cos,
 *   J_y(t)  = (1/(lx ly)) sum_{m>=0,n>=1} (n / (pi ly)) rts_mn f_mn(t) cos sin,
 *
 * at the nodes (i + 1/2, j + 1/2), and v = J(t) / rho(t).  The fields
 * depend on t, so every stage time of the integrator needs them anew.  The
 * improper integral to t = infinity is cut at a caller-given t_end.
 * ---------------------------------------------------------------------- */
int ffbo_diff_fields(int32_t lx, int32_t ly, const double *coef, double t, double *rho_t,
                     double *jx, double *jy)
{
    if (lx <= 0 || ly <= 0 || !(t >= 0.0)) return O_E_INVALID;
    const int64_t N = (int64_t)lx * ly;
    double *G = (double *)malloc(sizeof(double) * N);
    double *A = (double *)malloc(sizeof(double) * N);
    double *B = (double *)malloc(sizeof(double) * N);
    double *C = (double *)malloc(sizeof(double) * N);
    double *tx = make_table(lx), *ty = make_table(ly);
    if (!G || !A || !B || !C || !tx || !ty) {
        free(G); free(A); free(B); free(C); free(tx); free(ty);
        return O_E_NOMEM;
    }
    const double LX = lx, LY = ly;
    /* g_mn = rts_mn f_mn(t) */
    for (int32_t n = 0; n < ly; ++n)
        for (int32_t m = 0; m < lx; ++m) {
            double k2 = (double)m * m / (LX * LX) + (double)n * n / (LY * LY);
            G[(int64_t)n * lx + m] = coef[(int64_t)n * lx + m] * exp(-k2 * t);
        }
    /* pass over n for each node row j and x frequency m */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t m = 0; m < lx; ++m) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t n = 0; n < ly; ++n) {
                double g = G[(int64_t)n * lx + m];
                double cy = tcos(ty, ly, n, j), sy = tsin(ty, ly, n, j);
                a += g * cy;
                if (m > 0) b += ((double)m / (PI * LX)) * g * cy;
                if (n > 0) c += ((double)n / (PI * LY)) * g * sy;
            }
            A[(int64_t)j * lx + m] = a;
            B[(int64_t)j * lx + m] = b;
            C[(int64_t)j * lx + m] = c;
        }
    /* pass over m for each node (i, j) */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t i = 0; i < lx; ++i) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t m = 0; m < lx; ++m) {
                double cx = tcos(tx, lx, m, i), sx = tsin(tx, lx, m, i);
                a += A[(int64_t)j * lx + m] * cx;
                b += B[(int64_t)j * lx + m] * sx;
                c += C[(int64_t)j * lx + m] * cx;
            }
            rho_t[(int64_t)j * lx + i] = a / (double)N;
            jx[(int64_t)j * lx + i] = b / (double)N;
            jy[(int64_t)j * lx + i] = c / (double)N;
        }
    free(G); free(A); free(B); free(C); free(tx); free(ty);
    double mn = INFINITY;
    for (int64_t c = 0; c < N; ++c) if (rho_t[c] < mn) mn = rho_t[c];
    return (mn > 0.0) ? O_OK : O_E_NONPOSITIVE;
}

/* Fields recomputed at each new stage time; stages at equal times (the
 * last two of an attempt) share one evaluation. */
typedef struct {
    field_source base;
    int32_t lx, ly;
    const double *coef;
    double *rho_t, *jx, *jy;
    double last_t;
    int have;
    field_t F;
} diff_source;

static const field_t *diff_at(field_source *self, double ts, double *tv, int *status)
{
    diff_source *d = (diff_source *)self;
    if (!d->have || d->last_t != ts) {
        int st = ffbo_diff_fields(d->lx, d->ly, d->coef, ts, d->rho_t, d->jx, d->jy);
        if (st) { *status = st; return &d->F; }
        d->last_t = ts;
        d->have = 1;
    }
    *tv = 0.0;   /* rho_t of the field set is rho(ts) itself */
    return &d->F;
}

int ffbo_diff_integrate(int32_t lx, int32_t ly, const double *coef, double t_end, int64_t n,
                        double *xy, double tol, double h0, double safety, double fac_min,
                        double fac_max, double h_min, int32_t max_attempts,
                        const double *replay_h, int32_t n_replay, int32_t *accepted_out,
                        int32_t *rejected_out, double *h_out, int32_t h_cap)
{
    if (lx <= 0 || ly <= 0 || n < 0 || !(t_end > 0.0) || !(coef[0] > 0.0)) return O_E_INVALID;
    if (!replay_h && (!(tol > 0.0) || !(h0 > 0.0) || max_attempts <= 0)) return O_E_INVALID;
    for (int64_t k = 0; k < 2 * n; ++k)
        if (!isfinite(xy[k])) return O_E_NONFINITE;
    const int64_t N = (int64_t)lx * ly;
    diff_source src;
    memset(&src, 0, sizeof src);
    src.base.at = diff_at;
    src.lx = lx;
    src.ly = ly;
    src.coef = coef;
    src.rho_t = (double *)malloc(sizeof(double) * N);
    src.jx = (double *)malloc(sizeof(double) * N);
    src.jy = (double *)malloc(sizeof(double) * N);
    if (!src.rho_t || !src.jx || !src.jy) {
        free(src.rho_t); free(src.jx); free(src.jy);
        return O_E_NOMEM;
    }
    /* rho_bar only enters velocity_at through t * rho_bar with t = 0 */
    field_t F = {lx, ly, src.rho_t, src.jx, src.jy, coef[0] / (double)N};
    src.F = F;
    int st = dp_run(&src.base, n, xy, t_end, tol, h0, safety, fac_min, fac_max, h_min,
                    max_attempts, replay_h, n_replay, accepted_out, rejected_out, h_out, h_cap);
    free(src.rho_t); free(src.jx); free(src.jy);
    return st;
}

/* ------------------------------------------------------------------------
 * Inverse of the piecewise-linear approximation of T (Conclusion: the
 * graticule of the inverse transformation; T is approximated as piecewise
 * linear and that approximation is inverted).
 *
 * T is known at the nodes: nodes[j][i] (FP32 pairs) is the image of the
 * cell centre (i + 1/2, j + 1/2).  Reading: each cell between four nodes,
 * c = j (lx - 1) + i, is split along its (i,j)-(i+1,j+1) diagonal into
 * triangle 2c with corners (i,j), (i+1,j), (i+1,j+1) and triangle 2c + 1
 * with corners (i,j), (i+1,j+1), (i,j+1); on each, T is the affine map that
 * takes the three original corners to their images.
 *
 * For a query q the preimage is the original point whose image is q, taken
 * in the lowest-numbered triangle whose image contains q (edges included;
 * on a folded map several images may contain q).  A triangle with a
 * zero-area image contains nothing.  No triangle: tri = -1, pre = NaN.
 * The orientation of q against an edge is
 *   (b.x - a.x)(q.y - a.y) - (b.y - a.y)(q.x - a.x)
 * in FP64 on the FP32 inputs, with no fused multiply-add.
 * ---------------------------------------------------------------------- */
static double orient2(double ax, double ay, double bx, double by, double qx, double qy)
{
    double u = (bx - ax) * (qy - ay);
    double v = (by - ay) * (qx - ax);
    return u - v;
}

int ffbo_inverse(int32_t lx, int32_t ly, const float *nodes, int64_t nq, const float *queries,
                 int32_t *tri, double *pre)
{
    if (lx < 2 || ly < 2 || nq < 0) return O_E_INVALID;
    const int64_t ncell = (int64_t)(lx - 1) * (ly - 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nq; ++k) {
        const double qx = queries[2 * k], qy = queries[2 * k + 1];
        tri[k] = -1;
        pre[2 * k] = NAN;
        pre[2 * k + 1] = NAN;
        for (int64_t t = 0; t < 2 * ncell; ++t) {
            const int64_t c = t >> 1;
            const int32_t i = (int32_t)(c % (lx - 1)), j = (int32_t)(c / (lx - 1));
            /* original corners and their node indices */
            int32_t ci[3], cj[3];
            ci[0] = i; cj[0] = j;
            if ((t & 1) == 0) { ci[1] = i + 1; cj[1] = j; ci[2] = i + 1; cj[2] = j + 1; }
            else { ci[1] = i + 1; cj[1] = j + 1; ci[2] = i; cj[2] = j + 1; }
            double X[3], Y[3];
            for (int s = 0; s < 3; ++s) {
                const int64_t n = (int64_t)cj[s] * lx + ci[s];
                X[s] = nodes[2 * n];
                Y[s] = nodes[2 * n + 1];
            }
            const double o = orient2(X[0], Y[0], X[1], Y[1], X[2], Y[2]);
            if (o == 0.0) continue;
            const double d0 = orient2(X[1], Y[1], X[2], Y[2], qx, qy);
            const double d1 = orient2(X[2], Y[2], X[0], Y[0], qx, qy);
            const double d2 = orient2(X[0], Y[0], X[1], Y[1], qx, qy);
            const int inside = (o > 0.0) ? (d0 >= 0.0 && d1 >= 0.0 && d2 >= 0.0)
                                         : (d0 <= 0.0 && d1 <= 0.0 && d2 <= 0.0);
            if (!inside) continue;
            /* barycentric weights of q in the image, applied to the originals */
            const double l0 = d0 / o, l1 = d1 / o, l2 = d2 / o;
            double px = l0 * (ci[0] + 0.5);
            px += l1 * (ci[1] + 0.5);
            px += l2 * (ci[2] + 0.5);
            double py = l0 * (cj[0] + 0.5);
            py += l1 * (cj[1] + 0.5);
            py += l2 * (cj[2] + 0.5);
            tri[k] = (int32_t)t;
            pre[2 * k] = px;
            pre[2 * k + 1] = py;
            break;
        }
    }
    return O_OK;
}

/* ------------------------------------------------------------------------
 * Reverse mode of one round with the accepted step sizes frozen (the
 * gradient of a loss of the final areas with respect to the region
 * statistics).  Not part of the paper's method: written from the forward
 * definitions above by the chain rule, each function the transpose of the
 * linearised forward step it is named after.  Every function ADDS to its
 * output adjoints (lam_*), except ffbo_flux_adj, which writes lam_rho.
 * ---------------------------------------------------------------------- */

/* Areas: A_r = 1/2 sum_k (x_k y_{k+1} - x_{k+1} y_k) over the region's rings,
 * so dA/dx_k = (y_{k+1} - y_{k-1}) / 2 and dA/dy_k = (x_{k-1} - x_{k+1}) / 2. */
int ffbo_area_adj(int64_t nv, const double *xy, int32_t n_rings, const int32_t *ring_offsets,
                  const int32_t *ring_vidx, const int32_t *ring_region, int32_t n_regions,
                  const double *lam_area, double *lam_xy)
{
    int st = check_geometry(nv, n_rings, ring_offsets, ring_vidx, ring_region, n_regions);
    if (st) return st;
    for (int32_t g = 0; g < n_rings; ++g) {
        const int32_t b = ring_offsets[g], n = ring_offsets[g + 1] - b;
        const double l = lam_area[ring_region[g]];
        for (int32_t k = 0; k < n; ++k) {
            const int64_t p = ring_vidx[b + k];
            const double *prev = xy + 2 * (int64_t)ring_vidx[b + (k + n - 1) % n];
            const double *next = xy + 2 * (int64_t)ring_vidx[b + (k + 1) % n];
            lam_xy[2 * p] += 0.5 * l * (next[1] - prev[1]);
            lam_xy[2 * p + 1] += 0.5 * l * (prev[0] - next[0]);
        }
    }
    return O_OK;
}

/* Raster: rho_c = rho_pad + sum_r w_r cov_r(c), w_r = value_r / A_r - rho_pad,
 * rho_pad = sum(value) / sum(A), cov_r(c) the signed area of cell c inside
 * the region's rings.  With lam_w_r = sum_c lam_rho_c cov_r(c) (the integral
 * of the piecewise-constant lam over the region) and
 * lam_pad = sum_c lam_rho_c - sum_r lam_w_r:
 *   lam_value_r += lam_w_r / A_r + lam_pad / sum(A),
 *   lam_area_r  += -lam_w_r value_r / A_r^2 - lam_pad sum(value) / sum(A)^2.
 * Vertices: moving the end q of an edge p -> q (direction d = q - p, points
 * p + s d) moves each of its points by s dq, so the integral of lam over the
 * ring changes by (d_y, -d_x) . dq times the integral over s in [0, 1] of
 * lam(p + s d) s, and by the same with (1 - s) for the start p.  lam is
 * constant on the pieces of the edge between grid lines. */
static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int ffbo_density_adj(int32_t lx, int32_t ly, int64_t nv, const double *xy, int32_t n_rings,
                     const int32_t *ring_offsets, const int32_t *ring_vidx,
                     const int32_t *ring_region, int32_t n_regions, const double *value,
                     const double *area, const double *lam_rho, double *lam_value,
                     double *lam_area, double *lam_xy)
{
    if (lx <= 0 || ly <= 0) return O_E_INVALID;
    int st = check_geometry(nv, n_rings, ring_offsets, ring_vidx, ring_region, n_regions);
    if (st) return st;
    for (int64_t k = 0; k < nv; ++k) {
        double x = xy[2 * k], y = xy[2 * k + 1];
        if (!isfinite(x) || !isfinite(y)) return O_E_NONFINITE;
        if (x < 0.0 || x > lx || y < 0.0 || y > ly) return O_E_DOMAIN;
    }
    double sa = 0.0, sv = 0.0;
    for (int32_t r = 0; r < n_regions; ++r) {
        if (!(value[r] > 0.0) || !(area[r] > 0.0)) return O_E_NONPOSITIVE;
        sa += area[r];
        sv += value[r];
    }
    const double rho_pad = sv / sa;
    double *lam_w = (double *)calloc((size_t)n_regions, sizeof(double));
    if (!lam_w) return O_E_NOMEM;

    /* lam_w_r: the cell areas of the region's rings, clipped as in ffbo_density */
    int fail = 0;
    poly_t ring = {0}, t1 = {0}, band = {0}, t2 = {0}, cell = {0};
    for (int32_t g = 0; g < n_rings && !fail; ++g) {
        const int32_t b = ring_offsets[g], n = ring_offsets[g + 1] - b;
        if (poly_reserve(&ring, n)) { fail = 1; break; }
        double ylo = INFINITY, yhi = -INFINITY;
        for (int32_t k = 0; k < n; ++k) {
            ring.x[k] = xy[2 * (int64_t)ring_vidx[b + k]];
            ring.y[k] = xy[2 * (int64_t)ring_vidx[b + k] + 1];
            if (ring.y[k] < ylo) ylo = ring.y[k];
            if (ring.y[k] > yhi) yhi = ring.y[k];
        }
        ring.n = n;
        int32_t j0 = (int32_t)floor(ylo), j1 = (int32_t)ceil(yhi);
        if (j0 < 0) j0 = 0;
        if (j1 > ly) j1 = ly;
        double s = 0.0;
        for (int32_t j = j0; j < j1 && !fail; ++j) {
            if (clip_half(&ring, &t1, 1, (double)j, -1.0)) { fail = 1; break; }
            if (clip_half(&t1, &band, 1, (double)(j + 1), 1.0)) { fail = 1; break; }
            if (band.n < 3) continue;
            double xlo = INFINITY, xhi = -INFINITY;
            for (int32_t k = 0; k < band.n; ++k) {
                if (band.x[k] < xlo) xlo = band.x[k];
                if (band.x[k] > xhi) xhi = band.x[k];
            }
            int32_t i0 = (int32_t)floor(xlo), i1 = (int32_t)ceil(xhi);
            if (i0 < 0) i0 = 0;
            if (i1 > lx) i1 = lx;
            for (int32_t i = i0; i < i1; ++i) {
                if (clip_half(&band, &t2, 0, (double)i, -1.0)) { fail = 1; break; }
                if (clip_half(&t2, &cell, 0, (double)(i + 1), 1.0)) { fail = 1; break; }
                if (cell.n < 3) continue;
                s += lam_rho[(int64_t)j * lx + i] * poly_area(&cell, (double)i, (double)j);
            }
        }
        lam_w[ring_region[g]] += s;
    }
    free(ring.x); free(ring.y); free(t1.x); free(t1.y); free(band.x); free(band.y);
    free(t2.x); free(t2.y); free(cell.x); free(cell.y);
    if (fail) { free(lam_w); return O_E_NOMEM; }

    double lam_pad = 0.0;
    for (int64_t c = 0; c < (int64_t)lx * ly; ++c) lam_pad += lam_rho[c];
    for (int32_t r = 0; r < n_regions; ++r) lam_pad -= lam_w[r];
    for (int32_t r = 0; r < n_regions; ++r) {
        lam_value[r] += lam_w[r] / area[r] + lam_pad / sa;
        lam_area[r] += -lam_w[r] * value[r] / (area[r] * area[r]) - lam_pad * sv / (sa * sa);
    }

    /* vertices: boundary integrals of lam along every edge, weighted by w_r */
    double *cuts = NULL;
    int64_t cuts_cap = 0;
    for (int32_t g = 0; g < n_rings && !fail; ++g) {
        const int32_t b = ring_offsets[g], n = ring_offsets[g + 1] - b;
        const int32_t r = ring_region[g];
        const double w = value[r] / area[r] - rho_pad;
        for (int32_t k = 0; k < n; ++k) {
            const int64_t ip = ring_vidx[b + k], iq = ring_vidx[b + (k + 1) % n];
            const double px = xy[2 * ip], py = xy[2 * ip + 1];
            const double dx = xy[2 * iq] - px, dy = xy[2 * iq + 1] - py;
            /* parameters of the crossings with the grid lines, then the ends */
            const double xa = fmin(px, px + dx), xb = fmax(px, px + dx);
            const double ya = fmin(py, py + dy), yb = fmax(py, py + dy);
            const int64_t need = (int64_t)(floor(xb) - ceil(xa) + 1) +
                                 (int64_t)(floor(yb) - ceil(ya) + 1) + 2;
            if (need > cuts_cap) {
                double *nc = (double *)realloc(cuts, sizeof(double) * (size_t)need);
                if (!nc) { fail = 1; break; }
                cuts = nc;
                cuts_cap = need;
            }
            int64_t nc = 0;
            cuts[nc++] = 0.0;
            cuts[nc++] = 1.0;
            for (double X = ceil(xa); X <= xb; X += 1.0) {
                const double s = (X - px) / dx;
                if (dx != 0.0 && s > 0.0 && s < 1.0) cuts[nc++] = s;
            }
            for (double Y = ceil(ya); Y <= yb; Y += 1.0) {
                const double s = (Y - py) / dy;
                if (dy != 0.0 && s > 0.0 && s < 1.0) cuts[nc++] = s;
            }
            qsort(cuts, (size_t)nc, sizeof(double), cmp_double);
            double I0 = 0.0, I1 = 0.0;    /* integrals of lam (1 - s) and lam s */
            for (int64_t q = 0; q + 1 < nc; ++q) {
                const double s0 = cuts[q], s1 = cuts[q + 1];
                if (!(s1 > s0)) continue;
                const double sm = 0.5 * (s0 + s1);
                int32_t i = (int32_t)floor(px + sm * dx), j = (int32_t)floor(py + sm * dy);
                if (i < 0) i = 0;
                if (i > lx - 1) i = lx - 1;
                if (j < 0) j = 0;
                if (j > ly - 1) j = ly - 1;
                const double l = lam_rho[(int64_t)j * lx + i];
                const double m2 = 0.5 * (s1 * s1 - s0 * s0);
                I1 += l * m2;
                I0 += l * ((s1 - s0) - m2);
            }
            lam_xy[2 * ip] += w * dy * I0;
            lam_xy[2 * ip + 1] += -w * dx * I0;
            lam_xy[2 * iq] += w * dy * I1;
            lam_xy[2 * iq + 1] += -w * dx * I1;
        }
    }
    free(cuts);
    free(lam_w);
    return fail ? O_E_NOMEM : O_OK;
}

/* Flux series (ffbo_flux) transposed.  The forward is linear in rho:
 *   S = C_y C_x rho, rts = G o S, A = C_y^T rts, B = C_y^T (W_x o rts),
 *   C = S_y^T (W_y o rts), rho_s = C_x^T A / N, J_x = S_x^T B, J_y = C_x^T C,
 *   rho_bar = rts_00 / N,
 * with C_x[m][i] = cos(pi m (i+1/2)/lx), S_x[m][i] = sin(...), the same in y,
 * W_x = (ly/pi) m / (m^2 ly^2 + n^2 lx^2) (m > 0), W_y = (lx/pi) n / (...)
 * (n > 0) and G the Eq. 7 factor times the blur.  Its transpose:
 *   Abar = C_x lam_rs / N, Bbar = S_x lam_jx, Cbar = C_x lam_jy,
 *   rtsbar = C_y Abar + W_x o (C_y Bbar) + W_y o (S_y Cbar) (+ lam_rb / N at 00),
 *   lam_rho = C_x^T C_y^T (G o rtsbar).
 * Writes lam_rho [ly][lx]. */
int ffbo_flux_adj(int32_t lx, int32_t ly, double sigma, const double *lam_rs,
                  const double *lam_jx, const double *lam_jy, double lam_rb, double *lam_rho)
{
    if (lx <= 0 || ly <= 0 || !(sigma >= 0.0)) return O_E_INVALID;
    const int64_t N = (int64_t)lx * ly;
    double *A = (double *)malloc(sizeof(double) * N);
    double *B = (double *)malloc(sizeof(double) * N);
    double *C = (double *)malloc(sizeof(double) * N);
    double *R = (double *)malloc(sizeof(double) * N);
    double *T = (double *)malloc(sizeof(double) * N);
    double *tx = make_table(lx), *ty = make_table(ly);
    if (!A || !B || !C || !R || !T || !tx || !ty) {
        free(A); free(B); free(C); free(R); free(T); free(tx); free(ty);
        return O_E_NOMEM;
    }
    const double LX = lx, LY = ly;
    /* along x: Abar[j][m], Bbar[j][m], Cbar[j][m] */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t m = 0; m < lx; ++m) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t i = 0; i < lx; ++i) {
                const int64_t q = (int64_t)j * lx + i;
                const double cx = tcos(tx, lx, m, i), sx = tsin(tx, lx, m, i);
                a += lam_rs[q] * cx;
                b += lam_jx[q] * sx;
                c += lam_jy[q] * cx;
            }
            A[(int64_t)j * lx + m] = a / (double)N;
            B[(int64_t)j * lx + m] = b;
            C[(int64_t)j * lx + m] = c;
        }
    /* along y: rtsbar[n][m], times G */
#pragma omp parallel for schedule(static)
    for (int32_t n = 0; n < ly; ++n)
        for (int32_t m = 0; m < lx; ++m) {
            double a = 0.0, b = 0.0, c = 0.0;
            for (int32_t j = 0; j < ly; ++j) {
                const int64_t q = (int64_t)j * lx + m;
                const double cy = tcos(ty, ly, n, j), sy = tsin(ty, ly, n, j);
                a += A[q] * cy;
                b += B[q] * cy;
                c += C[q] * sy;
            }
            const double den = (double)m * m * LY * LY + (double)n * n * LX * LX;
            double rb = a;
            if (m > 0) rb += (LY / PI) * ((double)m / den) * b;
            if (n > 0) rb += (LX / PI) * ((double)n / den) * c;
            if (m == 0 && n == 0) rb += lam_rb / (double)N;
            const double f = 4.0 / ((m == 0 ? 2.0 : 1.0) * (n == 0 ? 2.0 : 1.0));
            const double k2 = (double)m * m / (LX * LX) + (double)n * n / (LY * LY);
            R[(int64_t)n * lx + m] = rb * f * exp(-PI * PI * sigma * sigma * k2 / 2.0);
        }
    /* lam_rho = C_x^T C_y^T R: first over n, then over m */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t m = 0; m < lx; ++m) {
            double s = 0.0;
            for (int32_t n = 0; n < ly; ++n) s += R[(int64_t)n * lx + m] * tcos(ty, ly, n, j);
            T[(int64_t)j * lx + m] = s;
        }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ly; ++j)
        for (int32_t i = 0; i < lx; ++i) {
            double s = 0.0;
            for (int32_t m = 0; m < lx; ++m) s += T[(int64_t)j * lx + m] * tcos(tx, lx, m, i);
            lam_rho[(int64_t)j * lx + i] = s;
        }
    free(A); free(B); free(C); free(R); free(T); free(tx); free(ty);
    return O_OK;
}

/* One velocity lookup (velocity_at) and its transpose: given kbar, the
 * adjoint of the returned v, add to the node field adjoints and return the
 * adjoint of the position (zero in a clamped coordinate).  With the node
 * velocities v_n = (s_x J_x, s_y J_y)_c / rt_c, rt_c = (1 - t) rho_s_c +
 * t rho_bar (ghost nodes mirror an inside node c with signs s_x, s_y) and
 * the bilinear weights w_n:  dv/dJ_x,c = w_n s_x / rt_c (x component),
 * dv/drho_s,c = -w_n v_n (1 - t) / rt_c, dv/drho_bar = -w_n v_n t / rt_c. */
typedef struct { double *rs, *jx, *jy, rb; } field_adj_t;

static void velocity_at_adj(const field_t *F, double t, double qx, double qy, double kbx,
                            double kby, field_adj_t *G, double *qbx, double *qby)
{
    const int inx = qx > 0.0 && qx < F->lx, iny = qy > 0.0 && qy < F->ly;
    if (qx < 0.0) qx = 0.0;
    if (qx > F->lx) qx = F->lx;
    if (qy < 0.0) qy = 0.0;
    if (qy > F->ly) qy = F->ly;
    const double u = qx - 0.5, w = qy - 0.5;
    const double fu = floor(u), fw = floor(w);
    const int32_t i0 = (int32_t)fu, j0 = (int32_t)fw;
    const double a = u - fu, b = w - fw;
    double vx[4], vy[4];
    const double wt[4] = {(1 - a) * (1 - b), a * (1 - b), (1 - a) * b, a * b};
    for (int q = 0; q < 4; ++q) {
        int32_t i = i0 + (q & 1), j = j0 + (q >> 1);
        double sx = 1.0, sy = 1.0;
        if (i < 0) { i = 0; sx = -sx; }
        if (i >= F->lx) { i = F->lx - 1; sx = -sx; }
        if (j < 0) { j = 0; sy = -sy; }
        if (j >= F->ly) { j = F->ly - 1; sy = -sy; }
        const int64_t c = (int64_t)j * F->lx + i;
        const double rt = (1.0 - t) * F->rho_s[c] + t * F->rho_bar;
        vx[q] = sx * F->jx[c] / rt;
        vy[q] = sy * F->jy[c] / rt;
        const double dot = kbx * vx[q] + kby * vy[q];
        G->jx[c] += wt[q] * kbx * sx / rt;
        G->jy[c] += wt[q] * kby * sy / rt;
        G->rs[c] += -wt[q] * dot * (1.0 - t) / rt;
        G->rb += -wt[q] * dot * t / rt;
    }
    /* dv/dq_x = (1 - b)(v_10 - v_00) + b (v_11 - v_01), dv/dq_y likewise */
    const double dxx = (1 - b) * (vx[1] - vx[0]) + b * (vx[3] - vx[2]);
    const double dxy = (1 - b) * (vy[1] - vy[0]) + b * (vy[3] - vy[2]);
    const double dyx = (1 - a) * (vx[2] - vx[0]) + a * (vx[3] - vx[1]);
    const double dyy = (1 - a) * (vy[2] - vy[0]) + a * (vy[3] - vy[1]);
    *qbx = inx ? kbx * dxx + kby * dxy : 0.0;
    *qby = iny ? kbx * dyx + kby * dyy : 0.0;
}

/* The integration from t = 0 with the given accepted steps h[0..S) (as
 * ffbo_integrate replays them: stage s of a step at y evaluates v at
 * Y_s = y + h sum_{q<s} a_sq k_q and time t + c_s h, the step ends at
 * y + h sum_s b_s k_s), transposed.  lam_xy [n][2]: in, dL/dy at the end;
 * out, dL/dy at the start.  The field adjoints lam_rs, lam_jx, lam_jy
 * ([ly][lx]) and *lam_rb are added to.  The states before every step are
 * recomputed and kept (n * S * 2 doubles). */
int ffbo_integrate_adj(int32_t lx, int32_t ly, const double *rho_s, const double *jx,
                       const double *jy, double rho_bar, int64_t n, const double *xy0,
                       const double *h, int32_t S, double *lam_xy, double *lam_rs,
                       double *lam_jx, double *lam_jy, double *lam_rb)
{
    if (lx <= 0 || ly <= 0 || n < 0 || S < 0 || !(rho_bar > 0.0)) return O_E_INVALID;
    const field_t F = {lx, ly, rho_s, jx, jy, rho_bar};
    double *ys = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1) * (size_t)(S + 1));
    double *ts = (double *)malloc(sizeof(double) * (size_t)(S + 1));
    if (!ys || !ts) { free(ys); free(ts); return O_E_NOMEM; }
    /* forward: the state before every step and the step start times */
    memcpy(ys, xy0, sizeof(double) * 2 * (size_t)n);
    double t = 0.0;
    for (int32_t s = 0; s < S; ++s) {
        ts[s] = t;
        const double *y = ys + 2 * (size_t)n * s;
        double *y1 = ys + 2 * (size_t)n * (s + 1);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            double kx[6], ky[6];
            double ex = y[2 * p], ey = y[2 * p + 1];
            for (int q = 0; q < 6; ++q) {
                double qx = y[2 * p], qy = y[2 * p + 1];
                for (int r = 0; r < q; ++r) {
                    qx += h[s] * DP_A[q][r] * kx[r];
                    qy += h[s] * DP_A[q][r] * ky[r];
                }
                velocity_at(&F, t + DP_C[q] * h[s], qx, qy, &kx[q], &ky[q]);
            }
            for (int q = 0; q < 6; ++q) {
                ex += h[s] * DP_A[6][q] * kx[q];
                ey += h[s] * DP_A[6][q] * ky[q];
            }
            y1[2 * p] = ex;
            y1[2 * p + 1] = ey;
        }
        t = (s == S - 1) ? 1.0 : t + h[s];
    }
    /* reverse: per point, the steps last to first; field adjoints are summed
     * in one buffer per thread and added up at the end */
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    const int64_t NF = (int64_t)lx * ly;
    double *acc = (double *)calloc((size_t)nt * 3 * (size_t)NF, sizeof(double));
    double *acc_rb = (double *)calloc((size_t)nt, sizeof(double));
    if (!acc || !acc_rb) { free(acc); free(acc_rb); free(ys); free(ts); return O_E_NOMEM; }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        field_adj_t G;
        G.rs = acc + (size_t)tid * 3 * (size_t)NF;
        G.jx = G.rs + NF;
        G.jy = G.jx + NF;
        G.rb = 0.0;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            double lx_ = lam_xy[2 * p], ly_ = lam_xy[2 * p + 1];
            for (int32_t s = S - 1; s >= 0; --s) {
                const double *y = ys + 2 * (size_t)n * s;
                const double hs = h[s];
                double kx[6], ky[6], Qx[6], Qy[6];
                for (int q = 0; q < 6; ++q) {
                    double qx = y[2 * p], qy = y[2 * p + 1];
                    for (int r = 0; r < q; ++r) {
                        qx += hs * DP_A[q][r] * kx[r];
                        qy += hs * DP_A[q][r] * ky[r];
                    }
                    Qx[q] = qx;
                    Qy[q] = qy;
                    velocity_at(&F, ts[s] + DP_C[q] * hs, qx, qy, &kx[q], &ky[q]);
                }
                /* kbar_q = h b_q lam' + h sum_{r>q} a_rq Ybar_r, Ybar_q = Jv_q^T kbar_q */
                double Yx[6], Yy[6];
                double nx = lx_, ny = ly_;
                for (int q = 5; q >= 0; --q) {
                    double kbx = hs * DP_A[6][q] * lx_, kby = hs * DP_A[6][q] * ly_;
                    for (int r = q + 1; r < 6; ++r) {
                        kbx += hs * DP_A[r][q] * Yx[r];
                        kby += hs * DP_A[r][q] * Yy[r];
                    }
                    velocity_at_adj(&F, ts[s] + DP_C[q] * hs, Qx[q], Qy[q], kbx, kby, &G,
                                    &Yx[q], &Yy[q]);
                    nx += Yx[q];
                    ny += Yy[q];
                }
                lx_ = nx;
                ly_ = ny;
            }
            lam_xy[2 * p] = lx_;
            lam_xy[2 * p + 1] = ly_;
        }
        acc_rb[tid] = G.rb;
    }
    for (int k = 0; k < nt; ++k) {
        const double *a = acc + (size_t)k * 3 * (size_t)NF;
        for (int64_t c = 0; c < NF; ++c) {
            lam_rs[c] += a[c];
            lam_jx[c] += a[NF + c];
            lam_jy[c] += a[2 * NF + c];
        }
        *lam_rb += acc_rb[k];
    }
    free(acc);
    free(acc_rb);
    free(ys);
    free(ts);
    return O_OK;
}
