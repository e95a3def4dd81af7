/*
 * rs_oracle.c -- plain, slow FP64 CPU oracle for inverse ray-shooting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Thompson, Fluke, Barnes & Barsdell 2009):
 *   - lens equation y = x - alpha(x)                           (section 1, eq. 1)
 *   - many-Schwarzschild deflection
 *       alpha(x) = sum_i m_i (x - x_i) / |x - x_i|^2            (section 1, eq. 2)
 *     summed in FP64, in lens-index order, with the operation split of
 *     appendix A: f = x - x_i, d = m_i / (f1 f1 + f2 f2), alpha += d f;
 *   - macro model with external shear gamma and smooth convergence
 *     sigma_c (= kappa_c): y = diag(1-gamma, 1+gamma) x - kappa_c x - alpha
 *                                                               (section 3.2, eq. 6)
 *     grouped as lambda_1 = (1 - gamma) - kappa_c, lambda_2 = (1 + gamma) - kappa_c;
 *   - inverse ray-shooting estimator: each ray adds one count to the source
 *     pixel it lands in; mu_ij = N_ij / N_av                  (section 1, eq. 4).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - rays sit one per cell of a regular grid, at the cell centre (offset
 *     u = 1/2) or, with jitter on, at a seeded uniform point of the cell (the
 *     paper draws ray positions at random, sections 2.1-2.2); coordinate i
 *     along an axis is the float32 rounding of lo + (i + u) (hi - lo) / n,
 *     evaluated in FP64 as t = (hi-lo)/n; v = (i+u)*t; w = lo+v with no
 *     contraction.  The offset of the ray of cell (i1, i2), r = i2 n1 + i1,
 *     along axis k (stream s = 8, 9) is u = (h >> 11) 2^-53 with
 *     h = mix(mix(seed G ^ (s << 32)) + (r + 1) G), G = 0x9E3779B97F4A7C15,
 *     mix = the SplitMix64 output function (Steele, Lea & Flood 2014);
 *   - pixels are half-open: p_k = floor((y_k - lo_k) * (n_k / (hi_k - lo_k)));
 *     a ray is counted iff y is finite and 0 <= p_k < n_k, otherwise it is
 *     "lost" (this includes a ray exactly on a lens, whose deflection is NaN);
 *   - lens records are float32 (x1, x2, m, pad), promoted exactly to FP64.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC.
 * Every function is single-threaded and re-entrant (callers may run several
 * disjoint windows in parallel threads).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* SplitMix64 output function, 64-bit wrapping. */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Offset in [0, 1) of the ray with grid index r along axis k (0 or 1) under seed. */
double orc_jitter_u(uint64_t seed, int k, int64_t r)
{
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t key = orc_mix64((seed * G) ^ ((uint64_t)(8 + k) << 32));
    uint64_t h = orc_mix64(key + (uint64_t)(r + 1) * G);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* Ray coordinate i of an axis [lo, hi) split into n cells, at offset u of the cell. */
static float orc_coord_u(double lo, double hi, int64_t n, int64_t i, double u)
{
    double t = (hi - lo) / (double)n;
    double v = ((double)i + u) * t;
    double w = lo + v;
    return (float)w;
}

static float orc_coord(double lo, double hi, int64_t n, int64_t i)
{
    return orc_coord_u(lo, hi, n, i, 0.5);
}

/* Both coordinates of grid ray (i1, i2); jitter 0 = cell centre. */
static void orc_ray(const double *glo, const double *ghi, const int64_t *gn, uint64_t seed, int jitter,
                    int64_t i1, int64_t i2, double *x1, double *x2)
{
    double u1 = 0.5, u2 = 0.5;
    if (jitter) {
        int64_t r = i2 * gn[0] + i1;
        u1 = orc_jitter_u(seed, 0, r);
        u2 = orc_jitter_u(seed, 1, r);
    }
    *x1 = (double)orc_coord_u(glo[0], ghi[0], gn[0], i1, u1);
    *x2 = (double)orc_coord_u(glo[1], ghi[1], gn[1], i2, u2);
}

/* Fill out[j] = coordinate (i0 + j) of the axis, j = 0 .. count-1. */
void orc_axis(double lo, double hi, int64_t n, int64_t i0, int64_t count, float *out)
{
    for (int64_t j = 0; j < count; ++j)
        out[j] = orc_coord(lo, hi, n, i0 + j);
}

/* Deflection (eq. 2) at (x1, x2) from lenses[0 .. n_lens-1], FP64, index order. */
static void orc_alpha(const float *lenses, int64_t n_lens, double x1, double x2,
                      double *a1, double *a2)
{
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < n_lens; ++i) {
        double f1 = x1 - (double)lenses[4 * i + 0];
        double f2 = x2 - (double)lenses[4 * i + 1];
        double d = (double)lenses[4 * i + 2] / (f1 * f1 + f2 * f2);
        s1 += d * f1;
        s2 += d * f2;
    }
    *a1 = s1;
    *a2 = s2;
}

/* Deflection at arbitrary FP64 points: pts and alpha are n_pts x 2. */
void orc_deflect_points(const float *lenses, int64_t n_lens, const double *pts, int64_t n_pts,
                        double *alpha)
{
    for (int64_t p = 0; p < n_pts; ++p)
        orc_alpha(lenses, n_lens, pts[2 * p], pts[2 * p + 1], &alpha[2 * p], &alpha[2 * p + 1]);
}

/* Source pixel of a source-plane point; -1 when the ray is lost. */
static int64_t orc_pixel(double y1, double y2, const double *mlo, const double *mhi,
                         const int32_t *mn)
{
    double s1 = (double)mn[0] / (mhi[0] - mlo[0]);
    double s2 = (double)mn[1] / (mhi[1] - mlo[1]);
    double f1 = floor((y1 - mlo[0]) * s1);
    double f2 = floor((y2 - mlo[1]) * s2);
    if (!(f1 >= 0.0 && f1 < (double)mn[0])) return -1;
    if (!(f2 >= 0.0 && f2 < (double)mn[1])) return -1;
    return (int64_t)f2 * (int64_t)mn[0] + (int64_t)f1;
}

/*
 * Trace the grid rays whose linear indices (i2 * n1 + i1 over the full grid)
 * are listed in ray_idx: y (n x 2, FP64) and the pixel (-1 = lost).
 */
void orc_trace(const float *lenses, int64_t n_lens, double kappa_c, double gamma,
               const double *glo, const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter,
               const double *mlo, const double *mhi, const int32_t *mn,
               const int64_t *ray_idx, int64_t n_rays, double *y, int64_t *pix)
{
    double lam1 = (1.0 - gamma) - kappa_c;
    double lam2 = (1.0 + gamma) - kappa_c;
    for (int64_t r = 0; r < n_rays; ++r) {
        int64_t i1 = ray_idx[r] % gn[0];
        int64_t i2 = ray_idx[r] / gn[0];
        double x1, x2;
        orc_ray(glo, ghi, gn, jitter_seed, jitter, i1, i2, &x1, &x2);
        double a1, a2;
        orc_alpha(lenses, n_lens, x1, x2, &a1, &a2);
        double y1 = lam1 * x1 - a1;
        double y2 = lam2 * x2 - a2;
        y[2 * r] = y1;
        y[2 * r + 1] = y2;
        pix[r] = orc_pixel(y1, y2, mlo, mhi, mn);
    }
}

/* Float32 ray positions (n x 2) of the listed grid rays (linear index i2 * n1 + i1). */
void orc_ray_positions(const double *glo, const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter,
                       const int64_t *ray_idx, int64_t n_rays, float *xy)
{
    for (int64_t r = 0; r < n_rays; ++r) {
        double x1, x2;
        orc_ray(glo, ghi, gn, jitter_seed, jitter, ray_idx[r] % gn[0], ray_idx[r] / gn[0], &x1, &x2);
        xy[2 * r] = (float)x1;
        xy[2 * r + 1] = (float)x2;
    }
}

/*
 * Shoot the window [wlo, wlo + wn) of the grid (row-major, axis 1 fastest)
 * and ADD its counts into counts[mn1 * mn0] (row-major, axis 1 fastest);
 * lost rays are added to *lost.  Returns the number of rays shot.
 */
int64_t orc_shoot(const float *lenses, int64_t n_lens, double kappa_c, double gamma,
                  const double *glo, const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter,
                  const int64_t *wlo, const int64_t *wn,
                  const double *mlo, const double *mhi, const int32_t *mn,
                  uint32_t *counts, uint64_t *lost)
{
    double lam1 = (1.0 - gamma) - kappa_c;
    double lam2 = (1.0 + gamma) - kappa_c;
    int64_t shot = 0;
    for (int64_t i2 = wlo[1]; i2 < wlo[1] + wn[1]; ++i2) {
        for (int64_t i1 = wlo[0]; i1 < wlo[0] + wn[0]; ++i1) {
            double x1, x2;
            orc_ray(glo, ghi, gn, jitter_seed, jitter, i1, i2, &x1, &x2);
            double a1, a2;
            orc_alpha(lenses, n_lens, x1, x2, &a1, &a2);
            int64_t p = orc_pixel(lam1 * x1 - a1, lam2 * x2 - a2, mlo, mhi, mn);
            if (p >= 0) counts[p] += 1u;
            else *lost += 1u;
            ++shot;
        }
    }
    return shot;
}
