/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the C oracle (test
 * infrastructure): it calls every entry point of oracle/rs_oracle.c on small inputs, including
 * the edge cases (no lenses, an empty window, a ray exactly on a lens, rays leaving the map,
 * ragged windows, jittered rays), and checks ray conservation.  Built and run by
 * tests/test_oracle_sanitize.py; any invalid access or undefined operation aborts the run.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t orc_mix64(uint64_t z);
double orc_jitter_u(uint64_t seed, int k, int64_t r);
void orc_axis(double lo, double hi, int64_t n, int64_t i0, int64_t count, float *out);
void orc_deflect_points(const float *lenses, int64_t n_lens, const double *pts, int64_t n_pts, double *out);
void orc_trace(const float *lenses, int64_t n_lens, double kappa_c, double gamma, const double *glo,
               const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter, const double *mlo,
               const double *mhi, const int32_t *mn, const int64_t *ray_idx, int64_t n_rays, double *y,
               int64_t *pix);
void orc_ray_positions(const double *glo, const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter,
                       const int64_t *ray_idx, int64_t n_rays, float *xy);
int64_t orc_shoot(const float *lenses, int64_t n_lens, double kappa_c, double gamma, const double *glo,
                  const double *ghi, const int64_t *gn, uint64_t jitter_seed, int jitter, const int64_t *wlo,
                  const int64_t *wn, const double *mlo, const double *mhi, const int32_t *mn, uint32_t *counts,
                  uint64_t *lost);

static int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                               \
        }                                                          \
    } while (0)

int main(void)
{
    /* three lenses; the grid's cell centre (i1, i2) = (2, 3) of a 9 x 7 grid on [-1,1]^2 is on lens 0 */
    const double glo[2] = {-1.0, -1.0}, ghi[2] = {1.0, 1.0};
    const int64_t gn[2] = {9, 7};
    float ax[9], ay[7];
    orc_axis(glo[0], ghi[0], gn[0], 0, gn[0], ax);
    orc_axis(glo[1], ghi[1], gn[1], 0, gn[1], ay);
    const float lenses[12] = {ax[2], ay[3], 1.0f, 0.0f, 0.37f, -0.61f, 0.5f, 0.0f, 5.0f, 5.0f, 0.25f, 0.0f};
    const double mlo[2] = {-2.0, -1.5}, mhi[2] = {2.0, 1.5};
    const int32_t mn[2] = {13, 5};
    uint32_t *counts = calloc((size_t)mn[0] * mn[1], sizeof *counts);
    uint64_t lost = 0;

    for (int jit = 0; jit < 2; ++jit) {
        for (int nl = 0; nl <= 3; ++nl) {
            const int64_t wlo[2] = {1, 2}, wn[2] = {7, 4};
            lost = 0;
            for (int64_t i = 0; i < (int64_t)mn[0] * mn[1]; ++i) counts[i] = 0;
            int64_t shot = orc_shoot(lenses, nl, 0.1, 0.2, glo, ghi, gn, 12345u, jit, wlo, wn, mlo, mhi, mn,
                                     counts, &lost);
            uint64_t sum = lost;
            for (int64_t i = 0; i < (int64_t)mn[0] * mn[1]; ++i) sum += counts[i];
            CHECK(shot == wn[0] * wn[1] && sum == (uint64_t)shot);
            /* an empty window shoots nothing */
            const int64_t wz[2] = {0, 3};
            CHECK(orc_shoot(lenses, nl, 0.0, 0.0, glo, ghi, gn, 1u, jit, wlo, wz, mlo, mhi, mn, counts, &lost) == 0);
        }
        /* every ray of the grid, traced one by one */
        const int64_t n = gn[0] * gn[1];
        int64_t *idx = malloc((size_t)n * sizeof *idx);
        double *y = malloc((size_t)n * 2 * sizeof *y);
        int64_t *pix = malloc((size_t)n * sizeof *pix);
        float *xy = malloc((size_t)n * 2 * sizeof *xy);
        for (int64_t i = 0; i < n; ++i) idx[i] = n - 1 - i;
        orc_trace(lenses, 3, 0.0, 0.0, glo, ghi, gn, 99u, jit, mlo, mhi, mn, idx, n, y, pix);
        orc_ray_positions(glo, ghi, gn, 99u, jit, idx, n, xy);
        for (int64_t i = 0; i < n; ++i) CHECK(pix[i] >= -1 && pix[i] < (int64_t)mn[0] * mn[1]);
        if (!jit) CHECK(pix[n - 1 - (3 * gn[0] + 2)] == -1);   /* the ray on lens 0 is lost */
        free(idx);
        free(y);
        free(pix);
        free(xy);
    }
    double pts[4] = {0.0, 0.0, 5.0, 5.0}, out[4];
    orc_deflect_points(lenses, 3, pts, 2, out);
    CHECK(isfinite(out[0]) && isfinite(out[1]) && !isfinite(out[2] + out[3]));
    CHECK(orc_mix64(0) == orc_mix64(0) && orc_jitter_u(1, 0, 5) >= 0.0 && orc_jitter_u(1, 1, 5) < 1.0);
    free(counts);
    printf("oracle driver: %s\n", fails ? "FAILED" : "ok");
    return fails ? 1 : 0;
}
