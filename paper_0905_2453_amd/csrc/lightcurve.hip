// Light curves from a magnification map: a source profile moved along straight tracks across
// the map, giving at each point the profile-weighted magnification (eq. 4 per pixel) and the
// magnitude change (section 1, the light-curve use of the maps).
#include <cmath>

#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kLcWaves = 4;
constexpr int kLcAxis = 128;   // support bounding-box side staged in LDS per wave

__device__ inline double wave_sum(double v)
{
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
    return v;
}

// One wave per track point.  Lane l takes the bounding-box pixels e = l, l + 64, ... (row-major)
// and the wave then reduces in a fixed butterfly order, so a result depends only on its inputs.
// A Gaussian weight is separable, exp(-(d1^2 + d2^2) / 2 s^2) = g(d1) g(d2): each wave stages the
// squared offsets and the one-axis factors of its box's columns and rows in LDS, leaving one
// product per pixel.  The inclusion test d1^2 + d2^2 <= R^2 uses the same FP64 expressions as the
// plain definition.  Boxes wider than the staging area take the per-pixel path.
__global__ void __launch_bounds__(64 * kLcWaves) k_light_curve(const LightArgs a)
{
    __shared__ double2 s_col[kLcWaves][kLcAxis];   // (d1^2, g(d1)) per box column
    __shared__ double2 s_row[kLcWaves][kLcAxis];   // (d2^2, g(d2)) per box row
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t gp = (int64_t)blockIdx.x * kLcWaves + wv;
    const bool active = gp < (int64_t)a.n_tracks * a.n_points;
    int64_t tr = 0;
    int k = 0;
    if (active) {
        if (gp < 0x7fffffff) {
            tr = (uint32_t)gp / (uint32_t)a.n_points;
            k = (int)((uint32_t)gp - (uint32_t)tr * (uint32_t)a.n_points);
        } else {
            tr = gp / a.n_points;
            k = (int)(gp - tr * a.n_points);
        }
    }
    const double *t = a.tracks + 4 * tr;
    const double f = a.n_points > 1 ? (double)k / (double)(a.n_points - 1) : 0.0;
    const double ys1 = t[0] + f * (t[2] - t[0]);
    const double ys2 = t[1] + f * (t[3] - t[1]);
    const double rs = a.support, rs2 = a.support * a.support;
    const double inv2s2 = a.inv2s2;
    const bool gauss = a.kind == 0;
    // Bounding box of the support in pixel indices, clamped to the map.  A pixel inside the
    // support has (p + 1/2) w >= y - R - lo, so p >= floor((y - R - lo) / w) with half a pixel to
    // spare: multiplying by a rounded 1/w cannot push the floor past a pixel that is inside
    // (and symmetrically at the upper end); the inclusion test below decides exactly.
    const double q1lo = floor((ys1 - rs - a.lo[0]) * a.inv_w[0]), q1hi = floor((ys1 + rs - a.lo[0]) * a.inv_w[0]);
    const double q2lo = floor((ys2 - rs - a.lo[1]) * a.inv_w[1]), q2hi = floor((ys2 + rs - a.lo[1]) * a.inv_w[1]);
    const int p1lo = (int)fmax(0.0, fmin(q1lo, (double)a.n[0]));
    const int p1hi = (int)fmax(-1.0, fmin(q1hi, (double)a.n[0] - 1));
    const int p2lo = (int)fmax(0.0, fmin(q2lo, (double)a.n[1]));
    const int p2hi = (int)fmax(-1.0, fmin(q2hi, (double)a.n[1] - 1));
    const int nx = active ? p1hi - p1lo + 1 : 0, ny = active ? p2hi - p2lo + 1 : 0;
    const bool staged = nx <= kLcAxis && ny <= kLcAxis;
    if (staged) {
        for (int c = lane; c < nx; c += 64) {
            const double d = (a.lo[0] + ((double)(p1lo + c) + 0.5) * a.w[0]) - ys1;
            const double d2 = d * d;
            s_col[wv][c] = make_double2(d2, gauss ? exp(-d2 * inv2s2) : 1.0);
        }
        for (int r = lane; r < ny; r += 64) {
            const double d = (a.lo[1] + ((double)(p2lo + r) + 0.5) * a.w[1]) - ys2;
            const double d2 = d * d;
            s_row[wv][r] = make_double2(d2, gauss ? exp(-d2 * inv2s2) : 1.0);
        }
    }
    __syncthreads();
    double num = 0.0, den = 0.0;
    if (nx > 0 && ny > 0) {
        if (staged) {
            const int total = nx * ny;
            // e = dr * nx + dc, advanced by 64 without a division per pixel
            int dr = lane / nx, dc = lane - (lane / nx) * nx;
            const int sr = 64 / nx, sc = 64 - (64 / nx) * nx;
            const uint32_t *base = a.counts + (int64_t)k * a.frame_stride + (int64_t)p2lo * a.n[0] + p1lo;
            for (int e = lane; e < total; e += 64) {
                const double2 cx = s_col[wv][dc], ry = s_row[wv][dr];
                if (cx.x + ry.x <= rs2) {
                    const double n = (double)base[(int64_t)dr * a.n[0] + dc];
                    if (gauss) {
                        const double wgt = cx.y * ry.y;
                        num += wgt * n;
                        den += wgt;
                    } else {
                        num += n;
                        den += 1.0;
                    }
                }
                dc += sc;
                dr += sr;
                if (dc >= nx) {
                    dc -= nx;
                    ++dr;
                }
            }
        } else {
            const int64_t total = (int64_t)nx * ny;
            for (int64_t e = lane; e < total; e += 64) {
                const int r = (int)(e / nx);
                const int p1 = p1lo + (int)(e - (int64_t)r * nx), p2 = p2lo + r;
                const double d1 = (a.lo[0] + ((double)p1 + 0.5) * a.w[0]) - ys1;
                const double d2 = (a.lo[1] + ((double)p2 + 0.5) * a.w[1]) - ys2;
                const double d2s = d1 * d1 + d2 * d2;
                if (d2s <= rs2) {
                    const double wgt = gauss ? exp(-d2s * inv2s2) : 1.0;
                    num += wgt * (double)a.counts[(int64_t)k * a.frame_stride + (int64_t)p2 * a.n[0] + p1];
                    den += wgt;
                }
            }
        }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (active && lane == 0) {
        const double mu = den > 0.0 ? num / (den * a.n_av) : __builtin_nan("");
        if (a.mu) a.mu[gp] = mu;
        if (a.mag) a.mag[gp] = -2.5 * log10(mu);
    }
}

// One lane per track point (used when there are many points with small supports): the lane
// walks its support box row by row, so no cross-lane reduction or staging is needed and
// consecutive lanes (consecutive points of a track) read neighbouring pixels.  The Gaussian
// factors along a row and down a column follow the exact recurrences
//   g(d + w) = g(d) r(d),  r(d + w) = r(d) exp(-w^2 / s^2),  r(d) = exp(-(2 d w + w^2) / 2 s^2),
// three FP64 multiplies per pixel instead of an exp; the inclusion test uses the same FP64
// expressions as the plain definition.
__global__ void __launch_bounds__(256) k_light_curve_lanes(const LightArgs a)
{
    const int64_t gp = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gp >= (int64_t)a.n_tracks * a.n_points) return;
    const int64_t tr = gp / a.n_points;
    const int k = (int)(gp - tr * a.n_points);
    const double *t = a.tracks + 4 * tr;
    const double f = a.n_points > 1 ? (double)k / (double)(a.n_points - 1) : 0.0;
    const double ys1 = t[0] + f * (t[2] - t[0]);
    const double ys2 = t[1] + f * (t[3] - t[1]);
    const double rs = a.support, rs2 = a.support * a.support;
    const bool gauss = a.kind == 0;
    const double q1lo = floor((ys1 - rs - a.lo[0]) * a.inv_w[0]), q1hi = floor((ys1 + rs - a.lo[0]) * a.inv_w[0]);
    const double q2lo = floor((ys2 - rs - a.lo[1]) * a.inv_w[1]), q2hi = floor((ys2 + rs - a.lo[1]) * a.inv_w[1]);
    const int p1lo = (int)fmax(0.0, fmin(q1lo, (double)a.n[0]));
    const int p1hi = (int)fmax(-1.0, fmin(q1hi, (double)a.n[0] - 1));
    const int p2lo = (int)fmax(0.0, fmin(q2lo, (double)a.n[1]));
    const int p2hi = (int)fmax(-1.0, fmin(q2hi, (double)a.n[1] - 1));
    double num = 0.0, den = 0.0;
    if (p1hi >= p1lo && p2hi >= p2lo) {
        const double w1 = a.w[0], w2 = a.w[1], h = a.inv2s2;
        // the recurrences stay finite while every exponent is moderate; otherwise (a source much
        // narrower than a pixel) each weight takes its own exp
        const double ext = rs + 2.0 * fmax(w1, w2);
        const bool rec = gauss && ext * ext * h < 600.0 && 2.0 * ext * fmax(w1, w2) * h < 600.0;
        const double dx0 = (a.lo[0] + ((double)p1lo + 0.5) * w1) - ys1;
        const double gx0 = rec ? exp(-dx0 * dx0 * h) : 1.0;
        const double rx0 = rec ? exp(-(2.0 * dx0 * w1 + w1 * w1) * h) : 1.0;
        const double kx = rec ? exp(-2.0 * w1 * w1 * h) : 1.0;
        const double dy0 = (a.lo[1] + ((double)p2lo + 0.5) * w2) - ys2;
        double gy = rec ? exp(-dy0 * dy0 * h) : 1.0;
        double ry = rec ? exp(-(2.0 * dy0 * w2 + w2 * w2) * h) : 1.0;
        const double ky = rec ? exp(-2.0 * w2 * w2 * h) : 1.0;
        for (int p2 = p2lo; p2 <= p2hi; ++p2) {
            const double dy = (a.lo[1] + ((double)p2 + 0.5) * w2) - ys2;
            const double dy2 = dy * dy;
            const uint32_t *row = a.counts + (int64_t)k * a.frame_stride + (int64_t)p2 * a.n[0];
            double gx = gx0, rx = rx0;
            for (int p1 = p1lo; p1 <= p1hi; ++p1) {
                const double dx = (a.lo[0] + ((double)p1 + 0.5) * w1) - ys1;
                const double d2s = dx * dx + dy2;
                if (d2s <= rs2) {
                    const double n = (double)row[p1];
                    if (gauss) {
                        const double wgt = rec ? gx * gy : exp(-d2s * h);
                        num += wgt * n;
                        den += wgt;
                    } else {
                        num += n;
                        den += 1.0;
                    }
                }
                if (rec) {
                    gx *= rx;
                    rx *= kx;
                }
            }
            if (rec) {
                gy *= ry;
                ry *= ky;
            }
        }
    }
    const double mu = den > 0.0 ? num / (den * a.n_av) : __builtin_nan("");
    if (a.mu) a.mu[gp] = mu;
    if (a.mag) a.mag[gp] = -2.5 * log10(mu);
}

}  // namespace

hipError_t launch_light_curve(const LightArgs &a, hipStream_t s)
{
    const int64_t pts = (int64_t)a.n_tracks * a.n_points;
    if (pts <= 0) return hipSuccess;
    // the support box spans at most this many pixels per axis
    const double bx = std::ceil(2.0 * a.support * a.inv_w[0]) + 2.0, by = std::ceil(2.0 * a.support * a.inv_w[1]) + 2.0;
    const bool lanes = a.path == 1 || (a.path == 0 && pts >= 16384 && bx * by <= 4096.0);
    if (lanes) {
        const int64_t blocks = (pts + 255) / 256;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_light_curve_lanes, dim3((unsigned)blocks), dim3(256), 0, s, a);
    } else {
        const int64_t blocks = (pts + kLcWaves - 1) / kLcWaves;
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_light_curve, dim3((unsigned)blocks), dim3(64 * kLcWaves), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace rs
