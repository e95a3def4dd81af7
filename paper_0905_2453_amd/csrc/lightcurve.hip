// Light curves from a magnification map: a source profile moved along straight tracks across
// the map, giving at each point the profile-weighted magnification (eq. 4 per pixel) and the
// magnitude change (section 1, the light-curve use of the maps).
#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kLcWaves = 4;

__device__ inline double wave_sum(double v)
{
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
    return v;
}

// One wave per track point.  Each lane accumulates the pixels e = lane, lane + 64, ... of the
// support's bounding box (row-major), then the wave reduces in a fixed butterfly order, so the
// result depends only on the inputs.
__global__ void __launch_bounds__(64 * kLcWaves) k_light_curve(const LightArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t gp = (int64_t)blockIdx.x * kLcWaves + (threadIdx.x >> 6);
    if (gp >= (int64_t)a.n_tracks * a.n_points) return;
    const int64_t tr = gp / a.n_points;
    const int k = (int)(gp - tr * a.n_points);
    const double *t = a.tracks + 4 * tr;
    const double f = a.n_points > 1 ? (double)k / (double)(a.n_points - 1) : 0.0;
    const double ys1 = t[0] + f * (t[2] - t[0]);
    const double ys2 = t[1] + f * (t[3] - t[1]);
    const double rs = a.support, rs2 = a.support * a.support;
    const double inv2s2 = 1.0 / (2.0 * a.size * a.size);
    // bounding box of the support in pixel indices, clamped to the map
    const double q1lo = floor((ys1 - rs - a.lo[0]) / a.w[0]), q1hi = floor((ys1 + rs - a.lo[0]) / a.w[0]);
    const double q2lo = floor((ys2 - rs - a.lo[1]) / a.w[1]), q2hi = floor((ys2 + rs - a.lo[1]) / a.w[1]);
    const int p1lo = (int)fmax(0.0, fmin(q1lo, (double)a.n[0]));
    const int p1hi = (int)fmax(-1.0, fmin(q1hi, (double)a.n[0] - 1));
    const int p2lo = (int)fmax(0.0, fmin(q2lo, (double)a.n[1]));
    const int p2hi = (int)fmax(-1.0, fmin(q2hi, (double)a.n[1] - 1));
    const int nx = p1hi - p1lo + 1, ny = p2hi - p2lo + 1;
    double num = 0.0, den = 0.0;
    if (nx > 0 && ny > 0) {
        const int total = nx * ny;
        for (int e = lane; e < total; e += 64) {
            const int r = e / nx;
            const int p1 = p1lo + (e - r * nx), p2 = p2lo + r;
            const double d1 = (a.lo[0] + ((double)p1 + 0.5) * a.w[0]) - ys1;
            const double d2 = (a.lo[1] + ((double)p2 + 0.5) * a.w[1]) - ys2;
            const double d2s = d1 * d1 + d2 * d2;
            if (d2s <= rs2) {
                const double wgt = a.kind == 0 ? exp(-d2s * inv2s2) : 1.0;
                num += wgt * (double)a.counts[(int64_t)p2 * a.n[0] + p1];
                den += wgt;
            }
        }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    if (lane == 0) {
        const double mu = den > 0.0 ? num / (den * a.n_av) : __builtin_nan("");
        if (a.mu) a.mu[gp] = mu;
        if (a.mag) a.mag[gp] = -2.5 * log10(mu);
    }
}

}  // namespace

hipError_t launch_light_curve(const LightArgs &a, hipStream_t s)
{
    const int64_t pts = (int64_t)a.n_tracks * a.n_points;
    if (pts <= 0) return hipSuccess;
    const int64_t blocks = (pts + kLcWaves - 1) / kLcWaves;
    hipLaunchKernelGGL(k_light_curve, dim3((unsigned)blocks), dim3(64 * kLcWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace rs
