// Direct inverse ray-shooting on gfx950: FP32 VALU direct sum with LDS-staged lens tiles,
// FP64 run combination, FP64 lens equation and LDS-privatised binning.
//
// Method: Thompson, Fluke, Barnes & Barsdell (2009), section 1 eqs. 1, 2, 4; section 2 eq. 5;
// section 3.2 eq. 6; the 10-flop interaction of appendix A.
//
// Work decomposition.  A workgroup of 4 wave64s owns a tile of (64 K1) grid columns x (4 K2)
// grid rows: lane l of wave w holds the K1 x K2 block of rays at columns c0 + K1 l + a (a < K1)
// and rows r0 + K2 w + b (b < K2).  Per lens, x1 - x1_i and its square are computed once per
// column and x2 - x2_i once per row.  With several columns per lane the mass is folded into
// those shared differences (m dx, m dy), so each ray-lens interaction costs one FMA (r^2), a
// reciprocal and two FMAs (alpha += (1/r^2) (m dx)), plus (3 K1 + 2 K2) / (K1 K2) shared
// operations; with one column the interaction keeps the multiply d = m / r^2.  Lenses stream through LDS in tiles of LT records (double buffered); every lane
// reads the same record, so each LDS read is a broadcast.  Partial sums run in float32 over
// T consecutive lenses, then are added to a per-ray FP64 accumulator.
#include <algorithm>
#include <mutex>

#include "rs_internal.h"

namespace rs {

namespace {

// Coordinate i of a grid axis at offset u in [0, 1) of its cell, FP64 then rounded to float32.
__device__ __forceinline__ float ray_coord(double lo, double t, int64_t i, double u = 0.5)
{
    double v = ((double)i + u) * t;
    double w = lo + v;
    return (float)w;
}

// Half-open source pixel of y; returns p2 * n1 + p1, or -1 when the ray is lost.
__device__ __forceinline__ int pixel_of(double y1, double y2, const DirectArgs &a, int &p1, int &p2)
{
    double f1 = floor((y1 - a.mlo1) * a.ms1);
    double f2 = floor((y2 - a.mlo2) * a.ms2);
    if (!(f1 >= 0.0 && f1 < (double)a.mn1 && f2 >= 0.0 && f2 < (double)a.mn2)) return -1;
    p1 = (int)f1;
    p2 = (int)f2;
    return p2 * a.mn1 + p1;
}

// 1 / (1 + mean relative error of v_rcp_f32), the error measured over every float32 mantissa
// in [1, 2) with weight 1/x.
constexpr double kRcpBiasComp = 1.0 + 6.41e-9;

// Ray and lens coordinates enter the lens loop scaled by 2^-4.  The scaling is exact, so every
// rounding is that of the unscaled arithmetic; it keeps the product of four squared distances (four
// rows sharing one reciprocal) in the float32 range for lenses up to about 1e6 from the rays.  The
// sums come out 2^4 times the deflection and are scaled back with the bias compensation.
constexpr float kLoopScale = 0.0625f;
constexpr double kLoopBack = kRcpBiasComp * 0.0625;

// One-column blocks add kQuadRuns consecutive float32 runs in float32 before the FP64 addition:
// one float32 add per run instead of a conversion and an FP64 add, at an error between that of
// single runs and of one run kQuadRuns times as long.
constexpr int kQuadRuns = 4;

// Lens i as the loop reads it: moved to the launch's time, coordinates scaled.
__device__ __forceinline__ float4 loop_lens(const DirectArgs &a, int64_t i)
{
    float4 l = moved_lens(a.lenses[i], a.vel, i, a.time);
    l.x *= kLoopScale;
    l.y *= kLoopScale;
    return l;
}

// Zero-mass padding of the last lens tile: at lens 0's position, so that its squared distances are
// ordinary numbers (products stay finite and its terms are exactly zero); a ray exactly there takes
// the per-ray recomputation below, as a ray on lens 0 does anyway.
__device__ __forceinline__ float4 pad_lens(const DirectArgs &a)
{
    float4 l = loop_lens(a, 0);
    l.z = 0.0f;
    l.w = 0.0f;
    return l;
}

template <int LT>
struct TileSmem {
    float4 lens[2][LT];
    uint32_t win[kMaxWindow * kMaxWindow];
    int cand[2][2 * kWaves];
    uint32_t lost;
};

// Shoot one block of rays per lane with the whole workgroup: lane rays are the window-relative
// columns c0 .. c0 + K1 - 1 and rows r0 .. r0 + K2 - 1 (r0 a multiple of 4); a ray counts only when
// its column is below cmax and its row in [rmin, rmax).  `slot` selects the partial map the counts
// go to.  Every thread of the workgroup must call it.
//
// Rays share reciprocals (simultaneous inversion).  With one column per lane, the four rows
// r0 + 4p .. r0 + 4p + 3 share one: with q0 .. q3 their squared distances to a lens, g = 1 /
// (q0 q1 q2 q3) gives 1 / q0 = g (q2 q3) q1 and so on, one v_rcp_f32 for four interactions; with
// several columns per lane (the mass folded into the shared differences), pairs of rows share
// one.  Window rows are aligned so that the groups are always grid rows 4p .. 4p + 3 (or pairs
// within them), which keeps every ray's arithmetic independent of the window and of the launch.
// A lane whose sums end non-finite (a product of zero: a ray on a lens) is recomputed with one
// reciprocal per ray, so a ray is lost exactly when its own distance is zero.  A product above
// the float32 range (all rays of the group more than about 1e6 Einstein radii from the lens)
// gives g = 0: such a lens deflects by less than 1e-6 m and is dropped.
template <int K1, int K2, int T, int LT, bool DUMP, bool JIT>
__device__ __forceinline__ void shoot_rays(const DirectArgs &a, int64_t c0, int64_t r0, int64_t cmax, int64_t rmin,
                                           int64_t rmax, uint32_t slot, TileSmem<LT> &sm)
{
    static_assert(K2 % 2 == 0, "rows pair up");
    constexpr int PER = LT / kThreads;
    constexpr int R = K1 * K2;
    constexpr bool FOLD = K1 >= 2;  // fold m into shared differences when a lane has several columns
    constexpr bool QUAD = K1 == 1 && K2 % 4 == 0;   // four rows per reciprocal
    constexpr int G = QUAD ? kQuadRuns : 1;         // float32 runs per FP64 addition
    static_assert(LT % kThreads == 0 && LT % (T * G) == 0, "tile shape");
    auto &s_lens = sm.lens;
    auto &s_win = sm.win;
    auto &s_cand = sm.cand;
    auto &s_lost = sm.lost;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // cell-centred rays share x1 down a column and x2 along a row; jittered rays (JIT) have
    // their own coordinates, xj1 / xj2 per ray slot
    float x1[K1], x2[K2], xj1[JIT ? R : 1], xj2[JIT ? R : 1];
#pragma unroll
    for (int i = 0; i < K1; ++i) x1[i] = ray_coord(a.glo1, a.gt1, a.wlo1 + c0 + i) * kLoopScale;
#pragma unroll
    for (int b = 0; b < K2; ++b) x2[b] = ray_coord(a.glo2, a.gt2, a.wlo2 + r0 + b) * kLoopScale;
    if constexpr (JIT) {
#pragma unroll
        for (int i = 0; i < K1; ++i)
#pragma unroll
            for (int b = 0; b < K2; ++b) {
                const int64_t g1 = a.wlo1 + c0 + i, g2 = a.wlo2 + r0 + b, r = g2 * a.gn1 + g1;
                xj1[i * K2 + b] = ray_coord(a.glo1, a.gt1, g1, jitter_u(a.jkey1, r)) * kLoopScale;
                xj2[i * K2 + b] = ray_coord(a.glo2, a.gt2, g2, jitter_u(a.jkey2, r)) * kLoopScale;
            }
    }

    for (int b = tid; b < kMaxWindow * kMaxWindow; b += kThreads) s_win[b] = 0u;
    if (tid == 0) s_lost = 0u;

    // ray (i, b) of the lane is slot i * K2 + b
    double A1[R], A2[R];
#pragma unroll
    for (int k = 0; k < R; ++k) { A1[k] = 0.0; A2[k] = 0.0; }

    const int64_t n_tiles = (a.n_lens + LT - 1) / LT;
    float4 reg[PER];
    if (n_tiles > 0) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            int64_t i = (int64_t)p * kThreads + tid;
            reg[p] = i < a.n_lens ? loop_lens(a, i) : pad_lens(a);
            s_lens[0][p * kThreads + tid] = reg[p];
        }
    }
    __syncthreads();

    for (int64_t t = 0; t < n_tiles; ++t) {
        const int buf = (int)(t & 1);
        const bool more = t + 1 < n_tiles;
        if (more) {
#pragma unroll
            for (int p = 0; p < PER; ++p) {
                int64_t i = (t + 1) * LT + (int64_t)p * kThreads + tid;
                reg[p] = i < a.n_lens ? loop_lens(a, i) : pad_lens(a);
            }
        }
        const float4 *L = s_lens[buf];
        // the last tile stops after the group of runs that holds the last lens: a group of
        // padding alone would add exact zeros
        const int64_t rest = a.n_lens - t * LT;
        const int lim = rest >= LT ? LT : (int)((rest + T * G - 1) / (T * G)) * (T * G);
        for (int r = 0; r < lim; r += T * G) {
            float m1[R], m2[R];
#pragma unroll
            for (int h = 0; h < G; ++h) {
                float s1[R], s2[R];
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    const float4 l = L[r + h * T + j];
                    if constexpr (JIT && QUAD) {
                        // every ray has its own coordinates; the four rows still share the reciprocal
#pragma unroll
                        for (int k = 0; k < R; k += 4) {
                            float dx[4], dy[4], q[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                dx[e] = xj1[k + e] - l.x;
                                dy[e] = xj2[k + e] - l.y;
                                q[e] = fmaf(dy[e], dy[e], dx[e] * dx[e]);
                            }
                            const float p01 = q[0] * q[1], p23 = q[2] * q[3];
                            const float g = l.z * __builtin_amdgcn_rcpf(p01 * p23);
                            const float g01 = g * p23, g23 = g * p01;
                            const float d[4] = {g01 * q[1], g01 * q[0], g23 * q[3], g23 * q[2]};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                s1[k + e] = j == 0 ? d[e] * dx[e] : fmaf(d[e], dx[e], s1[k + e]);
                                s2[k + e] = j == 0 ? d[e] * dy[e] : fmaf(d[e], dy[e], s2[k + e]);
                            }
                        }
                    } else if constexpr (JIT) {
                        // every ray has its own coordinates; rows still pair up for the reciprocal
#pragma unroll
                        for (int k = 0; k < R; k += 2) {
                            const float dxa = xj1[k] - l.x, dya = xj2[k] - l.y;
                            const float dxb = xj1[k + 1] - l.x, dyb = xj2[k + 1] - l.y;
                            const float ra = fmaf(dya, dya, dxa * dxa), rb = fmaf(dyb, dyb, dxb * dxb);
                            const float g = l.z * __builtin_amdgcn_rcpf(ra * rb);
                            const float da = g * rb, db = g * ra;
                            if (j == 0) {
                                s1[k] = da * dxa;
                                s2[k] = da * dya;
                                s1[k + 1] = db * dxb;
                                s2[k + 1] = db * dyb;
                            } else {
                                s1[k] = fmaf(da, dxa, s1[k]);
                                s2[k] = fmaf(da, dya, s2[k]);
                                s1[k + 1] = fmaf(db, dxb, s1[k + 1]);
                                s2[k + 1] = fmaf(db, dyb, s2[k + 1]);
                            }
                        }
                    } else if constexpr (FOLD) {
                        // shared per column: x1 - x1_i, its square and m (x1 - x1_i);
                        // per row: x2 - x2_i and m (x2 - x2_i)
                        float dx[K1], dx2[K1], mdx[K1], dy[K2], mdy[K2];
#pragma unroll
                        for (int i = 0; i < K1; ++i) {
                            dx[i] = x1[i] - l.x;
                            dx2[i] = dx[i] * dx[i];
                            mdx[i] = l.z * dx[i];
                        }
#pragma unroll
                        for (int b = 0; b < K2; ++b) {
                            dy[b] = x2[b] - l.y;
                            mdy[b] = l.z * dy[b];
                        }
#pragma unroll
                        for (int i = 0; i < K1; ++i) {
#pragma unroll
                            for (int b = 0; b < K2; b += 2) {
                                const int k = i * K2 + b;
                                const float ra = fmaf(dy[b], dy[b], dx2[i]), rb = fmaf(dy[b + 1], dy[b + 1], dx2[i]);
                                const float g = __builtin_amdgcn_rcpf(ra * rb);
                                const float qa = g * rb, qb = g * ra;
                                if (j == 0) {
                                    s1[k] = qa * mdx[i];
                                    s2[k] = qa * mdy[b];
                                    s1[k + 1] = qb * mdx[i];
                                    s2[k + 1] = qb * mdy[b + 1];
                                } else {
                                    s1[k] = fmaf(qa, mdx[i], s1[k]);
                                    s2[k] = fmaf(qa, mdy[b], s2[k]);
                                    s1[k + 1] = fmaf(qb, mdx[i], s1[k + 1]);
                                    s2[k + 1] = fmaf(qb, mdy[b + 1], s2[k + 1]);
                                }
                            }
                        }
                    } else if constexpr (QUAD) {
                        // one column per lane, four rows per reciprocal: d = m / r^2 per ray, then
                        // alpha += d (dx, dy)
                        const float dx = x1[0] - l.x;
                        const float dx2 = dx * dx;
#pragma unroll
                        for (int b = 0; b < K2; b += 4) {
                            float dy[4], q[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                dy[e] = x2[b + e] - l.y;
                                q[e] = fmaf(dy[e], dy[e], dx2);
                            }
                            const float p01 = q[0] * q[1], p23 = q[2] * q[3];
                            const float g = l.z * __builtin_amdgcn_rcpf(p01 * p23);
                            const float g01 = g * p23, g23 = g * p01;
                            const float d[4] = {g01 * q[1], g01 * q[0], g23 * q[3], g23 * q[2]};
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                s1[b + e] = j == 0 ? d[e] * dx : fmaf(d[e], dx, s1[b + e]);
                                s2[b + e] = j == 0 ? d[e] * dy[e] : fmaf(d[e], dy[e], s2[b + e]);
                            }
                        }
                    } else {
                        // one column per lane: d = m / r^2 per ray, then alpha += d (dx, dy)
                        const float dx = x1[0] - l.x;
                        const float dx2 = dx * dx;
#pragma unroll
                        for (int b = 0; b < K2; b += 2) {
                            const float dya = x2[b] - l.y, dyb = x2[b + 1] - l.y;
                            const float ra = fmaf(dya, dya, dx2), rb = fmaf(dyb, dyb, dx2);
                            const float g = l.z * __builtin_amdgcn_rcpf(ra * rb);
                            const float da = g * rb, db = g * ra;
                            if (j == 0) {
                                s1[b] = da * dx;
                                s2[b] = da * dya;
                                s1[b + 1] = db * dx;
                                s2[b + 1] = db * dyb;
                            } else {
                                s1[b] = fmaf(da, dx, s1[b]);
                                s2[b] = fmaf(da, dya, s2[b]);
                                s1[b + 1] = fmaf(db, dx, s1[b + 1]);
                                s2[b + 1] = fmaf(db, dyb, s2[b + 1]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    m1[k] = h == 0 ? s1[k] : m1[k] + s1[k];
                    m2[k] = h == 0 ? s2[k] : m2[k] + s2[k];
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                A1[k] += (double)m1[k];
                A2[k] += (double)m2[k];
            }
        }
        if (more) {
#pragma unroll
            for (int p = 0; p < PER; ++p) s_lens[buf ^ 1][p * kThreads + tid] = reg[p];
        }
        __syncthreads();
    }

    {
        // A group whose product left the finite range (a ray on a lens, or the group's rays all
        // very close to one) leaves a non-finite sum.  Redo this lane's rays with one reciprocal per
        // ray, in the same runs of T lenses and groups of G runs, reading the lenses from global
        // memory: every ray then gets exactly the per-ray result, and only a ray on a lens stays
        // non-finite.
        bool bad = false;
#pragma unroll
        for (int k = 0; k < R; ++k) bad = bad || !__builtin_isfinite(A1[k] + A2[k]);
        if (bad) {
#pragma unroll
            for (int k = 0; k < R; ++k) { A1[k] = 0.0; A2[k] = 0.0; }
            float m1[R], m2[R];
            for (int64_t r = 0; r < a.n_lens; r += T) {
                float s1[R], s2[R];
#pragma unroll
                for (int k = 0; k < R; ++k) { s1[k] = 0.0f; s2[k] = 0.0f; }
                const int64_t e = min(r + (int64_t)T, a.n_lens);
                for (int64_t li = r; li < e; ++li) {
                    const float4 l = loop_lens(a, li);
                    if constexpr (JIT) {
#pragma unroll
                        for (int k = 0; k < R; ++k) {
                            const float dx = xj1[k] - l.x, dy = xj2[k] - l.y;
                            const float d = l.z * __builtin_amdgcn_rcpf(fmaf(dy, dy, dx * dx));
                            s1[k] = fmaf(d, dx, s1[k]);
                            s2[k] = fmaf(d, dy, s2[k]);
                        }
                        continue;
                    }
#pragma unroll
                    for (int i = 0; i < K1; ++i) {
                        const float dx = x1[i] - l.x;
                        const float dx2 = dx * dx;
                        const float mdx = l.z * dx;
#pragma unroll
                        for (int b = 0; b < K2; ++b) {
                            const int k = i * K2 + b;
                            const float dy = x2[b] - l.y;
                            const float q = __builtin_amdgcn_rcpf(fmaf(dy, dy, dx2));
                            if constexpr (FOLD) {
                                s1[k] = fmaf(q, mdx, s1[k]);
                                s2[k] = fmaf(q, l.z * dy, s2[k]);
                            } else {
                                const float d = l.z * q;
                                s1[k] = fmaf(d, dx, s1[k]);
                                s2[k] = fmaf(d, dy, s2[k]);
                            }
                        }
                    }
                }
                // runs are grouped as in the lens loop: G runs added in float32, then in FP64
                const bool first = (r / T) % G == 0, last = (r / T) % G == G - 1 || e == a.n_lens;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    m1[k] = first ? s1[k] : m1[k] + s1[k];
                    m2[k] = first ? s2[k] : m2[k] + s2[k];
                }
                if (last) {
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        A1[k] += (double)m1[k];
                        A2[k] += (double)m2[k];
                    }
                }
            }
        }
    }

    // The hardware reciprocal is biased low: over all float32 mantissas, weighted as for
    // log-uniform arguments, its mean relative error is -6.41e-9.  Summed coherently over many
    // lenses this bias would dominate the float32 error of large deflections, so the FP64 sum
    // is rescaled by the inverse factor (two FP64 multiplies per ray, no per-lens cost), together
    // with the 2^-4 that undoes the coordinate scaling.
#pragma unroll
    for (int k = 0; k < R; ++k) {
        A1[k] *= kLoopBack;
        A2[k] *= kLoopBack;
    }

    // Lens equation (eq. 6) and source pixel, FP64.
    int key[R], q1[R], q2[R];
#pragma unroll
    for (int i = 0; i < K1; ++i) {
#pragma unroll
        for (int b = 0; b < K2; ++b) {
            const int k = i * K2 + b;
            const bool ok = (c0 + i < cmax) && (r0 + b >= rmin) && (r0 + b < rmax);
            const double y1 = a.lam1 * ((double)(JIT ? xj1[k] : x1[i]) * 16.0) - A1[k];
            const double y2 = a.lam2 * ((double)(JIT ? xj2[k] : x2[b]) * 16.0) - A2[k];
            int p1 = 0, p2 = 0;
            const int kv = pixel_of(y1, y2, a, p1, p2);
            key[k] = ok ? kv : -2;
            q1[k] = p1;
            q2[k] = p2;
            if (DUMP && ok) {
                const int64_t ri = (r0 + b - a.rskip) * a.wn1 + c0 + i;
                a.ray_y[2 * ri] = y1;
                a.ray_y[2 * ri + 1] = y2;
                a.ray_pix[ri] = kv;
            }
        }
    }

    // Window origin: per-axis median of 8 sample rays of the tile (robust to rays scattered
    // far by a close lens).
    const int W = a.window;
    int o1 = 0, o2 = 0;
    if (W > 0) {
        constexpr int ka = (K1 / 2) * K2 + K2 / 4, kb = (K1 / 2) * K2 + (3 * K2) / 4;
        if (lane == 16) {
            s_cand[0][2 * wave] = key[ka] >= 0 ? q1[ka] : INT_MIN;
            s_cand[1][2 * wave] = key[ka] >= 0 ? q2[ka] : INT_MIN;
        }
        if (lane == 48) {
            s_cand[0][2 * wave + 1] = key[kb] >= 0 ? q1[kb] : INT_MIN;
            s_cand[1][2 * wave + 1] = key[kb] >= 0 ? q2[kb] : INT_MIN;
        }
        __syncthreads();
        int v1[2 * kWaves], v2[2 * kWaves], n = 0;
#pragma unroll
        for (int c = 0; c < 2 * kWaves; ++c) {
            const int a1 = s_cand[0][c], a2 = s_cand[1][c];
            if (a1 != INT_MIN) { v1[n] = a1; v2[n] = a2; ++n; }
        }
        if (n > 0) {
            // insertion sorts of at most 8 values
            for (int i = 1; i < n; ++i) {
                int u = v1[i], w = v2[i], j = i - 1;
                while (j >= 0 && v1[j] > u) { v1[j + 1] = v1[j]; --j; }
                v1[j + 1] = u;
                j = i - 1;
                while (j >= 0 && v2[j] > w) { v2[j + 1] = v2[j]; --j; }
                v2[j + 1] = w;
            }
            o1 = v1[n / 2] - W / 2;
            o2 = v2[n / 2] - W / 2;
        }
    }

    // Binning: runs of equal keys among consecutive lanes are added once (wave aggregation),
    // into the LDS window when the pixel falls inside it, else into this die's partial map.
    uint32_t *part = a.partial + (size_t)slot * (size_t)a.pstride;
    uint32_t lost_cnt = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int kv = key[k];
        const int prev = __shfl_up(kv, 1);
        const bool head = (lane == 0) || (kv != prev);
        const unsigned long long H = __ballot(head);
        const unsigned long long above = lane == 63 ? 0ull : (H >> (lane + 1));
        const int next = above ? lane + 1 + __builtin_ctzll(above) : 64;
        const uint32_t cnt = (uint32_t)(next - lane);
        if (head) {
            if (kv >= 0) {
                const int w1 = q1[k] - o1, w2 = q2[k] - o2;
                if (W > 0 && (unsigned)w1 < (unsigned)W && (unsigned)w2 < (unsigned)W)
                    atomicAdd(&s_win[w2 * W + w1], cnt);
                else
                    atomicAdd(&part[kv], cnt);
            } else if (kv == -1) {
                lost_cnt += cnt;
            }
        }
    }
    if (lost_cnt) atomicAdd(&s_lost, lost_cnt);
    __syncthreads();

    // Flush the window's non-zero bins.
    if (W > 0) {
        for (int b = tid; b < W * W; b += kThreads) {
            const uint32_t v = s_win[b];
            if (v) atomicAdd(&part[(int64_t)(o2 + b / W) * a.mn1 + (o1 + b % W)], v);
        }
    }
    if (tid == 0 && s_lost) atomicAdd(a.lost, (unsigned long long)s_lost);
}

// Ray tile `tile` of the window: (64 K1) columns x (4 K2) rows, lane l of wave w holding the
// K1 x K2 block at columns c0 + K1 l, rows r0 + K2 w.
template <int K1, int K2, int T, int LT, bool DUMP, bool JIT>
__device__ __forceinline__ void shoot_tile(const DirectArgs &a, uint32_t tile, uint32_t slot, TileSmem<LT> &sm)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tx = (int)(tile % (uint32_t)a.tiles_x);
    const int ty = (int)(tile / (uint32_t)a.tiles_x);
    const int64_t c0 = (int64_t)tx * (64 * K1) + (int64_t)lane * K1;
    const int64_t r0 = (int64_t)ty * (kWaves * K2) + (int64_t)wave * K2;
    shoot_rays<K1, K2, T, LT, DUMP, JIT>(a, c0, r0, a.wn1, a.rskip, a.wn2, slot, sm);
}

template <int K1, int K2, int T, int LT, bool DUMP, bool JIT>
__global__ void __launch_bounds__(kThreads) k_direct(const DirectArgs a)
{
    __shared__ TileSmem<LT> sm;
    shoot_tile<K1, K2, T, LT, DUMP, JIT>(a, blockIdx.x, blockIdx.x & (kPartials - 1), sm);
}

// Persistent direct sum over the lane blocks of a list of culling cells (the cells a zoom
// keeps).  Cell q of the list covers the caller's window columns [mx c1, (mx + 1) c1) and rows
// [my c2, (my + 1) c2) (clipped to the window), i.e. rows shifted by rskip here; it is cut into
// S = sx sy lane blocks of K1 columns x K2 rows starting at the multiple of 4 at or below its first
// row (so the row groups are those of the plain launch), and block j of cell list[i] is lane
// slot i S + j.  Workgroup g takes slots g 256 .. g 256 + 255, then g + grid, ...
template <int K1, int K2, int T, int LT, bool JIT>
__global__ void __launch_bounds__(kThreads) k_direct_cells(const DirectArgs a, const CellBlocks cb)
{
    __shared__ TileSmem<LT> sm;
    const uint64_t n = (uint64_t)(*cb.count) * (uint64_t)cb.S;
    uint32_t it = 0;
    for (uint64_t base = (uint64_t)blockIdx.x * kThreads; base < n; base += (uint64_t)gridDim.x * kThreads, ++it) {
        const uint64_t q = base + threadIdx.x;
        int64_t c0 = 0, r0 = 0, cmax = 0, rmin = 0, rmax = 0;
        if (q < n) {
            const uint64_t i = q / (uint64_t)cb.S;
            const int64_t j = (int64_t)(q - i * (uint64_t)cb.S);
            const int64_t cell = cb.list[i];
            const int64_t mx = cell % cb.ncx, my = cell / cb.ncx;
            c0 = mx * cb.c1 + (j % cb.sx) * K1;
            rmin = my * cb.c2 + a.rskip;
            r0 = (rmin & ~int64_t(3)) + (j / cb.sx) * K2;
            cmax = min((mx + 1) * cb.c1, a.wn1);
            rmax = min((my + 1) * cb.c2 + a.rskip, a.wn2);
        }
        shoot_rays<K1, K2, T, LT, false, JIT>(a, c0, r0, cmax, rmin, rmax, (blockIdx.x + it) & (kPartials - 1),
                                             sm);
        __syncthreads();
    }
}

// Persistent kernel over a table of jobs: each workgroup takes (job, tile) work items from an
// atomic counter until none are left.  Items are numbered job by job in table order (the host
// orders jobs by decreasing work per tile), so the costliest tiles are taken first.  Counts go
// straight into each job's map.
template <int K1, int K2, int T, int LT>
__global__ void __launch_bounds__(kThreads) k_batched(const BatchArgs b)
{
    __shared__ TileSmem<LT> sm;
    __shared__ uint32_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(b.queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= b.n_items) break;
        // job j owns items [item_start[j], item_start[j+1])
        int lo = 0, hi = b.n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.item_start[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        if (b.jobs[lo].jitter)
            shoot_tile<K1, K2, T, LT, false, true>(b.jobs[lo], item - b.item_start[lo], 0u, sm);
        else
            shoot_tile<K1, K2, T, LT, false, false>(b.jobs[lo], item - b.item_start[lo], 0u, sm);
        __syncthreads();
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v) { p[threadIdx.x] = v; }

__global__ void __launch_bounds__(256) k_advance(const float4 *in, const float2 *vel, int64_t n, double time,
                                                 float4 *out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = moved_lens(in[i], vel, i, time);
}

__global__ void __launch_bounds__(256) k_zero(uint4 *p, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// counts[b] += sum over the kPartials maps; partial maps are kPartials x pstride words with
// pstride a multiple of 64, so every group of four bins is 16-byte aligned in the workspace.
__global__ void __launch_bounds__(256) k_reduce(const uint32_t *partial, int64_t bins, int64_t pstride,
                                                 uint32_t *counts)
{
    const int64_t n4 = (bins + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const bool vec = ((uintptr_t)counts & 15u) == 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        uint4 s = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int p = 0; p < kPartials; ++p) {
            const uint4 v = *reinterpret_cast<const uint4 *>(partial + (size_t)p * pstride + 4 * i);
            s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
        }
        const int64_t b = 4 * i;
        if (vec && b + 3 < bins) {
            uint4 *c = reinterpret_cast<uint4 *>(counts + b);
            uint4 o = *c;
            o.x += s.x; o.y += s.y; o.z += s.z; o.w += s.w;
            *c = o;
        } else {
            const uint32_t sv[4] = {s.x, s.y, s.z, s.w};
            for (int j = 0; j < 4 && b + j < bins; ++j) counts[b + j] += sv[j];
        }
    }
}

template <int K1, int K2, int T, int LT>
hipError_t launch_kt(const DirectArgs &a, int64_t n_tiles, hipStream_t s)
{
    const dim3 g((unsigned)n_tiles), blk(kThreads);
    if (a.jitter) {
        if (a.ray_y) hipLaunchKernelGGL((k_direct<K1, K2, T, LT, true, true>), g, blk, 0, s, a);
        else hipLaunchKernelGGL((k_direct<K1, K2, T, LT, false, true>), g, blk, 0, s, a);
    } else {
        if (a.ray_y) hipLaunchKernelGGL((k_direct<K1, K2, T, LT, true, false>), g, blk, 0, s, a);
        else hipLaunchKernelGGL((k_direct<K1, K2, T, LT, false, false>), g, blk, 0, s, a);
    }
    return hipGetLastError();
}

template <int K1, int K2>
hipError_t launch_k(const DirectArgs &a, int T, int LT, int64_t n_tiles, hipStream_t s)
{
    if (LT == 256) {
        if (T == 8) return launch_kt<K1, K2, 8, 256>(a, n_tiles, s);
        if (T == 16) return launch_kt<K1, K2, 16, 256>(a, n_tiles, s);
        if (T == 32) return launch_kt<K1, K2, 32, 256>(a, n_tiles, s);
    } else if (LT == 512) {
        if (T == 8) return launch_kt<K1, K2, 8, 512>(a, n_tiles, s);
        if (T == 16) return launch_kt<K1, K2, 16, 512>(a, n_tiles, s);
        if (T == 32) return launch_kt<K1, K2, 32, 512>(a, n_tiles, s);
    }
    return hipErrorInvalidValue;
}

template <int K1, int K2, int T, int LT>
hipError_t launch_ct(const DirectArgs &a, const CellBlocks &cb, int64_t max_groups, hipStream_t s)
{
    int occ = 0;
    if (a.jitter) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_direct_cells<K1, K2, T, LT, true>, kThreads, 0) !=
            hipSuccess)
            occ = 1;
    } else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_direct_cells<K1, K2, T, LT, false>, kThreads,
                                                            0) != hipSuccess) {
        occ = 1;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t grid = (int64_t)std::max(1, occ) * std::max(1, cus);
    if (grid > max_groups) grid = max_groups;
    const dim3 g((unsigned)grid), blk(kThreads);
    if (a.jitter) hipLaunchKernelGGL((k_direct_cells<K1, K2, T, LT, true>), g, blk, 0, s, a, cb);
    else hipLaunchKernelGGL((k_direct_cells<K1, K2, T, LT, false>), g, blk, 0, s, a, cb);
    return hipGetLastError();
}

template <int K1, int K2>
hipError_t launch_c(const DirectArgs &a, int T, int LT, const CellBlocks &cb, int64_t max_groups, hipStream_t s)
{
    if (LT == 256) {
        if (T == 8) return launch_ct<K1, K2, 8, 256>(a, cb, max_groups, s);
        if (T == 16) return launch_ct<K1, K2, 16, 256>(a, cb, max_groups, s);
        if (T == 32) return launch_ct<K1, K2, 32, 256>(a, cb, max_groups, s);
    } else if (LT == 512) {
        if (T == 8) return launch_ct<K1, K2, 8, 512>(a, cb, max_groups, s);
        if (T == 16) return launch_ct<K1, K2, 16, 512>(a, cb, max_groups, s);
        if (T == 32) return launch_ct<K1, K2, 32, 512>(a, cb, max_groups, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

template <int K1, int K2>
hipError_t launch_b(const BatchArgs &b, int T, int LT, int grid, hipStream_t s)
{
    if (LT == 256) {
        if (T == 8) hipLaunchKernelGGL((k_batched<K1, K2, 8, 256>), dim3(grid), dim3(kThreads), 0, s, b);
        else if (T == 16) hipLaunchKernelGGL((k_batched<K1, K2, 16, 256>), dim3(grid), dim3(kThreads), 0, s, b);
        else if (T == 32) hipLaunchKernelGGL((k_batched<K1, K2, 32, 256>), dim3(grid), dim3(kThreads), 0, s, b);
        else return hipErrorInvalidValue;
    } else if (LT == 512) {
        if (T == 8) hipLaunchKernelGGL((k_batched<K1, K2, 8, 512>), dim3(grid), dim3(kThreads), 0, s, b);
        else if (T == 16) hipLaunchKernelGGL((k_batched<K1, K2, 16, 512>), dim3(grid), dim3(kThreads), 0, s, b);
        else if (T == 32) hipLaunchKernelGGL((k_batched<K1, K2, 32, 512>), dim3(grid), dim3(kThreads), 0, s, b);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int K1, int K2>
int occ_b(int T, int LT)
{
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (LT == 256 && T == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 8, 256>, kThreads, 0);
    if (LT == 256 && T == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 16, 256>, kThreads, 0);
    if (LT == 256 && T == 32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 32, 256>, kThreads, 0);
    if (LT == 512 && T == 8) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 8, 512>, kThreads, 0);
    if (LT == 512 && T == 16) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 16, 512>, kThreads, 0);
    if (LT == 512 && T == 32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<K1, K2, 32, 512>, kThreads, 0);
    return e == hipSuccess ? n : 0;
}

bool ray_block_supported(int K1, int K2)
{
    return (K1 == 1 && K2 == 4) || (K1 == 2 && K2 == 2) || (K1 == 2 && K2 == 4) || (K1 == 4 && K2 == 2) ||
           (K1 == 4 && K2 == 4) || (K1 == 2 && K2 == 8);
}

hipError_t launch_direct(const DirectArgs &a, int K1, int K2, int T, int LT, int64_t n_tiles, hipStream_t s)
{
    if (n_tiles <= 0) return hipSuccess;
    if (K1 == 1 && K2 == 4) return launch_k<1, 4>(a, T, LT, n_tiles, s);
    if (K1 == 2 && K2 == 2) return launch_k<2, 2>(a, T, LT, n_tiles, s);
    if (K1 == 2 && K2 == 4) return launch_k<2, 4>(a, T, LT, n_tiles, s);
    if (K1 == 4 && K2 == 2) return launch_k<4, 2>(a, T, LT, n_tiles, s);
    if (K1 == 4 && K2 == 4) return launch_k<4, 4>(a, T, LT, n_tiles, s);
    if (K1 == 2 && K2 == 8) return launch_k<2, 8>(a, T, LT, n_tiles, s);
    return hipErrorInvalidValue;
}

#define RS_BLOCK_SWITCH(FN, ...)                                              \
    if (K1 == 1 && K2 == 4) return FN<1, 4>(__VA_ARGS__);                     \
    if (K1 == 2 && K2 == 2) return FN<2, 2>(__VA_ARGS__);                     \
    if (K1 == 2 && K2 == 4) return FN<2, 4>(__VA_ARGS__);                     \
    if (K1 == 4 && K2 == 2) return FN<4, 2>(__VA_ARGS__);                     \
    if (K1 == 4 && K2 == 4) return FN<4, 4>(__VA_ARGS__);                     \
    if (K1 == 2 && K2 == 8) return FN<2, 8>(__VA_ARGS__);

hipError_t launch_batched(const BatchArgs &b, int K1, int K2, int T, int LT, int grid, hipStream_t s)
{
    RS_BLOCK_SWITCH(launch_b, b, T, LT, grid, s)
    return hipErrorInvalidValue;
}

hipError_t launch_direct_cells(const DirectArgs &a, int K1, int K2, int T, int LT, const CellBlocks &cb,
                               int64_t max_groups, hipStream_t s)
{
    if (max_groups <= 0) return hipSuccess;
    RS_BLOCK_SWITCH(launch_c, a, T, LT, cb, max_groups, s)
    return hipErrorInvalidValue;
}

int batched_occupancy(int K1, int K2, int T, int LT)
{
    RS_BLOCK_SWITCH(occ_b, T, LT)
    return 0;
}

hipError_t launch_fill_u32(uint32_t *p, int n, uint32_t v, hipStream_t s)
{
    if (n <= 0 || n > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(n), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_advance(const float4 *in, const float2 *vel, int64_t n, double time, float4 *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_advance, dim3((unsigned)blocks), dim3(256), 0, s, in, vel, n, time, out);
    return hipGetLastError();
}

hipError_t launch_zero(uint32_t *p, int64_t n_words, hipStream_t s)
{
    const int64_t n4 = n_words / 4;
    if (n4 <= 0) return hipSuccess;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint4 *>(p), n4);
    return hipGetLastError();
}

hipError_t launch_reduce(const uint32_t *partial, int64_t bins, int64_t pstride, uint32_t *counts,
                         hipStream_t s)
{
    const int64_t n4 = (bins + 3) / 4;
    if (n4 <= 0) return hipSuccess;
    int64_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)blocks), dim3(256), 0, s, partial, bins, pstride, counts);
    return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free shooting

// The partial maps of rs_shoot_noalloc: kPartials maps of at most kNoAllocBins bins, in a fixed
// device array that every GPU the library runs on holds (its own copy) until the process ends.
// On the host this name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device, resolved once per device below.
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

hipError_t noalloc_scratch(uint32_t **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = static_cast<uint32_t *>(addr[dev]);
    return hipSuccess;
}

}  // namespace rs
