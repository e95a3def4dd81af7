// Interactive zoom (section 4: a selected area of a map recomputed at higher ray density).
//
// The zoom map is, by definition, the map that shooting EVERY ray of the fine grid would give on
// the selected source-plane window.  Only rays that can land in the window matter, so the fine
// grid is split into culling cells and each cell's whole image under the lens equation (eq. 6
// with the deflection of eq. 2) is bounded from one evaluation at the cell centre c:
//
//   y(x) = y(c) + J(c)(x - c) + R(x)     for the lenses at distance >= 3 rho from c
//                                         (rho = half-diagonal of the cell), with
//   J = diag(l1, l2) - grad alpha,  grad alpha_i = m_i / r^4 [[f2^2 - f1^2, -2 f1 f2], [-2 f1 f2, f1^2 - f2^2]]
//   |R| <= rho^2 sum m_i / (r_i - rho)^3 <= rho^2 (3/2)^3 sum m_i / r_i^3    (|d^2 alpha_i| = 2 m / r^3)
//
// while a lens closer than 3 rho moves the image by at most |alpha_i(x) - alpha_i(c)| <= 2 m_i / delta_i
// (delta_i = its distance to the cell rectangle); a lens inside the rectangle leaves the image
// unbounded.  A cell whose bounding box, widened by a rounding allowance, misses the window cannot
// contribute and is skipped; the rays of the kept cells are shot exactly as the plain path shoots
// them, so the zoom map equals the full fine-grid map on the window.
#include <algorithm>

#include "rs_internal.h"

namespace rs {

namespace {

constexpr int kZoomLT = 256;    // lenses per LDS tile
constexpr int kZoomRun = 16;    // float32 run length before the FP64 combine

__device__ __forceinline__ float4 zoom_pad_lens()
{
    return make_float4(kPadCoord, kPadCoord, 0.0f, 0.0f);
}

// One work item per cell of one culling level; kept cells are appended to that level's list.
//   level 0: every cell of the coarsest level;
//   level l > 0: the cells inside the cells kept at level l - 1: item t takes child t % P^2 of
//                kept cell lists[l - 1][t / P^2].
// A child's rectangle lies inside its parent's, so a cell whose image can meet the map is kept
// at every level above it.
//
// ks (1, 2, 4, 8 or 16) consecutive lanes share a cell, each summing every ks-th run of the lens
// tile, so coarse levels with few cells still fill the GPU; the partial sums then meet in a fixed
// butterfly and the first lane of the group decides.
__global__ void __launch_bounds__(kThreads) k_zoom_mark(const ZoomArgs z, int level, int ks)
{
    __shared__ float4 s_lens[2][kZoomLT];
    const int part = threadIdx.x & (ks - 1);
    const int64_t t_id = (int64_t)blockIdx.x * (kThreads / ks) + threadIdx.x / ks;
    const int64_t P = z.P, PP = z.P * z.P;
    const int64_t cw1 = z.lcw1[level], cw2 = z.lcw2[level];
    int64_t n_items, cx = 0, cy = 0, idx = 0;
    if (level == 0) {
        n_items = z.lnx[0] * z.lny[0];
        if (t_id < n_items) {
            cx = t_id % z.lnx[0];
            cy = t_id / z.lnx[0];
            idx = t_id;
        }
    } else {
        n_items = (int64_t)z.stats[4 + level - 1] * PP;
        if (t_id < n_items) {
            const int64_t par = z.lists[level - 1][t_id / PP], k = t_id % PP;
            cx = (par % z.lnx[level - 1]) * P + k % P;
            cy = (par / z.lnx[level - 1]) * P + k / P;
            idx = cy * z.lnx[level] + cx;
        }
    }
    if ((int64_t)blockIdx.x * (kThreads / ks) >= n_items) return;      // whole workgroup idle
    const bool active = t_id < n_items && cx * cw1 < z.wn1 && cy * cw2 < z.wn2;
    // fine-grid index range of the cell (global indices), its rectangle, centre and half-widths
    const int64_t g10 = z.wlo1 + min(cx * cw1, z.wn1), g11 = z.wlo1 + min((cx + 1) * cw1, z.wn1);
    const int64_t g20 = z.wlo2 + min(cy * cw2, z.wn2), g21 = z.wlo2 + min((cy + 1) * cw2, z.wn2);
    const double e1lo = z.glo1 + (double)g10 * z.gt1, e1hi = z.glo1 + (double)g11 * z.gt1;
    const double e2lo = z.glo2 + (double)g20 * z.gt2, e2hi = z.glo2 + (double)g21 * z.gt2;
    const float cf1 = (float)(0.5 * (e1lo + e1hi)), cf2 = (float)(0.5 * (e2lo + e2hi));
    // the rectangle around the float32 centre that holds every fine ray's float32 coordinates
    const double h1 = fmax(fabs(e1lo - (double)cf1), fabs(e1hi - (double)cf1)) + z.pad;
    const double h2 = fmax(fabs(e2lo - (double)cf2), fabs(e2hi - (double)cf2)) + z.pad;
    const double rho2 = h1 * h1 + h2 * h2;
    const float near2 = (float)(9.0 * rho2);
    const float fh1 = (float)h1, fh2 = (float)h2;

    double A1 = 0.0, A2 = 0.0, Jd = 0.0, Jo = 0.0, C3 = 0.0, P1 = 0.0, D2 = 0.0, nearsum = 0.0;
    bool inside = false;

    const int tid = threadIdx.x;
    const int64_t n_tiles = (z.n_lens + kZoomLT - 1) / kZoomLT;
    if (n_tiles > 0) {
        const int64_t i = tid;
        s_lens[0][tid] = i < z.n_lens ? moved_lens(z.lenses[i], z.vel, i, z.time) : zoom_pad_lens();
    }
    __syncthreads();
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int buf = (int)(t & 1);
        float4 nxt = zoom_pad_lens();
        const bool more = t + 1 < n_tiles;
        if (more) {
            const int64_t i = (t + 1) * kZoomLT + tid;
            if (i < z.n_lens) nxt = moved_lens(z.lenses[i], z.vel, i, z.time);
        }
        for (int r = part * kZoomRun; r < kZoomLT; r += ks * kZoomRun) {
            float s1 = 0.f, s2 = 0.f, sd = 0.f, so = 0.f, sc = 0.f, sp = 0.f, sq = 0.f;
            bool near_seen = false;
#pragma unroll
            for (int j = 0; j < kZoomRun; ++j) {
                const float4 l = s_lens[buf][r + j];
                const float f1 = cf1 - l.x, f2 = cf2 - l.y;
                const float f1s = f1 * f1, f2s = f2 * f2;
                const float r2 = f1s + f2s;
                const float s = __builtin_amdgcn_rsqf(r2);
                const float q = s * s;
                const float d = l.z * q;
                s1 = fmaf(d, f1, s1);
                s2 = fmaf(d, f2, s2);
                // the rounding-allowance sums take every lens (an over-estimate is safe)
                sp = fmaf(l.z, s, sp);
                sq += d;
                // the Taylor terms only the lenses at distance >= 3 rho
                const bool nr = r2 < near2;
                near_seen = near_seen || nr;
                const float dt = nr ? 0.0f : d;
                const float dq = dt * q;
                sd = fmaf(dq, f2s - f1s, sd);
                so = fmaf(dq, f1 * f2, so);
                sc = fmaf(dt, s, sc);
            }
            if (__any(near_seen)) {
                // near lenses (rare): bound each one's whole variation over the cell by 2 m / delta
                float ns = 0.0f;
#pragma unroll
                for (int j = 0; j < kZoomRun; ++j) {
                    const float4 l = s_lens[buf][r + j];
                    const float f1 = cf1 - l.x, f2 = cf2 - l.y;
                    const bool nr = f1 * f1 + f2 * f2 < near2 && l.z != 0.0f;
                    const float ex = fmaxf(fabsf(f1) - fh1, 0.0f), ey = fmaxf(fabsf(f2) - fh2, 0.0f);
                    const float dl2 = ex * ex + ey * ey;
                    inside = inside || (nr && !(dl2 > 0.0f));
                    ns += nr && dl2 > 0.0f ? l.z * __builtin_amdgcn_rsqf(dl2) : 0.0f;
                }
                nearsum += (double)ns;
            }
            A1 += (double)s1;
            A2 += (double)s2;
            Jd += (double)sd;
            Jo += (double)so;
            C3 += (double)sc;
            P1 += (double)sp;
            D2 += (double)sq;
        }
        if (more) s_lens[buf ^ 1][tid] = nxt;
        __syncthreads();
    }
    // the group's partial sums, combined in a fixed order
    int in_any = inside ? 1 : 0;
    for (int o = 1; o < ks; o <<= 1) {
        A1 += __shfl_xor(A1, o, 64);
        A2 += __shfl_xor(A2, o, 64);
        Jd += __shfl_xor(Jd, o, 64);
        Jo += __shfl_xor(Jo, o, 64);
        C3 += __shfl_xor(C3, o, 64);
        P1 += __shfl_xor(P1, o, 64);
        D2 += __shfl_xor(D2, o, 64);
        nearsum += __shfl_xor(nearsum, o, 64);
        in_any |= __shfl_xor(in_any, o, 64);
    }
    inside = in_any != 0;
    if (!active || part != 0) return;

    // centre image and the bounds, FP64
    const double y1 = z.lam1 * (double)cf1 - A1, y2 = z.lam2 * (double)cf2 - A2;
    const double J11 = fabs(z.lam1 - Jd), J22 = fabs(z.lam2 + Jd), J12 = 2.0 * fabs(Jo);
    const double tay = rho2 * 3.375 * C3;
    const double nv = 2.0 * nearsum;
    // rounding allowance: float32 arithmetic of the fine rays and of this centre evaluation
    const double scale = 1.5 * P1 + nearsum + fabs(z.lam1 * (double)cf1) + fabs(z.lam2 * (double)cf2) +
                         fabs(y1) + fabs(y2) + z.xmax * 2.25 * D2;
    const double slack = 1e-5 * scale + z.margin;
    const double E1 = (J11 * h1 + J12 * h2 + tay + nv + slack) * (1.0 + 1e-6);
    const double E2 = (J12 * h1 + J22 * h2 + tay + nv + slack) * (1.0 + 1e-6);
    bool keep = inside || !(fabs(y1) < 1e300 && fabs(y2) < 1e300 && E1 < 1e300 && E2 < 1e300);
    if (!keep)
        keep = (y1 + E1 >= z.zlo1) && (y1 - E1 <= z.zhi1) && (y2 + E2 >= z.zlo2) && (y2 - E2 <= z.zhi2);
    if (keep) {
        uint32_t *cnt = level == z.levels - 1 ? &z.stats[0] : &z.stats[4 + level];
        z.lists[level][atomicAdd(cnt, 1u)] = (uint32_t)idx;
    }
}

}  // namespace

hipError_t launch_zoom_mark(const ZoomArgs &z, hipStream_t s)
{
    int64_t items = z.lnx[0] * z.lny[0];
    if (items <= 0) return hipSuccess;
    for (int l = 0; l < z.levels; ++l) {
        // level l > 0 runs over at most every child of every cell of level l - 1; workgroups
        // past the kept children exit at once.  Lanes per cell: enough to give about 2^18
        // threads for the expected work (every cell at level 0, the children of about a third
        // of the cells above further down); the choice only affects speed.
        if (l > 0) items = z.lnx[l - 1] * z.lny[l - 1] * z.P * z.P;
        const int64_t expect = l == 0 ? items : std::max<int64_t>(1, items / 3);
        int ks = 1;
        while (ks < 16 && expect * ks < (int64_t(1) << 18)) ks <<= 1;
        const int64_t per_block = kThreads / ks;
        hipLaunchKernelGGL(k_zoom_mark, dim3((unsigned)((items + per_block - 1) / per_block)), dim3(kThreads), 0, s, z,
                           l, ks);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rs
