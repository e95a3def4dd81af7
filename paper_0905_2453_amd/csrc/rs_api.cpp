// Host runtime of librs: argument validation, launch geometry and the C ABI (include/rs.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "rs_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int dev_fail(hipError_t e, const char *what)
{
    return fail(RS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite(double v) { return std::isfinite(v); }

constexpr double kMaxCoord = 1.0e12;  // far below the position of the zero-mass padding lenses

// Resolved tuning of one direct-sum launch.
struct Tune {
    int K1 = 1, K2 = 4, T = 16, LT = 256, W = 64;
};

int resolve_opts(const rs_opts *o, Tune &t)
{
    if (!o) return RS_OK;
    if (o->block_cols || o->block_rows) {
        if (!rs::ray_block_supported(o->block_cols, o->block_rows))
            return fail(RS_EINVAL, "unsupported ray block %d x %d (use 1x4, 2x2, 2x4, 4x2, 4x4 or 2x8)",
                        o->block_cols, o->block_rows);
        t.K1 = o->block_cols;
        t.K2 = o->block_rows;
    }
    if (o->lens_tile) {
        if (o->lens_tile != 256 && o->lens_tile != 512)
            return fail(RS_EINVAL, "lens_tile must be 256 or 512 (got %d)", o->lens_tile);
        t.LT = o->lens_tile;
    }
    if (o->fp32_run) {
        if (o->fp32_run != 8 && o->fp32_run != 16 && o->fp32_run != 32)
            return fail(RS_EINVAL, "fp32_run must be 8, 16 or 32 (got %d)", o->fp32_run);
        t.T = o->fp32_run;
    }
    if (o->map_window) {
        if (o->map_window == -1) t.W = 0;
        else if (o->map_window == 16 || o->map_window == 32 || o->map_window == 64) t.W = o->map_window;
        else return fail(RS_EINVAL, "map_window must be 16, 32, 64 or -1 (got %d)", o->map_window);
    }
    if ((o->ray_y == nullptr) != (o->ray_pix == nullptr))
        return fail(RS_EINVAL, "ray_y and ray_pix must be given together");
    return RS_OK;
}

int validate_job(const rs_job *j)
{
    if (!j) return fail(RS_EINVAL, "job is NULL");
    if (j->n_lens < 0) return fail(RS_EINVAL, "n_lens < 0");
    if (j->n_lens > 0 && !j->lenses) return fail(RS_EINVAL, "lenses is NULL with n_lens > 0");
    if (!finite(j->macro.kappa_c) || !finite(j->macro.gamma)) return fail(RS_EINVAL, "macro not finite");
    const rs_raygrid &g = j->grid;
    for (int k = 0; k < 2; ++k) {
        if (!finite(g.lo[k]) || !finite(g.hi[k]) || !(g.hi[k] > g.lo[k]))
            return fail(RS_EINVAL, "grid axis %d: need finite lo < hi", k);
        if (std::fabs(g.lo[k]) > kMaxCoord || std::fabs(g.hi[k]) > kMaxCoord)
            return fail(RS_EINVAL, "grid axis %d: |coordinate| > 1e12", k);
        if (g.n[k] <= 0) return fail(RS_EINVAL, "grid axis %d: n <= 0", k);
        if (g.win_lo[k] < 0 || g.win_n[k] < 0 || g.win_lo[k] > g.n[k] || g.win_n[k] > g.n[k] - g.win_lo[k])
            return fail(RS_EINVAL, "grid axis %d: window outside the grid", k);
    }
    const rs_map &m = j->map;
    for (int k = 0; k < 2; ++k) {
        if (!finite(m.lo[k]) || !finite(m.hi[k]) || !(m.hi[k] > m.lo[k]))
            return fail(RS_EINVAL, "map axis %d: need finite lo < hi", k);
        if (m.n[k] <= 0) return fail(RS_EINVAL, "map axis %d: n <= 0", k);
    }
    if ((int64_t)m.n[0] * (int64_t)m.n[1] >= (int64_t(1) << 31))
        return fail(RS_ERANGE, "map has >= 2^31 pixels");
    if (!j->counts) return fail(RS_EINVAL, "counts is NULL");
    if (!j->n_lost) return fail(RS_EINVAL, "n_lost is NULL");
    if (g.win_n[0] * g.win_n[1] >= (int64_t(1) << 31))
        return fail(RS_ERANGE, "window has >= 2^31 rays; split it into several calls");
    return RS_OK;
}

int64_t partial_stride(const rs_job *j)
{
    const int64_t bins = (int64_t)j->map.n[0] * j->map.n[1];
    return (bins + 63) / 64 * 64;
}

}  // namespace

extern "C" {

const char *rs_status_str(int s)
{
    switch (s) {
    case RS_OK: return "RS_OK";
    case RS_EINVAL: return "RS_EINVAL";
    case RS_ERANGE: return "RS_ERANGE";
    case RS_EDEVICE: return "RS_EDEVICE";
    case RS_ESMALLBUF: return "RS_ESMALLBUF";
    case RS_ENOTFIT: return "RS_ENOTFIT";
    case RS_EINTERNAL: return "RS_EINTERNAL";
    default: return "RS_UNKNOWN";
    }
}

const char *rs_last_error(void) { return g_err; }

const char *rs_version(void) { return "librs 0.1 (gfx950)"; }

size_t rs_workspace_bytes(const rs_job *job, const rs_opts *opts)
{
    Tune t;
    if (validate_job(job) != RS_OK || resolve_opts(opts, t) != RS_OK) return 0;
    return (size_t)(rs::kPartials * partial_stride(job)) * sizeof(uint32_t) + 256;
}

int rs_shoot(const rs_job *job, void *workspace, size_t ws_bytes, void *stream, const rs_opts *opts)
{
    g_err[0] = '\0';
    int st = validate_job(job);
    if (st != RS_OK) return st;
    Tune t;
    if ((st = resolve_opts(opts, t)) != RS_OK) return st;
    const size_t need = rs_workspace_bytes(job, opts);
    if (!workspace) return fail(RS_EINVAL, "workspace is NULL");
    if (ws_bytes < need) return fail(RS_ESMALLBUF, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (opts && (opts->flags & RS_FLAG_FAULT_INJECT)) return fail(RS_EDEVICE, "injected fault (RS_FLAG_FAULT_INJECT)");

    const rs_raygrid &g = job->grid;
    if (g.win_n[0] == 0 || g.win_n[1] == 0) return RS_OK;

    uint32_t *part = reinterpret_cast<uint32_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    const int64_t pstride = partial_stride(job);
    const int64_t bins = (int64_t)job->map.n[0] * job->map.n[1];

    rs::DirectArgs a{};
    a.lenses = reinterpret_cast<const float4 *>(job->lenses);
    a.n_lens = job->n_lens;
    a.glo1 = g.lo[0];
    a.glo2 = g.lo[1];
    a.gt1 = (g.hi[0] - g.lo[0]) / (double)g.n[0];
    a.gt2 = (g.hi[1] - g.lo[1]) / (double)g.n[1];
    a.wlo1 = g.win_lo[0];
    a.wlo2 = g.win_lo[1];
    a.wn1 = g.win_n[0];
    a.wn2 = g.win_n[1];
    a.lam1 = (1.0 - job->macro.gamma) - job->macro.kappa_c;
    a.lam2 = (1.0 + job->macro.gamma) - job->macro.kappa_c;
    a.mlo1 = job->map.lo[0];
    a.mlo2 = job->map.lo[1];
    a.ms1 = (double)job->map.n[0] / (job->map.hi[0] - job->map.lo[0]);
    a.ms2 = (double)job->map.n[1] / (job->map.hi[1] - job->map.lo[1]);
    a.mn1 = job->map.n[0];
    a.mn2 = job->map.n[1];
    a.window = t.W;
    a.partial = part;
    a.pstride = pstride;
    a.lost = reinterpret_cast<unsigned long long *>(job->n_lost);
    a.ray_y = opts ? opts->ray_y : nullptr;
    a.ray_pix = opts ? opts->ray_pix : nullptr;

    const int64_t cols = 64 * (int64_t)t.K1;
    const int64_t tiles_x = (g.win_n[0] + cols - 1) / cols;
    const int64_t rows = (int64_t)rs::kWaves * t.K2;
    const int64_t tiles_y = (g.win_n[1] + rows - 1) / rows;
    if (tiles_x * tiles_y >= (int64_t(1) << 31)) return fail(RS_ERANGE, "too many ray tiles");
    a.tiles_x = (int32_t)tiles_x;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = rs::launch_zero(part, rs::kPartials * pstride, s);
    if (e != hipSuccess) return dev_fail(e, "zero partial maps");
    e = rs::launch_direct(a, t.K1, t.K2, t.T, t.LT, tiles_x * tiles_y, s);
    if (e != hipSuccess) return dev_fail(e, "direct-sum launch");
    e = rs::launch_reduce(part, bins, pstride, job->counts, s);
    if (e != hipSuccess) return dev_fail(e, "map reduce launch");
    return RS_OK;
}

}  // extern "C"
