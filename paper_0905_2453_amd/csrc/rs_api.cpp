// Host runtime of librs: argument validation, launch geometry and the C ABI (include/rs.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "rs_internal.h"
#include "rs_probe.h"

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

bool is_fin(double v) { return std::isfinite(v); }

constexpr double kMaxCoord = 1.0e12;  // far below the position of the zero-mass padding lenses

// Resolved tuning of one direct-sum launch.  T = 0 selects the float32 run length of the block
// shape: 8 lenses with one column per lane (four rows share a reciprocal), 16 with several (pairs).
struct Tune {
    int K1 = 1, K2 = 4, T = 0, LT = 256, W = 64;
    int run() const { return T ? T : (K1 == 1 ? 8 : 16); }
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
    if (!is_fin(j->macro.kappa_c) || !is_fin(j->macro.gamma)) return fail(RS_EINVAL, "macro not finite");
    const rs_raygrid &g = j->grid;
    for (int k = 0; k < 2; ++k) {
        if (!is_fin(g.lo[k]) || !is_fin(g.hi[k]) || !(g.hi[k] > g.lo[k]))
            return fail(RS_EINVAL, "grid axis %d: need finite lo < hi", k);
        if (std::fabs(g.lo[k]) > kMaxCoord || std::fabs(g.hi[k]) > kMaxCoord)
            return fail(RS_EINVAL, "grid axis %d: |coordinate| > 1e12", k);
        if (g.n[k] <= 0) return fail(RS_EINVAL, "grid axis %d: n <= 0", k);
        if (g.win_lo[k] < 0 || g.win_n[k] < 0 || g.win_lo[k] > g.n[k] || g.win_n[k] > g.n[k] - g.win_lo[k])
            return fail(RS_EINVAL, "grid axis %d: window outside the grid", k);
    }
    if ((g.jitter != 0 && g.jitter != 1) || g.reserved != 0) return fail(RS_EINVAL, "grid: jitter must be 0 or 1");
    if (g.n[0] > (int64_t(1) << 31) || g.n[1] > (int64_t(1) << 31) || g.n[0] * g.n[1] >= (int64_t(1) << 62))
        return fail(RS_ERANGE, "grid too large");
    const rs_map &m = j->map;
    for (int k = 0; k < 2; ++k) {
        if (!is_fin(m.lo[k]) || !is_fin(m.hi[k]) || !(m.hi[k] > m.lo[k]))
            return fail(RS_EINVAL, "map axis %d: need finite lo < hi", k);
        if (m.n[k] <= 0) return fail(RS_EINVAL, "map axis %d: n <= 0", k);
        if (!is_fin((double)m.n[k] / (m.hi[k] - m.lo[k])))
            return fail(RS_EINVAL, "map axis %d: pixels too small (n / (hi - lo) not finite)", k);
    }
    if ((int64_t)m.n[0] * (int64_t)m.n[1] >= (int64_t(1) << 31))
        return fail(RS_ERANGE, "map has >= 2^31 pixels");
    if (j->velocities && !is_fin(j->time)) return fail(RS_EINVAL, "time must be finite");
    if (!j->counts) return fail(RS_EINVAL, "counts is NULL");
    if (!j->n_lost) return fail(RS_EINVAL, "n_lost is NULL");
    if (g.win_n[0] * g.win_n[1] >= (int64_t(1) << 31))
        return fail(RS_ERANGE, "window has >= 2^31 rays; split it into several calls");
    return RS_OK;
}

// Rows of the ray window as the direct-sum kernels see it: reciprocals are shared by grid rows
// 4k..4k+3 (or pairs of them), so a window whose first row is not a multiple of 4 is widened by up
// to three masked rows.
int32_t row_skip(const rs_raygrid &g) { return g.win_n[1] > 0 ? (int32_t)(g.win_lo[1] & 3) : 0; }
int64_t kernel_rows(const rs_raygrid &g) { return g.win_n[1] + row_skip(g); }

int64_t partial_stride(const rs_job *j)
{
    const int64_t bins = (int64_t)j->map.n[0] * j->map.n[1];
    return (bins + 63) / 64 * 64;
}

// Device-side description of one job for a K1 x K2 ray block; counts go to `partial`.
rs::DirectArgs make_args(const rs_job *job, const Tune &t, uint32_t *partial, int64_t pstride,
                         const rs_opts *opts)
{
    const rs_raygrid &g = job->grid;
    rs::DirectArgs a{};
    a.lenses = reinterpret_cast<const float4 *>(job->lenses);
    a.n_lens = job->n_lens;
    a.glo1 = g.lo[0];
    a.glo2 = g.lo[1];
    a.gt1 = (g.hi[0] - g.lo[0]) / (double)g.n[0];
    a.gt2 = (g.hi[1] - g.lo[1]) / (double)g.n[1];
    a.rskip = row_skip(g);
    a.wlo1 = g.win_lo[0];
    a.wlo2 = g.win_lo[1] - a.rskip;
    a.wn1 = g.win_n[0];
    a.wn2 = kernel_rows(g);
    a.lam1 = (1.0 - job->macro.gamma) - job->macro.kappa_c;
    a.lam2 = (1.0 + job->macro.gamma) - job->macro.kappa_c;
    a.mlo1 = job->map.lo[0];
    a.mlo2 = job->map.lo[1];
    a.ms1 = (double)job->map.n[0] / (job->map.hi[0] - job->map.lo[0]);
    a.ms2 = (double)job->map.n[1] / (job->map.hi[1] - job->map.lo[1]);
    a.mn1 = job->map.n[0];
    a.mn2 = job->map.n[1];
    a.window = t.W;
    a.partial = partial;
    a.pstride = pstride;
    a.lost = reinterpret_cast<unsigned long long *>(job->n_lost);
    a.ray_y = opts ? opts->ray_y : nullptr;
    a.ray_pix = opts ? opts->ray_pix : nullptr;
    const int64_t cols = 64 * (int64_t)t.K1;
    a.tiles_x = (int32_t)((g.win_n[0] + cols - 1) / cols);
    a.gn1 = g.n[0];
    a.jitter = g.jitter;
    a.jkey1 = rs::jitter_key(g.jitter_seed, 0);
    a.jkey2 = rs::jitter_key(g.jitter_seed, 1);
    a.vel = reinterpret_cast<const float2 *>(job->velocities);
    a.time = job->time;
    return a;
}

int64_t tile_count(const rs_job *job, const Tune &t)
{
    const int64_t cols = 64 * (int64_t)t.K1;
    const int64_t rows = (int64_t)rs::kWaves * t.K2;
    return ((job->grid.win_n[0] + cols - 1) / cols) * ((kernel_rows(job->grid) + rows - 1) / rows);
}

// ---------------------------------------------------------------- batched launches

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BatchLayout {
    size_t queue_off, table_off, start_off, scratch_off, lost_off, total;
};

BatchLayout batch_layout(const rs_job *jobs, int32_t n_jobs)
{
    BatchLayout L{};
    size_t off = 0;
    L.queue_off = off;
    off += 256;
    L.table_off = off;
    off += align256((size_t)n_jobs * sizeof(rs::DirectArgs));
    L.start_off = off;
    off += align256(((size_t)n_jobs + 1) * sizeof(uint32_t));
    int64_t max_bins = 1;
    for (int32_t j = 0; j < n_jobs; ++j)
        max_bins = std::max<int64_t>(max_bins, (int64_t)jobs[j].map.n[0] * jobs[j].map.n[1]);
    L.scratch_off = off;
    off += align256((size_t)max_bins * sizeof(uint32_t));
    L.lost_off = off;
    off += 256;
    L.total = off + 256;  // slack to align the caller's base pointer
    return L;
}

std::mutex g_mu;
// Host staging copies of uploaded job tables, kept alive per workspace address.
std::map<void *, std::vector<uint8_t>> g_tables;

struct GraphKey {
    void *ws;
    int device, K1, K2, T, LT, W, grid, n_jobs;
    uint32_t n_items;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(ws, device, K1, K2, T, LT, W, grid, n_jobs, n_items) <
               std::tie(o.ws, o.device, o.K1, o.K2, o.T, o.LT, o.W, o.grid, o.n_jobs, o.n_items);
    }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;
constexpr size_t kMaxGraphs = 32;

struct PreparedBatch {
    rs::BatchArgs args{};
    uint64_t interactions = 0;  // ray-lens interactions of the items taken
    int grid = 0;
    int device = 0;
};

// Validate, order by decreasing work per tile, upload the job table into the workspace and fill
// the kernel arguments.  With `scratch`, every job's counts and lost counter are redirected to a
// scratch map inside the workspace (used by the autotuner).  At most `item_budget` ray-lens
// interactions worth of items are taken (0 = all).
int prepare_batch(const rs_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes, const Tune &t,
                  hipStream_t s, bool scratch, uint64_t item_budget, PreparedBatch &pb)
{
    if (n_jobs < 0) return fail(RS_EINVAL, "n_jobs < 0");
    if (n_jobs > 0 && !jobs) return fail(RS_EINVAL, "jobs is NULL");
    if (!workspace) return fail(RS_EINVAL, "workspace is NULL");
    for (int32_t j = 0; j < n_jobs; ++j) {
        const int st = validate_job(&jobs[j]);
        if (st != RS_OK) {
            char buf[512];
            snprintf(buf, sizeof buf, "job %d: %s", j, g_err);
            return fail(st, "%s", buf);
        }
    }
    const BatchLayout L = batch_layout(jobs, n_jobs);
    if (ws_bytes < L.total) return fail(RS_ESMALLBUF, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
    uint8_t *base = reinterpret_cast<uint8_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);

    std::vector<int32_t> order(n_jobs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return jobs[a].n_lens > jobs[b].n_lens; });

    const size_t table_bytes = (size_t)n_jobs * sizeof(rs::DirectArgs);
    const size_t start_bytes = ((size_t)n_jobs + 1) * sizeof(uint32_t);
    std::vector<uint8_t> host(table_bytes + start_bytes);
    auto *args = reinterpret_cast<rs::DirectArgs *>(host.data());
    auto *start = reinterpret_cast<uint32_t *>(host.data() + table_bytes);
    uint64_t items = 0, taken = 0, inter = 0;
    const uint64_t rays_per_tile = 64ull * (uint64_t)t.K1 * (uint64_t)rs::kWaves * (uint64_t)t.K2;
    start[0] = 0;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const rs_job *job = &jobs[order[k]];
        uint32_t *counts = job->counts;
        if (scratch) {
            rs_job tmp = *job;
            tmp.counts = reinterpret_cast<uint32_t *>(base + L.scratch_off);
            tmp.n_lost = reinterpret_cast<uint64_t *>(base + L.lost_off);
            args[k] = make_args(&tmp, t, tmp.counts, 0, nullptr);
        } else {
            args[k] = make_args(job, t, counts, 0, nullptr);
        }
        const int64_t nt = tile_count(job, t);
        items += (uint64_t)nt;
        if (items >= (uint64_t(1) << 31)) return fail(RS_ERANGE, "more than 2^31 ray tiles in one batch");
        start[k + 1] = (uint32_t)items;
        for (int64_t i = 0; i < nt; ++i) {
            if (item_budget && inter >= item_budget) break;
            inter += rays_per_tile * (uint64_t)job->n_lens;
            ++taken;
        }
    }
    if (!item_budget) taken = items;

    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return dev_fail(e, "device query");
    const int occ = rs::batched_occupancy(t.K1, t.K2, t.run(), t.LT);
    if (occ <= 0) return fail(RS_EINTERNAL, "no occupancy for the batched kernel");

    {
        std::lock_guard<std::mutex> lk(g_mu);
        std::vector<uint8_t> &keep = g_tables[workspace];
        keep.swap(host);
        if (table_bytes) {
            e = hipMemcpyAsync(base + L.table_off, keep.data(), table_bytes, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return dev_fail(e, "job table upload");
        }
        e = hipMemcpyAsync(base + L.start_off, keep.data() + table_bytes, start_bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return dev_fail(e, "job table upload");
    }
    pb.args.jobs = reinterpret_cast<const rs::DirectArgs *>(base + L.table_off);
    pb.args.item_start = reinterpret_cast<const uint32_t *>(base + L.start_off);
    pb.args.n_jobs = n_jobs;
    pb.args.n_items = (uint32_t)taken;
    pb.args.queue = reinterpret_cast<uint32_t *>(base + L.queue_off);
    pb.interactions = item_budget ? inter : 0;
    pb.grid = (int)std::min<uint64_t>(std::max<uint64_t>(taken, 1), (uint64_t)cus * (uint64_t)occ);
    pb.device = dev;
    return RS_OK;
}

// Reset the work counter and run the persistent kernel, captured once into a graph per
// (workspace, shape, grid, batch size) and replayed afterwards; the legacy default stream cannot
// be captured, so there the two kernels are launched directly.
int run_batch(const PreparedBatch &pb, const Tune &t, void *workspace, hipStream_t s, bool use_graph)
{
    if (pb.args.n_items == 0) return RS_OK;
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = rs::launch_fill_u32(pb.args.queue, 1, 0u, s);
        if (e == hipSuccess) e = rs::launch_batched(pb.args, t.K1, t.K2, t.run(), t.LT, pb.grid, s);
        return e;
    };
    if (!use_graph || s == nullptr) {
        const hipError_t e = enqueue();
        return e == hipSuccess ? RS_OK : dev_fail(e, "batched launch");
    }
    const GraphKey key{workspace, pb.device, t.K1, t.K2, t.run(), t.LT, t.W, pb.grid, pb.args.n_jobs, pb.args.n_items};
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) exec = it->second;
    }
    if (!exec) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return dev_fail(e, "begin capture");
        const hipError_t el = enqueue();
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(s, &graph);
        if (el != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return dev_fail(el, "batched launch (capture)");
        }
        if (e != hipSuccess) return dev_fail(e, "end capture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return dev_fail(e, "graph instantiate");
        std::lock_guard<std::mutex> lk(g_mu);
        if (g_graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(g_graphs.begin()->second);
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs[key] = exec;
    }
    const hipError_t e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? RS_OK : dev_fail(e, "graph launch");
}

std::string tune_key(const rs_job *jobs, int32_t n_jobs)
{
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::vector<double> nl, rays, bins;
    for (int32_t j = 0; j < n_jobs; ++j) {
        nl.push_back(std::log2(1.0 + (double)jobs[j].n_lens));
        rays.push_back(std::log2(1.0 + (double)jobs[j].grid.win_n[0] * (double)jobs[j].grid.win_n[1]));
        bins.push_back(std::log2(1.0 + (double)jobs[j].map.n[0] * (double)jobs[j].map.n[1]));
    }
    auto med = [](std::vector<double> v) {
        if (v.empty()) return 0L;
        std::sort(v.begin(), v.end());
        return (long)std::lround(v[v.size() / 2]);
    };
    std::ostringstream o;
    o << arch << "|lens2^" << med(nl) << "|rays2^" << med(rays) << "|map2^" << med(bins);
    return o.str();
}

// ---------------------------------------------------------------- learned far field

struct FarGeom {
    int64_t tiles_x, tiles_y, n_tiles;
    int32_t TX, TY;
    double cs;
};

int validate_ff(const rs_job *job, const rs_ff_config *c, FarGeom &g, bool eval = false)
{
    int st = validate_job(job);
    if (st != RS_OK) return st;
    if (!c) return fail(RS_EINVAL, "far-field config is NULL");
    if (job->velocities && !eval)
        return fail(RS_EINVAL, "the far-field fit takes a static field (velocities apply to rs_farfield_eval)");
    if (c->tile_rays[0] <= 0 || c->tile_rays[1] <= 0) return fail(RS_EINVAL, "tile_rays must be > 0");
    if ((int64_t)c->tile_rays[0] * c->tile_rays[1] > (int64_t(1) << 24))
        return fail(RS_ERANGE, "tile_rays: at most 2^24 rays per tile");
    if (!(c->r_near > 0.0) || !std::isfinite(c->r_near)) return fail(RS_EINVAL, "r_near must be finite and > 0");
    if (c->n_samples <= 0 || c->n_samples % 1024) return fail(RS_EINVAL, "n_samples must be a positive multiple of 1024");
    if (c->steps < 0) return fail(RS_EINVAL, "steps < 0");
    if (c->batch <= 0 || c->batch % 256 || c->n_samples % c->batch)
        return fail(RS_EINVAL, "batch must be a multiple of 256 dividing n_samples");
    if (!(c->lr >= 0.0f) || !std::isfinite(c->lr)) return fail(RS_EINVAL, "lr must be finite and >= 0");
    if (!(c->cell_size >= 0.0) || !std::isfinite(c->cell_size)) return fail(RS_EINVAL, "cell_size must be >= 0");
    if (c->shared_x != 0 && c->shared_x != 1) return fail(RS_EINVAL, "shared_x must be 0 or 1");
    g.TX = c->tile_rays[0];
    g.TY = c->tile_rays[1];
    g.tiles_x = (job->grid.win_n[0] + g.TX - 1) / g.TX;
    g.tiles_y = (job->grid.win_n[1] + g.TY - 1) / g.TY;
    g.n_tiles = g.tiles_x * g.tiles_y;
    if (g.n_tiles >= (int64_t(1) << 31)) return fail(RS_ERANGE, "too many far-field tiles");
    g.cs = c->cell_size > 0.0 ? c->cell_size : c->r_near / 4.0;
    return RS_OK;
}

uint64_t ff_hash(const rs_job *job, const rs_ff_config *c)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const uint8_t *b = static_cast<const uint8_t *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    mix(&job->grid, sizeof job->grid);
    mix(&job->n_lens, sizeof job->n_lens);
    mix(c->tile_rays, sizeof c->tile_rays);
    mix(&c->r_near, sizeof c->r_near);
    mix(&c->n_samples, sizeof c->n_samples);
    mix(&c->steps, sizeof c->steps);
    mix(&c->batch, sizeof c->batch);
    mix(&c->lr, sizeof c->lr);
    return h;
}

rs::FarArgs far_args(const rs_job *job, const rs_ff_config *c, const FarGeom &g)
{
    const rs_raygrid &gr = job->grid;
    rs::FarArgs f{};
    f.lenses = reinterpret_cast<const float4 *>(job->lenses);
    f.n_lens = job->n_lens;
    f.glo1 = gr.lo[0];
    f.glo2 = gr.lo[1];
    f.gt1 = (gr.hi[0] - gr.lo[0]) / (double)gr.n[0];
    f.gt2 = (gr.hi[1] - gr.lo[1]) / (double)gr.n[1];
    f.wlo1 = gr.win_lo[0];
    f.wlo2 = gr.win_lo[1];
    f.wn1 = gr.win_n[0];
    f.wn2 = gr.win_n[1];
    f.TX = g.TX;
    f.TY = g.TY;
    f.tiles_x = (int32_t)g.tiles_x;
    f.tiles_y = (int32_t)g.tiles_y;
    f.n_tiles = g.n_tiles;
    f.r_near = c->r_near;
    f.samples = c->samples;
    f.init_params = c->init_params;
    f.n_samples = c->n_samples;
    f.steps = c->steps;
    f.batch = c->batch;
    f.lr = c->lr;
    f.debug_grad = c->debug_grad;
    f.debug_targets = c->debug_targets;
    f.lam1 = (1.0 - job->macro.gamma) - job->macro.kappa_c;
    f.lam2 = (1.0 + job->macro.gamma) - job->macro.kappa_c;
    f.mlo1 = job->map.lo[0];
    f.mlo2 = job->map.lo[1];
    f.ms1 = (double)job->map.n[0] / (job->map.hi[0] - job->map.lo[0]);
    f.ms2 = (double)job->map.n[1] / (job->map.hi[1] - job->map.lo[1]);
    f.mn1 = job->map.n[0];
    f.mn2 = job->map.n[1];
    f.counts = job->counts;
    f.lost = reinterpret_cast<unsigned long long *>(job->n_lost);
    f.gn1 = gr.n[0];
    f.jitter = gr.jitter;
    f.jkey1 = rs::jitter_key(gr.jitter_seed, 0);
    f.jkey2 = rs::jitter_key(gr.jitter_seed, 1);
    return f;
}

size_t fit_ws_bytes(const FarGeom &g, const rs_ff_config *c)
{
    return align256((size_t)g.n_tiles * c->n_samples * 2 * sizeof(float)) +
           align256((size_t)g.n_tiles * 3 * rs::kNParams * sizeof(float)) + align256((size_t)c->steps * 4 * sizeof(float)) +
           256;
}

// Cell grid around the ray window grown by r_near (plus one cell): only lenses there can be near.
void cell_geom(const rs_job *job, const rs_ff_config *c, const FarGeom &g, double &ox, double &oy, int64_t &ncx,
               int64_t &ncy)
{
    const rs_raygrid &gr = job->grid;
    const double t1 = (gr.hi[0] - gr.lo[0]) / (double)gr.n[0], t2 = (gr.hi[1] - gr.lo[1]) / (double)gr.n[1];
    const double x0 = gr.lo[0] + (double)gr.win_lo[0] * t1, x1 = gr.lo[0] + (double)(gr.win_lo[0] + gr.win_n[0]) * t1;
    const double y0 = gr.lo[1] + (double)gr.win_lo[1] * t2, y1 = gr.lo[1] + (double)(gr.win_lo[1] + gr.win_n[1]) * t2;
    ox = x0 - c->r_near - g.cs;
    oy = y0 - c->r_near - g.cs;
    ncx = (int64_t)std::ceil((x1 + c->r_near + g.cs - ox) / g.cs);
    ncy = (int64_t)std::ceil((y1 + c->r_near + g.cs - oy) / g.cs);
}

// The three launches of one plain map: clear the kPartials partial maps at `part` (a fill kernel,
// never hipMemsetAsync), run the direct sum into them, add them into the caller's map.
int shoot_with_partials(const rs_job *job, const Tune &t, uint32_t *part, hipStream_t s, const rs_opts *opts)
{
    const int64_t pstride = partial_stride(job);
    const int64_t bins = (int64_t)job->map.n[0] * job->map.n[1];
    const rs::DirectArgs a = make_args(job, t, part, pstride, opts);
    hipError_t e = rs::launch_zero(part, rs::kPartials * pstride, s);
    if (e != hipSuccess) return dev_fail(e, "zero partial maps");
    e = rs::launch_direct(a, t.K1, t.K2, t.run(), t.LT, tile_count(job, t), s);
    if (e != hipSuccess) return dev_fail(e, "direct-sum launch");
    e = rs::launch_reduce(part, bins, pstride, job->counts, s);
    if (e != hipSuccess) return dev_fail(e, "map reduce launch");
    return RS_OK;
}

size_t eval_ws_bytes(const rs_job *job, const rs_ff_config *c, const FarGeom &g)
{
    double ox, oy;
    int64_t ncx, ncy;
    cell_geom(job, c, g, ox, oy, ncx, ncy);
    const size_t cells = (size_t)(ncx * ncy);
    return align256(cells * 4) * 2 + align256((cells + 1) * 4) + align256((size_t)std::max<int64_t>(job->n_lens, 1) * 4) +
           align256((size_t)g.n_tiles * 8 * sizeof(double)) + 256 + 256;
}

// Offset of the lens checksum word in the eval workspace (after the cell lists and affine bases).
size_t eval_checksum_off(const rs_job *job, const FarGeom &g, size_t cells)
{
    return align256(cells * 4) * 2 + align256((cells + 1) * 4) + align256((size_t)std::max<int64_t>(job->n_lens, 1) * 4) +
           align256((size_t)g.n_tiles * 8 * sizeof(double));
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
    if (tile_count(job, t) >= (int64_t(1) << 31)) return fail(RS_ERANGE, "too many ray tiles");
    uint32_t *part = reinterpret_cast<uint32_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    return shoot_with_partials(job, t, part, reinterpret_cast<hipStream_t>(stream), opts);
}

int rs_shoot_noalloc(const rs_job *job, void *stream, const rs_opts *opts)
{
    g_err[0] = '\0';
    int st = validate_job(job);
    if (st != RS_OK) return st;
    Tune t;
    if ((st = resolve_opts(opts, t)) != RS_OK) return st;
    if (partial_stride(job) > rs::kNoAllocBins)
        return fail(RS_ERANGE, "map of %lld bins: rs_shoot_noalloc takes at most %d (1024 x 1024); use rs_shoot",
                    (long long)((int64_t)job->map.n[0] * job->map.n[1]), rs::kNoAllocBins);
    if (opts && (opts->flags & RS_FLAG_FAULT_INJECT)) return fail(RS_EDEVICE, "injected fault (RS_FLAG_FAULT_INJECT)");
    const rs_raygrid &g = job->grid;
    if (g.win_n[0] == 0 || g.win_n[1] == 0) return RS_OK;
    if (tile_count(job, t) >= (int64_t(1) << 31)) return fail(RS_ERANGE, "too many ray tiles");
    uint32_t *part = nullptr;   // the library's fixed scratch array on the current device
    const hipError_t e = rs::noalloc_scratch(&part);
    if (e != hipSuccess) return dev_fail(e, "scratch address (hipGetSymbolAddress)");
    return shoot_with_partials(job, t, part, reinterpret_cast<hipStream_t>(stream), opts);
}

// ---------------------------------------------------------------- magnification (eq. 4)

int rs_magnification(const uint32_t *counts, const rs_raygrid *grid, const rs_map *map, double *mu,
                     double *n_av_out, void *stream)
{
    g_err[0] = '\0';
    if (!grid || !map) return fail(RS_EINVAL, "grid or map is NULL");
    for (int k = 0; k < 2; ++k) {
        if (!is_fin(grid->lo[k]) || !is_fin(grid->hi[k]) || !(grid->hi[k] > grid->lo[k]) || grid->n[k] <= 0)
            return fail(RS_EINVAL, "grid axis %d: need finite lo < hi and n > 0", k);
        if (!is_fin(map->lo[k]) || !is_fin(map->hi[k]) || !(map->hi[k] > map->lo[k]) || map->n[k] <= 0)
            return fail(RS_EINVAL, "map axis %d: need finite lo < hi and n > 0", k);
    }
    const int64_t bins = (int64_t)map->n[0] * map->n[1];
    if (bins >= (int64_t(1) << 31)) return fail(RS_ERANGE, "map has >= 2^31 pixels");
    // N_av: rays per pixel without lensing = pixel area / ray-cell area
    const double dx1 = (grid->hi[0] - grid->lo[0]) / (double)grid->n[0];
    const double dx2 = (grid->hi[1] - grid->lo[1]) / (double)grid->n[1];
    const double dy1 = (map->hi[0] - map->lo[0]) / (double)map->n[0];
    const double dy2 = (map->hi[1] - map->lo[1]) / (double)map->n[1];
    const double n_av = dy1 * dy2 / (dx1 * dx2);
    if (!is_fin(n_av) || !(n_av > 0.0)) return fail(RS_ERANGE, "N_av is not a finite positive number");
    if (n_av_out) *n_av_out = n_av;
    if (!counts || !mu) return fail(RS_EINVAL, "counts or mu is NULL");
    const hipError_t e = rs::launch_magnification(counts, bins, n_av, mu, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RS_OK : dev_fail(e, "magnification launch");
}

// ---------------------------------------------------------------- zoom

struct ZoomLayout {
    int64_t c1 = 0, c2 = 0, ncx = 0, ncy = 0, cells = 0, sx = 0, S = 0;
    int levels = rs::kZoomLevels;
    int64_t P = 2;                            // cells per parent side between levels
    int64_t lcw1[rs::kZoomLevels] = {}, lcw2[rs::kZoomLevels] = {}, lnx[rs::kZoomLevels] = {}, lny[rs::kZoomLevels] = {};
    size_t list_off[rs::kZoomLevels] = {};
    size_t part_off = 0, total = 0;
};

int zoom_layout(const rs_job *job, const rs_zoom *z, const Tune &t, ZoomLayout &L)
{
    if (!z) return fail(RS_EINVAL, "zoom is NULL");
    if (z->cell[0] < 0 || z->cell[1] < 0 || z->cell[0] > 65536 || z->cell[1] > 65536)
        return fail(RS_EINVAL, "zoom cell must be in [0, 65536]");
    if (!(z->margin >= 0.0) || !is_fin(z->margin)) return fail(RS_EINVAL, "zoom margin must be finite and >= 0");
    const rs_raygrid &g = job->grid;
    const double t1 = (g.hi[0] - g.lo[0]) / (double)g.n[0], t2 = (g.hi[1] - g.lo[1]) / (double)g.n[1];
    int64_t c1 = z->cell[0], c2 = z->cell[1];
    if (c1 == 0 && c2 == 0) {
        // about 64 fine rays per cell, square in the image plane, whole lane blocks
        c1 = std::max<int64_t>(1, std::min<int64_t>(4096, std::llround(std::sqrt(64.0 * t2 / t1))));
        c2 = std::max<int64_t>(1, std::min<int64_t>(4096, std::llround(64.0 / (double)c1)));
        c1 = (c1 + t.K1 - 1) / t.K1 * t.K1;
        c2 = (c2 + t.K2 - 1) / t.K2 * t.K2;
    } else if (c1 == 0 || c2 == 0) {
        return fail(RS_EINVAL, "zoom cell: give both sizes or neither");
    }
    L.c1 = c1;
    L.c2 = c2;
    L.ncx = (g.win_n[0] + c1 - 1) / c1;
    L.ncy = (g.win_n[1] + c2 - 1) / c2;
    L.cells = L.ncx * L.ncy;
    if (L.cells > (int64_t(1) << 30)) return fail(RS_ERANGE, "more than 2^30 culling cells; use larger cells");
    L.sx = (c1 + t.K1 - 1) / t.K1;
    // lane blocks start at the kernel row at or below a cell's first row that is a multiple of 4:
    // up to three more rows to cover when cells can start elsewhere
    const int64_t span2 = c2 + ((c2 % 4 != 0 || row_skip(g) != 0) ? 3 : 0);
    L.S = L.sx * ((span2 + t.K2 - 1) / t.K2);
    if ((uint64_t)L.cells * (uint64_t)L.S * (uint64_t)(t.K1 * t.K2) >= (uint64_t(1) << 40))
        return fail(RS_ERANGE, "too many ray slots");
    // level levels-1 is the cell grid; each coarser level groups P x P cells of the next
    size_t off = 256;
    for (int l = L.levels - 1; l >= 0; --l) {
        const int64_t f = (l == L.levels - 1) ? 1 : L.P * (L.lcw1[l + 1] / L.c1);
        L.lcw1[l] = c1 * f;
        L.lcw2[l] = c2 * f;
        L.lnx[l] = (g.win_n[0] + L.lcw1[l] - 1) / L.lcw1[l];
        L.lny[l] = (g.win_n[1] + L.lcw2[l] - 1) / L.lcw2[l];
    }
    for (int l = 0; l < L.levels; ++l) {
        L.list_off[l] = off;
        off += align256((size_t)(L.lnx[l] * L.lny[l]) * sizeof(uint32_t));
    }
    L.part_off = off;
    off += (size_t)(rs::kPartials * partial_stride(job)) * sizeof(uint32_t);
    L.total = off + 256;
    return RS_OK;
}

size_t rs_batched_workspace_bytes(const rs_job *jobs, int32_t n_jobs)
{
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return 0;
    for (int32_t j = 0; j < n_jobs; ++j)
        if (validate_job(&jobs[j]) != RS_OK) return 0;
    return batch_layout(jobs, n_jobs).total;
}

int rs_shoot_batched(const rs_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes, void *stream,
                     const rs_opts *opts)
{
    g_err[0] = '\0';
    Tune t;
    int st = resolve_opts(opts, t);
    if (st != RS_OK) return st;
    if (opts && (opts->ray_y || opts->ray_pix)) return fail(RS_EINVAL, "per-ray dumps are not available in batches");
    if (opts && (opts->flags & RS_FLAG_FAULT_INJECT)) {
        // validate first so the injected fault only stands for device failures
        if (n_jobs < 0 || (n_jobs > 0 && !jobs) || !workspace) return fail(RS_EINVAL, "bad batch arguments");
        return fail(RS_EDEVICE, "injected fault (RS_FLAG_FAULT_INJECT)");
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    PreparedBatch pb;
    st = prepare_batch(jobs, n_jobs, workspace, ws_bytes, t, s, false, 0, pb);
    if (st != RS_OK) return st;
    const bool graph = !(opts && (opts->flags & RS_FLAG_NO_GRAPH));
    return run_batch(pb, t, workspace, s, graph);
}

int rs_autotune_batched(const rs_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes, void *stream,
                        const char *cache_path, rs_opts *best)
{
    g_err[0] = '\0';
    if (!best) return fail(RS_EINVAL, "best is NULL");
    Tune base;
    int st = resolve_opts(best, base);
    if (st != RS_OK) return st;
    if (n_jobs <= 0 || !jobs) return fail(RS_EINVAL, "need at least one job");
    for (int32_t j = 0; j < n_jobs; ++j)
        if ((st = validate_job(&jobs[j])) != RS_OK) return st;
    const std::string key = tune_key(jobs, n_jobs);
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        bool found = false;
        int K1 = 0, K2 = 0, LT = 0, W = 0;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int a, b, c, d;
            if ((ls >> k >> a >> b >> c >> d) && k == key && rs::ray_block_supported(a, b)) {
                K1 = a; K2 = b; LT = c; W = d; found = true;
            }
        }
        if (found) {
            best->block_cols = K1;
            best->block_rows = K2;
            best->lens_tile = LT;
            best->map_window = W == 0 ? -1 : W;
            return RS_OK;
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int shapes[][2] = {{1, 4}, {2, 4}, {4, 4}, {2, 8}};
    const int windows[] = {32, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return dev_fail(e, "event create");
    double best_rate = -1.0;
    Tune win = base;
    const uint64_t budget = 200000000000ull;  // ~30 ms of work per candidate
    for (const auto &sh : shapes) {
        for (int W : windows) {
            Tune t = base;
            t.K1 = sh[0];
            t.K2 = sh[1];
            t.W = W;
            PreparedBatch pb;
            st = prepare_batch(jobs, n_jobs, workspace, ws_bytes, t, s, true, budget, pb);
            if (st != RS_OK) break;
            if ((st = run_batch(pb, t, workspace, s, false)) != RS_OK) break;  // warm-up
            e = hipEventRecord(e0, s);
            for (int r = 0; r < 2 && e == hipSuccess && st == RS_OK; ++r) st = run_batch(pb, t, workspace, s, false);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess || st != RS_OK) break;
            const double rate = 2.0 * (double)pb.interactions / std::max(1e-3, (double)ms);
            if (rate > best_rate) {
                best_rate = rate;
                win = t;
            }
        }
        if (e != hipSuccess || st != RS_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return dev_fail(e, "autotune timing");
    if (st != RS_OK) return st;
    best->block_cols = win.K1;
    best->block_rows = win.K2;
    best->lens_tile = win.LT;
    best->map_window = win.W == 0 ? -1 : win.W;
    if (cache_path && *cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << key << ' ' << win.K1 << ' ' << win.K2 << ' ' << win.LT << ' ' << win.W << '\n';
    }
    return RS_OK;
}

size_t rs_farfield_model_bytes(const rs_job *job, const rs_ff_config *cfg)
{
    FarGeom g;
    if (validate_ff(job, cfg, g, true) != RS_OK) return 0;
    return rs::kModelHeader + (size_t)g.n_tiles * rs::kTileRecord;
}

size_t rs_farfield_fit_workspace_bytes(const rs_job *job, const rs_ff_config *cfg)
{
    FarGeom g;
    if (validate_ff(job, cfg, g) != RS_OK) return 0;
    return fit_ws_bytes(g, cfg);
}

size_t rs_farfield_eval_workspace_bytes(const rs_job *job, const rs_ff_config *cfg)
{
    FarGeom g;
    if (validate_ff(job, cfg, g, true) != RS_OK) return 0;
    double ox, oy;
    int64_t ncx, ncy;
    cell_geom(job, cfg, g, ox, oy, ncx, ncy);
    if (ncx * ncy >= (int64_t(1) << 31)) return 0;
    return eval_ws_bytes(job, cfg, g);
}

int rs_farfield_fit(const rs_job *job, const rs_ff_config *cfg, void *model, size_t model_bytes, void *workspace,
                    size_t ws_bytes, void *stream)
{
    g_err[0] = '\0';
    FarGeom g;
    int st = validate_ff(job, cfg, g);
    if (st != RS_OK) return st;
    if (!cfg->samples || !cfg->init_params) return fail(RS_EINVAL, "samples and init_params are required");
    if (!model || !workspace) return fail(RS_EINVAL, "model and workspace are required");
    const size_t need_m = rs::kModelHeader + (size_t)g.n_tiles * rs::kTileRecord;
    if (model_bytes < need_m) return fail(RS_ESMALLBUF, "model %zu bytes < %zu needed", model_bytes, need_m);
    const size_t need_w = fit_ws_bytes(g, cfg);
    if (ws_bytes < need_w) return fail(RS_ESMALLBUF, "workspace %zu bytes < %zu needed", ws_bytes, need_w);
    if ((uintptr_t)model & 255) return fail(RS_EINVAL, "model must be 256-byte aligned");
    if (g.n_tiles == 0) return RS_OK;
    uint8_t *base = reinterpret_cast<uint8_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    rs::FarArgs f = far_args(job, cfg, g);
    if (cfg->shared_x) {
        // the shared first coordinates are a promise about the sample values: check it
        std::vector<float> smp((size_t)cfg->n_samples * 2);
        hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
        hipError_t e = hipMemcpyAsync(smp.data(), cfg->samples, smp.size() * sizeof(float), hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return dev_fail(e, "sample read");
        for (int g4 = 0; g4 < cfg->n_samples / 256; ++g4)
            for (int k = 1; k < 4; ++k)
                for (int i = 0; i < 64; ++i)
                    if (smp[2 * ((size_t)(4 * g4 + k) * 64 + i)] != smp[2 * ((size_t)(4 * g4) * 64 + i)])
                        return fail(RS_EINVAL, "samples %d and %d do not share their first coordinate",
                                    (4 * g4 + k) * 64 + i, 4 * g4 * 64 + i);
        f.grid_samples = 1;
    }
    f.model = static_cast<uint8_t *>(model);
    f.targets = reinterpret_cast<float *>(base);
    f.state = reinterpret_cast<float *>(base + align256((size_t)g.n_tiles * cfg->n_samples * 2 * sizeof(float)));
    f.sched = reinterpret_cast<float *>(reinterpret_cast<uint8_t *>(f.state) +
                                        align256((size_t)g.n_tiles * 3 * rs::kNParams * sizeof(float)));
    const hipError_t e = rs::launch_ff_fit(f, ff_hash(job, cfg), reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RS_OK : dev_fail(e, "far-field fit launch");
}

int rs_farfield_eval(const rs_job *job, const rs_ff_config *cfg, const void *model, size_t model_bytes,
                     void *workspace, size_t ws_bytes, void *stream, const rs_opts *opts)
{
    g_err[0] = '\0';
    FarGeom g;
    int st = validate_ff(job, cfg, g, true);
    if (st != RS_OK) return st;
    if (!model || !workspace) return fail(RS_EINVAL, "model and workspace are required");
    if (opts && ((opts->ray_y == nullptr) != (opts->ray_pix == nullptr)))
        return fail(RS_EINVAL, "ray_y and ray_pix must be given together");
    const size_t need_m = rs::kModelHeader + (size_t)g.n_tiles * rs::kTileRecord;
    if (model_bytes < need_m) return fail(RS_ESMALLBUF, "model %zu bytes < %zu needed", model_bytes, need_m);
    double ox, oy;
    int64_t ncx, ncy;
    cell_geom(job, cfg, g, ox, oy, ncx, ncy);
    if (ncx * ncy >= (int64_t(1) << 31)) return fail(RS_ERANGE, "cell grid too large; raise cell_size");
    const size_t need_w = eval_ws_bytes(job, cfg, g);
    if (ws_bytes < need_w) return fail(RS_ESMALLBUF, "workspace %zu bytes < %zu needed", ws_bytes, need_w);
    if (opts && (opts->flags & RS_FLAG_FAULT_INJECT)) return fail(RS_EDEVICE, "injected fault (RS_FLAG_FAULT_INJECT)");
    if (g.n_tiles == 0) return RS_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the model must have been fitted for this grid, tiling and configuration
    if (cfg->n_eval_tiles < 0 || (cfg->n_eval_tiles > 0 && !cfg->eval_tiles))
        return fail(RS_EINVAL, "eval_tiles / n_eval_tiles inconsistent");
    // ... and on this lens array: its checksum, computed now, must equal the one the fit stored
    uint8_t *base = reinterpret_cast<uint8_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    const size_t cells = (size_t)(ncx * ncy);
    uint64_t *csum = reinterpret_cast<uint64_t *>(base + eval_checksum_off(job, g, cells));
    uint64_t hdr[6] = {0, 0, 0, 0, 0, 0}, lens_sum = 0;
    std::vector<int32_t> tl(cfg->eval_tiles ? (size_t)cfg->n_eval_tiles : 0);
    hipError_t e = rs::launch_fill_u32(reinterpret_cast<uint32_t *>(csum), 2, 0u, s);
    if (e == hipSuccess)
        e = rs::launch_lens_checksum(reinterpret_cast<const float4 *>(job->lenses), job->n_lens,
                                     reinterpret_cast<unsigned long long *>(csum), s);
    if (e == hipSuccess) e = hipMemcpyAsync(hdr, model, sizeof hdr, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&lens_sum, csum, sizeof lens_sum, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !tl.empty())
        e = hipMemcpyAsync(tl.data(), cfg->eval_tiles, tl.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(e, "model header read");
    if (hdr[0] != rs::kModelMagic || hdr[1] != ff_hash(job, cfg))
        return fail(RS_ENOTFIT, "model was not fitted for this job and configuration");
    if (hdr[5] != lens_sum) return fail(RS_ENOTFIT, "model was fitted on a different lens array (checksum differs)");
    {
        std::vector<char> seen((size_t)g.n_tiles, 0);
        for (int32_t t : tl) {
            if (t < 0 || t >= g.n_tiles || seen[(size_t)t]) return fail(RS_EINVAL, "bad or repeated tile index %d", t);
            seen[(size_t)t] = 1;
        }
    }
    rs::FarArgs f = far_args(job, cfg, g);
    f.model = const_cast<uint8_t *>(static_cast<const uint8_t *>(model));
    f.ray_y = opts ? opts->ray_y : nullptr;
    f.ray_pix = opts ? opts->ray_pix : nullptr;
    f.affine_only = (opts && (opts->flags & RS_FLAG_AFFINE_ONLY)) ? 1 : 0;
    f.eval_tiles = cfg->eval_tiles;
    f.n_eval = cfg->eval_tiles ? cfg->n_eval_tiles : g.n_tiles;
    rs::CellArgs cg{};
    cg.lenses = f.lenses;
    cg.n_lens = job->n_lens;
    cg.ox = ox;
    cg.oy = oy;
    cg.cs = g.cs;
    cg.ncx = (int32_t)ncx;
    cg.ncy = (int32_t)ncy;
    cg.n_cells = (int32_t)cells;
    cg.count = reinterpret_cast<int32_t *>(base);
    cg.cursor = reinterpret_cast<int32_t *>(base + align256(cells * 4));
    cg.start = reinterpret_cast<int32_t *>(base + 2 * align256(cells * 4));
    cg.idx = reinterpret_cast<int32_t *>(base + 2 * align256(cells * 4) + align256((cells + 1) * 4));
    if (job->velocities) {
        f.vel = reinterpret_cast<const float2 *>(job->velocities);
        f.time = job->time;
        f.affine = reinterpret_cast<double *>(base + 2 * align256(cells * 4) + align256((cells + 1) * 4) +
                                              align256((size_t)std::max<int64_t>(job->n_lens, 1) * 4));
    }
    e = rs::launch_zero(reinterpret_cast<uint32_t *>(base), (int64_t)(2 * align256(cells * 4) / 4), s);
    if (e == hipSuccess) e = rs::launch_ff_eval(f, cg, s);
    return e == hipSuccess ? RS_OK : dev_fail(e, "far-field eval launch");
}

size_t rs_zoom_workspace_bytes(const rs_job *job, const rs_zoom *zoom, const rs_opts *opts)
{
    Tune t;
    ZoomLayout L;
    if (validate_job(job) != RS_OK || resolve_opts(opts, t) != RS_OK || zoom_layout(job, zoom, t, L) != RS_OK)
        return 0;
    return L.total;
}

int rs_shoot_zoom(const rs_job *job, const rs_zoom *zoom, void *workspace, size_t ws_bytes, void *stream,
                  const rs_opts *opts)
{
    g_err[0] = '\0';
    int st = validate_job(job);
    if (st != RS_OK) return st;
    Tune t;
    if ((st = resolve_opts(opts, t)) != RS_OK) return st;
    if (opts && (opts->ray_y || opts->ray_pix)) return fail(RS_EINVAL, "per-ray dumps are not available in a zoom");
    ZoomLayout L;
    if ((st = zoom_layout(job, zoom, t, L)) != RS_OK) return st;
    if (!workspace) return fail(RS_EINVAL, "workspace is NULL");
    if (ws_bytes < L.total) return fail(RS_ESMALLBUF, "workspace %zu bytes < %zu needed", ws_bytes, L.total);
    if (opts && (opts->flags & RS_FLAG_FAULT_INJECT)) return fail(RS_EDEVICE, "injected fault (RS_FLAG_FAULT_INJECT)");

    uint8_t *base = reinterpret_cast<uint8_t *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    uint32_t *stats = reinterpret_cast<uint32_t *>(base);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // statistics: [0] kept cells (the list length), [1] cells, [2] lane blocks per cell,
    // [3] rays per lane block, [4 + l] kept cells of the coarser level l < levels - 1
    static_assert(rs::kZoomLevels <= 5, "the statistics block holds four coarser levels");
    hipError_t e = rs::launch_fill_u32(stats, 8, 0u, s);
    if (e == hipSuccess) e = rs::launch_fill_u32(stats + 1, 1, (uint32_t)L.cells, s);
    if (e == hipSuccess) e = rs::launch_fill_u32(stats + 2, 1, (uint32_t)L.S, s);
    if (e == hipSuccess) e = rs::launch_fill_u32(stats + 3, 1, (uint32_t)(t.K1 * t.K2), s);
    if (e != hipSuccess) return dev_fail(e, "zoom statistics reset");
    const rs_raygrid &g = job->grid;
    if (g.win_n[0] == 0 || g.win_n[1] == 0) return RS_OK;

    uint32_t *part = reinterpret_cast<uint32_t *>(base + L.part_off);
    const int64_t pstride = partial_stride(job);
    const int64_t bins = (int64_t)job->map.n[0] * job->map.n[1];
    const rs::DirectArgs a = make_args(job, t, part, pstride, opts);

    rs::ZoomArgs z{};
    z.lenses = reinterpret_cast<const float4 *>(job->lenses);
    z.n_lens = job->n_lens;
    z.glo1 = a.glo1;
    z.glo2 = a.glo2;
    z.gt1 = a.gt1;
    z.gt2 = a.gt2;
    z.wlo1 = g.win_lo[0];
    z.wlo2 = g.win_lo[1];
    z.wn1 = g.win_n[0];
    z.wn2 = g.win_n[1];
    z.c1 = L.c1;
    z.c2 = L.c2;
    z.ncx = L.ncx;
    z.ncy = L.ncy;
    z.levels = L.levels;
    z.P = L.P;
    for (int l = 0; l < L.levels; ++l) {
        z.lcw1[l] = L.lcw1[l];
        z.lcw2[l] = L.lcw2[l];
        z.lnx[l] = L.lnx[l];
        z.lny[l] = L.lny[l];
        z.lists[l] = reinterpret_cast<uint32_t *>(base + L.list_off[l]);
    }
    z.lam1 = a.lam1;
    z.lam2 = a.lam2;
    z.zlo1 = job->map.lo[0];
    z.zlo2 = job->map.lo[1];
    z.zhi1 = job->map.hi[0];
    z.zhi2 = job->map.hi[1];
    z.margin = zoom->margin;
    // one float32 ulp of the largest grid coordinate: float32 ray coordinates lie within half of
    // it of their FP64 values, and the float32 cell centre within half of it of the true centre
    const double xmax = std::max(std::max(std::fabs(g.lo[0]), std::fabs(g.hi[0])),
                                 std::max(std::fabs(g.lo[1]), std::fabs(g.hi[1])));
    z.pad = std::ldexp(1.0, std::ilogb(std::max(xmax, 1e-30)) - 23);
    z.xmax = xmax;
    z.vel = a.vel;
    z.time = a.time;
    z.list = z.lists[L.levels - 1];
    z.stats = stats;

    rs::CellBlocks cb{};
    cb.list = z.list;
    cb.count = stats;
    cb.c1 = L.c1;
    cb.c2 = L.c2;
    cb.ncx = L.ncx;
    cb.sx = L.sx;
    cb.S = L.S;
    const int64_t max_groups = (L.cells * L.S + rs::kThreads - 1) / rs::kThreads;

    e = rs::launch_zero(part, rs::kPartials * pstride, s);
    if (e != hipSuccess) return dev_fail(e, "zero partial maps");
    e = rs::launch_zoom_mark(z, s);
    if (e != hipSuccess) return dev_fail(e, "zoom culling launch");
    e = rs::launch_direct_cells(a, t.K1, t.K2, t.run(), t.LT, cb, max_groups, s);
    if (e != hipSuccess) return dev_fail(e, "zoom direct-sum launch");
    e = rs::launch_reduce(part, bins, pstride, job->counts, s);
    if (e != hipSuccess) return dev_fail(e, "map reduce launch");
    return RS_OK;
}

int rs_zoom_stats(const void *workspace, uint64_t out[4], void *stream)
{
    g_err[0] = '\0';
    if (!workspace || !out) return fail(RS_EINVAL, "workspace and out are required");
    const void *base = reinterpret_cast<const void *>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    uint32_t st[4] = {0, 0, 0, 0};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(st, base, sizeof st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_fail(e, "zoom statistics read");
    out[0] = st[0];
    out[1] = st[1];
    out[2] = (uint64_t)st[0] * st[2] * st[3];
    out[3] = (uint64_t)st[1] * st[2] * st[3];
    return RS_OK;
}

int rs_plan_grid(const rs_map *map, const rs_macro *macro, double kappa_star, double lens_extent, double n_av,
                 double margin, rs_raygrid *out, double *n_av_out)
{
    g_err[0] = '\0';
    if (!map || !macro || !out) return fail(RS_EINVAL, "map, macro and out are required");
    for (int k = 0; k < 2; ++k)
        if (!is_fin(map->lo[k]) || !is_fin(map->hi[k]) || !(map->hi[k] > map->lo[k]) || map->n[k] <= 0)
            return fail(RS_EINVAL, "map axis %d invalid", k);
    if (!is_fin(macro->kappa_c) || !is_fin(macro->gamma)) return fail(RS_EINVAL, "macro not finite");
    if (!is_fin(kappa_star) || kappa_star < 0.0) return fail(RS_EINVAL, "kappa_star must be finite and >= 0");
    if (!is_fin(lens_extent) || lens_extent < 0.0) return fail(RS_EINVAL, "lens_extent must be finite and >= 0");
    if (!is_fin(n_av) || !(n_av > 0.0)) return fail(RS_EINVAL, "n_av must be finite and > 0");
    if (!is_fin(margin) || margin < 0.0) return fail(RS_EINVAL, "margin must be finite and >= 0");
    const double f = margin > 0.0 ? margin : 1.2;
    const double kappa = kappa_star + macro->kappa_c;
    const double lam[2] = {1.0 - kappa - macro->gamma, 1.0 - kappa + macro->gamma};
    double half[2], cen[2];
    for (int k = 0; k < 2; ++k) {
        const double l = std::fabs(lam[k]) >= 0.05 ? lam[k] : (lam[k] < 0.0 ? -0.05 : 0.05);
        half[k] = f * 0.5 * (map->hi[k] - map->lo[k]) / std::fabs(l);
        cen[k] = 0.5 * (map->lo[k] + map->hi[k]) / l;
    }
    const double pix = ((map->hi[0] - map->lo[0]) / map->n[0]) * ((map->hi[1] - map->lo[1]) / map->n[1]);
    const double t0 = std::sqrt(pix / n_av);
    if (!is_fin(pix) || !(pix > 0.0) || !is_fin(t0)) return fail(RS_ERANGE, "pixel area out of range");
    const double ext = std::max(std::fabs(cen[0]) + half[0], std::fabs(cen[1]) + half[1]) + lens_extent;
    if (!is_fin(ext) || ext > kMaxCoord) return fail(RS_EINVAL, "planned region too large");
    const double q = std::ldexp(1.0, std::ilogb(std::max(ext, 1e-30)) - 22);   // 2 ulp32 of ext
    const double t = std::floor(t0 / q) * q;
    if (!(t > 0.0)) return fail(RS_ERANGE, "n_av too high: cell below the float32 lattice of the region");
    if (!is_fin(t)) return fail(RS_ERANGE, "cell size out of range");
    for (int k = 0; k < 2; ++k) {
        const double n = std::max(1.0, std::ceil(2.0 * half[k] / t));
        if (n >= 2147483648.0) return fail(RS_ERANGE, "axis %d needs 2^31 rays or more", k);
        const double c = std::round(cen[k] / t) * t;
        out->n[k] = (int64_t)n;
        out->lo[k] = c - 0.5 * n * t;
        out->hi[k] = c + 0.5 * n * t;
        if (!is_fin(out->lo[k]) || !is_fin(out->hi[k]) || std::fabs(out->lo[k]) > kMaxCoord ||
            std::fabs(out->hi[k]) > kMaxCoord)
            return fail(RS_ERANGE, "planned region out of range");
        out->win_lo[k] = 0;
        out->win_n[k] = (int64_t)n;
    }
    out->jitter_seed = 0;
    out->jitter = 0;
    out->reserved = 0;
    if (n_av_out) *n_av_out = pix / (t * t);
    return RS_OK;
}

int rs_advance_lenses(const rs_lens *lenses, const float *velocities, int64_t n, double time, rs_lens *out,
                      void *stream)
{
    g_err[0] = '\0';
    if (n < 0) return fail(RS_EINVAL, "n < 0");
    if (n == 0) return RS_OK;
    if (!lenses || !velocities || !out) return fail(RS_EINVAL, "lenses, velocities and out are required");
    if (!is_fin(time)) return fail(RS_EINVAL, "time must be finite");
    const hipError_t e = rs::launch_advance(reinterpret_cast<const float4 *>(lenses),
                                            reinterpret_cast<const float2 *>(velocities), n, time,
                                            reinterpret_cast<float4 *>(out), reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RS_OK : dev_fail(e, "advance lenses launch");
}


int rs_light_curve(const uint32_t *counts, const rs_map *map, double n_av, const rs_source *src,
                   const double *tracks, int32_t n_tracks, int32_t n_points, int64_t frame_stride, double *mu,
                   double *mag, void *stream)
{
    g_err[0] = '\0';
    if (!map || !src) return fail(RS_EINVAL, "map and source are required");
    if (n_tracks < 0) return fail(RS_EINVAL, "n_tracks must be >= 0");
    if (n_points < 1) return fail(RS_EINVAL, "n_points must be >= 1");
    if ((int64_t)n_tracks * n_points > ((int64_t)1 << 36)) return fail(RS_EINVAL, "too many track points");
    for (int k = 0; k < 2; ++k)
        if (!std::isfinite(map->lo[k]) || !std::isfinite(map->hi[k]) || !(map->hi[k] > map->lo[k]) ||
            map->n[k] <= 0 || map->n[k] > 65536 || !std::isfinite((double)map->n[k] / (map->hi[k] - map->lo[k])))
            return fail(RS_EINVAL, "map axis %d invalid", k);
    if (!(n_av > 0.0) || !std::isfinite(n_av)) return fail(RS_EINVAL, "n_av must be finite and > 0");
    if (src->kind != 0 && src->kind != 1) return fail(RS_EINVAL, "source kind must be 0 or 1");
    if (!(src->size > 0.0) || !std::isfinite(src->size)) return fail(RS_EINVAL, "source size must be finite and > 0");
    if (!(src->cutoff >= 0.0) || !std::isfinite(src->cutoff)) return fail(RS_EINVAL, "cutoff must be finite and >= 0");
    if (src->layout < 0 || src->layout > 2) return fail(RS_EINVAL, "layout must be 0, 1 or 2");
    if (frame_stride != 0 && frame_stride < (int64_t)map->n[0] * map->n[1])
        return fail(RS_EINVAL, "frame_stride must be 0 or at least one map (%lld words)",
                    (long long)map->n[0] * map->n[1]);
    if (n_tracks == 0) return RS_OK;
    if (!counts || !tracks) return fail(RS_EINVAL, "counts and tracks are required");
    rs::LightArgs a{};
    a.counts = counts;
    for (int k = 0; k < 2; ++k) {
        a.lo[k] = map->lo[k];
        a.w[k] = (map->hi[k] - map->lo[k]) / (double)map->n[k];
        a.inv_w[k] = (double)map->n[k] / (map->hi[k] - map->lo[k]);
        a.n[k] = map->n[k];
    }
    a.n_av = n_av;
    a.inv2s2 = 1.0 / (2.0 * src->size * src->size);
    a.kind = src->kind;
    a.size = src->size;
    a.support = src->kind == 0 ? (src->cutoff > 0.0 ? src->cutoff : 4.0) * src->size : src->size;
    a.tracks = tracks;
    a.n_tracks = n_tracks;
    a.n_points = n_points;
    a.mu = mu;
    a.mag = mag;
    a.path = src->layout;
    a.frame_stride = frame_stride;
    const hipError_t e = rs::launch_light_curve(a, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? RS_OK : dev_fail(e, "light-curve launch");
}

int rs_probe_issue_rate(int op, double *lane_ops_per_s, double *seconds, void *stream)
{
    g_err[0] = '\0';
    if (op < RS_PROBE_FMAC_F32 || op > RS_PROBE_ADD_F64) return fail(RS_EINVAL, "unknown probe %d", op);
    if (!lane_ops_per_s) return fail(RS_EINVAL, "lane_ops_per_s is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return dev_fail(e, "device query");
    // 8 workgroups of 4 waves per compute unit: 8 waves per SIMD, enough to hide every latency
    const int blocks = 8 * cus;
    // about 20 ms per launch at the measured rates (reciprocals and FP64 adds issue slower)
    const int iters = (op == RS_PROBE_RCP_F32 || op == RS_PROBE_ADD_F64) ? 2048 : 8192;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = rs::launch_probe(op, blocks, iters, s);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(t0, s);
    if (e == hipSuccess) e = rs::launch_probe(op, blocks, iters, s);
    if (e == hipSuccess) e = hipEventRecord(t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return dev_fail(e, "probe launch");
    if (!(ms > 0.f)) return fail(RS_EDEVICE, "probe timing gave %g ms", (double)ms);
    const double ops = (double)blocks * 256.0 * (double)iters * (double)rs::probe_ops_per_iter(op);
    *lane_ops_per_s = ops / (1e-3 * (double)ms);
    if (seconds) *seconds = 1e-3 * (double)ms;
    return RS_OK;
}

void rs_release_graphs(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
    g_tables.clear();
}

}  // extern "C"
