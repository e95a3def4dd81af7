// Internal declarations shared by the host runtime and the HIP kernels of librs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rs.h"

namespace rs {

// A workgroup tile is (64 K1) grid columns x (kWaves K2) grid rows; see ray_block_shape.
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxWindow = 64;          // LDS map window side (bins)
constexpr int kPartials = 8;            // partial maps, one per accelerator complex die
constexpr float kPadCoord = 1.0e18f;    // position of the zero-mass lenses padding a tile
constexpr int kNoAllocBins = 1 << 20;   // largest map rs_shoot_noalloc takes (1024 x 1024 bins)
constexpr int64_t kNoAllocWords = (int64_t)kPartials * kNoAllocBins;   // its fixed scratch: 32 MiB

// Everything one direct-sum launch needs, already reduced to FP64 constants on the host.
struct DirectArgs {
    const float4 *lenses;   // n_lens records (x1, x2, m, pad)
    int64_t n_lens;
    double glo1, glo2;      // grid lower corner
    double gt1, gt2;        // grid cell size (hi - lo) / n, computed on the host in FP64
    int64_t wlo1, wlo2;     // ray window origin (grid indices); wlo2 is a multiple of 4 (see rskip)
    int64_t wn1, wn2;       // ray window size
    int32_t rskip;          // 0-3: the caller's window start row modulo 4; the window here then
                            // starts that many rows earlier and those rows are masked, so the
                            // rows that share a reciprocal (grid rows 4k..4k+3, or pairs of them)
                            // are the same in every launch shape
    int32_t tiles_x;        // ceil(wn1 / (64 K1))
    double lam1, lam2;      // (1 - gamma) - kappa_c, (1 + gamma) - kappa_c
    double mlo1, mlo2;      // map lower corner
    double ms1, ms2;        // n_k / (hi_k - lo_k)
    int32_t mn1, mn2;       // map size
    int32_t window;         // LDS window side, 0 = all bins go to global atomics
    uint32_t *partial;      // kPartials maps of mn1*mn2 bins, pstride words apart
    int64_t pstride;        // words between partial maps (multiple of 64)
    unsigned long long *lost;
    double *ray_y;          // optional per-ray dump (window-relative index)
    int32_t *ray_pix;
    int64_t gn1;            // full grid width (ray index for the jitter hash)
    uint64_t jkey1, jkey2;  // per-axis jitter keys; jitter = 0: cell centres
    int32_t jitter;
    const float2 *vel;      // lens velocities or null (static field)
    double time;            // lens i sits at x_i + v_i time
};

// Lens record i of a field that may move: positions advanced in FP64, rounded to float32.
__device__ __forceinline__ float4 moved_lens(float4 l, const float2 *vel, int64_t i, double time)
{
    if (vel) {
        const float2 v = vel[i];
        l.x = (float)((double)l.x + (double)v.x * time);
        l.y = (float)((double)l.y + (double)v.y * time);
    }
    return l;
}

// SplitMix64 output function (64-bit wrapping arithmetic).
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
// key of the jitter stream of axis k (0 or 1) under `seed`
__host__ __device__ inline uint64_t jitter_key(uint64_t seed, int k)
{
    return mix64(seed * kGolden ^ ((uint64_t)(8 + k) << 32));
}
// offset in [0, 1) of the ray with grid index r along the axis whose key is `key`
__device__ __forceinline__ double jitter_u(uint64_t key, int64_t r)
{
    return (double)(mix64(key + (uint64_t)(r + 1) * kGolden) >> 11) * 0x1.0p-53;
}

// A table of jobs for the persistent batched kernel (all in device memory).
struct BatchArgs {
    const DirectArgs *jobs;     // n_jobs descriptors
    const uint32_t *item_start; // n_jobs + 1 prefix sums of ray tiles per job
    int32_t n_jobs;
    uint32_t n_items;           // work items to take this launch (<= item_start[n_jobs])
    uint32_t *queue;            // work-item counter, zeroed before each launch
};

// ---------------------------------------------------------------- learned far field

// Network parameter layout (flat, logical order): W1 [64][16], b1 [64], W2 [64][64], b2 [64],
// W3 [2][64], b3 [2].
constexpr int kNParams = 5378;
constexpr int kNParamsPad = 5384;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5376;
// Model buffer: 256-byte header, then one record per tile: 10 doubles (c1, c2, h1, h2,
// alpha_far(c) 1 and 2, J11, J12, J22, s_t) padded to 128 bytes, the bfloat16 parameters
// (5378 x 2 bytes, padded to 16) and the 130 FP32 biases (b1, b2, b3).
constexpr size_t kModelHeader = 256;
constexpr size_t kTileWeightsOff = 128;
constexpr size_t kTileBiasOff = ((size_t)kNParams * 2 + 15) / 16 * 16;
constexpr size_t kTileRecord = (kTileWeightsOff + kTileBiasOff + 130 * 4 + 255) / 256 * 256;
constexpr uint64_t kModelMagic = 0x3130304646535252ull;  // "RRSFF001"

struct FarArgs {
    const float4 *lenses;
    int64_t n_lens;
    double glo1, glo2, gt1, gt2;  // grid lower corner and cell size
    int64_t wlo1, wlo2, wn1, wn2; // ray window
    int32_t TX, TY;               // rays per tile along each axis
    int32_t tiles_x, tiles_y;
    int64_t n_tiles;
    double r_near;
    // fit
    const float *samples;         // n_samples x 2 tile-local points in [-1, 1]^2
    const float *init_params;     // kNParams
    float *targets;               // n_tiles x n_samples x 2 (workspace)
    float *state;                 // n_tiles x kNParams x (FP32 master weight, Adam m, Adam v) (workspace)
    float *sched;                 // steps x 4: learning rate, 1 / (1 - beta1^t), 1 / (1 - beta2^t), 0 (workspace)
    int32_t n_samples, steps, batch;
    int32_t grid_samples;         // samples 64 (4 g + k) + i, k = 0..3, share their first coordinate
    float lr;
    float *debug_grad;            // optional n_tiles x kNParams: gradient of the first step
    float *debug_targets;         // optional n_tiles x n_samples x 2: unnormalised residuals
    uint8_t *model;
    // eval
    double lam1, lam2, mlo1, mlo2, ms1, ms2;
    int32_t mn1, mn2;
    uint32_t *counts;
    unsigned long long *lost;
    double *ray_y;
    int32_t *ray_pix;
    int32_t affine_only;
    const int32_t *eval_tiles;    // optional tile list (blockIdx.x -> tile)
    const float2 *vel;            // moving field (eval only): lens velocities, or null
    double time;
    double *affine;               // moving field: refreshed affine bases, n_tiles x 8 doubles
    int64_t n_eval;
    int64_t gn1;                  // full grid width, jitter keys and switch (as DirectArgs)
    uint64_t jkey1, jkey2;
    int32_t jitter;
};

// Uniform grid of lens cells around the ray window (near-field candidates).
struct CellArgs {
    const float4 *lenses;
    int64_t n_lens;
    double ox, oy, cs;
    int32_t ncx, ncy, n_cells;
    int32_t *count, *cursor, *start, *idx;  // n_cells, n_cells, n_cells + 1, n_lens
};

hipError_t launch_ff_fit(const FarArgs &f, uint64_t hash, hipStream_t s);
// *out += an order-independent 64-bit checksum of n lens records (the caller zeroes *out).
hipError_t launch_lens_checksum(const float4 *lenses, int64_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_ff_eval(const FarArgs &f, const CellArgs &g, hipStream_t s);

// ---------------------------------------------------------------- zoom

constexpr int kZoomLevels = 5;   // culling levels, each halving the cell side of the one above

struct ZoomArgs {
    const float4 *lenses;
    int64_t n_lens;
    double glo1, glo2, gt1, gt2;        // fine grid origin and spacing
    int64_t wlo1, wlo2, wn1, wn2;       // fine ray window
    int64_t c1, c2, ncx, ncy;           // fine rays per culling cell, cells per axis
    int32_t levels;                     // culling levels (coarsest first); the last is the cells
    int64_t P;                          // cells per parent side between consecutive levels
    int64_t lcw1[kZoomLevels], lcw2[kZoomLevels];   // fine rays per cell side, per level
    int64_t lnx[kZoomLevels], lny[kZoomLevels];     // cells per axis, per level
    double lam1, lam2;
    double zlo1, zlo2, zhi1, zhi2;      // zoom map rectangle
    double margin, pad, xmax;           // caller margin; float32 coordinate allowance; max |x|
    const float2 *vel;                  // lens velocities or null
    double time;
    uint32_t *lists[kZoomLevels];       // kept cells of each level; the last is `list`
    uint32_t *list;                     // kept cell indices (finest level)
    uint32_t *stats;                    // [0] cells kept (list length), [4 + l] kept at level l < levels - 1
};

hipError_t launch_zoom_mark(const ZoomArgs &z, hipStream_t s);
hipError_t launch_advance(const float4 *in, const float2 *vel, int64_t n, double time, float4 *out, hipStream_t s);
// Lane blocks (K1 columns x K2 rows) of the culling cells in list[0 .. *count).
struct CellBlocks {
    const uint32_t *list;
    const uint32_t *count;
    int64_t c1, c2, ncx;    // culling cell size (window columns, rows) and cells per row
    int64_t sx, S;          // lane blocks per cell row, lane blocks per cell
};

// Persistent direct sum over the lane blocks of the listed cells.
hipError_t launch_direct_cells(const DirectArgs &a, int K1, int K2, int T, int LT, const CellBlocks &cb,
                               int64_t max_groups, hipStream_t s);

// ---------------------------------------------------------------- light curves

struct LightArgs {
    const uint32_t *counts;
    double lo[2], w[2];     // map lower corner and pixel size (hi - lo) / n
    double inv_w[2];        // n / (hi - lo), for the support's bounding box only
    int32_t n[2];
    double n_av;
    int32_t kind;           // 0: Gaussian, 1: uniform disc
    double size, support;   // sigma or radius; support radius
    double inv2s2;          // 1 / (2 sigma^2)
    const double *tracks;   // n_tracks x (start1, start2, end1, end2), device
    int32_t n_tracks, n_points;
    double *mu, *mag;       // n_tracks x n_points each (either may be null)
    int32_t path;           // 0: chosen by size, 1: lane per point, 2: wave per point
    int64_t frame_stride;   // words between the maps of consecutive track points (0: one map)
};

hipError_t launch_light_curve(const LightArgs &a, hipStream_t s);

// Per-lane ray blocks (K1 columns x K2 rows) compiled into the library.
bool ray_block_supported(int K1, int K2);
// Launch the direct-sum kernel for a K1 x K2 ray block per lane, T-lens float32 runs and LT-lens
// LDS tiles.
hipError_t launch_direct(const DirectArgs &a, int K1, int K2, int T, int LT, int64_t n_tiles, hipStream_t s);
// Launch the persistent batched kernel on `grid` workgroups.
hipError_t launch_batched(const BatchArgs &b, int K1, int K2, int T, int LT, int grid, hipStream_t s);
// Resident workgroups per compute unit of the batched kernel (0 on error).
int batched_occupancy(int K1, int K2, int T, int LT);
// p[0..n) = v with a one-block kernel (graph-capture safe, n <= 1024).
hipError_t launch_fill_u32(uint32_t *p, int n, uint32_t v, hipStream_t s);
// Zero the partial maps (fill kernel; graph-capture safe).
hipError_t launch_zero(uint32_t *p, int64_t n_words, hipStream_t s);
// counts[b] += sum_s partial[s * pstride + b] for b < bins.
hipError_t launch_reduce(const uint32_t *partial, int64_t bins, int64_t pstride, uint32_t *counts,
                         hipStream_t s);
// mu[b] = counts[b] / n_av for b < bins (FP64).
hipError_t launch_magnification(const uint32_t *counts, int64_t bins, double n_av, double *mu, hipStream_t s);
// Issue-rate probes (rs_probe.h): lane instructions per loop iteration of probe `op`, and one launch.
int probe_ops_per_iter(int op);
hipError_t launch_probe(int op, int blocks, int iters, hipStream_t s);
// Device address of the fixed scratch array (kNoAllocWords words) on the current device, looked up
// with hipGetSymbolAddress on the first call per device.
hipError_t noalloc_scratch(uint32_t **ptr);

}  // namespace rs
