/*
 * rs.h -- C ABI of librs, an MI355X (gfx950) inverse ray-shooting library.
 *
 * The method is direct inverse ray-shooting for microlensing magnification
 * maps (Thompson, Fluke, Barnes & Barsdell 2009):
 *   lens equation                y = x - alpha(x)                 (section 1, eq. 1)
 *   many-Schwarzschild deflection alpha(x) = sum_i m_i (x - x_i) / |x - x_i|^2
 *                                                                  (section 1, eq. 2)
 *   direct sum split into lens subsets whose partial sums are added
 *                                                                  (section 2, eq. 5)
 *   macro model  y = diag(1-gamma, 1+gamma) x - kappa_c x - alpha  (section 3.2, eq. 6)
 *   estimator    mu_ij = N_ij / N_av, N_ij = rays in pixel (i, j)  (section 1, eq. 4)
 *
 * Conventions shared by every entry point
 *   - Lengths are in Einstein radii of a unit-mass lens.
 *   - Rays sit one per cell of a regular grid, at the cell centre or at a seeded
 *     random point of the cell (rs_raygrid): coordinate i of axis k is the float32
 *     rounding of lo_k + (i + u) (hi_k - lo_k) / n_k, evaluated in FP64 as
 *     t = (hi-lo)/n, v = (i + u) t, w = lo + v (no fused operations).
 *   - The deflection is summed in float32 over runs of consecutive lenses
 *     (lens-index order); each run's partial sum is added to a per-ray FP64
 *     accumulator (eq. 5 with FP64 combination).  The lens equation and the
 *     pixel index are evaluated in FP64.
 *   - Source pixels are half-open: p_k = floor((y_k - lo_k) * (n_k / (hi_k - lo_k))).
 *     A ray is counted iff y is finite and 0 <= p_k < n_k; otherwise it is
 *     "lost" (this includes a ray exactly on a lens).
 *   - Maps are uint32, row-major with axis 1 fastest: counts[p2 * n1 + p1].
 *     Every call ADDS into counts and n_lost; the caller zeroes them.
 *
 * Ownership and memory
 *   - Every pointer marked "device" is device memory owned by the caller.
 *     The library never allocates device memory: workspace sizes come from
 *     the *_bytes queries and the caller passes the buffers in.  The one
 *     exception is rs_shoot_noalloc's fixed scratch array, a device global of
 *     the library's code object (see there).
 *   - Host structs are read during the call only.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued asynchronously; kernel faults surface on the caller's next
 *     synchronisation.  Calls that share a workspace must be ordered.
 *
 * Errors
 *   Every function returns rs_status and never aborts, throws or prints.
 *   Invalid arguments are rejected before any HIP call.  rs_last_error()
 *   returns a thread-local description of the last failure on this thread.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RS_OK = 0,
    RS_EINVAL = -1,     /* invalid argument (NULL, negative or empty size, bad region, ...)  */
    RS_ERANGE = -2,     /* a size exceeds what one call supports (e.g. >= 2^31 rays)         */
    RS_EDEVICE = -3,    /* a HIP launch or runtime call failed (text in rs_last_error)       */
    RS_ESMALLBUF = -4,  /* workspace or model buffer smaller than its *_bytes query          */
    RS_ENOTFIT = -5,    /* a far-field model does not match the job / configuration          */
    RS_EINTERNAL = -6   /* unexpected internal state                                         */
} rs_status;

/* Human-readable name of a status code (static string). */
const char *rs_status_str(int status);
/* Thread-local detail of the last failure on the calling thread (static until the next call). */
const char *rs_last_error(void);
/* Library version string. */
const char *rs_version(void);

/* One point lens: position (x1, x2) and mass m (eq. 2); pad is ignored.  16 bytes. */
typedef struct {
    float x1, x2, m, pad;
} rs_lens;

/* Macro model of eq. 6: smooth convergence kappa_c (the paper's sigma_c) and external shear. */
typedef struct {
    double kappa_c, gamma;
} rs_macro;

/*
 * Image-plane ray grid: the rectangle [lo, hi) cut into n[0] x n[1] cells, one ray per cell.
 * Only the window [win_lo, win_lo + win_n) is shot by a call, so a large grid can be streamed
 * in pieces whose ray positions do not depend on the split.
 *
 * Ray placement.  jitter = 0: the cell centre (u_k = 1/2).  jitter = 1: one uniformly random
 * point per cell, the paper's Monte Carlo ray positions (section 2.1, 2.2) stratified by cell:
 * for the ray of cell (i1, i2), r = i2 * n[0] + i1, and axis k (s = 8 for axis 1, 9 for axis 2)
 *     key = mix(jitter_seed * G xor (s << 32)),  h = mix(key + (r + 1) * G),
 *     u_k = (h >> 11) * 2^-53,  G = 0x9E3779B97F4A7C15,
 * with mix the SplitMix64 output function (Steele, Lea & Flood 2014; 64-bit wrapping).
 * In both cases coordinate k is the float32 rounding of lo_k + (i_k + u_k) t_k, t_k =
 * (hi_k - lo_k) / n_k, evaluated in FP64 as v = ((double)i_k + u_k) t_k, w = lo_k + v.
 */
typedef struct {
    double lo[2], hi[2];
    int64_t n[2];
    int64_t win_lo[2], win_n[2];
    uint64_t jitter_seed;
    int32_t jitter;             /* 0: cell centres, 1: random point per cell */
    int32_t reserved;           /* must be 0 */
} rs_raygrid;

/* Source-plane map: the rectangle [lo, hi) cut into n[0] x n[1] half-open pixels. */
typedef struct {
    double lo[2], hi[2];
    int32_t n[2];
} rs_map;

/* One magnification-map job. */
typedef struct {
    const rs_lens *lenses;   /* device, n_lens records                                       */
    int64_t n_lens;          /* >= 0                                                         */
    rs_macro macro;
    rs_raygrid grid;
    rs_map map;
    uint32_t *counts;        /* device, map.n[1] * map.n[0], ACCUMULATED (+=)                */
    uint64_t *n_lost;        /* device, one counter, ACCUMULATED (+=)                        */
    /* Moving lenses (section 4: stars move between frames).  velocities: device, n_lens x
     * (v1, v2) float32, or NULL for a static field.  The job then shoots the field at `time`:
     * lens i sits at float32((double)x_i + (double)v_i * time) per axis (FP64, then rounded),
     * its mass unchanged.  rs_shoot, rs_shoot_batched and rs_shoot_zoom apply it while staging
     * lenses; rs_farfield_fit rejects it and rs_farfield_eval evaluates a fitted closure at
     * `time` (see there). */
    const float *velocities;
    double time;
} rs_job;

/* Flags for rs_opts.flags */
#define RS_FLAG_FAULT_INJECT 0x1u  /* fail with RS_EDEVICE after validation, before any HIP call */
#define RS_FLAG_NO_GRAPH 0x2u      /* rs_shoot_batched: launch directly instead of replaying a graph */
#define RS_FLAG_AFFINE_ONLY 0x4u   /* rs_farfield_eval: far field from the affine base alone (ablation) */

/*
 * Tuning and diagnostics for rs_shoot.  NULL, or a zero field, selects the
 * default.  Results depend on fp32_run (the length of the float32 runs before
 * each FP64 addition) and on whether the ray block has one column or several
 * (one column: four rows share a reciprocal; several columns: pairs of rows
 * share one and the mass is folded into the shared differences, which rounds
 * differently); lens_tile, map_window and the rows of a several-column block
 * change speed, not values.
 */
typedef struct {
    int32_t block_cols;      /* rays per lane: block_cols grid columns x block_rows grid rows;  */
    int32_t block_rows;      /* 1x4, 2x2, 2x4, 4x2, 4x4 or 2x8 (0, 0 = default)               */
    int32_t lens_tile;       /* lenses staged in LDS per tile: 256 or 512 (default 256)        */
    int32_t fp32_run;        /* lenses per float32 run: 8, 16 or 32 (default 8 with one column,
                                16 with several); one-column blocks add four runs in float32
                                before each FP64 addition, several-column blocks add each run  */
    int32_t map_window;      /* side of the LDS-privatised map window: 16, 32 or 64; -1 = off */
    double *ray_y;           /* optional device output, 2 doubles per ray of the window        */
    int32_t *ray_pix;        /* optional device output, pixel p2*n1+p1 per ray, -1 = lost      */
    uint32_t flags;          /* RS_FLAG_*                                                      */
} rs_opts;

/*
 * Workspace bytes rs_shoot needs for this job (8 partial maps, one per
 * accelerator complex die, plus alignment).  Returns 0 for an invalid job.
 */
size_t rs_workspace_bytes(const rs_job *job, const rs_opts *opts);

/*
 * Shoot the job's ray window and add its counts to job->counts and job->n_lost.
 * Direct inverse ray-shooting (eqs. 1, 2, 4, 5, 6).
 *   workspace: device, >= rs_workspace_bytes(job, opts) bytes, contents ignored
 *   (overwritten).  opts may be NULL.
 * Returns RS_EINVAL / RS_ERANGE / RS_ESMALLBUF before any HIP call on bad
 * arguments, RS_EDEVICE if a launch fails.  An empty window is a no-op.
 */
int rs_shoot(const rs_job *job, void *workspace, size_t ws_bytes, void *stream, const rs_opts *opts);

/*
 * rs_shoot without a workspace, for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid hipMalloc.  It computes
 * exactly what rs_shoot computes (same kernels, same counts and dumps), but its 8 partial maps
 * live in a fixed device array inside the library (32 MiB, held by every GPU the library runs
 * on until the process ends) instead of a caller workspace.  The map may have at most 2^20
 * bins (1024 x 1024); larger maps return RS_ERANGE before any HIP call (use rs_shoot).  The
 * first call on a device looks up the array's address there (hipGetSymbolAddress); no call
 * allocates or frees anything.  All calls on one GPU share that GPU's array and every call
 * clears the part it uses, so calls that overlap on one GPU (e.g. on two streams) race: order
 * them on one stream.  Errors as for rs_shoot.
 */
int rs_shoot_noalloc(const rs_job *job, void *stream, const rs_opts *opts);

/*
 * Magnification map (section 1, eq. 4): mu_ij = N_ij / N_av, where N_av, the number of rays a
 * pixel receives without lensing, is the pixel area over the ray-cell area,
 *     N_av = (dy1 dy2) / (dx1 dx2),  dy_k = (map hi_k - lo_k) / n_k,  dx_k = (grid hi_k - lo_k) / n_k,
 * evaluated in FP64 in that order (one ray per grid cell, centred or jittered alike; the grid's
 * window is ignored).
 *   counts: device, map->n[1] x map->n[0] uint32 (the layout rs_shoot fills)
 *   mu:     device output, the same number of doubles, mu[b] = (double)counts[b] / N_av (IEEE
 *           division); counts and mu must not overlap
 *   n_av_out: host, nullable; receives N_av (also when counts or mu is NULL, which then returns
 *           RS_EINVAL after filling it)
 * A map accumulated over k passes of the same grid holds k times the counts: divide mu by k.
 * Errors: RS_EINVAL for a bad grid or map or a NULL buffer, RS_ERANGE for >= 2^31 pixels or a
 * non-finite N_av, RS_EDEVICE if the launch fails.  Asynchronous on `stream`.
 */
int rs_magnification(const uint32_t *counts, const rs_raygrid *grid, const rs_map *map, double *mu,
                     double *n_av_out, void *stream);

/*
 * Many maps in one persistent launch (many independent map generations, section 4; each map is
 * eqs. 1, 2, 4, 5, 6 exactly as rs_shoot computes it, so its counts are bit-identical to a
 * rs_shoot call with the same block shape and fp32_run).
 *
 * Workspace bytes for a batch: work counter, job table, tile prefix sums and one scratch map
 * (for the autotuner).  Returns 0 for an invalid batch.
 */
size_t rs_batched_workspace_bytes(const rs_job *jobs, int32_t n_jobs);

/*
 * Shoot every job of the host array jobs[0 .. n_jobs) and add each job's counts to its own map.
 * Ray tiles of all jobs form one queue taken by a persistent kernel, costliest jobs first.  On a
 * non-NULL stream the two kernels (counter reset, persistent kernel) are captured once into a
 * HIP graph per (workspace address, block shape, grid, batch size) and replayed on later calls;
 * the job table is uploaded into the workspace before each launch, so later calls may change
 * the jobs' parameters and buffers.  opts: block shape, lens_tile, fp32_run, map_window and
 * RS_FLAG_NO_GRAPH; per-ray dumps are rejected (RS_EINVAL).  Calls sharing a workspace must be
 * ordered on one stream.  Returns as rs_shoot, with the failing job's index in rs_last_error.
 */
int rs_shoot_batched(const rs_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes, void *stream,
                     const rs_opts *opts);

/*
 * Pick the block shape and map window for a batch by timing candidates (1x4, 2x4, 4x4, 2x8 ray
 * blocks x 32/64 windows) on the batch's costliest tiles, with counts sent to the workspace's
 * scratch map (the jobs' maps are not touched).  *best supplies fp32_run and lens_tile and
 * receives block_cols, block_rows, lens_tile and map_window.  If cache_path (nullable) holds
 * an entry for this device and batch class (median lens count, ray count and map size, in
 * powers of two) it is used without timing; otherwise the result is appended to the file.
 * Synchronises the stream.
 */
int rs_autotune_batched(const rs_job *jobs, int32_t n_jobs, void *workspace, size_t ws_bytes, void *stream,
                        const char *cache_path, rs_opts *best);

/*
 * Learned far-field closure.  The ray window is cut into tiles of tile_rays[0] x tile_rays[1]
 * rays.  For each tile the lenses closer than r_near to the tile rectangle (the rectangle
 * covered by its ray cells; FP64 distance) are the near set, summed exactly per ray; the sum
 * over all other lenses (the far field, eq. 2 restricted to a lens subset as in eq. 5) is
 * replaced by
 *     alpha_far(c) + J_far(c) (x - c) + s_t * net((x - c) / h)
 * with c, h the tile centre and half-widths, alpha_far(c) and its Jacobian J_far(c) exact in
 * FP64, and net a 2 -> 16 -> 64 -> 64 -> 2 network (features sin, cos of (pi/2) 2^k u_d,
 * k = 0..3; SiLU) trained per tile on the far-field residual at n_samples exact samples
 * (float32 direct sums with FP64 combination, like rs_shoot), normalised by its RMS s_t.
 * Training: mini-batch Adam (0.9, 0.999, 1e-8), step t uses samples [(t-1) batch mod
 * n_samples, +batch), learning rate lr (1 + cos(pi (t-1) / steps)) / 2; GEMM operands in
 * bfloat16, sums in FP32, master weights FP32.
 */
typedef struct {
    int32_t tile_rays[2];       /* rays per tile along each axis, e.g. 64 x 64; <= 2^24 per tile  */
    double r_near;              /* near radius (Einstein radii), e.g. 8                            */
    int32_t n_samples;          /* fit samples per tile, multiple of 1024, e.g. 4096                */
    int32_t steps;              /* Adam steps (0 = keep the initial parameters), e.g. 2000          */
    int32_t batch;              /* samples per step: multiple of 256 dividing n_samples, e.g. 512   */
    float lr;                   /* peak learning rate, e.g. 1e-2                                    */
    double cell_size;           /* lens cell side for the near-set search (0 = r_near / 4)          */
    const float *samples;       /* device, n_samples x 2 tile-local points in [-1,1]^2 (input)       */
    const float *init_params;   /* device, 5378 initial parameters, the same for every tile (input) */
    float *debug_grad;          /* device, nullable: n_tiles x 5378, gradient of the first step      */
    float *debug_targets;       /* device, nullable: n_tiles x n_samples x 2 residual samples        */
    const int32_t *eval_tiles;  /* device, nullable: rs_farfield_eval shoots only these tile indices  */
    int32_t n_eval_tiles;       /* entries of eval_tiles (each in [0, n_tiles), distinct)             */
    int32_t shared_x;           /* 0: arbitrary samples.  1: samples 64 (4 g + k) + i, k = 0..3, share  */
                                /* their first coordinate (every g < n_samples / 256, i < 64): the fit */
                                /* checks this on the host (synchronising the stream) and shares      */
                                /* x - x_l between them.  The fitted model is bit-identical either way. */
} rs_ff_config;

/*
 * Model buffer (device, 256-byte aligned): a 256-byte header (magic, configuration hash, tile
 * counts) then one record per tile (tile index ty * tiles_x + tx) of rs_farfield_model_bytes /
 * n_tiles bytes: 10 doubles (c1, c2, h1, h2, alpha_far(c) 1, 2, J11, J12, J22, s_t) padded to
 * 128 bytes, the 5378 parameters as bfloat16 (W1 [64][16], b1, W2 [64][64], b2, W3 [2][64], b3)
 * padded to 16 bytes, then b1, b2, b3 again as 130 floats.  The hash covers the ray grid,
 * window, tiling, fit settings and lens count; the header also keeps a 64-bit checksum of the
 * lens records the fit saw, which rs_farfield_eval recomputes (one pass over the lens array).
 */
size_t rs_farfield_model_bytes(const rs_job *job, const rs_ff_config *cfg);
size_t rs_farfield_fit_workspace_bytes(const rs_job *job, const rs_ff_config *cfg);
size_t rs_farfield_eval_workspace_bytes(const rs_job *job, const rs_ff_config *cfg);

/*
 * Fit every tile's closure: affine base, exact far-field samples, normalisation, training.
 * job->counts / n_lost are not touched.  Asynchronous on `stream`.
 */
int rs_farfield_fit(const rs_job *job, const rs_ff_config *cfg, void *model, size_t model_bytes, void *workspace,
                    size_t ws_bytes, void *stream);

/*
 * Shoot the job's ray window with the fitted closure and add the counts to job->counts and
 * job->n_lost (same pixel rules as rs_shoot).  opts: ray_y / ray_pix dumps and
 * RS_FLAG_AFFINE_ONLY (network off: the method without the learned part).  With
 * cfg->eval_tiles only the listed tiles are shot (e.g. a seeded subset judged against
 * rs_shoot on the same tile windows).  Reads the model header and the tile list first
 * (synchronises the stream); RS_ENOTFIT on a model mismatch (grid, tiling, configuration or
 * lens records other than the fit's), RS_EINVAL on a bad tile index.
 * Moving field (section 4, one closure reused across frames): with job->velocities the job's
 * lens positions are those of the fit; each tile's near set is still chosen by them, its
 * lenses enter at their positions at job->time; the far set's affine base alpha_far(c),
 * J_far(c) is recomputed in FP64 at job->time, and the fitted network residual is kept.
 */
int rs_farfield_eval(const rs_job *job, const rs_ff_config *cfg, const void *model, size_t model_bytes,
                     void *workspace, size_t ws_bytes, void *stream, const rs_opts *opts);

/*
 * Ray budget (section 1, eq. 4: N_av, the rays per source pixel without lensing, sets the
 * map's Poisson noise; section 2: rays cover an image region somewhat larger than the
 * source region).  Plans a ray grid for `map` with at least `n_av` rays per pixel:
 *   lambda_k = (1 - kappa - gamma, 1 - kappa + gamma), kappa = kappa_star + macro->kappa_c
 *   (the field's mean lens mapping); half-widths X_k = margin L_k / (2 max(|lambda_k|, 0.05))
 *   around the preimage of the map centre, c_k / lambda_k (lambda_k floored the same way);
 *   square cells of side t <= sqrt(pixel area / n_av), t rounded down to a multiple of
 *   2 ulp32(max |coordinate| + lens_extent) so every ray coordinate sits on that lattice;
 *   n_k = ceil(2 X_k / t); the centre is snapped to the lattice too.
 * out receives lo, hi, n, the full window and jitter off; *n_av_out (if not NULL) the planned
 * pixel area / t^2.  margin 0 means 1.2.  lens_extent: largest |lens coordinate| (0 if unknown).
 * The lattice bounds a side at about 2^23 rays; near that limit the planned N_av exceeds the
 * target by more than the usual fraction of a percent.
 * Errors: RS_EINVAL for invalid arguments; RS_ERANGE if the cell would fall below the lattice.
 */
int rs_plan_grid(const rs_map *map, const rs_macro *macro, double kappa_star, double lens_extent, double n_av,
                 double margin, rs_raygrid *out, double *n_av_out);

/*
 * Moving lenses (section 4): out[i] = (float32(x1_i + v1_i t), float32(x2_i + v2_i t), m_i, pad_i),
 * the same positions a job with `velocities` and `time` shoots.  lenses, velocities (n x 2
 * float32) and out (n records) are device memory; out may equal lenses.  Asynchronous.
 */
int rs_advance_lenses(const rs_lens *lenses, const float *velocities, int64_t n, double time, rs_lens *out,
                      void *stream);

/*
 * Interactive zoom (section 4: a selected area of a map recomputed at higher detail).
 * `job` describes the dense problem: job->grid is the fine ray grid (and window) and job->map the
 * selected source-plane area at the wanted resolution.  The counts added to job->counts are
 * exactly those rs_shoot(job) would add, bit for bit, but only the rays that can reach the map
 * are shot: the window is split into culling cells of zoom->cell fine rays; each cell's image
 * under eq. 6 is bounded from its centre (deflection, its gradient, a second-order remainder
 * over the lenses beyond three half-diagonals, 2 m / distance for closer lenses; a cell that
 * holds a lens is always kept), widened by a float32 rounding allowance and zoom->margin.  The
 * bounds are taken coarse to fine over five levels: the coarsest groups 16 x 16 culling cells,
 * each later level halves the cell side (its cells are the 2 x 2 children of the cells kept at
 * the level above, and it looks only inside those), the last is the culling cells themselves;
 * the rays of the finest cells kept are shot with the plain path's arithmetic.
 * *job->n_lost receives only the shot rays that miss the map.  opts as for rs_shoot, except
 * that per-ray dumps are rejected (RS_EINVAL).
 */
typedef struct {
    int32_t cell[2];   /* fine rays per (finest) culling cell along each axis; {0, 0} = about   */
                       /* 64 rays, square in the image plane, rounded up to whole lane blocks */
    double margin;     /* extra source-plane distance added to every cell's bound, >= 0      */
} rs_zoom;

/* Workspace bytes for rs_shoot_zoom (0 if the arguments are invalid). */
size_t rs_zoom_workspace_bytes(const rs_job *job, const rs_zoom *zoom, const rs_opts *opts);

/* Asynchronous on `stream`; nothing is allocated.  Errors as for rs_shoot, plus RS_ERANGE for
 * more than 2^30 culling cells. */
int rs_shoot_zoom(const rs_job *job, const rs_zoom *zoom, void *workspace, size_t ws_bytes, void *stream,
                  const rs_opts *opts);

/* Statistics of the last rs_shoot_zoom on this workspace: out = {culling cells kept, culling
 * cells, ray slots shot, ray slots in all cells} (a ray slot is one ray of a lane block;
 * blocks at cell and window edges hold masked slots).  Synchronises `stream`. */
int rs_zoom_stats(const void *workspace, uint64_t out[4], void *stream);

/*
 * Light curves (section 1: a source profile moved across the magnification map, each position's
 * magnification turned into a magnitude change).  Pixel (p1, p2) has centre
 * c = lo_k + (p_k + 1/2) (hi_k - lo_k) / n_k and magnification N / n_av (eq. 4).  Track t runs
 * from s = tracks[4t .. 4t+1] to e = tracks[4t+2 .. 4t+3]; its point k of n_points is
 * y = s + (k / (n_points - 1)) (e - s)  (y = s when n_points = 1).  The source magnification is
 *   mu = sum_p w_p N_p / (n_av sum_p w_p)
 * over the map pixels whose centre lies in the profile's support, |c - y|^2 <= support^2, with
 * w = exp(-|c - y|^2 / (2 sigma^2)) for a Gaussian (support = cutoff sigma, cutoff 0 -> 4) or
 * w = 1 for a uniform disc (support = radius).  The magnitude change is -2.5 log10(mu).  A point
 * whose support holds no pixel centre gives NaN.
 */
typedef struct {
    int32_t kind;               /* 0: Gaussian, 1: uniform disc                                */
    double size;                /* sigma (Gaussian) or radius (disc), source-plane units, > 0  */
    double cutoff;              /* Gaussian support in sigmas (0 = 4); ignored for a disc      */
    int32_t layout;             /* evaluation layout: 0 = chosen by size, 1 = one lane per     */
                                /* point, 2 = one wave per point (results agree to rounding)   */
} rs_source;

/*
 * counts: device map, map->n[1] rows of map->n[0] uint32 (the layout rs_shoot fills).
 * tracks: device, n_tracks x 4 doubles (start1, start2, end1, end2), finite.
 * mu, mag: device outputs of n_tracks x n_points doubles, track-major (either may be NULL).
 * frame_stride: 0 reads one map for every point; otherwise point k of every track reads the
 * map at counts + k frame_stride (a time-evolving field, section 4: one frame per point, e.g.
 * the maps of a batch of moving-lens jobs); frame_stride >= map->n[0] map->n[1].
 * Nothing is allocated; asynchronous on `stream`.  n_tracks = 0 is a no-op.
 * Errors: RS_EINVAL for a bad map, n_av <= 0, source, sizes or stride; RS_EDEVICE if the launch
 * fails.  A non-finite track coordinate is not detected (the tracks live on the device) and
 * gives NaN.
 */
int rs_light_curve(const uint32_t *counts, const rs_map *map, double n_av, const rs_source *src,
                   const double *tracks, int32_t n_tracks, int32_t n_points, int64_t frame_stride, double *mu,
                   double *mag, void *stream);

/* Destroy the cached batch graphs and staged job tables (e.g. before freeing workspaces). */
void rs_release_graphs(void);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
