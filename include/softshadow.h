/* softshadow: soft shadows on a planetary heightfield by dynamic programming
 * over a maximum mipmap, after Jung, Schrempp and Son, "Optimally Fast Soft
 * Shadows on Curved Terrain with Dynamic Programming and Maximum Mipmaps".
 *
 * C ABI of libsoftshadow.so (HIP, gfx950).  Conventions for every call:
 *
 *  - Heights are float32, row-major [rows][width], metres above a reference
 *    sphere of radius body_radius_m.  Texel (column i, row j) covers
 *    [i, i+1) x [j, j+1) in texel units and its centre is a ray origin.
 *    Sizes: width, rows <= 65536 and width * rows < 2^30 (otherwise
 *    SS_ERR_INVALID_ARG, or -1 / 0 from the layout functions).
 *  - The tile is a gnomonic patch: the tile-centre frame has z along the local
 *    vertical, x along +column, y along +row; the texel grid lies on the plane
 *    tangent to the sphere at the tile centre and spacing texel_m is measured
 *    there (Sec. 3.2, texture-space ray; Sec. 4, cube-sphere faces).
 *  - Every pointer named d_* is DEVICE memory owned by the caller; the library
 *    never frees it.  Host structs (ss_tile, ss_sun, ss_params) are read during
 *    the call only.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work on it: they return before the GPU finishes and never synchronise the
 *    device, except where a function says otherwise.  Apart from
 *    ss_batched_plan_create (which tunes and synchronises) and
 *    ss_batched_plan_launch (which launches the plan's own graph), every call
 *    that takes a stream only launches kernels on it (no allocation, no host
 *    wait, no memset or copy node), so it may be recorded into a caller's HIP
 *    graph by stream capture.
 *  - Return value: SS_OK (0) or a negative SS_ERR_* status; arguments are
 *    validated on the host before anything is enqueued, so an error leaves
 *    every output untouched.  No C++ exception crosses the ABI.
 *  - Calls are reentrant; calls that share output buffers must be ordered by
 *    the caller (same stream or events).
 */
#ifndef SOFTSHADOW_H
#define SOFTSHADOW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SS_OK 0
#define SS_ERR_INVALID_ARG (-1)  /* a pointer, size or parameter is out of range */
#define SS_ERR_HIP (-2)          /* the HIP runtime reported an error; see ss_status_string */
#define SS_ERR_WORKSPACE (-3)    /* workspace missing or smaller than required */
#define SS_ERR_UNSUPPORTED (-4)  /* a combination the library does not implement */

#define SS_MODE_DP 0             /* dynamic-programming descent (Sec. 3.2, Alg. 1) */
#define SS_MODE_UNIFORM 1        /* uniform stepping baseline (Sec. 2, Fig. 1b; Sec. 6.3) */
#define SS_MODE_EXACT 2          /* exact minimum over the half-texel sample grid of Alg. 1's
                                    final samples, by branch and bound over the tap-bound
                                    pyramid (Sec. 2: global minimisation) */
#define SS_MODE_POINT 3          /* Alg. 1 read literally: three point samples of the max-mip
                                    per level at fixed offsets behind the previous choice */

#define SS_SCHED_GEOMETRIC 0     /* segment j traces N'_0 + j levels (capped at the mipmap) */
#define SS_SCHED_EQUAL 1         /* every segment traces N'_0 levels (the paper's {5,5,5}) */
#define SS_SCHED_LIST 2          /* segment j traces n_prime_list[j] levels, n_segments of them
                                    (1..16; the paper's {5,5,5,3}, Sec. 6.3) */

/* Sun direction in the tile-centre frame (Sec. 3.1: shadow ray toward the disc
 * centre; Sec. 3.4: apparent disc radius r_L).  |elev_rad| < pi/2; azimuth is
 * measured from +column toward +row; ang_radius_rad > 0. */
typedef struct {
  double elev_rad;
  double azim_rad;
  double ang_radius_rad;
} ss_sun;

/* Method parameters.  Zero-initialised fields take the defaults noted. */
typedef struct {
  double body_radius_m;    /* > 0; INFINITY selects a flat plane (test geometry) */
  double max_len_m;        /* horizontal ray cap; <= 0: rays run to the tile edge */
  int32_t n_prime0;        /* levels of the first segment, N'_0 (Sec. 3.2; 0 -> 5) */
  int32_t schedule;        /* SS_SCHED_* (Sec. 3.3 interval concatenation) */
  int32_t n_segments;      /* > 0 fixes the number of concatenated runs; 0: reach max_len_m.
                              At most 48 runs: a run spans at most the tile's top mip level
                              (2^(L-1) texels), so a cap far longer than the tile (e.g. 2 km
                              on a 16-texel tile) is SS_ERR_UNSUPPORTED; rays stop at the tile
                              edge anyway, so such tiles take a cap <= their extent or none */
  int32_t mode;            /* SS_MODE_* */
  double uniform_step;     /* SS_MODE_UNIFORM: step in texels of horizontal travel, >= 1/64 (0 -> 1) */
  int32_t prune;           /* 1: skip work that cannot change the result (bitwise-identical) */
  int32_t ray_tile;        /* ray-tile shape code, 0 = default (results never depend on it) */
  int32_t n_prime_list[16];/* SS_SCHED_LIST: levels per segment, each >= 1 */
} ss_params;

/* One heightfield tile.  `maxmip` holds levels >= 1 of its maximum mipmap in
 * the packed layout below (built by ss_maxmip_build); `bound` holds its
 * tap-bound pyramid (built by ss_bound_build), read by SS_MODE_EXACT only and
 * may be NULL otherwise.  The per-tile calls only read both; the batched call
 * and a plan's graph (re)build them from `height`, so they are not const.
 *
 * Ray window: rays start only at texels (i, j) with ray_x0 <= i < ray_x0 +
 * ray_w and ray_y0 <= j < ray_y0 + ray_h, while they see the whole tile.  A
 * tile made of a core plus a halo of neighbouring terrain (up to the ray cap
 * toward the sun) gives the core's shadows as if the terrain went on past its
 * edge; it is also how one tile splits over GPUs.  Per-ray buffers (d_shadow,
 * d_sample, d_grad_shadow) are then [ray_h][ray_w]; d_grad_height stays
 * [rows][width].  All four zero: the whole tile.  The window must lie inside
 * the tile. */
typedef struct {
  const float* height;     /* device, [rows][width] */
  float* maxmip;           /* device, ss_maxmip_floats(width, rows) floats */
  int32_t width, rows;     /* >= 1 */
  double texel_m;          /* > 0 */
  float* bound;            /* device, ss_bound_floats(width, rows) floats, or NULL */
  int32_t ray_x0, ray_y0, ray_w, ray_h;  /* ray window, all 0 = whole tile */
} ss_tile;

/* ---- maximum mipmap (Sec. 3.2, "Maximum mipmaps") ------------------------ */

/* Number of levels including level 0: 1 + ceil(log2(max(width, rows))).
 * Returns 0 when a size is < 1. */
int32_t ss_maxmip_levels(int32_t width, int32_t rows);

/* Level m >= 1 has ceil(width/2^m) x ceil(rows/2^m) texels, row-major, starting
 * at float offset ss_maxmip_level_offset(width, rows, m) (a multiple of 64).
 * ss_maxmip_floats is the total size.  Invalid arguments give -1. */
int64_t ss_maxmip_level_offset(int32_t width, int32_t rows, int32_t level);
int64_t ss_maxmip_floats(int32_t width, int32_t rows);

/* Builds levels >= 1: each texel is the maximum of the (up to four) texels it
 * covers one level down; texels beyond a ragged edge are absent; -0 is stored
 * as +0.  Bit-exact.  fuse_depth = levels written per launch (1..6, 0 = tuned).
 * width or rows == 0 is an empty no-op. */
int32_t ss_maxmip_build(const float* d_height, int32_t width, int32_t rows, float* d_maxmip,
                        int32_t fuse_depth, void* stream);

/* ---- tap-bound pyramid (for SS_MODE_EXACT) ------------------------------- */

/* A bilinear sample (Sec. 3.4) located anywhere in texel (x, y), or up to half
 * a texel outside it, reads only texels of the 3 x 3 block around (x, y).
 * Level 0 of the tap-bound pyramid holds, per texel, the largest height of that
 * block clipped to the tile; level m >= 1 is the maximum mipmap of level 0
 * (Sec. 3.2), so a level-m entry bounds every tap of every sample that falls in
 * its 2^m x 2^m texels.  Layout: level 0 ([rows][width]) at float offset 0,
 * level m >= 1 at ss_bound_level_offset(width, rows, m) = B +
 * ss_maxmip_level_offset(width, rows, m) with B = width*rows rounded up to a
 * multiple of 64; ss_bound_floats is the total (-1 for invalid sizes).  -0 is
 * stored as +0.  Bit-exact; sun-independent, so it is built once per tile. */
int64_t ss_bound_floats(int32_t width, int32_t rows);
int64_t ss_bound_level_offset(int32_t width, int32_t rows, int32_t level);
int32_t ss_bound_build(const float* d_height, int32_t width, int32_t rows, float* d_bound,
                       void* stream);

/* ---- shadow factor (Sec. 3.1-3.4, Alg. 1) -------------------------------- */

/* For every texel centre p: cast the shadow ray p + t L toward the sun centre,
 * find the clearance by the segment schedule (Sec. 3.3) and the descent through
 * the maximum mipmap (Sec. 3.2) -- or by uniform steps in SS_MODE_UNIFORM, or
 * as the exact minimum over the half-texel grid t_n = (n+1) delta/2 in
 * SS_MODE_EXACT (bit-identical to SS_MODE_UNIFORM with uniform_step 0.5) --,
 * and write the visible fraction of the sun disc (Sec. 3.4, Eq. 6 circular
 * segment) to d_shadow[j*width + i] in [0, 1] (1 = fully lit).  Overwrites
 * d_shadow.  tile->maxmip must hold the built mipmap of tile->height, and in
 * SS_MODE_EXACT tile->bound its tap-bound pyramid (NULL: SS_ERR_INVALID_ARG).
 * SS_MODE_POINT runs Alg. 1's point-sample descent on the same segments:
 * level k of a segment of N' levels reads the maximum mipmap (level N'-1-k,
 * nearest texel) under the ray tip at three grid samples 2^(N'-1-k) half
 * texels apart ending at the previous choice plus that spacing, the last level
 * reads the heightfield bilinearly, and the chosen sample's clearance counts. */
int32_t ss_shadow_cast(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                       float* d_shadow, void* stream);

/* Instrumented variant: same output; adds the number of max-mip lower-bound
 * evaluations (SS_MODE_EXACT: tap-bound tests) to d_eval_count[0] and of
 * bilinear clearance samples (the descent's final samples, uniform steps, or
 * the exact mode's evaluated grid samples) to d_eval_count[1]. */
int32_t ss_shadow_cast_counted(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                               float* d_shadow, unsigned long long* d_eval_count, void* stream);

/* Adjoint of ss_shadow_cast (every mode).  Recomputes every ray's
 * decisions (rays with a zero upstream gradient are skipped: they contribute
 * nothing), then ACCUMULATES (+=) dL/dh into d_grad_height [rows][width] and
 * dL/d(elev, azim) into d_grad_sun[2] (FP64), given dL/ds in d_grad_shadow.
 * The max-mipmap enters only through discrete choices and has zero gradient.
 * Accumulation uses atomics, so the summation order is not fixed. */
int32_t ss_shadow_cast_backward(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                                const float* d_grad_shadow, float* d_grad_height,
                                double* d_grad_sun, void* stream);

/* ss_shadow_cast_backward given the forward's output d_shadow (ss_shadow_cast
 * with the same tile, sun and params): s is exactly 0 or 1 only where the
 * clearance puts the whole sun disc below or above it (|d| >= 1), where s has
 * no derivative, so those rays (and rays whose upstream gradient is 0) are not
 * replayed.  The accumulated gradients equal ss_shadow_cast_backward's up to
 * the order of the atomic sums; the cost follows the penumbra, not the tile.
 * d_shadow is [ray_h][ray_w] like d_grad_shadow. */
int32_t ss_shadow_cast_backward_penumbra(const ss_tile* tile, const ss_sun* sun,
                                         const ss_params* params, const float* d_shadow,
                                         const float* d_grad_shadow, float* d_grad_height,
                                         double* d_grad_sun, void* stream);

/* ---- tiles in other gnomonic frames (Sec. 3.3 virtual texture, Sec. 4) ---- */

/* A tile frame: the plane tangent to the reference sphere at the unit vector
 * `centre` (planet frame), with unit axes ex (+column) and ey (+row)
 * orthogonal to it and to each other (each within 1e-9), texel spacing
 * texel_m in that plane and the plane coordinates origin_m of the grid centre.
 * Texel (i, j) stands for the surface direction of R centre + X ex + Y ey,
 * X = origin_m[0] + (i + 1/2 - width/2) texel_m (Y likewise).  A tile of this
 * library (gnomonic about its own centre) has origin_m = (0, 0); a sub-tile of
 * a cube face shares the face's centre and axes and has its own origin_m. */
typedef struct {
  int32_t width, rows;
  double texel_m;
  double centre[3];
  double ex[3], ey[3];
  double origin_m[2];
} ss_frame;

/* Resamples a source tile into a destination tile in another frame (Sec. 3.3:
 * the visible tiles are stitched into one texture; Sec. 4: tiles lie on
 * different cube faces).  Every destination texel whose direction projects
 * centrally into the source tile [0, width) x [0, rows) (in front of its
 * plane) receives the source's bilinear height there (texel centres, taps
 * clamped to the tile, the shadow path's sampling rule); other texels are not
 * written, so several sources composite in call order.  Heights are radial and
 * carry over unchanged.  Positions and the blend are FP64 in a fixed order,
 * rounded once to float32, so the result is a function of the definition
 * alone.  d_src and d_dst must not overlap.  Build a core tile plus a halo
 * from its neighbours this way, then shade the core with a ray window. */
int32_t ss_resample(const float* d_src, const ss_frame* src, float* d_dst, const ss_frame* dst,
                    double body_radius_m, void* stream);

/* ---- view rays (Sec. 4, view ray casting) -------------------------------- */

#define SS_VIEW_HIER 0   /* skip empty space over the tap-bound pyramid */
#define SS_VIEW_DENSE 1  /* test every grid sample between the clip points */

/* Pinhole camera in the tile frame (metres).  The eye is given relative to the
 * point where the tile's z axis meets the reference surface (the sphere centre
 * is at (0, 0, -body_radius_m); on the plane, the tile centre at height 0).
 * Pixel (px, py), row py from the top, looks along fwd + sx right + sy up,
 * normalised, with sx = 2 (px + 1/2) / width - 1, sy = 1 - 2 (py + 1/2) /
 * height; a pixel whose vector is zero sees nothing.  All values are rounded
 * to float32 for the kernels. */
typedef struct {
  int32_t width, height;    /* image, 1..16384 each */
  double eye_m[3];          /* |eye| < body_radius_m / 4 on the sphere */
  double fwd[3], right[3], up[3];  /* finite; fwd nonzero */
  double step_m;            /* sample spacing along the view ray, >= texel_m / 64 */
  double far_m;             /* samples beyond this ray length do not count; <= 0: none */
  int32_t mode;             /* SS_VIEW_* (results identical; the cost differs) */
} ss_camera;

/* First hit of every pixel's view ray with the bilinear terrain (Sec. 4: the
 * view ray meets the same height field the shadow rays see; the shadow ray
 * then starts there).  The ray eye + t V is sampled at t_n = n * step_m; a
 * sample counts when its texel coordinates lie in the tile and t_n <= far_m;
 * the hit is the first counting sample with H - b <= 0 (H the height above the
 * reference surface, b the bilinear terrain over texel centres, taps clamped
 * to the tile), refined by the zero of the line through (t_{n-1}, f_{n-1}) and
 * (t_n, f_n) (t_{n-1} itself when f_{n-1} <= 0; 0 for n = 0).
 * SS_VIEW_HIER starts where the terrain can be, as the paper's pre-displaced
 * mesh does: it skips every tap-bound pyramid cell the ray passes above.
 * Writes d_t[py][px] (ray length of the hit, +inf for none) and d_xy[py][px]
 * (float2 texel coordinates of the hit, NaN for none; the input format of
 * ss_shadow_points); d_steps, if not NULL, gets int32 pairs (grid samples
 * tested, pyramid cells visited; the count is negated in the second entry if
 * a ray hit its iteration bound, which valid input never does).  tile->bound
 * (ss_bound_build) is required; tile->maxmip and the ray window are unused. */
int32_t ss_view_cast(const ss_tile* tile, double body_radius_m, const ss_camera* cam,
                     float* d_t, float* d_xy, int32_t* d_steps, void* stream);

/* Shadow factor at n arbitrary surface points: d_xy holds n (x, y) float pairs
 * in continuous texel coordinates (texel i covers [i, i+1); 8-byte aligned),
 * each ray starts on the bilinear terrain there (Sec. 3.4's sampling) and runs
 * the chosen mode exactly as a texel-centre ray does; d_shadow[n] receives s.
 * Points outside the tile are clamped to its edge; a point with a NaN
 * coordinate (a view ray's miss) gets s = NaN.  The ray window is ignored.
 * Texel centres (i + 1/2, j + 1/2) give ss_shadow_cast's values.  n is at most
 * SS_MAX_POINTS.  This is the call a view-ray caster feeds (Sec. 4: shadows at
 * the visible surface points of a frame). */
#define SS_MAX_POINTS (1LL << 36)

int32_t ss_shadow_points(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                         const float* d_xy, int64_t n, float* d_shadow, void* stream);

/* Adjoint of ss_shadow_points (every mode) with the points held fixed:
 * ACCUMULATES (+=) dL/dh into d_grad_height [rows][width] and dL/d(elev, azim)
 * into d_grad_sun[2] (FP64), given dL/ds in d_grad_shadow[n].  A ray's origin
 * sits on the bilinear terrain at its point, so dL/d(origin height) goes to
 * the four texels that bilinear sample reads; the rest is the texel-centre
 * adjoint.  width = 0: a list of points; width > 0: an image of that many
 * columns (n a multiple of it, at most 16384 rows), worked in 8 x 8 pixel
 * tiles.  NaN points and zero upstream gradients contribute nothing.
 * d_grad_sun must be 8-byte aligned.  Accumulation uses atomics, so the
 * summation order is not fixed. */
int32_t ss_shadow_points_backward(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                                  const float* d_xy, int64_t n, int32_t width,
                                  const float* d_grad_shadow, float* d_grad_height,
                                  double* d_grad_sun, void* stream);

/* ss_shadow_points over an image of points: d_xy is [height][width] float2
 * (ss_view_cast's output), d_shadow [height][width]; width, height 1..16384.
 * The values are ss_shadow_points' on the same points bit for bit; work is
 * grouped in 8 x 8 pixel tiles, whose hits are neighbours on the terrain. */
int32_t ss_shadow_points_image(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                               const float* d_xy, int32_t width, int32_t height, float* d_shadow,
                               void* stream);

/* Forward that also records, for every ray, the index n of its deciding
 * sample (the one whose clearance gave s): t = delta/2 + n * step with
 * step = delta/2, or the uniform step in SS_MODE_UNIFORM; -1 when no sample
 * decided (s = 1 with no terrain in view).  d_sample is int32 [rows][width],
 * overwritten.  d_shadow is bit-identical to ss_shadow_cast's.  The record is
 * what ss_shadow_cast_backward_saved needs, 4 bytes per ray. */
int32_t ss_shadow_cast_save(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                            float* d_shadow, int32_t* d_sample, void* stream);

/* ss_shadow_cast_backward from a record of ss_shadow_cast_save with the same
 * tile, sun and params: the same accumulation (+=) without replaying the
 * forward's decisions.  Up to the order of the atomic sums it equals
 * ss_shadow_cast_backward. */
int32_t ss_shadow_cast_backward_saved(const ss_tile* tile, const ss_sun* sun,
                                      const ss_params* params, const int32_t* d_sample,
                                      const float* d_grad_shadow, float* d_grad_height,
                                      double* d_grad_sun, void* stream);

/* ---- batched: many suns over tiles of uneven size ------------------------ */

/* Bytes of device workspace ss_shadow_cast_batched needs (-1: bad sizes). */
int64_t ss_batched_workspace_bytes(int32_t n_tiles, int32_t n_suns);

/* Builds every tile's maximum mipmap (written to tiles[t].maxmip), then
 * computes d_shadow[t*n_suns + k]
 * (host array of device pointers, each [rows_t][width_t]) for tile t and sun
 * k in one launch over every (tile, sun, ray block): by default one workgroup
 * per ray block of every pair, or, with the environment variable
 * SS_BATCH_FORM=persistent (and always for batches of 2^31 ray blocks or
 * more), a persistent kernel whose workgroups take ray blocks from per-XCD
 * queues in d_workspace.  Outputs are bit-identical to ss_shadow_cast with the
 * same parameters in either form.  d_workspace (256-byte aligned) is used by
 * the work this call enqueues; the per-pair set-up reaches it through kernel
 * arguments, so the call allocates nothing, never waits on the device and may
 * be captured into a caller's HIP graph (a replay redoes the whole call).
 * Every mode; SS_MODE_EXACT needs each tile's `bound` buffer, which the call
 * (and a plan's graph) rebuilds from the heights like the maximum mipmap. */
int32_t ss_shadow_cast_batched(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                               int32_t n_suns, const ss_params* params, float* const* d_shadow,
                               void* d_workspace, int64_t workspace_bytes, void* stream);

/* ss_shadow_cast_batched for callers that cannot allocate device memory or
 * hand over a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same work and bit-identical outputs,
 * with the tables kept in a library-owned device array of
 * SS_NOALLOC_SCRATCH_BYTES per GPU (allocated with the library, held until the
 * process ends).  The call allocates nothing and never waits.  Batches whose
 * ss_batched_workspace_bytes(n_tiles, n_suns) exceeds the array get
 * SS_ERR_WORKSPACE before anything is enqueued (2 MiB holds about 1900
 * (tile, sun) pairs).  Every call on one GPU uses that GPU's one array, so
 * calls on one GPU must not overlap in time (order them on one stream or with
 * events); overlapping calls race on the tables. */
#define SS_NOALLOC_SCRATCH_BYTES (2u << 20)
int32_t ss_shadow_cast_batched_noalloc(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                                       int32_t n_suns, const ss_params* params,
                                       float* const* d_shadow, void* stream);

/* A captured HIP graph of the batched call for fixed buffers.  Create picks the
 * ray-tile shape and mipmap fusion depth by timing the candidates on these
 * inputs (it synchronises `stream` while tuning), then captures the maxmip
 * builds and the batched launch (in the form SS_BATCH_FORM selects).  Launch replays the graph on `stream`; the
 * workspace belongs to the plan until it is destroyed.  Choices are kept per
 * process, keyed by the device architecture, the tile sizes and spacings, the
 * sun count, the method parameters and the form; with the environment variable
 * SS_TUNE_CACHE naming a file they also persist across processes (read once,
 * new choices appended as JSON lines {"key": ..., "ray_tile": n,
 * "fuse_depth": f}).  The choices never change results. */
typedef struct ss_plan ss_plan;
int32_t ss_batched_plan_create(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                               int32_t n_suns, const ss_params* params, float* const* d_shadow,
                               void* d_workspace, int64_t workspace_bytes, void* stream,
                               ss_plan** plan_out);
int32_t ss_batched_plan_launch(ss_plan* plan, void* stream);
/* The choices the tuner made: ray-tile code and fusion depth. */
int32_t ss_batched_plan_config(const ss_plan* plan, int32_t* ray_tile, int32_t* fuse_depth);
int32_t ss_batched_plan_destroy(ss_plan* plan);

/* ---- diagnostics --------------------------------------------------------- */

/* Memory-system probe used to put the descent's gather rate in context (not
 * part of the method): n_threads lanes (a multiple of 256) each sum `iters`
 * floats (rounded up to a multiple of 8, eight loads in flight) of d_src at
 * pseudo-random indices below the largest power of two
 * <= n_floats, or, with window > 0 (a power of two <= n_floats), inside one
 * window of that many floats per lane; d_out[n_threads] receives the sums. */
int32_t ss_probe_gather(const float* d_src, int64_t n_floats, int64_t window, int32_t iters,
                        float* d_out, int64_t n_threads, void* stream);

/* Coherent gather probe, the access pattern of the shadow rays' 8 x 8 ray
 * tiles (not part of the method): n_threads lanes (a multiple of 256) each sum
 * `iters` floats (rounded up to a multiple of 8); the 64 lanes of a wavefront
 * read one 8 x 8 patch of the [rows][width] image d_src per step (lane k at
 * row k / 8, column k % 8 of the patch), the patch origin pseudo-random per
 * wavefront and step; width, rows in 8..65536.  d_out[n_threads] receives the
 * sums.  Rate = n_threads iters / time 4-byte gathers per second. */
int32_t ss_probe_gather_tiles(const float* d_src, int32_t width, int32_t rows, int32_t iters,
                              float* d_out, int64_t n_threads, void* stream);

/* FP32 VALU probe used to check the arithmetic peak a roofline divides by (not
 * part of the method): n_workgroups x 256 lanes each run 32 x iters non-packed
 * FP32 FMAs in eight independent chains; d_out[n_workgroups * 256] receives
 * the lanes' sums.  Rate = 8192 n_workgroups iters / time lane-FMAs per second. */
int32_t ss_probe_valu(int32_t iters, int64_t n_workgroups, float* d_out, void* stream);

/* Text for a status code (for SS_ERR_HIP: the last HIP error of this thread). */
const char* ss_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif
