/* Reference oracle for the soft-shadow hot path: public C interface.
 *
 * TEST INFRASTRUCTURE.  This is a plain, slow FP64 CPU implementation written
 * from the paper (Jung, Schrempp, Son: "Optimally Fast Soft Shadows on Curved
 * Terrain with Dynamic Programming and Maximum Mipmaps").  Only the tests, the
 * package smoke check and the bench's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * Conventions: heights are float32, row-major [rows][width], metres above the
 * reference sphere.  Texel (column i, row j) covers [i, i+1) x [j, j+1) in
 * continuous texel coordinates; its centre is a ray origin.
 */
#ifndef SS_ORACLE_H
#define SS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXSEG 64
#define OR_MAXLEV 32

typedef struct {
  int32_t width, rows;
  double texel_m;         /* texel spacing on the tangent plane at the tile centre */
  double radius_m;        /* body radius; +INFINITY selects the flat-plane mode */
  double elev_rad;        /* sun elevation in the tile-centre frame */
  double azim_rad;        /* sun azimuth from +column toward +row */
  double ang_radius_rad;  /* apparent radius of the sun disc */
  double max_len_m;       /* horizontal ray cap; <= 0: rays run to the tile edge */
  int32_t n_prime0;       /* mip levels traced by the first segment */
  int32_t schedule;       /* 0: N'_j = N'_0 + j (geometric); 1: N'_j = N'_0 (equal);
                             2: N'_j = n_prime_list[j] for n_segments runs */
  int32_t n_segments;     /* > 0 overrides the segment count derived from the cap */
  int32_t mode;           /* 0: dynamic-programming descent; 1: uniform stepping;
                             2: exact minimum over the half-texel grid (dense stepping);
                             3: Alg. 1's point-sample descent */
  double uniform_step;    /* uniform step, texels of horizontal travel */
  double uniform_tmax_m;  /* > 0 overrides the uniform cap on ray length t */
  int32_t n_prime_list[16]; /* schedule 2: levels of each run */
} or_params;

typedef struct {
  int32_t seg;           /* segment that gave the minimum (uniform: -1); -2 when lit by default */
  int32_t n;             /* index of the deciding sample on the t grid */
  double t;              /* ray length of that sample */
  double dh;             /* clearance height of that sample */
  double alpha;          /* angular clearance (radians), +INF when no valid sample */
  int32_t base_i, base_j;/* base texel of the descent in that segment */
  int32_t evals;         /* lower-bound evaluations + final samples (uniform: steps) */
  double margin_lb;      /* smallest best/runner-up gap of any lower-bound argmin (m) */
  double margin_dh;      /* smallest best/runner-up gap of any final-sample argmin (m) */
  double margin_round;   /* smallest distance of a rounding argument from its boundary */
  double margin_seg;     /* gap between the two smallest segment clearances (rad);
                            stepping modes: between the two smallest step clearances */
  double margin_geo;     /* smallest spacing of crossing events / (1 + texels travelled) */
  double margin_tap;     /* distance of the deciding sample from a tap line / (1 + texels travelled) */
} or_trace;

typedef struct or_ctx or_ctx;

int32_t or_maxmip_levels(int32_t width, int32_t rows);
int64_t or_maxmip_offset(int32_t width, int32_t rows, int32_t level); /* floats, levels >= 1 */
int64_t or_maxmip_floats(int32_t width, int32_t rows);

/* Builds the maximum mipmap of h (kept by reference: h must outlive the context). */
or_ctx* or_ctx_create(const float* h, int32_t width, int32_t rows);
void or_ctx_destroy(or_ctx* c);
/* Copies levels >= 1 into out (layout of or_maxmip_offset). */
void or_ctx_copy_maxmip(const or_ctx* c, float* out);

/* Shadow factor for n_rays texels (linear index j*width+i; NULL = all texels
 * in order).  s_out[k] in [0,1]; alpha_out and trace_out may be NULL. */
/* Shadow rays from n surface points xy[2k], xy[2k+1] (continuous texel
 * coordinates inside the tile; the origin height is the bilinear terrain
 * there).  Returns -2 if a point lies outside. */
int32_t or_shadow_points(const or_ctx* c, const or_params* p, const double* xy, int64_t n,
                         double* s_out, double* alpha_out, or_trace* trace_out);
int32_t or_shadow(const or_ctx* c, const or_params* p, const int64_t* rays, int64_t n_rays,
                  double* s_out, double* alpha_out, or_trace* trace_out);

/* Set of angular clearances the method yields for one ray when every decision
 * whose FP64 margin is below a tolerance may go either way.  Height margins
 * (lower bounds, final clearances) use eh_abs + eh_rel * t metres, positions
 * (crossings, rounding, tile edge) et_abs + et_rel * t/delta texels, t the
 * ray length there.  Modes 0 (descent), 1 (uniform stepping) and 2 (the
 * minimum over the half-texel grid); for the last two the only decisions are
 * whether a step lies inside the tile and within the cap.  Returns the number
 * of values written (<= max_out), -1 when the branch cap was exceeded, -2 for
 * another mode or a bad ray. */
int32_t or_alternatives(const or_ctx* c, const or_params* p, int64_t ray,
                        double eh_abs, double eh_rel, double et_abs, double et_rel,
                        double* alpha_out, int32_t max_out);

/* ---- view rays (Sec. 4, view ray casting); definitions in view.c ---- */
typedef struct {
  int32_t width, height;    /* image, pixels */
  double eye[3];            /* tile frame, metres, relative to the point where the
                               tile's z axis meets the reference surface */
  double fwd[3], right[3], up[3]; /* pixel ray: fwd + sx right + sy up (normalised) */
  double step_m;            /* sample spacing along the view ray */
  double far_m;             /* samples beyond this ray length do not count; <= 0: none */
} or_camera;

typedef struct {
  double eh_abs, eh_rel;    /* height tolerance eh_abs + eh_rel (|eye| + t), metres */
  double ep_abs, ep_rel;    /* position tolerance ep_abs + ep_rel (|eye| + t), metres */
  int64_t max_samples;      /* safety cap per ray (status -1 when exceeded) */
} or_view_tol;

#define OR_VIEW_MAXADM 8
typedef struct {
  int32_t n_hit;            /* first certain hit sample, -1: none (a miss is admissible) */
  int32_t n_adm;            /* admissible first-hit samples (may exceed OR_VIEW_MAXADM) */
  int32_t adm[OR_VIEW_MAXADM];
  int32_t adm_overflow;
  int32_t status;
  double t_hit;             /* refined hit (INFINITY: none) */
  double qx, qy;            /* texel coordinates at t_hit (NaN: none) */
  double f_prev, f_hit;     /* f at t_{n-1} and t_n */
  double eps;               /* height tolerance at the hit sample */
  double dqdt;              /* |dq/dt| at t_hit, texels per metre */
} or_view_hit;

/* pixels: n (px, py) pairs, or NULL for all width*height pixels row by row.
 * Returns 0, -1 for bad arguments, -2 for a pixel outside the image. */
int32_t or_view(const or_ctx* c, double radius_m, double texel_m, const or_camera* cam,
                const int32_t* pixels, int64_t n, const or_view_tol* tol, or_view_hit* out);
void or_view_direction(const or_camera* cam, int32_t px, int32_t py, double* V);
/* out6: qx, qy, H, terrain, f = H - terrain, defined (P_z > 0) */
void or_view_probe(const or_ctx* c, double radius_m, double texel_m, const or_camera* cam,
                   int32_t px, int32_t py, double t, double* out6);

/* ---- tiles in different gnomonic frames (Sec. 3.3, Sec. 4); resample.c ---- */
typedef struct {
  int32_t width, rows;
  double texel_m;
  double centre[3];         /* unit tangent point, planet frame */
  double ex[3], ey[3];      /* unit plane axes: +column, +row */
  double origin_m[2];       /* plane coordinates of the grid centre */
} or_frame;

/* Destination texels whose direction projects into the source tile get the
 * source's bilinear height (FP64, rounded once into dst); others are left
 * alone.  Any of dst, dst64, covered, edge_margin may be NULL. */
int32_t or_resample(const float* src, const or_frame* fs, const or_frame* fd, double radius_m,
                    float* dst, double* dst64, uint8_t* covered, double* edge_margin);
void or_frame_source_coords(const or_frame* fs, const or_frame* fd, double R, int i, int j,
                            double* qx, double* qy, double* front);

/* Inspection helpers used by the pins. */
double or_disc_fraction(double d);
int32_t or_schedule(const or_params* p, int32_t* m0_out, double* tau_out, double* delta_out);
void or_ray_consts(const or_ctx* c, const or_params* p, int32_t i, int32_t j, double* out16);
void or_probe(const or_ctx* c, const or_params* p, int32_t i, int32_t j, double t, double* out8);
int32_t or_path_cells(const or_ctx* c, const or_params* p, int32_t i, int32_t j, int32_t level,
                      double ta, double tb, int32_t* cells_out, double* t_out, int32_t max_out);

#ifdef __cplusplus
}
#endif
#endif
