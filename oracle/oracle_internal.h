/* Internal helpers of the reference oracle (shared by oracle.c and alternatives.c). */
#ifndef SS_ORACLE_INTERNAL_H
#define SS_ORACLE_INTERNAL_H

#include "oracle.h"

struct or_ctx {
  int W, H, L;
  int w[OR_MAXLEV], h[OR_MAXLEV];
  const float* level[OR_MAXLEV]; /* level 0 is the caller's heightfield */
  float* store;
};

/* Per (tile, sun) quantities. */
typedef struct {
  const or_ctx* c;
  const or_params* p;
  int planar;
  double R, D;           /* body radius, texel spacing */
  double Lv[3];          /* unit vector toward the sun centre, tile frame */
  double delta;          /* ray length per texel of horizontal travel */
  double tau0;           /* first sample: half a texel of travel */
  int nseg;
  int m0[OR_MAXSEG];     /* top mip level of each segment (N'_j - 1) */
  double tau[OR_MAXSEG + 1];
  double tcap_uniform;
} setup_t;

/* Per ray quantities. */
typedef struct {
  const setup_t* s;
  int i, j;
  double hp;
  double n[3];           /* unit radial normal at the origin */
  double p[3];           /* ray origin */
  double rho;            /* |p| */
  double sp, cp;         /* n.L and |n x L| */
  double t_hmin;         /* ray length where the tip height H(t) is smallest */
  double texit;          /* ray length where the path leaves the tile */
} ray_t;

typedef struct {
  int cx, cy;            /* cell indices at the current level */
  double t_in, t_out;    /* part of the ray inside the cell */
} cand_t;

#define OR_MAXCAND 16

void or_setup(setup_t* s, const or_ctx* c, const or_params* p);
void or_ray_init(ray_t* r, const setup_t* s, int i, int j);
void or_ray_init_at(ray_t* r, const setup_t* s, double qx, double qy, double hp);
void or_ray_point(const ray_t* r, double t, double* qx, double* qy, double* Ht);
double or_t_on_line(const ray_t* r, int axis, double g);
int or_motion_sign(const ray_t* r, int axis);
int or_inside(const setup_t* s, double qx, double qy);
double or_bilinear(const setup_t* s, double qx, double qy);
double or_alpha_of(const ray_t* r, double t, double dh);
double or_t_grid(const setup_t* s, long n);
double or_lower_bound(const ray_t* r, int m, const cand_t* c);
int or_cells_on_path(const ray_t* r, int m, double ta, double tb, const cand_t* parent,
                     cand_t* out, double* min_gap);

#endif
