/* Reference oracle for the soft-shadow hot path (FP64, one ray at a time).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the bench's CPU
 * baseline use it; the product path never does.  Every function below follows
 * the paper passage named in its comment.  Where the paper is silent or
 * garbled, the reading taken is stated in the comment.
 *
 * Pins (tests/test_oracle_*.py): maximum mipmap against a direct block-max
 * definition and its invariants; geometry against closed forms (gnomonic round
 * trip, planar and bare-sphere tip height, projective form of the texture
 * path); the clearance angle against a direct 3-D angle; the disc fraction
 * against circular-segment geometry; the descent's cell walk against dense
 * sampling of the path; the whole method against flat ground, a half-set sun,
 * the straight-ridge penumbra closed form, and the exact invariant that the
 * descent's clearance is never below dense half-texel stepping.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

/* ------------------------------------------------------------------ */
/* Maximum mipmap (Sec. 3.2, "Maximum mipmaps"): each texel of level m */
/* holds the largest height of the level-(m-1) texels it covers.       */
/* ------------------------------------------------------------------ */

int32_t or_maxmip_levels(int32_t width, int32_t rows) {
  int32_t big = width > rows ? width : rows;
  int32_t L = 1;
  while ((1LL << (L - 1)) < big) L++;
  return L;
}

static void level_dims(int32_t W, int32_t H, int32_t m, int* wm, int* hm) {
  int w = W, h = H;
  for (int k = 0; k < m; ++k) {
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  *wm = w;
  *hm = h;
}

int64_t or_maxmip_offset(int32_t width, int32_t rows, int32_t level) {
  int64_t off = 0;
  for (int32_t m = 1; m < level; ++m) {
    int wm, hm;
    level_dims(width, rows, m, &wm, &hm);
    off += (int64_t)wm * hm;
  }
  return off;
}

int64_t or_maxmip_floats(int32_t width, int32_t rows) {
  return or_maxmip_offset(width, rows, or_maxmip_levels(width, rows));
}

or_ctx* or_ctx_create(const float* h, int32_t width, int32_t rows) {
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  if (!c) return NULL;
  c->W = width;
  c->H = rows;
  c->L = or_maxmip_levels(width, rows);
  int64_t total = or_maxmip_floats(width, rows);
  c->store = (float*)malloc(sizeof(float) * (size_t)(total > 0 ? total : 1));
  if (!c->store) {
    free(c);
    return NULL;
  }
  c->level[0] = h;
  c->w[0] = width;
  c->h[0] = rows;
  for (int m = 1; m < c->L; ++m) {
    level_dims(width, rows, m, &c->w[m], &c->h[m]);
    float* dst = c->store + or_maxmip_offset(width, rows, m);
    const float* src = c->level[m - 1];
    int ws = c->w[m - 1], hs = c->h[m - 1];
    for (int j = 0; j < c->h[m]; ++j) {
      for (int i = 0; i < c->w[m]; ++i) {
        float best = -INFINITY;
        for (int dj = 0; dj < 2; ++dj) {
          for (int di = 0; di < 2; ++di) {
            int cj = 2 * j + dj, ci = 2 * i + di;
            if (cj >= hs || ci >= ws) continue; /* absent child of a ragged edge */
            float v = src[(int64_t)cj * ws + ci] + 0.0f; /* -0 becomes +0 */
            if (v > best) best = v;
          }
        }
        dst[(int64_t)j * c->w[m] + i] = best;
      }
    }
    c->level[m] = dst;
  }
  return c;
}

void or_ctx_destroy(or_ctx* c) {
  if (!c) return;
  free(c->store);
  free(c);
}

void or_ctx_copy_maxmip(const or_ctx* c, float* out) {
  int64_t total = or_maxmip_floats(c->W, c->H);
  if (total > 0) memcpy(out, c->store, sizeof(float) * (size_t)total);
}

/* ------------------------------------------------------------------ */
/* Sun disc occlusion (Sec. 3.4, Eq. 6 first term): the visible part  */
/* of a unit disc above a chord at signed distance d below its centre. */
/* ------------------------------------------------------------------ */

double or_disc_fraction(double d) {
  if (d <= -1.0) return 0.0;
  if (d >= 1.0) return 1.0;
  return (M_PI - acos(d) + d * sqrt(1.0 - d * d)) / M_PI;
}

/* ------------------------------------------------------------------ */
/* Per (tile, sun) set-up.                                              */
/* ------------------------------------------------------------------ */

/* Segment schedule (Sec. 3.3, "Long shadows"): segment j traces N'_j levels
 * from m0 = N'_j - 1 and covers one level-m0 texel of travel, T_j = 2^m0 delta;
 * the next segment starts where the previous ended.  The segment count is the
 * smallest that reaches the horizontal cap (or spans the tile diagonal). */
void or_setup(setup_t* s, const or_ctx* c, const or_params* p) {
  memset(s, 0, sizeof(*s));
  s->c = c;
  s->p = p;
  s->planar = isinf(p->radius_m) ? 1 : 0;
  s->R = p->radius_m;
  s->D = p->texel_m;
  double ce = cos(p->elev_rad);
  s->Lv[0] = ce * cos(p->azim_rad);
  s->Lv[1] = ce * sin(p->azim_rad);
  s->Lv[2] = sin(p->elev_rad);
  /* Appendix (deriving T): one texel of horizontal travel at the tile centre. */
  s->delta = p->texel_m / ce;
  s->tau0 = 0.5 * s->delta;
  int L = c ? c->L : or_maxmip_levels(p->width, p->rows);
  /* without a cap the segments cover the tile diagonal (plus the half-texel start) */
  double need = p->max_len_m > 0.0 ? p->max_len_m / p->texel_m
                                   : sqrt((double)p->width * p->width + (double)p->rows * p->rows) + 2.0;
  double covered = 0.0;
  s->tau[0] = s->tau0;
  int j = 0;
  for (;;) {
    int np = p->schedule == 1 ? p->n_prime0 : p->n_prime0 + j;
    if (p->schedule == 2) np = p->n_prime_list[j < 16 ? j : 15];
    if (np > L) np = L;
    if (np < 1) np = 1;
    s->m0[j] = np - 1;
    s->tau[j + 1] = s->tau[j] + ldexp(s->delta, s->m0[j]);
    covered += ldexp(1.0, s->m0[j]);
    j++;
    if (p->n_segments > 0) {
      if (j >= p->n_segments) break;
    } else if (covered >= need) {
      break;
    }
    if (j >= OR_MAXSEG) break;
  }
  s->nseg = j;
  /* Uniform steps stop at the cap; without one at the tile edge, and at the
   * latest after the tile diagonal (the segments' extent), since on the sphere
   * a ray toward a texel's zenith never leaves the tile in texture space. */
  if (p->uniform_tmax_m > 0.0)
    s->tcap_uniform = p->uniform_tmax_m;
  else if (p->max_len_m > 0.0)
    s->tcap_uniform = p->max_len_m / p->texel_m * s->delta;
  else
    s->tcap_uniform = s->tau[s->nseg];
}

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 3.2 texture-space ray; Sec. 4 cube-sphere faces):     */
/* a gnomonic tile.  The tile frame has z through the tile centre, the  */
/* tangent plane at distance R carries the texel grid, and a point P    */
/* maps to texel coordinates by central projection onto that plane.    */
/* ------------------------------------------------------------------ */

void or_ray_init(ray_t* r, const setup_t* s, int i, int j) {
  const or_ctx* c = s->c;
  or_ray_init_at(r, s, i + 0.5, j + 0.5, c ? (double)c->level[0][(int64_t)j * c->W + i] : 0.0);
  r->i = i;
  r->j = j;
}

/* A ray from the surface point above continuous texel coordinates (qx, qy)
 * at height hp (texel centres: (i + 1/2, j + 1/2) and the texel's height). */
void or_ray_init_at(ray_t* r, const setup_t* s, double qx, double qy, double hp) {
  memset(r, 0, sizeof(*r));
  r->s = s;
  r->i = (int)floor(qx);
  r->j = (int)floor(qy);
  r->hp = hp;
  double X = (qx - 0.5 * s->p->width) * s->D;
  double Y = (qy - 0.5 * s->p->rows) * s->D;
  const double* L = s->Lv;
  if (s->planar) {
    r->n[0] = 0.0;
    r->n[1] = 0.0;
    r->n[2] = 1.0;
    r->p[0] = X;
    r->p[1] = Y;
    r->p[2] = r->hp;
    r->rho = INFINITY;
    r->t_hmin = L[2] >= 0.0 ? -INFINITY : INFINITY;
  } else {
    double l = sqrt(X * X + Y * Y + s->R * s->R);
    r->n[0] = X / l;
    r->n[1] = Y / l;
    r->n[2] = s->R / l;
    r->rho = s->R + r->hp;
    for (int k = 0; k < 3; ++k) r->p[k] = r->rho * r->n[k];
  }
  r->sp = r->n[0] * L[0] + r->n[1] * L[1] + r->n[2] * L[2];
  double cx = r->n[1] * L[2] - r->n[2] * L[1];
  double cy = r->n[2] * L[0] - r->n[0] * L[2];
  double cz = r->n[0] * L[1] - r->n[1] * L[0];
  r->cp = sqrt(cx * cx + cy * cy + cz * cz);
  /* |p + tL|^2 = rho^2 + 2 t rho sp + t^2 is smallest at t = -rho sp. */
  if (!s->planar) r->t_hmin = -r->rho * r->sp;
  /* Leaving the tile: the first boundary line met in the direction of motion. */
  r->texit = INFINITY;
  for (int a = 0; a < 2; ++a) {
    int sg = or_motion_sign(r, a);
    if (sg == 0) continue;
    double g = sg > 0 ? (a == 0 ? (double)s->p->width : (double)s->p->rows) : 0.0;
    double t = or_t_on_line(r, a, g);
    /* On the sphere the texture-space line approaches a limit point as t grows;
     * a boundary beyond it is never reached (the solution has t <= 0). */
    if (t > 0.0 && t < r->texit) r->texit = t;
  }
}

/* Ray tip R(t) = p + t L: texel coordinates and height above the sphere. */
void or_ray_point(const ray_t* r, double t, double* qx, double* qy, double* Ht) {
  const setup_t* s = r->s;
  double P0 = r->p[0] + t * s->Lv[0];
  double P1 = r->p[1] + t * s->Lv[1];
  double P2 = r->p[2] + t * s->Lv[2];
  if (s->planar) {
    *qx = P0 / s->D + 0.5 * s->p->width;
    *qy = P1 / s->D + 0.5 * s->p->rows;
    *Ht = P2;
  } else {
    *qx = s->R * P0 / (P2 * s->D) + 0.5 * s->p->width;
    *qy = s->R * P1 / (P2 * s->D) + 0.5 * s->p->rows;
    *Ht = sqrt(P0 * P0 + P1 * P1 + P2 * P2) - s->R;
  }
}

/* Ray length at which texel coordinate `axis` equals g (line crossing). */
double or_t_on_line(const ray_t* r, int axis, double g) {
  const setup_t* s = r->s;
  double half = axis == 0 ? 0.5 * s->p->width : 0.5 * s->p->rows;
  double G = (g - half) * s->D;
  if (s->planar) return (G - r->p[axis]) / s->Lv[axis];
  /* R (p_a + t L_a) = G (p_z + t L_z) */
  return (G * r->p[2] - s->R * r->p[axis]) / (s->R * s->Lv[axis] - G * s->Lv[2]);
}

/* Sign of d q_axis / dt; constant along the ray because central projection
 * maps the straight ray onto a straight texture-space line. */
int or_motion_sign(const ray_t* r, int axis) {
  const setup_t* s = r->s;
  double v = s->planar ? s->Lv[axis] : s->Lv[axis] * r->p[2] - r->p[axis] * s->Lv[2];
  return v > 0.0 ? 1 : (v < 0.0 ? -1 : 0);
}

int or_inside(const setup_t* s, double qx, double qy) {
  return qx >= 0.0 && qx < (double)s->p->width && qy >= 0.0 && qy < (double)s->p->rows;
}

/* Bilinear height over texel centres (i+1/2, j+1/2), clamped to the edge. */
double or_bilinear(const setup_t* s, double qx, double qy) {
  const or_ctx* c = s->c;
  double x = qx - 0.5, y = qy - 0.5;
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  long i0 = (long)x0, j0 = (long)y0;
  long i1 = i0 + 1, j1 = j0 + 1;
  long Wm = c->W - 1, Hm = c->H - 1;
  i0 = i0 < 0 ? 0 : (i0 > Wm ? Wm : i0);
  i1 = i1 < 0 ? 0 : (i1 > Wm ? Wm : i1);
  j0 = j0 < 0 ? 0 : (j0 > Hm ? Hm : j0);
  j1 = j1 < 0 ? 0 : (j1 > Hm ? Hm : j1);
  const float* h = c->level[0];
  double h00 = h[j0 * c->W + i0], h10 = h[j0 * c->W + i1];
  double h01 = h[j1 * c->W + i0], h11 = h[j1 * c->W + i1];
  return (1.0 - fy) * ((1.0 - fx) * h00 + fx * h10) + fy * ((1.0 - fx) * h01 + fx * h11);
}

/* Angular clearance of the terrain point O below the ray tip, seen from p:
 * the signed angle between L and O - p, positive when O is below the ray.
 * With O = R(t) - dh * R(t)/|R(t)|:  (O-p).L = t - dh (rho sp + t)/|R| and the
 * component toward the sky is -dh rho cp/|R|.  To first order this is the
 * paper's J* (N.N_L) = (dh/t) cp (Sec. 3.4, Eq. 5). */
double or_alpha_of(const ray_t* r, double t, double dh) {
  const setup_t* s = r->s;
  if (s->planar) return atan2(dh * r->cp, t - dh * r->sp);
  double P0 = r->p[0] + t * s->Lv[0];
  double P1 = r->p[1] + t * s->Lv[1];
  double P2 = r->p[2] + t * s->Lv[2];
  double len = sqrt(P0 * P0 + P1 * P1 + P2 * P2);
  return atan2(dh * r->rho * r->cp, t * len - dh * (r->rho * r->sp + t));
}

/* The half-texel grid of ray lengths: t_n = tau0 + n delta/2. */
double or_t_grid(const setup_t* s, long n) { return s->tau0 + (double)n * (0.5 * s->delta); }

/* Lower bound of the clearance over a candidate texel (Sec. 3.2, Eq. 4 with
 * the maximum mipmap): smallest tip height over the part of the ray inside the
 * texel minus the texel's maximum height.  H(t) is convex in t. */
double or_lower_bound(const ray_t* r, int m, const cand_t* c) {
  double tc = r->t_hmin;
  if (tc < c->t_in) tc = c->t_in;
  if (tc > c->t_out) tc = c->t_out;
  double qx, qy, Ht;
  or_ray_point(r, tc, &qx, &qy, &Ht);
  const or_ctx* cx = r->s->c;
  double M = cx->level[m][(int64_t)c->cy * cx->w[m] + c->cx];
  return Ht - M;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* Texel traversal (Sec. 3.2, "Texel traversal", Fig. 3b): every level-m texel
 * under the footprint of the ray for t in [ta, tb], each with the part of the
 * ray inside it.  Crossings of the level's grid lines split [ta, tb]; each
 * piece of positive length belongs to the texel holding its midpoint.  With a
 * parent the pieces are restricted to the parent's children (Sec. 3.2 proof:
 * the ray inside texel i at one level crosses texels 2i, 2i+1, ... at the next). */
int or_cells_on_path(const ray_t* r, int m, double ta, double tb, const cand_t* parent,
                     cand_t* out, double* min_gap) {
  const or_ctx* c = r->s->c;
  double S = ldexp(1.0, m);
  double qa[2], qb[2], Hd;
  or_ray_point(r, ta, &qa[0], &qa[1], &Hd);
  or_ray_point(r, tb, &qb[0], &qb[1], &Hd);
  double ev[2 * OR_MAXCAND + 2];
  int ne = 0;
  ev[ne++] = ta;
  for (int a = 0; a < 2; ++a) {
    double lo = qa[a] < qb[a] ? qa[a] : qb[a];
    double hi = qa[a] < qb[a] ? qb[a] : qa[a];
    for (double k = floor(lo / S) + 1.0; k * S < hi; k += 1.0) {
      double t = or_t_on_line(r, a, k * S);
      if (t < ta) t = ta;
      if (t > tb) t = tb;
      if (ne < 2 * OR_MAXCAND) ev[ne++] = t;
    }
  }
  ev[ne++] = tb;
  qsort(ev + 1, (size_t)(ne - 2), sizeof(double), cmp_double);
  if (min_gap) {
    /* spacing of the real decisions: crossings inside (ta, tb) and the ends.
     * A crossing that coincides with an end to rounding is the parent's own
     * boundary line seen again one level down, not a decision. */
    double tiny = 1e-9 * (fabs(ta) + fabs(tb) + r->s->delta);
    double prev = ta;
    for (int k = 1; k < ne; ++k) {
      int is_end = (k == ne - 1);
      if (!is_end && (ev[k] - ta <= tiny || tb - ev[k] <= tiny)) continue;
      /* in texels, relative to the texels travelled (FP32 position error grows
       * with the offset from the origin) */
      double g = (ev[k] - prev) / (r->s->delta + ev[k]);
      if (g < *min_gap) *min_gap = g;
      prev = ev[k];
    }
  }
  int n = 0;
  for (int k = 0; k + 1 < ne; ++k) {
    double u = ev[k], v = ev[k + 1];
    if (!(v > u)) continue;
    double qx, qy;
    or_ray_point(r, 0.5 * (u + v), &qx, &qy, &Hd);
    int cx = (int)floor(qx / S), cy = (int)floor(qy / S);
    if (cx < 0 || cy < 0 || cx >= c->w[m] || cy >= c->h[m]) continue;
    if (parent && (cx / 2 != parent->cx || cy / 2 != parent->cy)) continue;
    if (n > 0 && out[n - 1].cx == cx && out[n - 1].cy == cy) {
      out[n - 1].t_out = v; /* same texel on both sides of a coincident crossing */
      continue;
    }
    if (n < OR_MAXCAND) {
      out[n].cx = cx;
      out[n].cy = cy;
      out[n].t_in = u;
      out[n].t_out = v;
      n++;
    }
  }
  return n;
}

/* ------------------------------------------------------------------ */
/* Dynamic-programming descent of one segment (Sec. 3.2, Alg. 1, with  */
/* the candidate texels of the proof and Fig. 3b).                      */
/* ------------------------------------------------------------------ */

typedef struct {
  double alpha;
  double t, dh;
  long n;
  int base_i, base_j;
  int evals;
  double margin_lb, margin_dh, margin_round, margin_geo;
} seg_result;

static void dp_segment(const ray_t* r, int jseg, seg_result* out) {
  const setup_t* s = r->s;
  out->alpha = INFINITY;
  out->n = -1;
  out->base_i = out->base_j = -1;
  out->evals = 0;
  double ta = s->tau[jseg];
  double tb = ta + ldexp(s->delta, s->m0[jseg]);
  if (!(ta < r->texit)) return; /* segment starts outside the tile */
  if (tb > r->texit) tb = r->texit;
  int m = s->m0[jseg];
  cand_t cand[OR_MAXCAND];
  int n = or_cells_on_path(r, m, ta, tb, NULL, cand, &out->margin_geo);
  cand_t best;
  for (;;) {
    /* Strict '<' evaluated from the far end toward the origin, as in Alg. 1:
     * an exact tie keeps the farther texel. */
    int b = -1;
    double blb = INFINITY, second = INFINITY;
    for (int k = n - 1; k >= 0; --k) {
      double lb = or_lower_bound(r, m, &cand[k]);
      out->evals++;
      if (lb < blb) {
        second = blb;
        blb = lb;
        b = k;
      } else if (lb < second) {
        second = lb;
      }
    }
    if (b < 0) return;
    if (second - blb < out->margin_lb) out->margin_lb = second - blb;
    best = cand[b];
    if (m == 0) break;
    n = or_cells_on_path(r, m - 1, best.t_in, best.t_out, &best, cand, &out->margin_geo);
    m -= 1;
  }
  /* Final level (Alg. 1 at m = 0): three samples half a texel apart around the
   * chosen base texel, on the grid t_n; the clearance uses the bilinear height
   * of the terrain below the ray tip. */
  double tmid = 0.5 * (best.t_in + best.t_out);
  double arg = (tmid - s->tau0) / (0.5 * s->delta) + 0.5;
  long nc = (long)floor(arg);
  double fr = fabs(arg - floor(arg));
  if (fr > 0.5) fr = 1.0 - fr;
  if (fr < out->margin_round) out->margin_round = fr;
  out->base_i = best.cx;
  out->base_j = best.cy;
  double bdh = INFINITY, second = INFINITY;
  long bn = -1;
  for (long nn = nc + 1; nn >= nc - 1; --nn) {
    if (nn < 0) continue;
    double t = or_t_grid(s, nn);
    double qx, qy, Ht;
    or_ray_point(r, t, &qx, &qy, &Ht);
    if (!or_inside(s, qx, qy)) continue;
    double dh = Ht - or_bilinear(s, qx, qy);
    out->evals++;
    if (dh < bdh) {
      second = bdh;
      bdh = dh;
      bn = nn;
    } else if (dh < second) {
      second = dh;
    }
  }
  if (bn < 0) return;
  if (second - bdh < out->margin_dh) out->margin_dh = second - bdh;
  out->n = bn;
  out->t = or_t_grid(s, bn);
  out->dh = bdh;
  out->alpha = or_alpha_of(r, out->t, out->dh);
}

/* Alg. 1 read literally: the point-sample variant of the descent.  Positions
 * along run j are indices n on the half-texel grid t_n = tau0 + n delta/2; the
 * algorithm's normalised t in [0, 1] is (n - a_j) / 2^(m0+1), a_j the run's
 * first index.  Level k (mip m = m0 - k) reads the maximum mipmap at the texel
 * holding the ray tip at n = a_j + K, a_j + K - 2^m, a_j + K - 2^(m+1), in that
 * order (the far one first, so strict '<' keeps it on a tie); the smallest
 * H - max h gives K*, and the next level starts at K* + 2^m.  K starts at
 * 2^(m0+1) (t = 1).  The last level (m = 0) samples the heightfield
 * bilinearly, and the chosen sample's exact angle is the run's clearance, as
 * in the texel descent.  A level with no sample inside the tile ends the run. */
static void point_segment(const ray_t* r, int jseg, seg_result* out) {
  const setup_t* s = r->s;
  const or_ctx* c = s->c;
  out->alpha = INFINITY;
  out->n = -1;
  out->base_i = out->base_j = -1;
  out->evals = 0;
  const int m0 = s->m0[jseg];
  long a = 0;
  for (int i = 0; i < jseg; ++i) a += 2L << s->m0[i];
  long K = 2L << m0;
  for (int m = m0; m >= 0; --m) {
    const long step = 1L << m;
    double best = INFINITY, second = INFINITY;
    long kstar = -1;
    double bqx = 0.0, bqy = 0.0;
    for (int i = 0; i < 3; ++i) {
      long n = a + K - i * step;
      double t = or_t_grid(s, n);
      double qx, qy, Ht;
      or_ray_point(r, t, &qx, &qy, &Ht);
      /* where a rounding of q could change the texel read or the tile test */
      double fx = ldexp(qx, -m) - floor(ldexp(qx, -m)), fy = ldexp(qy, -m) - floor(ldexp(qy, -m));
      double g = fmin(fmin(fx, 1.0 - fx), fmin(fy, 1.0 - fy)) * ldexp(1.0, m);
      g = fmin(g, fmin(fmin(fabs(qx), fabs(qx - s->p->width)), fmin(fabs(qy), fabs(qy - s->p->rows))));
      g /= 1.0 + t / s->delta;
      if (m > 0 && g < out->margin_geo) out->margin_geo = g;
      if (!or_inside(s, qx, qy)) continue;
      double v;
      if (m > 0) {
        int cx = (int)floor(ldexp(qx, -m)), cy = (int)floor(ldexp(qy, -m));
        v = Ht - c->level[m][(int64_t)cy * c->w[m] + cx];
      } else {
        v = Ht - or_bilinear(s, qx, qy);
      }
      out->evals++;
      if (v < best) {
        second = best;
        best = v;
        kstar = K - i * step;
        bqx = qx;
        bqy = qy;
      } else if (v < second) {
        second = v;
      }
    }
    if (kstar < 0) return;
    if (m > 0) {
      if (second - best < out->margin_lb) out->margin_lb = second - best;
      K = kstar + step;
      continue;
    }
    if (second - best < out->margin_dh) out->margin_dh = second - best;
    out->n = a + kstar;
    out->t = or_t_grid(s, out->n);
    out->dh = best;
    out->alpha = or_alpha_of(r, out->t, best);
    out->base_i = (int)floor(bqx);
    out->base_j = (int)floor(bqy);
  }
}

typedef void (*segment_fn)(const ray_t* r, int jseg, seg_result* out);

static double shadow_runs(const ray_t* r, segment_fn segment, or_trace* tr);

static double shadow_dp(const ray_t* r, or_trace* tr) { return shadow_runs(r, dp_segment, tr); }

static double shadow_runs(const ray_t* r, segment_fn segment, or_trace* tr) {
  const setup_t* s = r->s;
  double alpha = INFINITY, second = INFINITY;
  or_trace t0;
  memset(&t0, 0, sizeof(t0));
  t0.seg = -2;
  t0.n = -1;
  t0.base_i = t0.base_j = -1;
  t0.alpha = INFINITY;
  t0.margin_lb = t0.margin_dh = t0.margin_round = t0.margin_seg = t0.margin_geo = INFINITY;
  for (int j = 0; j < s->nseg; ++j) {
    seg_result sr;
    sr.margin_lb = sr.margin_dh = sr.margin_round = sr.margin_geo = INFINITY;
    segment(r, j, &sr);
    t0.evals += sr.evals;
    if (sr.margin_lb < t0.margin_lb) t0.margin_lb = sr.margin_lb;
    if (sr.margin_dh < t0.margin_dh) t0.margin_dh = sr.margin_dh;
    if (sr.margin_round < t0.margin_round) t0.margin_round = sr.margin_round;
    if (sr.margin_geo < t0.margin_geo) t0.margin_geo = sr.margin_geo;
    /* Concatenated runs (Sec. 3.3): the shadow takes the smallest clearance. */
    if (sr.alpha < alpha) {
      second = alpha;
      alpha = sr.alpha;
      t0.seg = j;
      t0.n = (int32_t)sr.n;
      t0.t = sr.t;
      t0.dh = sr.dh;
      t0.base_i = sr.base_i;
      t0.base_j = sr.base_j;
    } else if (sr.alpha < second) {
      second = sr.alpha;
    }
  }
  t0.alpha = alpha;
  t0.margin_seg = second - alpha;
  t0.margin_tap = INFINITY;
  if (t0.n >= 0) {
    /* the bilinear height is continuous across the lines through texel
     * centres, its slope is not */
    double qx, qy, Hd;
    or_ray_point(r, t0.t, &qx, &qy, &Hd);
    double fx = qx - 0.5 - floor(qx - 0.5), fy = qy - 0.5 - floor(qy - 0.5);
    double m = fmin(fmin(fx, 1.0 - fx), fmin(fy, 1.0 - fy));
    t0.margin_tap = m / (1.0 + t0.t / s->delta);
  }
  if (tr) *tr = t0;
  return alpha;
}

/* Uniform stepping (Sec. 2 and Fig. 1b; the paper's baseline in Sec. 6.3):
 * constant steps du along the ray, clearance angle at every step, minimum.
 * With du = delta/2 the steps are exactly the half-texel grid t_n = (n+1)
 * delta/2 on which the descent places its final samples, so the minimum is
 * the global minimum over that grid (the exact mode's definition). */
static double shadow_uniform(const ray_t* r, double du, or_trace* tr) {
  const setup_t* s = r->s;
  double alpha = INFINITY, second = INFINITY;
  or_trace t0;
  memset(&t0, 0, sizeof(t0));
  t0.seg = -2;
  t0.n = -1;
  t0.base_i = t0.base_j = -1;
  t0.margin_lb = t0.margin_dh = t0.margin_round = t0.margin_seg = t0.margin_geo = INFINITY;
  for (long k = 0;; ++k) {
    double t = s->tau0 + (double)k * du;
    if (t > s->tcap_uniform) break;
    double qx, qy, Ht;
    or_ray_point(r, t, &qx, &qy, &Ht);
    if (!or_inside(s, qx, qy)) break;
    double dh = Ht - or_bilinear(s, qx, qy);
    double a = or_alpha_of(r, t, dh);
    t0.evals++;
    if (a < alpha) {
      second = alpha;
      alpha = a;
      t0.seg = -1;
      t0.n = (int32_t)k;
      t0.t = t;
      t0.dh = dh;
    } else if (a < second) {
      second = a;
    }
  }
  t0.alpha = alpha;
  /* how clearly the deciding step wins (rad), and its distance from a line
   * through texel centres (where the bilinear slope jumps) per texel travelled */
  t0.margin_seg = second - alpha;
  t0.margin_tap = INFINITY;
  if (t0.n >= 0) {
    double qx, qy, Hd;
    or_ray_point(r, t0.t, &qx, &qy, &Hd);
    double fx = qx - 0.5 - floor(qx - 0.5), fy = qy - 0.5 - floor(qy - 0.5);
    double m = fmin(fmin(fx, 1.0 - fx), fmin(fy, 1.0 - fy));
    t0.margin_tap = m / (1.0 + t0.t / s->delta);
  }
  if (tr) *tr = t0;
  return alpha;
}

int32_t or_shadow(const or_ctx* c, const or_params* p, const int64_t* rays, int64_t n_rays,
                  double* s_out, double* alpha_out, or_trace* trace_out) {
  if (!c || !p || p->width != c->W || p->rows != c->H) return -1;
  setup_t s;
  or_setup(&s, c, p);
  int64_t total = rays ? n_rays : (int64_t)c->W * c->H;
  for (int64_t k = 0; k < total; ++k) {
    int64_t lin = rays ? rays[k] : k;
    if (lin < 0 || lin >= (int64_t)c->W * c->H) return -2;
    ray_t r;
    or_ray_init(&r, &s, (int)(lin % c->W), (int)(lin / c->W));
    or_trace tr;
    double alpha;
    if (p->mode == 1)
      alpha = shadow_uniform(&r, p->uniform_step * s.delta, &tr);
    else if (p->mode == 2)
      alpha = shadow_uniform(&r, 0.5 * s.delta, &tr);
    else if (p->mode == 3)
      alpha = shadow_runs(&r, point_segment, &tr);
    else
      alpha = shadow_dp(&r, &tr);
    double sv = 1.0;
    if (isfinite(alpha)) {
      double d = alpha / p->ang_radius_rad;
      if (d < -1.0) d = -1.0;
      if (d > 1.0) d = 1.0;
      sv = or_disc_fraction(d);
    }
    if (s_out) s_out[k] = sv;
    if (alpha_out) alpha_out[k] = alpha;
    if (trace_out) trace_out[k] = tr;
  }
  return 0;
}

/* Shadow rays from arbitrary surface points: origin (qx, qy) in continuous
 * texel coordinates (inside the tile), height the bilinear terrain there. */
int32_t or_shadow_points(const or_ctx* c, const or_params* p, const double* xy, int64_t n,
                         double* s_out, double* alpha_out, or_trace* trace_out) {
  if (!c || !p || p->width != c->W || p->rows != c->H) return -1;
  setup_t s;
  or_setup(&s, c, p);
  for (int64_t k = 0; k < n; ++k) {
    double qx = xy[2 * k], qy = xy[2 * k + 1];
    if (!or_inside(&s, qx, qy)) return -2;
    ray_t r;
    or_ray_init_at(&r, &s, qx, qy, or_bilinear(&s, qx, qy));
    or_trace tr;
    double alpha;
    if (p->mode == 1)
      alpha = shadow_uniform(&r, p->uniform_step * s.delta, &tr);
    else if (p->mode == 2)
      alpha = shadow_uniform(&r, 0.5 * s.delta, &tr);
    else if (p->mode == 3)
      alpha = shadow_runs(&r, point_segment, &tr);
    else
      alpha = shadow_dp(&r, &tr);
    double sv = 1.0;
    if (isfinite(alpha)) {
      double d = alpha / p->ang_radius_rad;
      if (d < -1.0) d = -1.0;
      if (d > 1.0) d = 1.0;
      sv = or_disc_fraction(d);
    }
    if (s_out) s_out[k] = sv;
    if (alpha_out) alpha_out[k] = alpha;
    if (trace_out) trace_out[k] = tr;
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Inspection helpers for the pins.                                     */
/* ------------------------------------------------------------------ */

int32_t or_schedule(const or_params* p, int32_t* m0_out, double* tau_out, double* delta_out) {
  setup_t s;
  or_setup(&s, NULL, p);
  for (int j = 0; j < s.nseg; ++j) {
    if (m0_out) m0_out[j] = s.m0[j];
    if (tau_out) tau_out[j] = s.tau[j];
  }
  if (tau_out) tau_out[s.nseg] = s.tau[s.nseg];
  if (delta_out) *delta_out = s.delta;
  return s.nseg;
}

void or_ray_consts(const or_ctx* c, const or_params* p, int32_t i, int32_t j, double* out) {
  setup_t s;
  or_setup(&s, c, p);
  ray_t r;
  or_ray_init(&r, &s, i, j);
  double v[16] = {r.n[0], r.n[1], r.n[2], r.p[0], r.p[1], r.p[2], r.rho, r.sp,
                  r.cp,   r.t_hmin, r.texit, s.Lv[0], s.Lv[1], s.Lv[2], s.delta, r.hp};
  memcpy(out, v, sizeof(v));
}

void or_probe(const or_ctx* c, const or_params* p, int32_t i, int32_t j, double t, double* out) {
  setup_t s;
  or_setup(&s, c, p);
  ray_t r;
  or_ray_init(&r, &s, i, j);
  double qx, qy, Ht;
  or_ray_point(&r, t, &qx, &qy, &Ht);
  int in = or_inside(&s, qx, qy);
  double hb = in ? or_bilinear(&s, qx, qy) : NAN;
  double dh = Ht - hb;
  out[0] = qx;
  out[1] = qy;
  out[2] = Ht;
  out[3] = hb;
  out[4] = dh;
  out[5] = in ? or_alpha_of(&r, t, dh) : NAN;
  out[6] = in;
  out[7] = r.texit;
}

int32_t or_path_cells(const or_ctx* c, const or_params* p, int32_t i, int32_t j, int32_t level,
                      double ta, double tb, int32_t* cells_out, double* t_out, int32_t max_out) {
  setup_t s;
  or_setup(&s, c, p);
  ray_t r;
  or_ray_init(&r, &s, i, j);
  cand_t cand[OR_MAXCAND];
  int n = or_cells_on_path(&r, level, ta, tb, NULL, cand, NULL);
  int k;
  for (k = 0; k < n && k < max_out; ++k) {
    cells_out[2 * k] = cand[k].cx;
    cells_out[2 * k + 1] = cand[k].cy;
    t_out[2 * k] = cand[k].t_in;
    t_out[2 * k + 1] = cand[k].t_out;
  }
  return n;
}
