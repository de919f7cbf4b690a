/* Reference oracle: view rays onto the heightfield (TEST INFRASTRUCTURE).
 *
 * Sec. 4 (view ray casting) shoots, for every pixel, a ray from the eye and
 * intersects it with the same bilinear height field that the shadow rays see;
 * the shadow ray (Sec. 3) then starts at that intersection.  The paper leaves
 * the sampling of the view ray open (its shader marches from pre-displaced
 * vertices).  The definition followed here, written out densely:
 *
 *   - pixel (px, py) looks along V = fwd + sx right + sy up, normalised, with
 *     sx = 2 (px + 1/2) / width - 1 and sy = 1 - 2 (py + 1/2) / height;
 *   - the ray P(t) = eye + t V is sampled at t_n = n * step, n = 0, 1, 2, ...;
 *   - a sample counts when its texel coordinates q lie in the tile
 *     [0, width) x [0, rows) and t_n <= far (far <= 0: no limit);
 *   - f(t) = H(P(t)) - b(q(P(t))), H the height above the reference sphere
 *     (the plane z = 0 in flat mode), b the bilinear terrain (texel centres,
 *     clamped to the edge);
 *   - the hit is the first counting sample with f <= 0; it is refined by the
 *     zero of the straight line through (t_{n-1}, f_{n-1}) and (t_n, f_n):
 *     t_hit = t_{n-1} + step * f_{n-1} / (f_{n-1} - f_n) when f_{n-1} > 0,
 *     else t_{n-1} (t_hit = 0 for n = 0).  f_{n-1} uses the clamped terrain
 *     also when t_{n-1} lies outside the tile.
 *
 * Frame and mapping are the shadow oracle's (gnomonic tile, Sec. 3.2 and 4):
 * the eye is given relative to the point where the tile's z axis meets the
 * reference surface, i.e. the sphere centre sits at (0, 0, -R).
 *
 * Decisions with a small margin are reported instead of taken: a sample with
 * |f| <= eps, or whose q lies within a position tolerance of the tile edge,
 * may go either way; the answer is the set of admissible first-hit indices
 * (those ambiguous samples before the first certain hit, then that hit).
 */
#include <math.h>
#include <string.h>

#include "oracle_internal.h"

typedef struct {
  const or_ctx* c;
  const or_camera* cam;
  int planar;
  double R, D;
  double hmax;
} view_setup;

/* Bilinear terrain over texel centres (i + 1/2, j + 1/2), clamped to the edge;
 * *slope receives the largest tap difference per metre (for tolerances). */
static double terrain(const view_setup* v, double qx, double qy, double* slope) {
  const or_ctx* c = v->c;
  double x = qx - 0.5, y = qy - 0.5;
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  long i0 = (long)x0, j0 = (long)y0, i1 = i0 + 1, j1 = j0 + 1;
  long Wm = c->W - 1, Hm = c->H - 1;
  i0 = i0 < 0 ? 0 : (i0 > Wm ? Wm : i0);
  i1 = i1 < 0 ? 0 : (i1 > Wm ? Wm : i1);
  j0 = j0 < 0 ? 0 : (j0 > Hm ? Hm : j0);
  j1 = j1 < 0 ? 0 : (j1 > Hm ? Hm : j1);
  const float* h = c->level[0];
  double h00 = h[j0 * c->W + i0], h10 = h[j0 * c->W + i1];
  double h01 = h[j1 * c->W + i0], h11 = h[j1 * c->W + i1];
  if (slope) {
    double g = fabs(h10 - h00);
    g = fmax(g, fabs(h11 - h01));
    g = fmax(g, fabs(h01 - h00));
    g = fmax(g, fabs(h11 - h10));
    *slope = g / v->D;
  }
  return (1.0 - fy) * ((1.0 - fx) * h00 + fx * h10) + fy * ((1.0 - fx) * h01 + fx * h11);
}

/* Point of the ray at t: texel coordinates, height above the reference
 * surface, and whether the central projection is defined (P_z > 0). */
static int view_point(const view_setup* v, const double* E, const double* V, double t,
                      double* qx, double* qy, double* H) {
  double P0 = E[0] + t * V[0], P1 = E[1] + t * V[1], P2 = E[2] + t * V[2];
  double W2 = 0.5 * v->c->W, H2 = 0.5 * v->c->H;
  if (v->planar) {
    *qx = P0 / v->D + W2;
    *qy = P1 / v->D + H2;
    *H = P2;
    return 1;
  }
  double Z = v->R + P2; /* distance along z from the sphere centre */
  *qx = v->R * P0 / (Z * v->D) + W2;
  *qy = v->R * P1 / (Z * v->D) + H2;
  *H = sqrt(P0 * P0 + P1 * P1 + Z * Z) - v->R;
  return Z > 0.0;
}

/* Sign of d q_axis / d t (constant along the ray while P_z > 0). */
static int view_motion(const view_setup* v, const double* E, const double* V, int axis) {
  double s = v->planar ? V[axis] : V[axis] * (v->R + E[2]) - E[axis] * V[2];
  return s > 0.0 ? 1 : (s < 0.0 ? -1 : 0);
}

void or_view_direction(const or_camera* cam, int32_t px, int32_t py, double* V) {
  double sx = 2.0 * (px + 0.5) / cam->width - 1.0;
  double sy = 1.0 - 2.0 * (py + 0.5) / cam->height;
  double n2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    V[k] = cam->fwd[k] + sx * cam->right[k] + sy * cam->up[k];
    n2 += V[k] * V[k];
  }
  double inv = 1.0 / sqrt(n2);
  for (int k = 0; k < 3; ++k) V[k] *= inv;
}

static double view_f(const view_setup* v, const double* E, const double* V, double t,
                     double* qx, double* qy, double* slope, int* defined) {
  double H;
  *defined = view_point(v, E, V, t, qx, qy, &H);
  return H - terrain(v, *qx, *qy, slope);
}

static void view_pixel(const view_setup* v, int32_t px, int32_t py, const or_view_tol* tol,
                       or_view_hit* out) {
  const or_camera* cam = v->cam;
  const double* E = cam->eye;
  double V[3];
  or_view_direction(cam, px, py, V);
  double eyen = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
  double step = cam->step_m;
  int sgn[2] = {view_motion(v, E, V, 0), view_motion(v, E, V, 1)};
  double lim[2] = {(double)v->c->W, (double)v->c->H};
  memset(out, 0, sizeof(*out));
  out->n_hit = -1;
  out->t_hit = INFINITY;
  out->qx = out->qy = NAN;
  double f_prev = NAN;
  for (long n = 0;; ++n) {
    if (n > tol->max_samples) {
      out->status = -1;
      return;
    }
    double t = (double)n * step;
    if (cam->far_m > 0.0 && t > cam->far_m + tol->ep_abs) break;
    double qx, qy, slope;
    int defined;
    double f = view_f(v, E, V, t, &qx, &qy, &slope, &defined);
    if (!defined) break;
    double ep = tol->ep_abs + tol->ep_rel * (eyen + t); /* metres */
    double eq = ep / v->D;                               /* texels */
    double eps = tol->eh_abs + tol->eh_rel * (eyen + t) + slope * ep;
    double q[2] = {qx, qy};
    /* stop once the sample is clearly outside and moving away (the texture
     * path is a straight line traversed monotonically) */
    int gone = 0;
    for (int a = 0; a < 2; ++a) {
      if (q[a] < -eq && sgn[a] <= 0) gone = 1;
      if (q[a] > lim[a] + eq && sgn[a] >= 0) gone = 1;
    }
    /* or above every terrain height and rising (H is convex along the ray) */
    double qx2, qy2, H1, H0;
    view_point(v, E, V, t, &qx2, &qy2, &H0);
    view_point(v, E, V, t + step, &qx2, &qy2, &H1);
    if (H0 > v->hmax + eps && H1 >= H0) gone = 1;
    if (gone) break;
    int in_certain = qx >= eq && qx < lim[0] - eq && qy >= eq && qy < lim[1] - eq;
    int in_maybe = qx > -eq && qx < lim[0] + eq && qy > -eq && qy < lim[1] + eq;
    int far_maybe = cam->far_m > 0.0 && fabs(t - cam->far_m) <= tol->ep_abs;
    if (far_maybe) in_certain = 0;
    if (in_certain && f < -eps) {
      out->n_hit = (int32_t)n;
      if (out->n_adm < OR_VIEW_MAXADM) out->adm[out->n_adm] = (int32_t)n;
      else out->adm_overflow = 1;
      out->n_adm++;
      double w = (n > 0 && f_prev > 0.0) ? f_prev / (f_prev - f) : 0.0;
      double t0 = n > 0 ? (double)(n - 1) * step : 0.0;
      out->t_hit = t0 + step * w;
      out->f_prev = n > 0 ? f_prev : NAN;
      out->f_hit = f;
      out->eps = eps;
      double H;
      view_point(v, E, V, out->t_hit, &out->qx, &out->qy, &H);
      double ax, ay, bx, by, Ha, Hb;
      double dt = 1e-3 * step;
      view_point(v, E, V, out->t_hit - dt, &ax, &ay, &Ha);
      view_point(v, E, V, out->t_hit + dt, &bx, &by, &Hb);
      out->dqdt = hypot(bx - ax, by - ay) / (2.0 * dt);
      return;
    }
    if (in_maybe && f <= eps) {
      if (out->n_adm < OR_VIEW_MAXADM) out->adm[out->n_adm] = (int32_t)n;
      else out->adm_overflow = 1;
      out->n_adm++;
    }
    f_prev = f;
  }
  /* no certain hit: a miss is admissible too (n_hit stays -1) */
}

int32_t or_view(const or_ctx* c, double radius_m, double texel_m, const or_camera* cam,
                const int32_t* pixels, int64_t n, const or_view_tol* tol, or_view_hit* out) {
  if (!c || !cam || !tol || !out || texel_m <= 0.0 || radius_m <= 0.0 || cam->step_m <= 0.0 ||
      cam->width < 1 || cam->height < 1)
    return -1;
  view_setup v;
  v.c = c;
  v.cam = cam;
  v.planar = isinf(radius_m) ? 1 : 0;
  v.R = radius_m;
  v.D = texel_m;
  v.hmax = c->level[c->L - 1][0];
  if (!v.planar && cam->eye[2] <= -0.5 * radius_m) return -1;
  for (int64_t k = 0; k < n; ++k) {
    int32_t px, py;
    if (pixels) {
      px = pixels[2 * k];
      py = pixels[2 * k + 1];
    } else {
      px = (int32_t)(k % cam->width);
      py = (int32_t)(k / cam->width);
    }
    if (px < 0 || py < 0 || px >= cam->width || py >= cam->height) return -2;
    view_pixel(&v, px, py, tol, &out[k]);
  }
  return 0;
}

/* f, q and H along one pixel's ray at a given t (inspection for the pins). */
void or_view_probe(const or_ctx* c, double radius_m, double texel_m, const or_camera* cam,
                   int32_t px, int32_t py, double t, double* out6) {
  view_setup v;
  v.c = c;
  v.cam = cam;
  v.planar = isinf(radius_m) ? 1 : 0;
  v.R = radius_m;
  v.D = texel_m;
  v.hmax = c->level[c->L - 1][0];
  double V[3], qx, qy, H;
  or_view_direction(cam, px, py, V);
  int def = view_point(&v, cam->eye, V, t, &qx, &qy, &H);
  out6[0] = qx;
  out6[1] = qy;
  out6[2] = H;
  out6[3] = terrain(&v, qx, qy, NULL);
  out6[4] = H - out6[3];
  out6[5] = def;
}
