/* Reference oracle: moving heights between gnomonic tiles (TEST INFRASTRUCTURE).
 *
 * Sec. 3.3 (virtual texture mapping) and Sec. 4 (cube-sphere faces) stitch the
 * visible tiles into one texture; tiles on different cube faces live on
 * different projection planes.  A tile frame here is a plane tangent to the
 * sphere at a unit vector c, with orthonormal in-plane axes ex (+column) and
 * ey (+row), a texel spacing D measured in that plane and the plane
 * coordinates (o_x, o_y) of the grid centre (zero for a tile centred on its
 * tangent point, non-zero for a sub-tile of a cube face).  Texel (i, j) of a
 * W x H grid sits at plane point
 *     P = R c + X ex + Y ey,  X = o_x + (i + 1/2 - W/2) D,  Y likewise,
 * and stands for the surface point in direction P / |P|; heights are radial,
 * so they carry over unchanged between frames.
 *
 * Resampling a source tile into a destination tile: for each destination
 * texel, project its direction centrally onto the source plane (scale P so
 * that P . c_s = R), read the source texel coordinates and, if they lie in
 * [0, W_s) x [0, H_s), take the source's bilinear height there (texel
 * centres, taps clamped to the tile: the sampling rule of the shadow path).
 * Everything in FP64, rounded once to float32.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double bilinear(const float* h, int W, int H, double qx, double qy) {
  double x = qx - 0.5, y = qy - 0.5;
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  long i0 = (long)x0, j0 = (long)y0, i1 = i0 + 1, j1 = j0 + 1;
  i0 = i0 < 0 ? 0 : (i0 > W - 1 ? W - 1 : i0);
  i1 = i1 < 0 ? 0 : (i1 > W - 1 ? W - 1 : i1);
  j0 = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
  j1 = j1 < 0 ? 0 : (j1 > H - 1 ? H - 1 : j1);
  double h00 = h[j0 * W + i0], h10 = h[j0 * W + i1];
  double h01 = h[j1 * W + i0], h11 = h[j1 * W + i1];
  return (1.0 - fy) * ((1.0 - fx) * h00 + fx * h10) + fy * ((1.0 - fx) * h01 + fx * h11);
}

/* Plane point of destination texel (i, j) (metres, planet frame). */
static void texel_point(const or_frame* f, double R, int i, int j, double* P) {
  double X = f->origin_m[0] + ((double)i + 0.5 - 0.5 * f->width) * f->texel_m;
  double Y = f->origin_m[1] + ((double)j + 0.5 - 0.5 * f->rows) * f->texel_m;
  for (int k = 0; k < 3; ++k) P[k] = R * f->centre[k] + X * f->ex[k] + Y * f->ey[k];
}

void or_frame_source_coords(const or_frame* fs, const or_frame* fd, double R, int i, int j,
                            double* qx, double* qy, double* front) {
  double P[3];
  texel_point(fd, R, i, j, P);
  double z = dot3(P, fs->centre);
  *front = z;
  double s = R / z;
  double Xs = s * dot3(P, fs->ex), Ys = s * dot3(P, fs->ey);
  *qx = (Xs - fs->origin_m[0]) / fs->texel_m + 0.5 * fs->width;
  *qy = (Ys - fs->origin_m[1]) / fs->texel_m + 0.5 * fs->rows;
}

int32_t or_resample(const float* src, const or_frame* fs, const or_frame* fd, double radius_m,
                    float* dst, double* dst64, uint8_t* covered, double* edge_margin) {
  if (!src || !fs || !fd || !(radius_m > 0.0) || isinf(radius_m) || fs->width < 1 ||
      fs->rows < 1 || fd->width < 1 || fd->rows < 1 || !(fs->texel_m > 0.0) ||
      !(fd->texel_m > 0.0))
    return -1;
  for (int j = 0; j < fd->rows; ++j) {
    for (int i = 0; i < fd->width; ++i) {
      long k = (long)j * fd->width + i;
      double qx, qy, front;
      or_frame_source_coords(fs, fd, radius_m, i, j, &qx, &qy, &front);
      int in = front > 0.0 && qx >= 0.0 && qx < fs->width && qy >= 0.0 && qy < fs->rows;
      /* distance (texels) of the decision from the coverage boundary */
      double m = fmin(fmin(fabs(qx), fabs(qx - fs->width)), fmin(fabs(qy), fabs(qy - fs->rows)));
      if (edge_margin) edge_margin[k] = front > 0.0 ? m : 0.0;
      if (covered) covered[k] = (uint8_t)in;
      if (!in) continue;
      double v = bilinear(src, fs->width, fs->rows, qx, qy);
      if (dst64) dst64[k] = v;
      if (dst) dst[k] = (float)v;
    }
  }
  return 0;
}
