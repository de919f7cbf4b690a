// Heights moved between gnomonic tile frames (Sec. 3.3: visible tiles stitched
// into one texture; Sec. 4: cube-sphere faces) on gfx950.
//
// A frame is the plane tangent to the sphere at unit vector c with unit axes
// ex (+column) and ey (+row), texel spacing D in the plane and the plane
// coordinates (ox, oy) of its grid centre.  Destination texel (i, j) stands
// for the surface direction of P = R c + X ex + Y ey with
// X = ox + (i + 1/2 - W/2) D (Y likewise); its source texel coordinates come
// from central projection onto the source plane (P scaled so that P . c_s =
// R), and if they fall inside the source tile the texel receives the source's
// bilinear height there (texel centres, taps clamped).  Heights are radial,
// so they carry over unchanged.
//
// Positions and the blend are FP64, evaluated in a fixed order without
// contraction and rounded once to float32: a stitched halo is then the same
// float in every implementation of this definition, so shadows across seams
// do not depend on how the halo was built.  The kernel is HBM-bound (one
// 4-byte write per destination texel, neighbouring texels read neighbouring
// source texels); FP64 at 78.6 TFLOP/s stays below that.
#include "kernels.h"

namespace ss {

namespace {

__device__ __forceinline__ double dot3(const double* a, const double* b) {
#pragma clang fp contract(off)
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__global__ __launch_bounds__(256) void resample_kernel(ResampleK K) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= K.Wd || j >= K.Hd) return;
  const double X = K.oxd + ((double)i + 0.5 - 0.5 * (double)K.Wd) * K.Dd;
  const double Y = K.oyd + ((double)j + 0.5 - 0.5 * (double)K.Hd) * K.Dd;
  double P[3];
  for (int k = 0; k < 3; ++k) P[k] = K.R * K.cd[k] + X * K.exd[k] + Y * K.eyd[k];
  const double z = dot3(P, K.cs);
  if (!(z > 0.0)) return;
  const double s = K.R / z;
  const double Xs = s * dot3(P, K.exs), Ys = s * dot3(P, K.eys);
  const double qx = (Xs - K.oxs) / K.Ds + 0.5 * (double)K.Ws;
  const double qy = (Ys - K.oys) / K.Ds + 0.5 * (double)K.Hs;
  if (!(qx >= 0.0 && qx < (double)K.Ws && qy >= 0.0 && qy < (double)K.Hs)) return;
  const double x = qx - 0.5, y = qy - 0.5;
  const double x0 = floor(x), y0 = floor(y);
  const double fx = x - x0, fy = y - y0;
  // x0 >= -1 and < Ws here, so the clamps keep every tap inside the source
  const int i0 = max((int)x0, 0), i1 = min((int)x0 + 1, K.Ws - 1);
  const int j0 = max((int)y0, 0), j1 = min((int)y0 + 1, K.Hs - 1);
  const long long W = K.Ws;
  const double h00 = K.src[j0 * W + i0], h10 = K.src[j0 * W + i1];
  const double h01 = K.src[j1 * W + i0], h11 = K.src[j1 * W + i1];
  const double v = (1.0 - fy) * ((1.0 - fx) * h00 + fx * h10) + fy * ((1.0 - fx) * h01 + fx * h11);
  K.dst[(long long)j * K.Wd + i] = (float)v;
}

}  // namespace

hipError_t launch_resample(const ResampleK& K, hipStream_t stream) {
  if (K.Wd <= 0 || K.Hd <= 0) return hipSuccess;
  const dim3 grid((unsigned)((K.Wd + 15) / 16), (unsigned)((K.Hd + 15) / 16)), block(256);
  hipLaunchKernelGGL(resample_kernel, grid, block, 0, stream, K);
  return hipGetLastError();
}

}  // namespace ss
