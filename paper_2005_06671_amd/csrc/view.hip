// View rays onto the heightfield (Sec. 4, view ray casting) on gfx950.
//
// Pixel (px, py) looks along V = fwd + sx right + sy up (normalised),
// sx = 2 (px + 1/2) / width - 1, sy = 1 - 2 (py + 1/2) / height.  The ray
// P(t) = eye + t V is sampled at t_n = n * step; a sample counts when its
// texel coordinates lie in the tile and t_n <= far; the hit is the first
// counting sample below the bilinear terrain, f(t_n) = H - b(q) <= 0, refined
// by the zero of the straight line through (t_{n-1}, f_{n-1}) and (t_n, f_n).
//
// The paper starts its view rays from cube-sphere vertices pre-displaced by
// the height field so that few steps remain.  Here a compute kernel has no
// rasteriser; the same purpose -- start where the terrain can be -- is served
// by the tap-bound pyramid (every bilinear tap of every sample in a level-m
// cell is at most that cell's entry): the ray is clipped to the tile and to
// the shell below the highest terrain, then walks the pyramid front to back,
// skips every cell it passes above (with a margin covering FP32 rounding),
// moves forward inside a cell to where the ray can first come down to the
// cell's bound, and tests grid samples only inside level-0 cells.  Because the
// skip is conservative and the samples are the same, the dense mode (every
// grid sample between the clip points) gives bit-identical results.
//
// Frame: the gnomonic tile of the shadow path; the eye is relative to the
// point where the tile's z axis meets the reference surface (the sphere
// centre is at (0, 0, -R)), so every quantity stays small in FP32.
#include "kernels.h"

namespace ss {

namespace {

template <bool SPHERE>
struct VRay {
  float ex, ey, ez;     // eye
  float vx, vy, vz;     // unit direction
  int sgx, sgy;         // motion direction of q along the ray (-1, 0, 1)
  float t_hmin;         // ray length of the lowest point (sphere), or +-inf
  float b;              // (S0 + eye) . V on the sphere: d|P|/dt = (b + t) / |P|
};

// Per-level tables in LDS: the walk's level differs between lanes, and
// indexing the kernel arguments with it would put a dependent memory load in
// front of every bound.
struct VTab {
  int off[SS_MAXLEV], lw[SS_MAXLEV], lh[SS_MAXLEV];
  float ip[SS_MAXLEV];  // 2^-m
};

__device__ __forceinline__ void vtab_fill(const ViewK& K, VTab& lt) {
  const int m = threadIdx.x;
  if (m < SS_MAXLEV) {
    lt.off[m] = K.loff[m];
    lt.lw[m] = K.lw[m];
    lt.lh[m] = K.lh[m];
    lt.ip[m] = K.inv_pow2[m];
  }
}

__device__ __forceinline__ float vbound(const ViewK& K, const VTab& lt, int m, int cx, int cy) {
  const float* base = m == 0 ? K.bnd : K.bmm + lt.off[m];
  return base[__umul24((unsigned)cy, (unsigned)lt.lw[m]) + (unsigned)cx];
}

// Texel coordinates of the ray point at t.
template <bool SPHERE>
__device__ __forceinline__ void vq(const ViewK& K, const VRay<SPHERE>& r, float t, float& qx,
                                   float& qy) {
  const float dx = fmaf(t, r.vx, r.ex), dy = fmaf(t, r.vy, r.ey);
  if (SPHERE) {
    const float dz = fmaf(t, r.vz, r.ez);
    const float w = 1.0f / fmaf(dz, K.invR, 1.0f);
    qx = fmaf(dx * K.invT, w, K.cx0);
    qy = fmaf(dy * K.invT, w, K.cy0);
  } else {
    qx = fmaf(dx, K.invT, K.cx0);
    qy = fmaf(dy, K.invT, K.cy0);
  }
}

// Height of the ray point at t above the reference surface:
// |S0 + D| - R = (2 R dz + |D|^2) / (|S0 + D| + R) with D = eye + t V.
template <bool SPHERE>
__device__ __forceinline__ float vH(const ViewK& K, const VRay<SPHERE>& r, float t) {
  const float dz = fmaf(t, r.vz, r.ez);
  if (!SPHERE) return dz;
  const float dx = fmaf(t, r.vx, r.ex), dy = fmaf(t, r.vy, r.ey);
  const float u = dz * K.invR;
  const float rr = fmaf(dx, dx, dy * dy);
  const float num = fmaf(dz, 2.0f + u, rr * K.invR);
  const float s2 = rr * (K.invR * K.invR);
  const float den = 1.0f + sqrtf(fmaf(1.0f + u, 1.0f + u, s2));
  return num / den;
}

// Bilinear terrain over texel centres, taps clamped to the tile.
__device__ __forceinline__ float vterrain(const ViewK& K, float qx, float qy) {
  const float x = qx - 0.5f, y = qy - 0.5f;
  const float x0 = floorf(x), y0 = floorf(y);
  const float fx = x - x0, fy = y - y0;
  // clamp in float first: q can be far outside for samples off the tile
  const int i0 = (int)fminf(fmaxf(x0, 0.0f), (float)(K.W - 1));
  const int i1 = (int)fminf(fmaxf(x0 + 1.0f, 0.0f), (float)(K.W - 1));
  const int j0 = (int)fminf(fmaxf(y0, 0.0f), (float)(K.H - 1));
  const int j1 = (int)fminf(fmaxf(y0 + 1.0f, 0.0f), (float)(K.H - 1));
  const unsigned W = (unsigned)K.W;
  const float h00 = K.h[__umul24((unsigned)j0, W) + i0], h10 = K.h[__umul24((unsigned)j0, W) + i1];
  const float h01 = K.h[__umul24((unsigned)j1, W) + i0], h11 = K.h[__umul24((unsigned)j1, W) + i1];
  const float a = fmaf(fx, h10 - h00, h00), b = fmaf(fx, h11 - h01, h01);
  return fmaf(fy, b - a, a);
}

template <bool SPHERE>
__device__ __forceinline__ float vf(const ViewK& K, const VRay<SPHERE>& r, float t) {
  float qx, qy;
  vq<SPHERE>(K, r, t, qx, qy);
  return vH<SPHERE>(K, r, t) - vterrain(K, qx, qy);
}

// Ray length where texel coordinate x (axis 0) or y (axis 1) equals g.
template <bool SPHERE>
__device__ __forceinline__ float vcross(const ViewK& K, const VRay<SPHERE>& r, int axis, float g) {
  const float G = (g - (axis == 0 ? K.cx0 : K.cy0)) * K.texel;
  const float e = axis == 0 ? r.ex : r.ey, v = axis == 0 ? r.vx : r.vy;
  if (!SPHERE) return (G - e) / v;
  // R (e + t v) = G (R + ez + t vz)
  return fmaf(G, r.ez * K.invR, G - e) / fmaf(-G * K.invR, r.vz, v);
}

// Ray length where the ray reaches line g moving with sign sg, or +inf when
// it never does: on the sphere the texture path runs toward a limit point,
// and a line beyond it is not reached (the denominator's sign then disagrees
// with the motion).  When it is reached the result is >= the current t up to
// rounding, which the caller clamps.
template <bool SPHERE>
__device__ __forceinline__ float vreach(const ViewK& K, const VRay<SPHERE>& r, int axis, float g,
                                        int sg) {
  const float G = (g - (axis == 0 ? K.cx0 : K.cy0)) * K.texel;
  const float e = axis == 0 ? r.ex : r.ey, v = axis == 0 ? r.vx : r.vy;
  const float den = SPHERE ? fmaf(-G * K.invR, r.vz, v) : v;
  if (!(den * (float)sg > 0.0f)) return INFINITY;
  return SPHERE ? fmaf(G, r.ez * K.invR, G - e) / den : (G - e) / den;
}

// Motion sign of q along an axis; below the threshold the ray's whole path
// moves less than a small fraction of a texel and counts as still.
template <bool SPHERE>
__device__ __forceinline__ int vsign(const ViewK& K, const VRay<SPHERE>& r, int axis) {
  const float e = axis == 0 ? r.ex : r.ey, v = axis == 0 ? r.vx : r.vy;
  const float s = SPHERE ? fmaf(v, r.ez * K.invR, v) - e * r.vz * K.invR : v;
  return s > 1e-6f ? 1 : (s < -1e-6f ? -1 : 0);
}

// Part of the ray (t >= 0) whose texel coordinate on one axis lies in
// [0, lim): [lo, hi), empty when lo >= hi.  tpz bounds the branch where the
// central projection is defined.
template <bool SPHERE>
__device__ __forceinline__ void vclip(const ViewK& K, const VRay<SPHERE>& r, int axis, int sg,
                                      float q0, float lim, float tpz, float& lo, float& hi) {
  lo = 0.0f;
  hi = tpz;
  if (sg == 0) {
    if (!(q0 >= 0.0f && q0 < lim)) hi = -1.0f;
    return;
  }
  const float g_in = sg > 0 ? 0.0f : lim, g_out = sg > 0 ? lim : 0.0f;
  const bool before = sg > 0 ? q0 < 0.0f : q0 >= lim;   // not yet at the entry line
  const bool after = sg > 0 ? q0 >= lim : q0 < 0.0f;    // past the exit line
  if (after) {
    hi = -1.0f;
    return;
  }
  if (before) {
    const float c = vcross<SPHERE>(K, r, axis, g_in);
    if (!(c > 0.0f && c < tpz)) {
      hi = -1.0f;
      return;
    }
    lo = c;
  }
  const float c = vcross<SPHERE>(K, r, axis, g_out);
  if (c > 0.0f && c < tpz) hi = c;
}

struct VHit {
  int n;        // hit sample, -1: none
  int samples;  // f evaluations
  int cells;    // pyramid cells tested
};

__device__ __forceinline__ int vk(const ViewK& K, float t) {
  // t is finite or +inf; the clamp keeps the index representable
  return (int)fminf(ceilf(t * K.inv_step), 2.0e9f);
}

// Dense mode: every grid sample in [t0, t1).
template <bool SPHERE>
__device__ VHit view_dense(const ViewK& K, const VRay<SPHERE>& r, float t0, float t1) {
  VHit h{-1, 0, 0};
  const int n0 = vk(K, t0), n1 = min(vk(K, t1), n0 + K.max_samples);
  for (int n = n0; n < n1; ++n) {
    h.samples++;
    if (vf<SPHERE>(K, r, (float)n * K.step) <= 0.0f) {
      h.n = n;
      break;
    }
  }
  return h;
}

// Hierarchical mode: front-to-back walk over the tap-bound pyramid.
template <bool SPHERE>
__device__ VHit view_hier(const ViewK& K, const VTab& lt, const VRay<SPHERE>& r, float t0,
                          float t1, float eyen) {
  VHit h{-1, 0, 0};
  float t = t0;
  // start three levels below the top (cells of 1/8 of the tile): every ray
  // below the shell would descend through the top levels anyway, and after a
  // skip the walk climbs again where the terrain allows
  int m = max(K.L - 4, 0), cx = 0, cy = 0;
  if (m < K.L - 1) {
    float qx, qy;
    vq<SPHERE>(K, r, t, qx, qy);
    cx = min(max((int)floorf(qx * lt.ip[m]), 0), lt.lw[m] - 1);
    cy = min(max((int)floorf(qy * lt.ip[m]), 0), lt.lh[m] - 1);
  }
  for (int it = 0; it < K.max_iter; ++it) {
    h.cells++;
    // exit of the current cell through its far lines in the motion direction
    const float gx = (float)((r.sgx > 0 ? cx + 1 : cx) << m);
    const float gy = (float)((r.sgy > 0 ? cy + 1 : cy) << m);
    const float tx = r.sgx != 0 ? vreach<SPHERE>(K, r, 0, gx, r.sgx) : INFINITY;
    const float ty = r.sgy != 0 ? vreach<SPHERE>(K, r, 1, gy, r.sgy) : INFINITY;
    const float te = fmaxf(fminf(tx, ty), t);
    const float tb = fminf(te, t1);
    const float tm = fminf(fmaxf(r.t_hmin, t), tb);
    const float Hmin = vH<SPHERE>(K, r, tm);
    const float margin = fmaf(K.m_rel, eyen + tb, K.m_abs);
    const float Bm = vbound(K, lt, m, cx, cy) + margin;
    bool pass = Hmin > Bm;
    if (!pass) {
      // the ray's height is convex in t, so its tangent at t is a lower bound:
      // until the tangent comes down to Bm the ray passes above every tap of
      // the cell, and those samples are skipped (the slope, (b + t) / |P| on
      // the sphere, carries an allowance for its FP32 error of ~1e-7)
      const float Ht = vH<SPHERE>(K, r, t);
      const float slope = SPHERE ? (r.b + t) / (K.R + Ht) : r.vz;
      const float rate = 2e-7f - slope;
      if (Ht > Bm && rate > 0.0f) t = fminf(t + (Ht - Bm) / rate, tb);
    }
    if (!pass && m > 0) {
      // descend into the child that holds q(t) (clamped to this cell)
      float qx, qy;
      vq<SPHERE>(K, r, t, qx, qy);
      --m;
      const int kx = (int)floorf(qx * lt.ip[m]), ky = (int)floorf(qy * lt.ip[m]);
      cx = min(max(kx, 2 * cx), min(2 * cx + 1, lt.lw[m] - 1));
      cy = min(max(ky, 2 * cy), min(2 * cy + 1, lt.lh[m] - 1));
      continue;
    }
    if (!pass) {
      // level 0: the grid samples whose t falls in this cell's part of the ray
      const int n0 = vk(K, t), n1 = min(vk(K, tb), n0 + K.max_samples);
      for (int n = n0; n < n1; ++n) {
        h.samples++;
        if (vf<SPHERE>(K, r, (float)n * K.step) <= 0.0f) {
          h.n = n;
          return h;
        }
      }
    }
    if (te >= t1) return h;
    t = te;
    const bool stx = tx <= ty, sty = ty <= tx;
    if (stx) cx += r.sgx;
    if (sty) cy += r.sgy;
    if (cx < 0 || cy < 0 || cx >= lt.lw[m] || cy >= lt.lh[m]) return h;
    // one level up when the step left the parent cell
    const bool up = m < K.L - 1 && ((stx && ((cx & 1) == (r.sgx > 0 ? 0 : 1))) ||
                                    (sty && ((cy & 1) == (r.sgy > 0 ? 0 : 1))));
    if (up) {
      ++m;
      cx >>= 1;
      cy >>= 1;
    }
  }
  h.cells = -h.cells;  // iteration cap reached (never on valid input)
  return h;
}

template <bool SPHERE, int MODE>
__global__ __launch_bounds__(256) void view_kernel(ViewK K, float* __restrict__ out_t,
                                                   float2* __restrict__ out_xy,
                                                   int2* __restrict__ out_steps) {
  __shared__ VTab lt;
  if (MODE == SS_VIEW_HIER) {
    vtab_fill(K, lt);
    __syncthreads();
  }
  // a wavefront covers an 8 x 8 pixel tile, a workgroup 16 x 16 pixels
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bx = blockIdx.x % K.nbx, by = blockIdx.x / K.nbx;
  const int px = bx * 16 + (wv & 1) * 8 + (lane & 7);
  const int py = by * 16 + (wv >> 1) * 8 + (lane >> 3);
  if (px >= K.img_w || py >= K.img_h) return;
  const float sx = fmaf((float)px + 0.5f, K.inv_w2, -1.0f);
  const float sy = fmaf(-((float)py + 0.5f), K.inv_h2, 1.0f);
  float vx = fmaf(sy, K.ux, fmaf(sx, K.rx, K.fx));
  float vy = fmaf(sy, K.uy, fmaf(sx, K.ry, K.fy));
  float vz = fmaf(sy, K.uz, fmaf(sx, K.rz, K.fz));
  const float n2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
  VHit h{-1, 0, 0};
  VRay<SPHERE> r;
  r.ex = K.ex;
  r.ey = K.ey;
  r.ez = K.ez;
  float t_lo = 0.0f, t_hi = -1.0f;
  if (n2 > 0.0f) {
    const float inv = 1.0f / sqrtf(n2);
    r.vx = vx * inv;
    r.vy = vy * inv;
    r.vz = vz * inv;
    r.sgx = vsign<SPHERE>(K, r, 0);
    r.sgy = vsign<SPHERE>(K, r, 1);
    // the branch where the projection is defined, and the lowest point
    float tpz = INFINITY;
    if (SPHERE) {
      if (r.vz < 0.0f) tpz = (0.5f * K.R + r.ez) / -r.vz;
      r.b = fmaf(K.R, r.vz, fmaf(r.ex, r.vx, fmaf(r.ey, r.vy, r.ez * r.vz)));
      r.t_hmin = -r.b;
    } else {
      r.t_hmin = r.vz < 0.0f ? INFINITY : -INFINITY;
    }
    float q0x, q0y;
    vq<SPHERE>(K, r, 0.0f, q0x, q0y);
    float lx, hx, ly, hy;
    vclip<SPHERE>(K, r, 0, r.sgx, q0x, (float)K.W, tpz, lx, hx);
    vclip<SPHERE>(K, r, 1, r.sgy, q0y, (float)K.H, tpz, ly, hy);
    t_lo = fmaxf(lx, ly);
    t_hi = fminf(fminf(hx, hy), K.far);
    // the shell below the highest terrain (the pyramid's top entry)
    const float hs = (K.L == 1 ? K.bnd : K.bmm + K.loff[K.L - 1])[0];
    if (SPHERE) {
      const float b = fmaf(K.R, r.vz, fmaf(r.ex, r.vx, fmaf(r.ey, r.vy, r.ez * r.vz)));
      const float e2 = fmaf(r.ex, r.ex, fmaf(r.ey, r.ey, r.ez * r.ez));
      const float c0 = fmaf(2.0f * K.R, r.ez - hs, fmaf(-hs, hs, e2));
      const float disc = fmaf(b, b, -c0);
      if (disc < 0.0f) {
        t_hi = -1.0f;
      } else {
        const float sq = sqrtf(disc);
        float s1, s2;
        if (b < 0.0f) {
          s2 = sq - b;
          s1 = c0 / s2;
        } else {
          s1 = -b - sq;
          s2 = s1 != 0.0f ? c0 / s1 : 0.0f;
        }
        t_lo = fmaxf(t_lo, s1);
        t_hi = fminf(t_hi, s2);
      }
    } else {
      if (r.vz < 0.0f) {
        t_lo = fmaxf(t_lo, (r.ez - hs) / -r.vz);
      } else if (r.vz > 0.0f) {
        t_hi = fminf(t_hi, (hs - r.ez) / r.vz);
      } else if (r.ez > hs) {
        t_hi = -1.0f;
      }
    }
    t_lo = fmaxf(t_lo, 0.0f);
    if (t_lo < t_hi) {
      const float eyen = sqrtf(fmaf(r.ex, r.ex, fmaf(r.ey, r.ey, r.ez * r.ez)));
      h = MODE == SS_VIEW_DENSE ? view_dense<SPHERE>(K, r, t_lo, t_hi)
                                : view_hier<SPHERE>(K, lt, r, t_lo, t_hi, eyen);
    }
  }
  const unsigned k = __umul24((unsigned)py, (unsigned)K.img_w) + (unsigned)px;
  if (h.n >= 0) {
    float th = 0.0f;
    if (h.n > 0) {
      const float tp = (float)(h.n - 1) * K.step;
      const float fp = vf<SPHERE>(K, r, tp);
      const float fn = vf<SPHERE>(K, r, (float)h.n * K.step);
      const float w = fp > 0.0f ? fp / (fp - fn) : 0.0f;
      th = fmaf(w, K.step, tp);
    }
    float qx, qy;
    vq<SPHERE>(K, r, th, qx, qy);
    out_t[k] = th;
    out_xy[k] = make_float2(qx, qy);
  } else {
    out_t[k] = INFINITY;
    out_xy[k] = make_float2(NAN, NAN);
  }
  if (out_steps) out_steps[k] = make_int2(h.samples, h.cells);
}

template <bool SPHERE>
void view_launch(const ViewK& K, int mode, float* t, float* xy, int* steps, hipStream_t s) {
  const dim3 grid((unsigned)(K.nbx * K.nby)), block(256);
  float2* q = reinterpret_cast<float2*>(xy);
  int2* st = reinterpret_cast<int2*>(steps);
  if (mode == SS_VIEW_DENSE)
    hipLaunchKernelGGL((view_kernel<SPHERE, SS_VIEW_DENSE>), grid, block, 0, s, K, t, q, st);
  else
    hipLaunchKernelGGL((view_kernel<SPHERE, SS_VIEW_HIER>), grid, block, 0, s, K, t, q, st);
}

}  // namespace

hipError_t launch_view(const ViewK& K, bool sphere, int mode, float* t, float* xy, int* steps,
                       hipStream_t stream) {
  if (K.img_w <= 0 || K.img_h <= 0) return hipSuccess;
  if (sphere)
    view_launch<true>(K, mode, t, xy, steps, stream);
  else
    view_launch<false>(K, mode, t, xy, steps, stream);
  return hipGetLastError();
}

}  // namespace ss
