// Per-ray device code: geometry, the descent through the maximum mipmap,
// final samples, clearance angle and disc occlusion.  Used by the forward,
// adjoint and persistent kernels, so every caller makes the same decisions.
//
// Everything is FP32 and relative to the ray origin p (texel centre):
//   * texture-space offsets  d(u) = K u  with  u = t / (1 + c t)  (central
//     projection maps the straight ray to a straight texture line);
//   * tip height above p     dH(t) = t (2 s + x) / (sqrt(1 + x (2 s + x)) + 1),
//     x = t / rho, the cancellation-free form of |p + t L| - |p|;
//   * bilinear heights minus h_p.
// Absolute coordinates would lose the metre-scale detail near the origin
// (an FP32 ulp at the Moon's radius is 0.125 m).
#pragma once

#include "common.h"

#define SS_INF __builtin_inff()

__device__ __forceinline__ float ss_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float ss_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <bool SPHERE>
struct Ray {
  int i, j;
  float hp;          // origin height
  float Kx, Ky;      // texture-space velocity per unit u (texels)
  float invKx, invKy;
  float c;           // projective constant: u = t / (1 + c t)
  float sp, cp;      // n.L and |n x L| at the origin (radial normal n)
  float invrho;      // 1 / |p|
  float uexit;       // u where the path leaves the tile
  float uhmin;       // u where the tip height is smallest (-inf: rising from the start)
  int sx, sy;        // direction of travel along columns / rows
};

template <bool SPHERE>
__device__ __forceinline__ void ray_init(const TileK& T, int i, int j, float hp, Ray<SPHERE>& r) {
  r.i = i;
  r.j = j;
  r.hp = hp;
  const float X = ((float)i + 0.5f - 0.5f * (float)T.W) * T.texel;
  const float Y = ((float)j + 0.5f - 0.5f * (float)T.H) * T.texel;
  if (SPHERE) {
    // n = (a, b, 1)/g with a = X/R, b = Y/R, g = |(a, b, 1)|; rho = R (1 + h_p/R)
    const float a = X * T.invR, b = Y * T.invR;
    const float g = sqrtf(1.0f + a * a + b * b);
    const float ig = 1.0f / g;
    const float r1 = 1.0f + hp * T.invR;
    r.sp = (a * T.Lx + b * T.Ly + T.Lz) * ig;
    const float cx = b * T.Lz - T.Ly, cy = T.Lx - a * T.Lz, cz = a * T.Ly - b * T.Lx;
    r.cp = sqrtf(cx * cx + cy * cy + cz * cz) * ig;
    const float sc = g / (r1 * T.texel);
    r.Kx = (T.Lx - a * T.Lz) * sc;
    r.Ky = (T.Ly - b * T.Lz) * sc;
    r.c = T.Lz * g / r1 * T.invR;
    r.invrho = T.invR / r1;
    // |p + t L| is smallest at t = -rho s (ahead of p only when the sun is
    // below the local horizon)
    if (r.sp < 0.0f) {
      const float th = -r.sp / r.invrho;
      r.uhmin = th / (1.0f + r.c * th);
    } else {
      r.uhmin = -SS_INF;
    }
  } else {
    r.sp = T.Lz;
    r.cp = sqrtf(T.Lx * T.Lx + T.Ly * T.Ly);
    r.Kx = T.Lx / T.texel;
    r.Ky = T.Ly / T.texel;
    r.c = 0.0f;
    r.invrho = 0.0f;
    r.uhmin = T.Lz >= 0.0f ? -SS_INF : SS_INF;
  }
  r.sx = r.Kx > 0.0f ? 1 : (r.Kx < 0.0f ? -1 : 0);
  r.sy = r.Ky > 0.0f ? 1 : (r.Ky < 0.0f ? -1 : 0);
  r.invKx = r.sx ? 1.0f / r.Kx : 0.0f;
  r.invKy = r.sy ? 1.0f / r.Ky : 0.0f;
  // leaving the tile: first boundary in the direction of travel
  float ux = SS_INF, uy = SS_INF;
  if (r.sx > 0) ux = ((float)(T.W - i) - 0.5f) / r.Kx;
  if (r.sx < 0) ux = ((float)(-i) - 0.5f) / r.Kx;
  if (r.sy > 0) uy = ((float)(T.H - j) - 0.5f) / r.Ky;
  if (r.sy < 0) uy = ((float)(-j) - 0.5f) / r.Ky;
  r.uexit = fminf(ux, uy);
}

template <bool SPHERE>
__device__ __forceinline__ float u_to_t(const Ray<SPHERE>& r, float u) {
  return SPHERE ? u * ss_rcp(1.0f - r.c * u) : u;
}

template <bool SPHERE>
__device__ __forceinline__ float t_to_u(const Ray<SPHERE>& r, float t) {
  return SPHERE ? t * ss_rcp(1.0f + r.c * t) : t;
}

// Tip height above the origin height: |p + t L| - |p| (sphere), t L_z (plane).
template <bool SPHERE>
__device__ __forceinline__ float tip_rise(const Ray<SPHERE>& r, const TileK& T, float t) {
  if (SPHERE) {
    const float x = t * r.invrho;
    const float q = 2.0f * r.sp + x;
    return t * q * ss_rcp(ss_sqrt(1.0f + x * q) + 1.0f);
  }
  return t * T.Lz;
}

__device__ __forceinline__ const float* level_ptr(const TileK& T, int m) {
  return m == 0 ? T.h : T.mm + T.loff[m];
}

// Keeps an index inside [0, n): a negative index wraps to a huge unsigned
// value and lands on n - 1.  Only rounding at a tile edge can produce an index
// outside the level, so this is a memory-safety guard, not a behaviour.
__device__ __forceinline__ unsigned inside(int v, int n) { return min((unsigned)v, (unsigned)(n - 1)); }

__device__ __forceinline__ float mip_at(const TileK& T, int m, int cx, int cy) {
  const unsigned w = (unsigned)T.lw[m];
  return level_ptr(T, m)[inside(cy, T.lh[m]) * w + inside(cx, T.lw[m])];
}

// Lower bound of the clearance over the part [u0, u1] of the ray inside a
// level-m texel: smallest tip height there minus the texel's maximum height
// (Sec. 3.2, Eq. 4 with the maximum mipmap), relative to h_p.
template <bool SPHERE>
__device__ __forceinline__ float lower_bound(const Ray<SPHERE>& r, const TileK& T, int m, int cx,
                                             int cy, float u0, float u1) {
  const float uc = fminf(fmaxf(r.uhmin, u0), u1);
  const float t = u_to_t(r, uc);
  return tip_rise(r, T, t) - (mip_at(T, m, cx, cy) - r.hp);
}

// The same bound when the tip rise at the texel's entry is already known (the
// tip height rises from the start, so the entry is where it is smallest).
__device__ __forceinline__ float lower_bound_at(const TileK& T, float rise, int m, int cx, int cy,
                                                float hp) {
  return rise - (mip_at(T, m, cx, cy) - hp);
}

// Bilinear sample of the terrain below the ray tip at ray length t (u = u(t)):
// clearance height and the tap layout (for the adjoint).
struct Sample {
  float dh;
  float fx, fy;
  int x0, y0;   // unclamped lower-left tap (texel indices)
};

template <bool SPHERE>
__device__ __forceinline__ Sample sample_at(const Ray<SPHERE>& r, const TileK& T, float t, float u) {
  Sample s;
  const float dx = r.Kx * u, dy = r.Ky * u;
  const float flx = floorf(dx), fly = floorf(dy);
  s.fx = dx - flx;
  s.fy = dy - fly;
  s.x0 = r.i + (int)flx;
  s.y0 = r.j + (int)fly;
  // clamp to the edge (the tap index is -1 only left of the first centre)
  const unsigned x0 = (unsigned)min(max(s.x0, 0), T.W - 1), x1 = inside(s.x0 + 1, T.W);
  const unsigned y0 = (unsigned)min(max(s.y0, 0), T.H - 1), y1 = inside(s.y0 + 1, T.H);
  const float* h = T.h;
  const unsigned W = (unsigned)T.W;
  const float h00 = h[y0 * W + x0] - r.hp, h10 = h[y0 * W + x1] - r.hp;
  const float h01 = h[y1 * W + x0] - r.hp, h11 = h[y1 * W + x1] - r.hp;
  const float hb = (1.0f - s.fy) * ((1.0f - s.fx) * h00 + s.fx * h10) +
                   s.fy * ((1.0f - s.fx) * h01 + s.fx * h11);
  s.dh = tip_rise(r, T, t) - hb;
  return s;
}

// Visible part of the sun disc above a chord at d disc radii below its centre
// (Sec. 3.4, Eq. 6 first term; circular segment).
__device__ __forceinline__ float disc_fraction(float alpha, const TileK& T) {
  if (!(alpha < SS_INF)) return 1.0f;
  const float d = fminf(fmaxf(alpha * T.inv_rL, -1.0f), 1.0f);
  return (3.14159265358979f - acosf(d) + d * sqrtf(fmaxf(0.0f, 1.0f - d * d))) *
         0.318309886183791f;
}

// Clearance of a sample: the signed angle at p between L and the terrain point
// below the ray tip (positive: below the ray), atan2(num, den) with the terms
// below; to first order (dh / t) |n x L| (Sec. 3.4, Eq. 5).  Runs are compared by the
// tangent key num/den (den > 0; +inf / -inf when the angle is beyond +-pi/2),
// which orders like the angle, so atan runs once per ray.
struct SegOut {
  float key;
  float t;        // ray length of the deciding sample
  float u;
  int valid;
};

template <bool SPHERE>
__device__ __forceinline__ void clearance_terms(const Ray<SPHERE>& r, float t, float dh, float& num,
                                                float& den) {
  if (SPHERE) {
    const float x = t * r.invrho;
    const float w = ss_sqrt(1.0f + x * (2.0f * r.sp + x));
    num = dh * r.cp;
    den = t * w - dh * (r.sp + x);
  } else {
    num = dh * r.cp;
    den = t - dh * r.sp;
  }
}

__device__ __forceinline__ float tangent_key(float num, float den) {
  return den > 0.0f ? num * ss_rcp(den) : (num >= 0.0f ? SS_INF : -SS_INF);
}

// One concatenated run (Sec. 3.3): descent from level m0 = T.m0[j] over the
// texels the ray crosses (Sec. 3.2, Fig. 3b), strict argmin from the far end
// (kept here as '<=' scanning from the near end), then three samples half a
// texel apart around the chosen base texel (Alg. 1, final level).
template <bool SPHERE>
__device__ __forceinline__ void descend_run(const TileK& T, const Ray<SPHERE>& r, int jseg, SegOut& out,
                                            unsigned& n_lb, unsigned& n_smp) {
  out.valid = 0;
  const float ta = T.tau[jseg], tb = T.tau[jseg + 1];
  const float ua = t_to_u(r, ta);
  const float ub = fminf(t_to_u(r, tb), r.uexit);
  const int m = T.m0[jseg];
  const int S = 1 << m;
  // top level: walk the level-m texels crossed for u in [ua, ub]
  int cx = (r.i >> m) + (int)floorf(ldexpf((float)(r.i & (S - 1)) + 0.5f + r.Kx * ua, -m));
  int cy = (r.j >> m) + (int)floorf(ldexpf((float)(r.j & (S - 1)) + 0.5f + r.Ky * ua, -m));
  float best = SS_INF, bu0 = ua, bu1 = ua, brise = 0.0f;
  int bx = cx, by = cy, have = 0;
  float u0 = ua;
  const bool rising = r.uhmin <= ua;  // tip height grows over the whole run
  for (int it = 0; it < 8; ++it) {
    const float ux = r.sx > 0 ? ((float)(((cx + 1) << m) - r.i) - 0.5f) * r.invKx
                   : (r.sx < 0 ? ((float)((cx << m) - r.i) - 0.5f) * r.invKx : SS_INF);
    const float uy = r.sy > 0 ? ((float)(((cy + 1) << m) - r.j) - 0.5f) * r.invKy
                   : (r.sy < 0 ? ((float)((cy << m) - r.j) - 0.5f) * r.invKy : SS_INF);
    const float u1 = fminf(fminf(ux, uy), ub);
    // a piece in a texel outside the level is a rounding sliver at the tile edge
    const bool in_level = (unsigned)cx < (unsigned)T.lw[m] && (unsigned)cy < (unsigned)T.lh[m];
    if (u1 > u0 && in_level) {
      const float uc = fminf(fmaxf(r.uhmin, u0), u1);
      const float rise = tip_rise(r, T, u_to_t(r, uc));
      const float lb = lower_bound_at(T, rise, m, cx, cy, r.hp);
      n_lb++;
      if (lb <= best) {
        best = lb;
        bx = cx;
        by = cy;
        bu0 = u0;
        bu1 = u1;
        brise = rise;
        have = 1;
      }
    }
    if (u1 > u0) u0 = u1;
    if (!(u1 < ub)) break;
    const bool stepx = ux <= uy, stepy = uy <= ux;
    if (stepx) cx += r.sx;
    if (stepy) cy += r.sy;
  }
  if (!have) return;
  // descend: the children of the chosen texel crossed by the ray, split at the
  // parent's two mid-lines (at most three pieces)
  for (int lv = m; lv > 0; --lv) {
    const int half = 1 << (lv - 1);
    const float mxr = (float)((2 * bx + 1) * half - r.i) - 0.5f;
    const float myr = (float)((2 * by + 1) * half - r.j) - 0.5f;
    const float umx = r.sx ? mxr * r.invKx : SS_INF;
    const float umy = r.sy ? myr * r.invKy : SS_INF;
    const float c1 = fminf(fmaxf(fminf(umx, umy), bu0), bu1);
    const float c2 = fminf(fmaxf(fmaxf(umx, umy), bu0), bu1);
    const float pa[3] = {bu0, c1, c2};
    const float pb[3] = {c1, c2, bu1};
    // tip rise at each piece's entry: the first piece enters where the parent
    // did (already known); identical to evaluating it again
    float rise[3];
    if (rising) {
      rise[0] = brise;
      rise[1] = tip_rise(r, T, u_to_t(r, c1));
      rise[2] = tip_rise(r, T, u_to_t(r, c2));
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        rise[k] = tip_rise(r, T, u_to_t(r, fminf(fmaxf(r.uhmin, pa[k]), pb[k])));
    }
    float nbest = SS_INF, n0 = bu0, n1 = bu1, nrise = brise;
    int nx = 2 * bx, ny = 2 * by, nh = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float u = pa[k], v = pb[k];
      const float um = 0.5f * (u + v);
      const int ccx = 2 * bx + ((r.Kx * um >= mxr) ? 1 : 0);
      const int ccy = 2 * by + ((r.Ky * um >= myr) ? 1 : 0);
      const float lb = lower_bound_at(T, rise[k], lv - 1, ccx, ccy, r.hp);
      // children beyond a ragged edge are absent
      const bool ok = v > u && ccx < T.lw[lv - 1] && ccy < T.lh[lv - 1];
      n_lb += ok ? 1u : 0u;
      if (ok && lb <= nbest) {
        nbest = lb;
        nx = ccx;
        ny = ccy;
        n0 = u;
        n1 = v;
        nrise = rise[k];
        nh = 1;
      }
    }
    if (!nh) return;
    bx = nx;
    by = ny;
    bu0 = n0;
    bu1 = n1;
    brise = nrise;
  }
  // final samples on the half-texel grid t_n = (n + 1) delta/2 around the
  // middle of the base texel's stretch of ray
  const float tin = u_to_t(r, bu0), tout = u_to_t(r, bu1);
  const float tmid = 0.5f * (tin + tout);
  const int nc = (int)floorf((tmid - T.half_delta) * T.two_over_delta + 0.5f);
  float bdh = SS_INF, bt = 0.0f, bu = 0.0f;
  int found = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int n = nc - 1 + k;
    const float t = (float)(n + 1) * T.half_delta;
    const float u = t_to_u(r, t);
    if (n >= 0 && u < r.uexit) {
      const Sample s = sample_at(r, T, t, u);
      n_smp++;
      if (s.dh <= bdh) {
        bdh = s.dh;
        bt = t;
        bu = u;
        found = 1;
      }
    }
  }
  if (!found) return;
  float num, den;
  clearance_terms(r, bt, bdh, num, den);
  out.key = tangent_key(num, den);
  out.t = bt;
  out.u = bu;
  out.valid = 1;
}

// True when every sample at ray length >= t clears the angle whose tangent is
// need_tan (an angle in (-pi/2, pi/2)), given that no terrain rises above
// `top` (relative to h_p, >= 0): the clearance of the point at that height
// below the tip grows with t on the plane and on the sphere.  Used for the
// result-invariant early exits.
template <bool SPHERE>
__device__ __forceinline__ bool clears(const Ray<SPHERE>& r, const TileK& T, float t, float top,
                                       float need_tan) {
  const float d = tip_rise(r, T, t) - top;
  if (!(d > 0.0f)) return false;
  float num, den;
  clearance_terms(r, t, d, num, den);
  return den <= 0.0f || num >= need_tan * den;  // den <= 0: at least pi/2
}

// tan(min(alpha, r_L) + margin) for the tangent key of alpha (tan addition).
__device__ __forceinline__ float need_tangent(const TileK& T, float key) {
  const float k = fmaxf(fminf(key, T.tan_rL), -1e30f);
  return (k + T.tan_margin) * ss_rcp(1.0f - k * T.tan_margin);
}

// Highest terrain (relative to h_p, at least 0) that any bilinear tap of run
// j's final samples can touch: the samples lie on the ray for t in
// [tlo, tau_{j+1} + 3 delta/4] inside the tile, and a sample at texture point q
// reads taps within [q - 3/2, q + 1/2] per axis.  That box spans at most two
// texels per axis of level max(m0 + 1, 3), whose maxima bound it.
template <bool SPHERE>
__device__ __forceinline__ float run_top(const TileK& T, const Ray<SPHERE>& r, int j, float tlo) {
  const int mb = max(T.m0[j] + 1, 3);
  if (mb >= T.L) return fmaxf(mip_at(T, T.L - 1, 0, 0), r.hp) - r.hp;
  const float ulo = t_to_u(r, tlo);
  const float uhi = fminf(t_to_u(r, T.tau[j + 1] + 1.5f * T.half_delta), r.uexit);
  const float xa = r.Kx * ulo, xb = r.Kx * uhi, ya = r.Ky * ulo, yb = r.Ky * uhi;
  // FP32 slack on the offsets (relative ~1e-6) plus a hundredth of a texel
  const float sx = 0.01f + 1e-5f * fmaxf(fabsf(xa), fabsf(xb));
  const float sy = 0.01f + 1e-5f * fmaxf(fabsf(ya), fabsf(yb));
  const float x0 = (float)r.i + 0.5f + fminf(xa, xb) - 1.5f - sx;
  const float x1 = (float)r.i + 0.5f + fmaxf(xa, xb) + 0.5f + sx;
  const float y0 = (float)r.j + 0.5f + fminf(ya, yb) - 1.5f - sy;
  const float y1 = (float)r.j + 0.5f + fmaxf(ya, yb) + 0.5f + sy;
  const int ix0 = min(max((int)floorf(x0), 0), T.W - 1) >> mb;
  const int ix1 = min(max((int)floorf(x1), 0), T.W - 1) >> mb;
  const int iy0 = min(max((int)floorf(y0), 0), T.H - 1) >> mb;
  const int iy1 = min(max((int)floorf(y1), 0), T.H - 1) >> mb;
  if (ix1 > ix0 + 1 || iy1 > iy0 + 1) return fmaxf(mip_at(T, T.L - 1, 0, 0), r.hp) - r.hp;
  const float m = fmaxf(fmaxf(mip_at(T, mb, ix0, iy0), mip_at(T, mb, ix1, iy0)),
                        fmaxf(mip_at(T, mb, ix0, iy1), mip_at(T, mb, ix1, iy1)));
  return fmaxf(m, r.hp) - r.hp;
}

struct RayResult {
  float alpha;
  float t, u;
  int valid;
};

__device__ __forceinline__ float angle_of(float key) {
  return key == SS_INF ? SS_INF : (key == -SS_INF ? -SS_INF : atanf(key));
}

// Smallest clearance over the concatenated runs (Sec. 3.3).
template <bool SPHERE>
__device__ __forceinline__ RayResult shadow_dp(const TileK& T, const Ray<SPHERE>& r, float top,
                                               unsigned& n_lb, unsigned& n_smp) {
  RayResult res;
  res.t = 0.0f;
  res.u = 0.0f;
  res.valid = 0;
  float best = SS_INF;                    // tangent key of the smallest clearance so far
  float need = need_tangent(T, SS_INF);   // tan(min(alpha, r_L) + margin)
  for (int j = 0; j < T.nseg; ++j) {
    const float ta = T.tau[j];
    if (!(t_to_u(r, ta) < r.uexit)) break;  // the run starts outside the tile
    if (T.prune) {
      // every final sample of run j lies at t >= tau_j - 3 delta/4
      const float tlo = fmaxf(T.half_delta, ta - 1.5f * T.half_delta);
      if (clears(r, T, tlo, top, need)) break;                     // nothing ahead is high enough
      if (clears(r, T, tlo, run_top(T, r, j, tlo), need)) continue;  // nor in this run
    }
    SegOut so;
    descend_run(T, r, j, so, n_lb, n_smp);
    if (so.valid && so.key < best) {
      best = so.key;
      res.t = so.t;
      res.u = so.u;
      res.valid = 1;
      need = need_tangent(T, best);
    }
    if (T.prune && best <= -T.tan_rL) break;  // umbra: nothing can change s = 0
  }
  res.alpha = angle_of(best);
  return res;
}

// Uniform stepping (Sec. 2, Fig. 1b): every step, smallest clearance, kept as
// a tangent key; atan is taken once.
template <bool SPHERE>
__device__ __forceinline__ float shadow_uniform(const TileK& T, const Ray<SPHERE>& r, float top,
                                                unsigned& n_smp) {
  float best = SS_INF;
  float t = T.half_delta;
  for (int k = 0; k < (1 << 22); ++k, t = T.half_delta + (float)k * T.ustep) {
    if (t > T.ucap) break;
    const float u = t_to_u(r, t);
    if (!(u < r.uexit)) break;
    if (T.prune && (k & 15) == 0) {
      if (best <= -T.tan_rL) break;
      if (clears(r, T, t, top, need_tangent(T, best))) break;
    }
    const Sample s = sample_at(r, T, t, u);
    n_smp++;
    float num, den;
    clearance_terms(r, t, s.dh, num, den);
    best = fminf(best, tangent_key(num, den));
  }
  return angle_of(best);
}
