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

// Workgroup ids are dealt round-robin over the 8 XCDs.  xcd_remap gives each
// XCD one contiguous run of [0, nb) (the first nb % 8 XCDs one id more);
// xcd_remap_grouped does so inside each group of grp ids (grp a multiple of 8,
// so an id keeps its XCD).  Both are bijections of [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
  return x * per + min(x, rem) + k;
}

__device__ __forceinline__ int xcd_remap_grouped(int b, int nb, int grp) {
  const int lo = (b / grp) * grp;
  return lo + xcd_remap(b - lo, min(grp, nb - lo));
}

__device__ __forceinline__ float ss_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float ss_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

template <bool SPHERE>
struct Ray {
  int i, j;          // texel holding the origin
  float ox, oy;      // origin minus that texel's centre, in texels (-0 at centres)
  float hp;          // reference height: relative heights are taken from it
  float dz;          // origin height above hp (-0 at centres, whose height is hp)
  float Kx, Ky;      // texture-space velocity per unit u (texels)
  float invKx, invKy;
  float c;           // projective constant: u = t / (1 + c t)
  float sp, cp;      // n.L and |n x L| at the origin (radial normal n)
  float sp2;         // 2 sp
  float invrho;      // 1 / |p|
  float uexit;       // u where the path leaves the tile
  float uhmin;       // u where the tip height is smallest (-inf: rising from the start)
  int sx, sy;        // direction of travel along columns / rows
};

// Ray from the surface point at texel (i, j)'s centre plus (ox, oy) texels,
// at height hp + dz.  Positions are taken relative to the texel centre and
// shifted by (ox, oy); heights relative to hp, a stored height, with the
// origin dz above it.  At centres ox = oy = dz = -0, which every sum below
// drops exactly, so those rays compute as if the terms were absent.
template <bool SPHERE>
__device__ __forceinline__ void ray_init(const TileK& T, int i, int j, float hp, Ray<SPHERE>& r,
                                         float ox = -0.0f, float oy = -0.0f, float dz = -0.0f) {
  r.i = i;
  r.j = j;
  r.ox = ox;
  r.oy = oy;
  r.hp = hp;
  r.dz = dz;
  const float X = ((float)i + 0.5f + ox - 0.5f * (float)T.W) * T.texel;
  const float Y = ((float)j + 0.5f + oy - 0.5f * (float)T.H) * T.texel;
  if (SPHERE) {
    // n = (a, b, 1)/g with a = X/R, b = Y/R, g = |(a, b, 1)|; rho = R (1 + h_p/R)
    const float a = X * T.invR, b = Y * T.invR;
    const float g = sqrtf(1.0f + a * a + b * b);
    const float ig = 1.0f / g;
    const float r1 = 1.0f + (hp + dz) * T.invR;
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
  r.sp2 = 2.0f * r.sp;
  r.sx = r.Kx > 0.0f ? 1 : (r.Kx < 0.0f ? -1 : 0);
  r.sy = r.Ky > 0.0f ? 1 : (r.Ky < 0.0f ? -1 : 0);
  // +inf on an axis the path never moves along: every crossing time on it is
  // then +-inf (the numerators are half-integers, never 0)
  r.invKx = r.sx ? 1.0f / r.Kx : SS_INF;
  r.invKy = r.sy ? 1.0f / r.Ky : SS_INF;
  // leaving the tile: first boundary in the direction of travel
  float ux = SS_INF, uy = SS_INF;
  if (r.sx > 0) ux = ((float)(T.W - i) - 0.5f - ox) / r.Kx;
  if (r.sx < 0) ux = ((float)(-i) - 0.5f - ox) / r.Kx;
  if (r.sy > 0) uy = ((float)(T.H - j) - 0.5f - oy) / r.Ky;
  if (r.sy < 0) uy = ((float)(-j) - 0.5f - oy) / r.Ky;
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

// Tip height above the reference height hp: the rise above the origin,
// |p + t L| - |p| (sphere) or t L_z (plane), plus the origin's dz.
template <bool SPHERE>
__device__ __forceinline__ float tip_rise(const Ray<SPHERE>& r, const TileK& T, float t) {
  if (SPHERE) {
    const float x = t * r.invrho;
    const float q = 2.0f * r.sp + x;
    return t * q * ss_rcp(ss_sqrt(1.0f + x * q) + 1.0f) + r.dz;
  }
  return t * T.Lz + r.dz;
}

// The same tip height at the texture parameter u (t = u / A, A = 1 - c u):
// |p + t L| - |p| = u P / ((S + A) A) with P = 2 s A + u/rho and
// S = sqrt(A^2 + (u/rho) P), still free of cancellation; one reciprocal
// fewer than converting u to t first.
template <bool SPHERE>
__device__ __forceinline__ float tip_rise_u(const Ray<SPHERE>& r, const TileK& T, float u) {
  if (SPHERE) {
    const float A = fmaf(-r.c, u, 1.0f);
    const float v = u * r.invrho;
    const float P = fmaf(r.sp2, A, v);
    const float S = ss_sqrt(fmaf(A, A, v * P));
    return u * P * ss_rcp((S + A) * A) + r.dz;
  }
  return u * T.Lz + r.dz;
}

__device__ __forceinline__ const float* level_ptr(const TileK& T, int m) {
  return m == 0 ? T.h : T.mm + T.loff[m];
}

// Keeps an index inside [0, n): a negative index wraps to a huge unsigned
// value and lands on n - 1.  Only rounding at a tile edge can produce an index
// outside the level, so this is a memory-safety guard, not a behaviour.
__device__ __forceinline__ unsigned inside(int v, int n) { return min((unsigned)v, (unsigned)(n - 1)); }

// Row-major index y w + x.  Rows and widths stay below 2^24, so the full-rate
// 24-bit multiply gives the exact product (the 32-bit one issues at quarter
// rate).
__device__ __forceinline__ unsigned idx2(unsigned y, unsigned w, unsigned x) {
  return __umul24(y, w) + x;
}

__device__ __forceinline__ float mip_at(const TileK& T, int m, int cx, int cy) {
  const unsigned w = (unsigned)T.lw[m];
  return level_ptr(T, m)[idx2(inside(cy, T.lh[m]), w, inside(cx, T.lw[m]))];
}

// One mip level as a buffer resource: 32-bit offsets, and an offset past the
// end reads 0 instead of faulting (the hardware range check), so gathers for
// candidates that are then discarded need no clamping.
struct Level {
  __amdgpu_buffer_rsrc_t rs;
  int w;
};

__device__ __forceinline__ Level level_of(const TileK& T, int m) {
  Level L;
  L.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(level_ptr(T, m)), 0,
                                           T.lw[m] * T.lh[m] * 4, 0x00020000);
  L.w = T.lw[m];
  return L;
}

// (A texel outside the level may give any offset; the range check makes the
// load return 0 or an in-range value, and such candidates are discarded.)
__device__ __forceinline__ float level_at(const Level& L, int cx, int cy) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                       L.rs, (int)(idx2((unsigned)cy, (unsigned)L.w, (unsigned)cx) * 4u), 0, 0));
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
  const float dx = fmaf(r.Kx, u, r.ox), dy = fmaf(r.Ky, u, r.oy);
  const float flx = floorf(dx), fly = floorf(dy);
  s.fx = dx - flx;
  s.fy = dy - fly;
  s.x0 = r.i + (int)flx;
  s.y0 = r.j + (int)fly;
  // clamp to the edge (the tap index is -1 only left of the first centre)
  const unsigned x0 = (unsigned)min(max(s.x0, 0), T.W - 1), x1 = inside(s.x0 + 1, T.W);
  const unsigned y0 = (unsigned)min(max(s.y0, 0), T.H - 1), y1 = inside(s.y0 + 1, T.H);
  const Level L0 = level_of(T, 0);
  const float h00 = level_at(L0, x0, y0) - r.hp, h10 = level_at(L0, x1, y0) - r.hp;
  const float h01 = level_at(L0, x0, y1) - r.hp, h11 = level_at(L0, x1, y1) - r.hp;
  const float hb = (1.0f - s.fy) * ((1.0f - s.fx) * h00 + s.fx * h10) +
                   s.fy * ((1.0f - s.fx) * h01 + s.fx * h11);
  s.dh = tip_rise(r, T, t) - hb;
  return s;
}

// Height of the bilinear terrain at continuous texel coordinates (qx, qy)
// above the reference height ref (texel i covers [i, i+1); taps clamp to the
// edge, as for the samples).  Differences of nearby heights are exact in
// FP32, so the result carries no rounding of the absolute height.
__device__ __forceinline__ float terrain_above(const TileK& T, float qx, float qy, float ref) {
  const float x = qx - 0.5f, y = qy - 0.5f;
  const float flx = floorf(x), fly = floorf(y);
  const float fx = x - flx, fy = y - fly;
  const int x0 = (int)flx, y0 = (int)fly;
  const unsigned xa = (unsigned)min(max(x0, 0), T.W - 1), xb = (unsigned)min(max(x0 + 1, 0), T.W - 1);
  const unsigned ya = (unsigned)min(max(y0, 0), T.H - 1), yb = (unsigned)min(max(y0 + 1, 0), T.H - 1);
  const unsigned W = (unsigned)T.W;
  const float h00 = T.h[idx2(ya, W, xa)] - ref, h10 = T.h[idx2(ya, W, xb)] - ref;
  const float h01 = T.h[idx2(yb, W, xa)] - ref, h11 = T.h[idx2(yb, W, xb)] - ref;
  return (1.0f - fy) * ((1.0f - fx) * h00 + fx * h10) + fy * ((1.0f - fx) * h01 + fx * h11);
}

// Visible part of the sun disc above a chord at d disc radii below its centre
// (Sec. 3.4, Eq. 6 first term; circular segment).  s is exactly 0 or 1 when
// |d| >= 1 (the disc wholly below or above the clearance, zero derivative) and
// strictly inside (0, 1) otherwise, so the adjoint can tell the rays it may
// skip from the forward's output alone.
__device__ __forceinline__ float disc_fraction(float alpha, const TileK& T) {
  if (!(alpha < SS_INF)) return 1.0f;
  const float dd = alpha * T.inv_rL;
  if (dd <= -1.0f) return 0.0f;
  if (dd >= 1.0f) return 1.0f;
  const float v = (3.14159265358979f - acosf(dd) + dd * sqrtf(fmaxf(0.0f, 1.0f - dd * dd))) *
                  0.318309886183791f;
  return fminf(fmaxf(v, 1.17549435e-38f), 0.99999994f);
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
  int n;          // its index on the half-texel grid
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
  const bool rising = r.uhmin <= ua;  // tip height grows over the whole run
  // the next grid line ahead of the current texel on each axis (+1 when the
  // path moves forward or not at all)
  const int ex = r.Kx >= 0.0f ? 1 : 0, ey = r.Ky >= 0.0f ? 1 : 0;
  // top level: walk the level-m texels crossed for u in [ua, ub]
  int cx = (r.i >> m) + (int)floorf(ldexpf((float)(r.i & (S - 1)) + 0.5f + r.ox + r.Kx * ua, -m));
  int cy = (r.j >> m) + (int)floorf(ldexpf((float)(r.j & (S - 1)) + 0.5f + r.oy + r.Ky * ua, -m));
  // those grid lines relative to the origin texel centre, in texels; they
  // are half-integers, exact in FP32, and move by +-2^m per step
  float gx = (float)(((cx + ex) << m) - r.i) - 0.5f - r.ox;
  float gy = (float)(((cy + ey) << m) - r.j) - 0.5f - r.oy;
  const float stx = (float)(r.sx * S), sty = (float)(r.sy * S);
  const Level Ltop = level_of(T, m);
  const unsigned lwm = (unsigned)T.lw[m], lhm = (unsigned)T.lh[m];
  float best = SS_INF, bu0 = ua, bu1 = ua, brise = 0.0f;
  int bx = cx, by = cy, have = 0;
  float u0 = ua;
  for (int it = 0; it < 8; ++it) {
    const float ux = gx * r.invKx;
    const float uy = gy * r.invKy;
    const float u1 = fminf(fminf(ux, uy), ub);
    // a piece in a texel outside the level is a rounding sliver at the tile edge
    const bool ok = u1 > u0 && (unsigned)cx < lwm && (unsigned)cy < lhm;
    // where the tip is lowest on [u0, u1] (a piece that is not ok is discarded)
    const float uc = __builtin_amdgcn_fmed3f(r.uhmin, u0, u1);
    // lower bound of the clearance over the piece: lowest tip height minus
    // the texel's maximum height (Sec. 3.2, Eq. 4 with the maximum mipmap)
    const float rise = tip_rise_u(r, T, uc);
    const float lb = rise - (level_at(Ltop, cx, cy) - r.hp);
    n_lb += ok ? 1u : 0u;
    const bool take = ok && lb <= best;
    best = take ? lb : best;
    bx = take ? cx : bx;
    by = take ? cy : by;
    bu0 = take ? u0 : bu0;
    bu1 = take ? u1 : bu1;
    brise = take ? rise : brise;
    have |= take ? 1 : 0;
    u0 = fmaxf(u0, u1);
    if (!(u1 < ub)) break;
    const bool mx = ux <= uy, my = uy <= ux;
    cx += mx ? r.sx : 0;
    gx += mx ? stx : 0.0f;
    cy += my ? r.sy : 0;
    gy += my ? sty : 0.0f;
  }
  if (!have) return;
  // descend: the children of the chosen texel crossed by the ray.  The
  // parent's two mid-lines split its stretch [bu0, bu1] into at most three
  // pieces, in order: before both crossings, after the first, after both.  The
  // child before a mid-line (in the direction of travel) is the low one when
  // moving forward or not at all; each crossing flips that axis, so the
  // children follow from which mid-line comes first.  A crossing outside the
  // stretch (an infinite one on an axis the path does not move along, too)
  // leaves its piece empty.
  const int bfx = 1 - ex, bfy = 1 - ey;  // child bits before the mid-lines
  // parent's low edge relative to the origin texel centre, in texels
  float fx = (float)((bx << m) - r.i) - 0.5f - r.ox;
  float fy = (float)((by << m) - r.j) - 0.5f - r.oy;
  for (int lv = m; lv > 0; --lv) {
    const int half = 1 << (lv - 1);
    const float fh = (float)half;
    const Level Lc = level_of(T, lv - 1);
    const int px = 2 * bx, py = 2 * by;
    const float mxr = fx + fh, myr = fy + fh;  // mid-lines (exact)
    const float umx = mxr * r.invKx, umy = myr * r.invKy;
    const bool xfirst = umx <= umy;
    const float c1 = __builtin_amdgcn_fmed3f(fminf(umx, umy), bu0, bu1);
    const float c2 = __builtin_amdgcn_fmed3f(fmaxf(umx, umy), bu0, bu1);
    const int xa = px + bfx, ya = py + bfy;  // before both
    const int xc = px + ex, yc = py + ey;    // after both
    const int xb = xfirst ? xc : xa, yb = xfirst ? ya : yc;
    const float M0 = level_at(Lc, xa, ya), M1 = level_at(Lc, xb, yb), M2 = level_at(Lc, xc, yc);
    // tip rise at each piece's entry: the first piece enters where the parent
    // did (already known); identical to evaluating it again
    float r0, r1, r2;
    if (rising) {
      r0 = brise;
      r1 = tip_rise_u(r, T, c1);
      r2 = tip_rise_u(r, T, c2);
    } else {
      r0 = tip_rise_u(r, T, fminf(fmaxf(r.uhmin, bu0), c1));
      r1 = tip_rise_u(r, T, fminf(fmaxf(r.uhmin, c1), c2));
      r2 = tip_rise_u(r, T, fminf(fmaxf(r.uhmin, c2), bu1));
    }
    // children beyond a ragged edge are absent; px and py always exist, so
    // only the high children px + 1, py + 1 can be missing
    const bool hx = px + 1 < T.lw[lv - 1], hy = py + 1 < T.lh[lv - 1];
    const bool ina = (ex == 1 || hx) && (ey == 1 || hy);  // before both
    const bool inc = (ex == 0 || hx) && (ey == 0 || hy);  // after both
    const bool inb = xfirst ? ((ex == 0 || hx) && (ey == 1 || hy)) : ((ex == 1 || hx) && (ey == 0 || hy));
    const bool ok0 = c1 > bu0 && ina;
    const bool ok1 = c2 > c1 && inb;
    const bool ok2 = bu1 > c2 && inc;
    // an absent piece has bound +inf; present ones are finite
    const float lb0 = ok0 ? r0 - (M0 - r.hp) : SS_INF;
    const float lb1 = ok1 ? r1 - (M1 - r.hp) : SS_INF;
    const float lb2 = ok2 ? r2 - (M2 - r.hp) : SS_INF;
    n_lb += (ok0 ? 1u : 0u) + (ok1 ? 1u : 0u) + (ok2 ? 1u : 0u);
    // strict argmin from the far end == '<=' from the near end
    const bool t1 = lb1 <= lb0;
    const float b01 = t1 ? lb1 : lb0;
    const bool t2 = lb2 <= b01;
    if (!((t2 ? lb2 : b01) < SS_INF)) return;  // no piece inside the level
    const int nx = t2 ? xc : (t1 ? xb : xa);
    const int ny = t2 ? yc : (t1 ? yb : ya);
    fx = nx != px ? mxr : fx;
    fy = ny != py ? myr : fy;
    bx = nx;
    by = ny;
    brise = t2 ? r2 : (t1 ? r1 : r0);
    const float nu0 = t2 ? c2 : (t1 ? c1 : bu0);
    const float nu1 = t2 ? bu1 : (t1 ? c2 : c1);
    bu0 = nu0;
    bu1 = nu1;
  }
  // final samples on the half-texel grid t_n = (n + 1) delta/2 around the
  // middle of the base texel's stretch of ray
  const float tin = u_to_t(r, bu0), tout = u_to_t(r, bu1);
  const float tmid = 0.5f * (tin + tout);
  const int nc = (int)floorf((tmid - T.half_delta) * T.two_over_delta + 0.5f);
  float bdh = SS_INF, bt = 0.0f, bu = 0.0f;
  int found = 0, bn = -1;
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
        bn = n;
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
  out.n = bn;
  out.valid = 1;
}

// One run of Alg. 1 read literally: point samples instead of the texels the
// ray crosses.  Positions along run j are indices n on the half-texel grid
// t_n = (n + 1) delta/2 (the algorithm's normalised t in [0, 1] is
// (n - a_j) / 2^(m0+1)).  Level m = m0 .. 1 reads the maximum mipmap at the
// level-m texel under the ray tip at n = a_j + K, a_j + K - 2^m and
// a_j + K - 2^(m+1) (far to near; strict '<' keeps the far one on a tie) and
// continues from the smallest H - max h at K* with K = K* + 2^m; K starts at
// 2^(m0+1).  Level 0 samples the heightfield bilinearly at the three grid
// points and the chosen sample's clearance is the run's.  A level with no
// sample inside the tile ends the run.
template <bool SPHERE>
__device__ __forceinline__ void point_run(const TileK& T, const Ray<SPHERE>& r, int jseg,
                                          SegOut& out, unsigned& n_lb, unsigned& n_smp) {
  out.valid = 0;
  const int m0 = T.m0[jseg];
  const int a = T.a0[jseg];
  int K = 2 << m0;
  for (int m = m0; m >= 1; --m) {
    const int step = 1 << m;
    const Level Lm = level_of(T, m);
    float best = SS_INF;
    int kstar = -1;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int kk = K - q * step;
      const float t = (float)(a + kk + 1) * T.half_delta;
      const float u = t_to_u(r, t);
      // texel under the tip (positions before the edge are >= 0 by construction)
      const int cx = (int)floorf((float)r.i + 0.5f + r.ox + r.Kx * u) >> m;
      const int cy = (int)floorf((float)r.j + 0.5f + r.oy + r.Ky * u) >> m;
      const bool ok = u < r.uexit && (unsigned)cx < (unsigned)T.lw[m] && (unsigned)cy < (unsigned)T.lh[m];
      const float v = tip_rise(r, T, t) - (level_at(Lm, cx, cy) - r.hp);
      n_lb += ok ? 1u : 0u;
      const bool take = ok && v < best;
      best = take ? v : best;
      kstar = take ? kk : kstar;
    }
    if (kstar < 0) return;
    K = kstar + step;
  }
  float bdh = SS_INF, bt = 0.0f, bu = 0.0f;
  int found = 0, bn = -1;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float t = (float)(a + K - q + 1) * T.half_delta;
    const float u = t_to_u(r, t);
    if (u < r.uexit) {
      const Sample s = sample_at(r, T, t, u);
      n_smp++;
      if (s.dh < bdh) {
        bdh = s.dh;
        bt = t;
        bu = u;
        bn = a + K - q;
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
  out.n = bn;
  out.valid = 1;
}

// True when every sample at ray length >= t clears the angle whose tangent is
// need_tan (an angle in (-pi/2, pi/2)), given that no terrain rises above
// `top` (relative to the reference height hp, and at least the origin's dz,
// i.e. not below the origin): the clearance of the point at that height below
// the tip grows with t on the plane and on the sphere.  Used for the
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

struct RayResult {
  float alpha;
  float key;      // tangent key of alpha (orders like alpha)
  float t, u;     // deciding sample
  int n;          // its index on the step grid t = delta/2 + n step
  int valid;
};

__device__ __forceinline__ float angle_of(float key) {
  return key == SS_INF ? SS_INF : (key == -SS_INF ? -SS_INF : atanf(key));
}

// Smallest clearance over the concatenated runs (Sec. 3.3), each by the
// texel descent (POINT = false) or Alg. 1's point samples (POINT = true).
template <bool SPHERE, bool POINT = false>
__device__ __forceinline__ RayResult shadow_dp(const TileK& T, const Ray<SPHERE>& r, float top,
                                               unsigned& n_lb, unsigned& n_smp) {
  RayResult res;
  res.t = 0.0f;
  res.u = 0.0f;
  res.n = -1;
  res.valid = 0;
  float best = SS_INF;                    // tangent key of the smallest clearance so far
  float need = need_tangent(T, SS_INF);   // tan(min(alpha, r_L) + margin)
  for (int j = 0; j < T.nseg; ++j) {
    const float ta = T.tau[j];
    if (!(t_to_u(r, ta) < r.uexit)) break;  // the run starts outside the tile
    if (T.prune) {
      // every final sample of run j lies at t >= tau_j - 3 delta/4
      const float tlo = fmaxf(T.half_delta, ta - 1.5f * T.half_delta);
      if (clears(r, T, tlo, top, need)) break;  // nothing ahead is high enough
    }
    SegOut so;
    if (POINT)
      point_run(T, r, j, so, n_lb, n_smp);
    else
      descend_run(T, r, j, so, n_lb, n_smp);
    if (so.valid && so.key < best) {
      best = so.key;
      res.t = so.t;
      res.u = so.u;
      res.n = so.n;
      res.valid = 1;
      need = need_tangent(T, best);
    }
    if (T.prune && best <= -T.tan_rL) break;  // umbra: nothing can change s = 0
  }
  res.key = best;
  res.alpha = angle_of(best);
  return res;
}

// Ray length of step k: t_k = delta/2 + k step, rounded once, so that the
// exact mode (step delta/2) and uniform stepping at half a texel place their
// samples at bit-identical t.
__device__ __forceinline__ float step_t(const TileK& T, int k, float step) {
  return fmaf((float)k, step, T.half_delta);
}

// Uniform stepping (Sec. 2, Fig. 1b): every step, smallest clearance, kept as
// a tangent key; atan is taken once.  The first smallest step decides.
template <bool SPHERE>
__device__ __forceinline__ RayResult shadow_uniform(const TileK& T, const Ray<SPHERE>& r, float top,
                                                    unsigned& n_smp) {
  RayResult res;
  res.t = 0.0f;
  res.u = 0.0f;
  res.n = -1;
  res.valid = 0;
  float best = SS_INF;
  for (int k = 0; k < (1 << 22); ++k) {
    const float t = step_t(T, k, T.ustep);
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
    const float key = tangent_key(num, den);
    if (key < best) {
      best = key;
      res.t = t;
      res.u = u;
      res.n = k;
      res.valid = 1;
    }
  }
  res.key = best;
  res.alpha = angle_of(best);
  return res;
}

// Entry m >= 0 of the tap-bound pyramid: the largest height any bilinear tap
// of a sample inside level-m texel (cx, cy) can read (also for samples up to
// half a texel outside it).
// The exact walk's pyramid level differs between lanes, so reading the level's
// offset from the kernel arguments would put a dependent memory load before
// every bound; kernels that run the walk copy the offsets to LDS first.
__device__ __forceinline__ void bound_tab_fill(const TileK& T, int* tab) {
  if (threadIdx.x < SS_MAXLEV) tab[threadIdx.x] = T.loff[threadIdx.x];
}

__device__ __forceinline__ float bound_at(const TileK& T, const int* tab, int m, int cx, int cy) {
  const float* base = m == 0 ? T.bnd : T.bmm + tab[m];
  const int w = (T.W + (1 << m) - 1) >> m;
  return base[idx2((unsigned)cy, (unsigned)w, (unsigned)cx)];
}

// Exact mode: the smallest clearance over every sample of the grid
// t_n = (n + 1) delta/2 up to the cap or the tile edge -- the grid of the
// descent's final samples (Alg. 1), i.e. uniform stepping at half a texel --
// found by branch and bound over the tap-bound pyramid (the global
// minimisation of Sec. 2 made exact).  A per-lane walk front to back over
// the sample index n and a pyramid level m:
//   * the level-m texel holding sample n bounds the terrain under every
//     sample whose position lies in it; if the point at that height below the
//     tip at t_n already clears the angle that could still matter, every
//     sample up to the texel's exit is skipped and the walk climbs a level;
//   * otherwise it descends a level, and at level 0 evaluates sample n.
// Every iteration either advances n or lowers m, so the walk ends.  The skips
// use the same margin as the other result-invariant exits, so the output is
// bit-identical to uniform stepping at half a texel (prune = 0 evaluates
// every sample).
//
// Branch and bound prunes best with a good incumbent: the descent (Sec. 3.2)
// runs first and its deciding sample, a sample of the same grid computed by
// the same arithmetic, seeds the minimum when it lies within the cap.  A ray
// the descent already finds in umbra is then done.
template <bool SPHERE>
__device__ __forceinline__ RayResult shadow_exact(const TileK& T, const Ray<SPHERE>& r, float top,
                                                  unsigned& n_tst, unsigned& n_smp,
                                                  const int* tab) {
  RayResult res;
  res.t = 0.0f;
  res.u = 0.0f;
  res.n = -1;
  res.valid = 0;
  float best = SS_INF;
  if (T.prune) {
    unsigned n_lb = 0, n_dp = 0;
    const RayResult d = shadow_dp(T, r, top, n_lb, n_dp);
    n_tst += n_lb;
    n_smp += n_dp;
    if (d.valid && d.t <= T.ucap) {
      res = d;
      best = d.key;
    }
  }
  float need = need_tangent(T, best);
  const int mtop = T.L - 1;
  const int ex = r.Kx >= 0.0f ? 1 : 0, ey = r.Ky >= 0.0f ? 1 : 0;
  // where the samples end: the cap, or the tile edge
  const float uend = fminf(r.uexit, t_to_u(r, T.ucap));
  int n = 0, m = 0;
  // the level-0 texel whose test last failed: its next sample is evaluated
  // without testing again (a test only ever skips work, so this changes no
  // result; the texel's second sample rarely clears where the first did not)
  int fx0 = -1, fy0 = -1;
  const bool umbra = T.prune && best <= -T.tan_rL;  // settled by the descent
  for (int it = 0; it < (umbra ? 0 : (1 << 24)); ++it) {
    const float t = step_t(T, n, T.half_delta);
    if (t > T.ucap) break;
    const float u = t_to_u(r, t);
    if (!(u < r.uexit)) break;
    // texel under sample n (rounding past the edge is clamped)
    const int ix = min(max((int)floorf((float)r.i + 0.5f + r.ox + r.Kx * u), 0), T.W - 1);
    const int iy = min(max((int)floorf((float)r.j + 0.5f + r.oy + r.Ky * u), 0), T.H - 1);
    const int cx = ix >> m, cy = iy >> m;
    bool skip = false;
    if (T.prune && !(m == 0 && ix == fx0 && iy == fy0)) {
      n_tst++;
      // relative to the origin the bound must be at least 0 (see clears)
      const float b0 = fmaxf(bound_at(T, tab, m, cx, cy) - r.hp, 0.0f);
      const float top = r.dz > b0 ? r.dz : b0;
      skip = clears(r, T, t, top, need);
    }
    if (skip) {
      // first grid sample at or past the texel's exit (a sample a rounding
      // error past the exit is still under the bound's half-texel margin)
      const float ux = ((float)(((cx + ex) << m) - r.i) - 0.5f - r.ox) * r.invKx;
      const float uy = ((float)(((cy + ey) << m) - r.j) - 0.5f - r.oy) * r.invKy;
      const float tb = u_to_t(r, fminf(fminf(ux, uy), uend));
      const float nb = ceilf(tb * T.two_over_delta) - 1.0f;
      n = max(n + 1, (int)fminf(nb, 16777216.0f));
      m = min(m + 1, mtop);
    } else if (m > 0) {
      --m;
    } else {
      fx0 = ix;
      fy0 = iy;
      const Sample s = sample_at(r, T, t, u);
      n_smp++;
      float num, den;
      clearance_terms(r, t, s.dh, num, den);
      const float key = tangent_key(num, den);
      if (key < best) {
        best = key;
        res.t = t;
        res.u = u;
        res.n = n;
        res.valid = 1;
        need = need_tangent(T, best);
        if (T.prune && best <= -T.tan_rL) break;  // umbra: nothing can change s = 0
      }
      ++n;
    }
  }
  res.key = best;
  res.alpha = angle_of(best);
  return res;
}

// The shadow clearance of one ray by the chosen method.
template <bool SPHERE, int MODE>
__device__ __forceinline__ RayResult trace_ray(const TileK& T, const Ray<SPHERE>& r, unsigned& n_lb,
                                               unsigned& n_smp, const int* tab) {
  // no terrain rises above `top` (relative to h_p, at least 0)
  const float t0 = T.prune ? fmaxf(mip_at(T, T.L - 1, 0, 0), r.hp) - r.hp : 0.0f;
  const float top = r.dz > t0 ? r.dz : t0;
  if (MODE == SS_MODE_EXACT) return shadow_exact(T, r, top, n_lb, n_smp, tab);
  if (MODE == SS_MODE_POINT) return shadow_dp<SPHERE, true>(T, r, top, n_lb, n_smp);
  if (MODE == SS_MODE_UNIFORM) return shadow_uniform(T, r, top, n_smp);
  return shadow_dp<SPHERE, false>(T, r, top, n_lb, n_smp);
}
