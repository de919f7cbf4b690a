// Shadow-factor kernels for gfx950: forward (descent or uniform stepping),
// its instrumented twin, and the adjoint.
//
// One lane = one ray (texel centre); one wavefront = a TW x TH ray tile; a
// 256-thread workgroup = 2 x 2 wavefront tiles.  Workgroup ids are dealt
// round-robin over the 8 XCDs and run roughly in order, about one device-full
// at a time.  They are remapped within groups of one device-full (T.wg_group
// ids): inside a group each XCD takes one contiguous run of ray blocks, so the
// XCDs work side by side on one slab of the tile with their rays' neighbours in
// their own L2.  One contiguous band of the whole tile per XCD kept the same
// locality but left the XCDs with unequal work (the slowest band set the
// launch time): on the 4096^2 tile's 8 suns the groups are 18% faster.
#include "kernels.h"
#include "ray.h"

namespace ss {


__device__ __forceinline__ unsigned wave_sum_u32(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Texel of this lane in ray block b (2 x 2 wavefront tiles of TW x 64/TW).
template <int TW>
__device__ __forceinline__ void coords_of(int b, int nbx, int& i, int& j) {
  constexpr int TH = 64 / TW;
  const int bxi = b % nbx, byi = b / nbx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  i = bxi * (2 * TW) + (wave & 1) * TW + lane % TW;
  j = byi * (2 * TH) + (wave >> 1) * TH + lane / TW;
}

template <int TW>
__device__ __forceinline__ void ray_coords(int nbx, int nblocks, int grp, int& i, int& j) {
  coords_of<TW>(xcd_remap_grouped((int)blockIdx.x, nblocks, grp), nbx, i, j);
}

// FLAGS: FWD_COUNT adds the work units to counter[0..1]; FWD_SAVE writes each
// ray's deciding sample index (-1: none) to sample[].
enum { FWD_PLAIN = 0, FWD_COUNT = 1, FWD_SAVE = 2 };

template <bool SPHERE, int TW, int MODE, int FLAGS>
__global__ __launch_bounds__(256) void shadow_kernel(TileK T, float* __restrict__ out,
                                                     unsigned long long* counter,
                                                     int* __restrict__ sample, int nbx,
                                                     int nblocks) {
  constexpr bool COUNT = FLAGS == FWD_COUNT;
  __shared__ int tab[SS_MAXLEV];
  if (MODE == SS_MODE_EXACT) {
    bound_tab_fill(T, tab);
    __syncthreads();
  }
  int li, lj;
  ray_coords<TW>(nbx, nblocks, T.wg_group, li, lj);
  unsigned n_lb = 0, n_smp = 0;
  if (li < T.RW && lj < T.RH) {
    const int i = T.rx0 + li, j = T.ry0 + lj;
    const float hp = T.h[j * T.W + i];
    Ray<SPHERE> r;
    ray_init(T, i, j, hp, r);
    const RayResult res = trace_ray<SPHERE, MODE>(T, r, n_lb, n_smp, tab);
    out[lj * T.RW + li] = disc_fraction(res.alpha, T);
    if (FLAGS == FWD_SAVE) sample[lj * T.RW + li] = res.valid ? res.n : -1;
  }
  if (COUNT) {
    const unsigned a = wave_sum_u32(n_lb), b = wave_sum_u32(n_smp);
    if ((threadIdx.x & 63) == 0) {
      if (a) atomicAdd(&counter[0], (unsigned long long)a);
      if (b) atomicAdd(&counter[1], (unsigned long long)b);
    }
  }
}

// Adjoint: recompute the forward decisions (or read the deciding sample the
// forward recorded, SAVED), then apply the chain rule through that sample.  With the decisions fixed, s depends on the origin
// height (through rho and the texture path), the four bilinear taps, and the
// sun direction (through L, s_p, c_p, the texture path and t* = (n*+1) delta/2
// with delta = texel / cos e).  Each partial below is the derivative of the
// forward expression it sits next to.
struct SunTrig {
  float se, ce, sa, ca, tan_e;
};

// The chain rule through one ray's deciding sample: adds to dL/dh at the
// sample's four taps and to the sun gradient, and returns dL/d(origin height).
// X, Y: the origin's plane position; r1 = 1 + (origin height) / R.
template <bool SPHERE>
__device__ __forceinline__ float adjoint_sample(const TileK& T, const SunTrig& st,
                                                const Ray<SPHERE>& r, const RayResult& res,
                                                float g, float X, float Y, float r1,
                                                float* __restrict__ gh, double& ge, double& ga) {
  const float dd = res.alpha * T.inv_rL;
  if (!(res.valid && g != 0.0f && fabsf(dd) < 1.0f)) return 0.0f;
  const float t = res.t, u = res.u;
  const Sample s = sample_at(r, T, t, u);
  const float dh = s.dh;
  const float galpha = g * 2.0f * sqrtf(1.0f - dd * dd) * (0.318309886183791f * T.inv_rL);
  float num, den, x = 0.0f, w = 1.0f;
  if (SPHERE) {
    x = t * r.invrho;
    w = sqrtf(1.0f + x * (2.0f * r.sp + x));
    num = dh * r.cp;
    den = t * w - dh * (r.sp + x);
  } else {
    num = dh * r.cp;
    den = t - dh * r.sp;
  }
  const float inv2 = 1.0f / (num * num + den * den);
  const float a_n = galpha * den * inv2;
  const float a_d = -galpha * num * inv2;
  float a_dh, a_cp, a_sp, a_t, a_hp = 0.0f;
  float a_Lx = 0.0f, a_Ly = 0.0f, a_Lz = 0.0f;
  // bilinear taps
  const int xa = min(max(s.x0, 0), T.W - 1), xb = min(max(s.x0 + 1, 0), T.W - 1);
  const int ya = min(max(s.y0, 0), T.H - 1), yb = min(max(s.y0 + 1, 0), T.H - 1);
  const float h00 = T.h[ya * T.W + xa], h10 = T.h[ya * T.W + xb];
  const float h01 = T.h[yb * T.W + xa], h11 = T.h[yb * T.W + xb];
  const float gxh = (1.0f - s.fy) * (h10 - h00) + s.fy * (h11 - h01);
  const float gyh = (1.0f - s.fx) * (h01 - h00) + s.fx * (h11 - h10);
  if (SPHERE) {
    const float aa = X * T.invR, bb = Y * T.invR;
    const float gg = sqrtf(1.0f + aa * aa + bb * bb);
    const float G = gg / (r1 * T.texel);
    a_dh = a_n * r.cp - a_d * (r.sp + x);
    a_cp = a_n * dh;
    a_t = a_d * w;
    float a_w = a_d * t;
    a_sp = -a_d * dh;
    float a_x = -a_d * dh;
    // dh = dH(t, rho, sp) - (hb - hp)
    const float a_hb = -a_dh;
    a_hp += a_dh;
    const float spx = r.sp + x;
    const float wm1 = x * (2.0f * r.sp + x) / (w + 1.0f);
    a_t += a_dh * spx / w;
    a_sp += a_dh * t / w;
    float a_rho = a_dh * (wm1 - x * spx / w);
    a_x += a_w * spx / w;
    a_sp += a_w * x / w;
    a_t += a_x * r.invrho;
    a_rho -= a_x * x * r.invrho;
    // texture position d = K u(t)
    const float a_dx = a_hb * gxh, a_dy = a_hb * gyh;
    const float omc = 1.0f - r.c * u;  // = 1 / (1 + c t)
    const float k1 = omc * omc;
    const float aK = a_dx * r.Kx + a_dy * r.Ky;
    a_t += aK * k1;
    a_rho -= aK * k1 * x;
    a_Lx += a_dx * G * u;
    a_Ly += a_dy * G * u;
    a_Lz += -G * u * (a_dx * aa + a_dy * bb) - aK * k1 * t * t * (gg * T.invR / r1);
    // s_p = (aa Lx + bb Ly + Lz)/g and c_p = sqrt(1 - s_p^2)
    a_sp += -a_cp * r.sp / r.cp;
    const float ig = 1.0f / gg;
    a_Lx += a_sp * aa * ig;
    a_Ly += a_sp * bb * ig;
    a_Lz += a_sp * ig;
    a_hp += a_rho;
    // taps
    atomicAdd(&gh[ya * T.W + xa], a_hb * (1.0f - s.fx) * (1.0f - s.fy));
    atomicAdd(&gh[ya * T.W + xb], a_hb * s.fx * (1.0f - s.fy));
    atomicAdd(&gh[yb * T.W + xa], a_hb * (1.0f - s.fx) * s.fy);
    atomicAdd(&gh[yb * T.W + xb], a_hb * s.fx * s.fy);
  } else {
    a_dh = a_n * r.cp - a_d * r.sp;
    a_cp = a_n * dh;
    a_sp = -a_d * dh;
    a_t = a_d;
    a_t += a_dh * T.Lz;
    a_Lz += a_dh * t;
    const float a_hb = -a_dh;
    a_hp += a_dh;
    const float a_dx = a_hb * gxh, a_dy = a_hb * gyh;
    const float it = 1.0f / T.texel;
    a_t += (a_dx * T.Lx + a_dy * T.Ly) * it;
    a_Lx += a_dx * t * it;
    a_Ly += a_dy * t * it;
    a_Lz += a_sp;
    if (r.cp > 0.0f) {
      a_Lx += a_cp * T.Lx / r.cp;
      a_Ly += a_cp * T.Ly / r.cp;
    }
    atomicAdd(&gh[ya * T.W + xa], a_hb * (1.0f - s.fx) * (1.0f - s.fy));
    atomicAdd(&gh[ya * T.W + xb], a_hb * s.fx * (1.0f - s.fy));
    atomicAdd(&gh[yb * T.W + xa], a_hb * (1.0f - s.fx) * s.fy);
    atomicAdd(&gh[yb * T.W + xb], a_hb * s.fx * s.fy);
  }
  // t = texel (1/2 + k step) / cos e (every mode) grows with e; L(e, a)
  // on the unit sphere
  const double dte = (double)a_t * (double)t * (double)st.tan_e;
  ge += dte + (double)a_Lx * (-(double)st.se * st.ca) + (double)a_Ly * (-(double)st.se * st.sa) +
        (double)a_Lz * (double)st.ce;
  ga += (double)a_Lx * (-(double)st.ce * st.sa) + (double)a_Ly * ((double)st.ce * st.ca);
  return a_hp;
}

// sfwd (may be null): the forward's shadow factors; a ray whose value is 0 or
// 1 has |d| >= 1 (disc_fraction) and no derivative, so it is not replayed, nor
// is one whose upstream gradient is 0: neither contributes anything.
template <bool SPHERE, int MODE, bool SAVED>
__device__ __forceinline__ void adjoint_ray(const TileK& T, const SunTrig& st, int li, int lj,
                                            const float* __restrict__ gs,
                                            const int* __restrict__ sample,
                                            const float* __restrict__ sfwd,
                                            float* __restrict__ gh, double& ge, double& ga,
                                            const int* tab) {
  if (li < T.RW && lj < T.RH) {
    const int i = T.rx0 + li, j = T.ry0 + lj;
    const float g = gs[lj * T.RW + li];
    if (g == 0.0f) return;
    if (sfwd) {
      const float sv = sfwd[lj * T.RW + li];
      if (sv == 0.0f || sv == 1.0f) return;
    }
    const float hp = T.h[j * T.W + i];
    Ray<SPHERE> r;
    ray_init(T, i, j, hp, r);
    RayResult res;
    if (SAVED) {
      // the recorded sample, with the forward's own arithmetic: t rounded once
      // from its index, u(t), the clearance key and its angle
      const int n = sample[lj * T.RW + li];
      res.valid = n >= 0 && g != 0.0f;
      res.alpha = SS_INF;
      if (res.valid) {
        res.t = fmaf((float)n, MODE == SS_MODE_UNIFORM ? T.ustep : T.half_delta, T.half_delta);
        res.u = t_to_u(r, res.t);
        const Sample s0 = sample_at(r, T, res.t, res.u);
        float num0, den0;
        clearance_terms(r, res.t, s0.dh, num0, den0);
        res.alpha = angle_of(tangent_key(num0, den0));
      }
    } else {
      unsigned n_lb = 0, n_smp = 0;
      res = trace_ray<SPHERE, MODE>(T, r, n_lb, n_smp, tab);
    }
    float X = 0.0f, Y = 0.0f;
    if (SPHERE) {
      X = ((float)i + 0.5f - 0.5f * (float)T.W) * T.texel;
      Y = ((float)j + 0.5f - 0.5f * (float)T.H) * T.texel;
    }
    const float a_hp = adjoint_sample<SPHERE>(T, st, r, res, g, X, Y, 1.0f + hp * T.invR, gh, ge,
                                              ga);
    if (a_hp != 0.0f) atomicAdd(&gh[j * T.W + i], a_hp);
  }
}

// Each workgroup adds its sun gradient once (waves reduce through LDS), and
// with a recorded forward, where a ray costs little, it takes four
// consecutive ray blocks: the two fp64 sums every workgroup shares are then
// hit by one atomic pair per 4096 rays instead of one per wavefront.  A
// replaying adjoint keeps one block per workgroup for parallelism.
template <bool SAVED>
struct AdjBlocks {
  static constexpr int n = SAVED ? 4 : 1;
};

template <bool SPHERE, int TW, int MODE, bool SAVED>
__global__ __launch_bounds__(256) void adjoint_kernel(TileK T, SunTrig st,
                                                      const float* __restrict__ gs,
                                                      const int* __restrict__ sample,
                                                      const float* __restrict__ sfwd,
                                                      float* __restrict__ gh,
                                                      double* __restrict__ gsun, int nbx,
                                                      int nblocks) {
  __shared__ double red[2][4];
  __shared__ int tab[SS_MAXLEV];
  if (MODE == SS_MODE_EXACT && !SAVED) {
    bound_tab_fill(T, tab);
    __syncthreads();
  }
  double ge = 0.0, ga = 0.0;
  const int b = xcd_remap_grouped((int)blockIdx.x, (int)gridDim.x, T.wg_group);
  for (int g = 0; g < AdjBlocks<SAVED>::n; ++g) {
    const int vb = b * AdjBlocks<SAVED>::n + g;
    if (vb >= nblocks) break;
    int i, j;
    coords_of<TW>(vb, nbx, i, j);
    adjoint_ray<SPHERE, MODE, SAVED>(T, st, i, j, gs, sample, sfwd, gh, ge, ga, tab);
  }
  ge = wave_sum_f64(ge);
  ga = wave_sum_f64(ga);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = ge;
    red[1][wave] = ga;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double se = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double sa = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    if (se != 0.0 || sa != 0.0) {
      atomicAdd(&gsun[0], se);
      atomicAdd(&gsun[1], sa);
    }
  }
}

// Adjoint given the forward's values on large tiles (ss_shadow_cast_backward_
// penumbra): a workgroup takes SS_PEN_BLOCKS consecutive ray blocks (its id
// remapped as the other per-tile kernels remap theirs), lists in LDS the rays
// whose s lies strictly inside (0, 1) and whose upstream gradient is nonzero
// (a ballot per wavefront, so neighbouring rays stay neighbours in the list),
// then replays only those, 256 at a time, so the replaying wavefronts run
// full.  It pays where penumbra is sparse and the launch has many workgroups
// per device-full to balance the uneven lists (the launcher's threshold);
// smaller launches keep adjoint_kernel's per-lane skip.
#define SS_PEN_BLOCKS 8

template <bool SPHERE, int MODE>
__global__ __launch_bounds__(256) void adjoint_penumbra_kernel(TileK T, SunTrig st,
                                                               const float* __restrict__ gs,
                                                               const float* __restrict__ sfwd,
                                                               float* __restrict__ gh,
                                                               double* __restrict__ gsun, int nbx,
                                                               int nblocks) {
  __shared__ double red[2][4];
  __shared__ int tab[SS_MAXLEV];
  __shared__ unsigned list[SS_PEN_BLOCKS * 256];
  __shared__ unsigned count;
  if (threadIdx.x == 0) count = 0u;
  if (MODE == SS_MODE_EXACT) bound_tab_fill(T, tab);
  __syncthreads();
  const int grp = xcd_remap_grouped((int)blockIdx.x, (int)gridDim.x, T.wg_group);
  const int lane = threadIdx.x & 63;
  for (int g = 0; g < SS_PEN_BLOCKS; ++g) {
    const int vb = grp * SS_PEN_BLOCKS + g;
    bool take = false;
    int li = 0, lj = 0;
    if (vb < nblocks) {
      coords_of<8>(vb, nbx, li, lj);
      if (li < T.RW && lj < T.RH) {
        const int k = lj * T.RW + li;
        const float sv = sfwd[k];
        take = gs[k] != 0.0f && sv != 0.0f && sv != 1.0f;
      }
    }
    const unsigned long long m = __ballot(take);
    if (m) {
      unsigned base = 0u;
      if (lane == 0) base = atomicAdd(&count, (unsigned)__popcll(m));
      base = __shfl(base, 0, 64);
      if (take)
        list[base + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] =
            (unsigned)li | ((unsigned)lj << 16);
    }
  }
  __syncthreads();
  const unsigned n = count;
  double ge = 0.0, ga = 0.0;
  for (unsigned q = threadIdx.x; q < n; q += 256u) {
    const unsigned e = list[q];
    adjoint_ray<SPHERE, MODE, false>(T, st, (int)(e & 0xffffu), (int)(e >> 16), gs, nullptr,
                                     nullptr, gh, ge, ga, tab);
  }
  ge = wave_sum_f64(ge);
  ga = wave_sum_f64(ga);
  const int wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = ge;
    red[1][wave] = ga;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double se = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double sa = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    if (se != 0.0 || sa != 0.0) {
      atomicAdd(&gsun[0], se);
      atomicAdd(&gsun[1], sa);
    }
  }
}

// Shadow rays from arbitrary surface points: point k at continuous texel
// coordinates xy[k] (clamped to the tile), on the bilinear terrain there.
template <bool SPHERE, int MODE>
__device__ __forceinline__ float shade_point(const TileK& T, float2 q, const int* tab) {
  if (q.x != q.x || q.y != q.y) return NAN;  // a view ray's miss: nothing to shade
  const float qx = fminf(fmaxf(q.x, 0.0f), (float)T.W), qy = fminf(fmaxf(q.y, 0.0f), (float)T.H);
  const int i = min((int)floorf(qx), T.W - 1), j = min((int)floorf(qy), T.H - 1);
  // heights relative to the texel's own, the origin dz above it
  const float ref = T.h[j * T.W + i];
  Ray<SPHERE> r;
  ray_init(T, i, j, ref, r, qx - ((float)i + 0.5f), qy - ((float)j + 0.5f),
           terrain_above(T, qx, qy, ref));
  unsigned n_lb = 0, n_smp = 0;
  return disc_fraction(trace_ray<SPHERE, MODE>(T, r, n_lb, n_smp, tab).alpha, T);
}

// IMAGE: the points form an image [n / img_w][img_w] and a wavefront takes an
// 8 x 8 pixel tile (a workgroup 16 x 16): neighbouring pixels' hits are
// neighbours on the terrain, so their shadow rays walk the same cells (a row
// of 64 pixels spreads them out).  Otherwise lane k takes point k.
template <bool SPHERE, int MODE, bool IMAGE>
__global__ __launch_bounds__(256) void points_kernel(TileK T, const float2* __restrict__ xy,
                                                     long long n, int img_w, int nbx,
                                                     float* __restrict__ out) {
  __shared__ int tab[SS_MAXLEV];
  if (MODE == SS_MODE_EXACT) {
    bound_tab_fill(T, tab);
    __syncthreads();
  }
  long long k;
  if (IMAGE) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = (int)(blockIdx.x % (unsigned)nbx), by = (int)(blockIdx.x / (unsigned)nbx);
    const int px = bx * 16 + (wv & 1) * 8 + (lane & 7);
    const int py = by * 16 + (wv >> 1) * 8 + (lane >> 3);
    if (px >= img_w) return;
    k = (long long)py * img_w + px;  // >= n for rows past the image
  } else {
    k = (long long)blockIdx.x * 256 + threadIdx.x;
  }
  if (k >= n) return;
  out[k] = shade_point<SPHERE, MODE>(T, xy[k], tab);
}

// Adjoint of shadow rays from surface points, the points held fixed: the
// chain rule of adjoint_sample, with dL/d(origin height) spread over the
// bilinear taps at the point (the origin sits on the bilinear terrain there).
// Work is mapped as in points_kernel; the sun gradient is reduced per
// workgroup as in adjoint_kernel.
template <bool SPHERE, int MODE, bool IMAGE>
__global__ __launch_bounds__(256) void points_adjoint_kernel(TileK T, SunTrig st,
                                                             const float2* __restrict__ xy,
                                                             long long n, int img_w, int nbx,
                                                             const float* __restrict__ gs,
                                                             float* __restrict__ gh,
                                                             double* __restrict__ gsun) {
  __shared__ double red[2][4];
  __shared__ int tab[SS_MAXLEV];
  if (MODE == SS_MODE_EXACT) {
    bound_tab_fill(T, tab);
    __syncthreads();
  }
  long long k;
  bool ok;
  if (IMAGE) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = (int)(blockIdx.x % (unsigned)nbx), by = (int)(blockIdx.x / (unsigned)nbx);
    const int px = bx * 16 + (wv & 1) * 8 + (lane & 7);
    const int py = by * 16 + (wv >> 1) * 8 + (lane >> 3);
    k = (long long)py * img_w + px;
    ok = px < img_w && k < n;
  } else {
    k = (long long)blockIdx.x * 256 + threadIdx.x;
    ok = k < n;
  }
  double ge = 0.0, ga = 0.0;
  if (ok) {
    const float2 q = xy[k];
    const float g = gs[k];
    if (q.x == q.x && q.y == q.y && g != 0.0f) {
      const float qx = fminf(fmaxf(q.x, 0.0f), (float)T.W);
      const float qy = fminf(fmaxf(q.y, 0.0f), (float)T.H);
      const int i = min((int)floorf(qx), T.W - 1), j = min((int)floorf(qy), T.H - 1);
      const float ref = T.h[j * T.W + i];
      const float ox = qx - ((float)i + 0.5f), oy = qy - ((float)j + 0.5f);
      const float dz = terrain_above(T, qx, qy, ref);
      Ray<SPHERE> r;
      ray_init(T, i, j, ref, r, ox, oy, dz);
      unsigned n_lb = 0, n_smp = 0;
      const RayResult res = trace_ray<SPHERE, MODE>(T, r, n_lb, n_smp, tab);
      float X = 0.0f, Y = 0.0f;
      if (SPHERE) {
        X = ((float)i + 0.5f + ox - 0.5f * (float)T.W) * T.texel;
        Y = ((float)j + 0.5f + oy - 0.5f * (float)T.H) * T.texel;
      }
      const float a_o = adjoint_sample<SPHERE>(T, st, r, res, g, X, Y,
                                               1.0f + (ref + dz) * T.invR, gh, ge, ga);
      if (a_o != 0.0f) {
        // the origin height is the bilinear terrain at q (taps as terrain_above)
        const float x = qx - 0.5f, y = qy - 0.5f;
        const float flx = floorf(x), fly = floorf(y);
        const float fx = x - flx, fy = y - fly;
        const int x0 = (int)flx, y0 = (int)fly;
        const int xa = min(max(x0, 0), T.W - 1), xb = min(max(x0 + 1, 0), T.W - 1);
        const int ya = min(max(y0, 0), T.H - 1), yb = min(max(y0 + 1, 0), T.H - 1);
        atomicAdd(&gh[ya * T.W + xa], a_o * (1.0f - fx) * (1.0f - fy));
        atomicAdd(&gh[ya * T.W + xb], a_o * fx * (1.0f - fy));
        atomicAdd(&gh[yb * T.W + xa], a_o * (1.0f - fx) * fy);
        atomicAdd(&gh[yb * T.W + xb], a_o * fx * fy);
      }
    }
  }
  ge = wave_sum_f64(ge);
  ga = wave_sum_f64(ga);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = ge;
    red[1][wave] = ga;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double se = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double sa = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    if (se != 0.0 || sa != 0.0) {
      atomicAdd(&gsun[0], se);
      atomicAdd(&gsun[1], sa);
    }
  }
}

template <bool SPHERE, int MODE>
static void points_adjoint_launch(const TileK& T, const SunTrig& st, const float* xy,
                                  long long n, int img_w, const float* gs, float* gh,
                                  double* gsun, hipStream_t stream) {
  const float2* q = reinterpret_cast<const float2*>(xy);
  if (img_w > 0) {
    const int nbx = (img_w + 15) / 16;
    const long long rows = n / img_w, nby = (rows + 15) / 16;
    hipLaunchKernelGGL((points_adjoint_kernel<SPHERE, MODE, true>), dim3((unsigned)(nbx * nby)),
                       dim3(256), 0, stream, T, st, q, n, img_w, nbx, gs, gh, gsun);
  } else {
    hipLaunchKernelGGL((points_adjoint_kernel<SPHERE, MODE, false>),
                       dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, T, st, q, n, 0, 1,
                       gs, gh, gsun);
  }
}

template <bool SPHERE>
static void points_adjoint_mode(const TileK& T, const SunTrig& st, int mode, const float* xy,
                                long long n, int img_w, const float* gs, float* gh, double* gsun,
                                hipStream_t stream) {
  switch (mode) {
    case SS_MODE_EXACT:
      points_adjoint_launch<SPHERE, SS_MODE_EXACT>(T, st, xy, n, img_w, gs, gh, gsun, stream);
      break;
    case SS_MODE_POINT:
      points_adjoint_launch<SPHERE, SS_MODE_POINT>(T, st, xy, n, img_w, gs, gh, gsun, stream);
      break;
    case SS_MODE_UNIFORM:
      points_adjoint_launch<SPHERE, SS_MODE_UNIFORM>(T, st, xy, n, img_w, gs, gh, gsun, stream);
      break;
    default:
      points_adjoint_launch<SPHERE, SS_MODE_DP>(T, st, xy, n, img_w, gs, gh, gsun, stream);
      break;
  }
}

hipError_t launch_points_adjoint(const TileK& T, bool sphere, int mode, double elev, double azim,
                                 const float* xy, long long n, int img_w, const float* gs,
                                 float* gh, double* gsun, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  SunTrig st;
  st.se = (float)sin(elev);
  st.ce = (float)cos(elev);
  st.sa = (float)sin(azim);
  st.ca = (float)cos(azim);
  st.tan_e = (float)tan(elev);
  if (sphere)
    points_adjoint_mode<true>(T, st, mode, xy, n, img_w, gs, gh, gsun, stream);
  else
    points_adjoint_mode<false>(T, st, mode, xy, n, img_w, gs, gh, gsun, stream);
  return hipGetLastError();
}

template <bool SPHERE, int MODE>
static void points_launch(const TileK& T, const float* xy, long long n, int img_w,
                          float* out, hipStream_t stream) {
  const float2* q = reinterpret_cast<const float2*>(xy);
  if (img_w > 0) {
    const int nbx = (img_w + 15) / 16;
    const long long rows = n / img_w, nby = (rows + 15) / 16;
    hipLaunchKernelGGL((points_kernel<SPHERE, MODE, true>), dim3((unsigned)(nbx * nby)),
                       dim3(256), 0, stream, T, q, n, img_w, nbx, out);
  } else {
    hipLaunchKernelGGL((points_kernel<SPHERE, MODE, false>), dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, stream, T, q, n, 0, 1, out);
  }
}

template <bool SPHERE>
static void points_mode(const TileK& T, int mode, const float* xy, long long n, int img_w,
                        float* out, hipStream_t stream) {
  switch (mode) {
    case SS_MODE_EXACT: points_launch<SPHERE, SS_MODE_EXACT>(T, xy, n, img_w, out, stream); break;
    case SS_MODE_POINT: points_launch<SPHERE, SS_MODE_POINT>(T, xy, n, img_w, out, stream); break;
    case SS_MODE_UNIFORM:
      points_launch<SPHERE, SS_MODE_UNIFORM>(T, xy, n, img_w, out, stream);
      break;
    default: points_launch<SPHERE, SS_MODE_DP>(T, xy, n, img_w, out, stream); break;
  }
}

hipError_t launch_points(const TileK& T, bool sphere, int mode, const float* xy, long long n,
                         int img_w, float* out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (sphere)
    points_mode<true>(T, mode, xy, n, img_w, out, stream);
  else
    points_mode<false>(T, mode, xy, n, img_w, out, stream);
  return hipGetLastError();
}

static int tile_width_of(int code) {
  switch (code) {
    case SS_TILE_16x4: return 16;
    case SS_TILE_4x16: return 4;
    case SS_TILE_32x2: return 32;
    default: return 8;
  }
}

void grid_for(const TileK& T, int ray_tile, int* nbx, int* nblocks) {
  const int tw = tile_width_of(ray_tile), th = 64 / tw;
  const int bx = (T.RW + 2 * tw - 1) / (2 * tw);
  const int by = (T.RH + 2 * th - 1) / (2 * th);
  *nbx = bx;
  *nblocks = bx * by;
}

template <bool SPHERE, int TW, int MODE>
static void launch_fwd_m(const TileK& T, int flags, float* out, unsigned long long* counter,
                         int* sample, int nbx, int nb, hipStream_t stream) {
  dim3 grid(nb), block(256);
  if (flags == FWD_COUNT)
    hipLaunchKernelGGL((shadow_kernel<SPHERE, TW, MODE, FWD_COUNT>), grid, block, 0, stream, T, out,
                       counter, sample, nbx, nb);
  else if (flags == FWD_SAVE)
    hipLaunchKernelGGL((shadow_kernel<SPHERE, TW, MODE, FWD_SAVE>), grid, block, 0, stream, T, out,
                       counter, sample, nbx, nb);
  else
    hipLaunchKernelGGL((shadow_kernel<SPHERE, TW, MODE, FWD_PLAIN>), grid, block, 0, stream, T, out,
                       counter, sample, nbx, nb);
}

template <bool SPHERE, int TW>
static hipError_t launch_fwd_tw(const TileK& T, int mode, int flags, float* out,
                                unsigned long long* counter, int* sample, hipStream_t stream) {
  int nbx, nb;
  grid_for(T, TW == 16 ? SS_TILE_16x4 : TW == 4 ? SS_TILE_4x16 : TW == 32 ? SS_TILE_32x2 : SS_TILE_8x8,
           &nbx, &nb);
  if (nb == 0) return hipSuccess;
  switch (mode) {
    case SS_MODE_EXACT: launch_fwd_m<SPHERE, TW, SS_MODE_EXACT>(T, flags, out, counter, sample, nbx, nb, stream); break;
    case SS_MODE_POINT: launch_fwd_m<SPHERE, TW, SS_MODE_POINT>(T, flags, out, counter, sample, nbx, nb, stream); break;
    case SS_MODE_UNIFORM: launch_fwd_m<SPHERE, TW, SS_MODE_UNIFORM>(T, flags, out, counter, sample, nbx, nb, stream); break;
    default: launch_fwd_m<SPHERE, TW, SS_MODE_DP>(T, flags, out, counter, sample, nbx, nb, stream); break;
  }
  return hipGetLastError();
}

template <bool SPHERE>
static hipError_t launch_fwd_s(const TileK& T, int mode, int ray_tile, int flags, float* out,
                               unsigned long long* counter, int* sample, hipStream_t stream) {
  switch (ray_tile) {
    case SS_TILE_16x4: return launch_fwd_tw<SPHERE, 16>(T, mode, flags, out, counter, sample, stream);
    case SS_TILE_4x16: return launch_fwd_tw<SPHERE, 4>(T, mode, flags, out, counter, sample, stream);
    case SS_TILE_32x2: return launch_fwd_tw<SPHERE, 32>(T, mode, flags, out, counter, sample, stream);
    default: return launch_fwd_tw<SPHERE, 8>(T, mode, flags, out, counter, sample, stream);
  }
}

hipError_t launch_forward(const TileK& T, bool sphere, int mode, int ray_tile, bool count,
                          float* out, unsigned long long* counter, int* sample,
                          hipStream_t stream) {
  const int flags = count ? FWD_COUNT : (sample ? FWD_SAVE : FWD_PLAIN);
  return sphere ? launch_fwd_s<true>(T, mode, ray_tile, flags, out, counter, sample, stream)
                : launch_fwd_s<false>(T, mode, ray_tile, flags, out, counter, sample, stream);
}

template <bool SPHERE, int MODE>
static void adjoint_launch(const TileK& T, const SunTrig& st, const float* gs, const int* sample,
                           const float* sfwd, float* gh, double* gsun, int nbx, int nb,
                           hipStream_t stream) {
  // the compacting form once the launch has at least 16 device-fulls of its workgroups
  // (2^18 ray blocks, 8192^2 rays): fewer, and the uneven lists leave CUs idle at the end
  if (sfwd && !sample && (long long)nb >= 16LL * SS_PEN_BLOCKS * T.wg_group)
    hipLaunchKernelGGL((adjoint_penumbra_kernel<SPHERE, MODE>),
                       dim3((nb + SS_PEN_BLOCKS - 1) / SS_PEN_BLOCKS), dim3(256), 0, stream, T,
                       st, gs, sfwd, gh, gsun, nbx, nb);
  else if (sample)
    hipLaunchKernelGGL((adjoint_kernel<SPHERE, 8, MODE, true>),
                       dim3((nb + AdjBlocks<true>::n - 1) / AdjBlocks<true>::n), dim3(256), 0,
                       stream, T, st, gs, sample, sfwd, gh, gsun, nbx, nb);
  else
    hipLaunchKernelGGL((adjoint_kernel<SPHERE, 8, MODE, false>), dim3(nb), dim3(256), 0, stream, T,
                       st, gs, sample, sfwd, gh, gsun, nbx, nb);
}

template <bool SPHERE>
static void adjoint_mode(const TileK& T, int mode, const SunTrig& st, const float* gs,
                         const int* sample, const float* sfwd, float* gh, double* gsun, int nbx,
                         int nb, hipStream_t stream) {
  if (mode == SS_MODE_EXACT)
    adjoint_launch<SPHERE, SS_MODE_EXACT>(T, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
  else if (mode == SS_MODE_POINT)
    adjoint_launch<SPHERE, SS_MODE_POINT>(T, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
  else if (mode == SS_MODE_UNIFORM)
    adjoint_launch<SPHERE, SS_MODE_UNIFORM>(T, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
  else
    adjoint_launch<SPHERE, SS_MODE_DP>(T, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
}

hipError_t launch_adjoint(const TileK& T, bool sphere, int mode, double elev, double azim,
                          const float* gs, const int* sample, const float* sfwd, float* gh,
                          double* gsun, hipStream_t stream) {
  SunTrig st;
  st.se = (float)sin(elev);
  st.ce = (float)cos(elev);
  st.sa = (float)sin(azim);
  st.ca = (float)cos(azim);
  st.tan_e = (float)tan(elev);
  int nbx, nb;
  grid_for(T, SS_TILE_8x8, &nbx, &nb);
  if (nb == 0) return hipSuccess;
  if (sphere)
    adjoint_mode<true>(T, mode, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
  else
    adjoint_mode<false>(T, mode, st, gs, sample, sfwd, gh, gsun, nbx, nb, stream);
  return hipGetLastError();
}

}  // namespace ss
