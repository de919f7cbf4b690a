// C ABI of libsoftshadow: validation, FP64 per-(tile, sun) set-up, launches,
// the batched call and its captured-graph plan with the tuner.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace ss;

static thread_local hipError_t g_last_hip = hipSuccess;

static int32_t hip_fail(hipError_t e) {
  g_last_hip = e;
  return SS_ERR_HIP;
}

#define SS_HIP(call)                         \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

// ------------------------------------------------------------------------
// Mipmap layout: level m >= 1 at a 64-float aligned offset.
// ------------------------------------------------------------------------

static int levels_of(int32_t W, int32_t H) {
  const int32_t big = W > H ? W : H;
  int L = 1;
  while ((1LL << (L - 1)) < big) L++;
  return L;
}

static void dims_of(int32_t W, int32_t H, int m, int* w, int* h) {
  int64_t a = W, b = H;
  for (int k = 0; k < m; ++k) {
    a = (a + 1) / 2;
    b = (b + 1) / 2;
  }
  *w = (int)a;
  *h = (int)b;
}

// Each side at most 65536 and fewer than 2^30 texels: the kernels address a
// level through a buffer resource whose size and offsets are 32-bit byte
// counts.
static bool size_ok(int32_t W, int32_t H) {
  return W >= 1 && H >= 1 && W <= 65536 && H <= 65536 && (int64_t)W * H < (1LL << 30);
}

extern "C" int32_t ss_maxmip_levels(int32_t width, int32_t rows) {
  if (!size_ok(width, rows)) return 0;
  return levels_of(width, rows);
}

extern "C" int64_t ss_maxmip_level_offset(int32_t width, int32_t rows, int32_t level) {
  if (!size_ok(width, rows)) return -1;
  const int L = levels_of(width, rows);
  if (level < 1 || level > L) return -1;
  int64_t off = 0;
  for (int m = 1; m < level; ++m) {
    int w, h;
    dims_of(width, rows, m, &w, &h);
    off += ((int64_t)w * h + 63) / 64 * 64;
  }
  return off;
}

extern "C" int64_t ss_maxmip_floats(int32_t width, int32_t rows) {
  if (!size_ok(width, rows)) return -1;
  return ss_maxmip_level_offset(width, rows, levels_of(width, rows));
}

static int32_t maxmip_build(const float* d_height, int32_t W, int32_t H, float* d_mm, int fuse,
                            hipStream_t stream) {
  const int L = levels_of(W, H);
  if (fuse < 1 || fuse > 6) fuse = 6;
  int src_m = 0;
  while (src_m < L - 1) {
    const int F = (L - 1 - src_m) < fuse ? (L - 1 - src_m) : fuse;
    int sw, sh;
    dims_of(W, H, src_m, &sw, &sh);
    const float* src = src_m == 0 ? d_height : d_mm + ss_maxmip_level_offset(W, H, src_m);
    int off[6], w[6], h[6];
    for (int k = 0; k < F; ++k) {
      off[k] = (int)ss_maxmip_level_offset(W, H, src_m + 1 + k);
      dims_of(W, H, src_m + 1 + k, &w[k], &h[k]);
    }
    SS_HIP(launch_maxmip(src, sw, sh, d_mm, off, w, h, F, stream));
    src_m += F;
  }
  return SS_OK;
}

extern "C" int32_t ss_maxmip_build(const float* d_height, int32_t width, int32_t rows,
                                   float* d_maxmip, int32_t fuse_depth, void* stream) {
  if (width == 0 || rows == 0) return (width >= 0 && rows >= 0) ? SS_OK : SS_ERR_INVALID_ARG;
  if (!size_ok(width, rows) || !d_height) return SS_ERR_INVALID_ARG;
  if (fuse_depth < 0 || fuse_depth > 6) return SS_ERR_INVALID_ARG;
  if (ss_maxmip_floats(width, rows) > 0 && !d_maxmip) return SS_ERR_INVALID_ARG;
  return maxmip_build(d_height, width, rows, d_maxmip, fuse_depth ? fuse_depth : 6,
                      (hipStream_t)stream);
}

// ------------------------------------------------------------------------
// Tap-bound pyramid: level 0 then the maximum mipmap of level 0.
// ------------------------------------------------------------------------

static int64_t bound_base(int32_t W, int32_t H) { return ((int64_t)W * H + 63) / 64 * 64; }

extern "C" int64_t ss_bound_floats(int32_t width, int32_t rows) {
  if (!size_ok(width, rows)) return -1;
  return bound_base(width, rows) + ss_maxmip_floats(width, rows);
}

extern "C" int64_t ss_bound_level_offset(int32_t width, int32_t rows, int32_t level) {
  if (!size_ok(width, rows)) return -1;
  if (level == 0) return 0;
  const int64_t o = ss_maxmip_level_offset(width, rows, level);
  return o < 0 ? -1 : bound_base(width, rows) + o;
}

extern "C" int32_t ss_bound_build(const float* d_height, int32_t width, int32_t rows,
                                  float* d_bound, void* stream) {
  if (width == 0 || rows == 0) return (width >= 0 && rows >= 0) ? SS_OK : SS_ERR_INVALID_ARG;
  if (!size_ok(width, rows) || !d_height || !d_bound) return SS_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  SS_HIP(launch_block3_max(d_height, width, rows, d_bound, s));
  return maxmip_build(d_bound, width, rows, d_bound + bound_base(width, rows), 6, s);
}

// ------------------------------------------------------------------------
// Per-(tile, sun) set-up in FP64 (Sec. 3.3 schedule; Appendix step length).
// ------------------------------------------------------------------------

struct Resolved {
  int n_prime0, schedule, n_segments, mode, prune, ray_tile;
  int n_prime_list[16];
  double uniform_step;
  bool sphere;
};

static int32_t resolve_params(const ss_params* p, Resolved* r) {
  if (!p) return SS_ERR_INVALID_ARG;
  if (!(p->body_radius_m > 0.0) || isnan(p->body_radius_m)) return SS_ERR_INVALID_ARG;
  if (isnan(p->max_len_m) || isinf(p->max_len_m)) return SS_ERR_INVALID_ARG;
  if (p->n_prime0 < 0 || p->n_prime0 > 64) return SS_ERR_INVALID_ARG;
  if (p->schedule != SS_SCHED_GEOMETRIC && p->schedule != SS_SCHED_EQUAL &&
      p->schedule != SS_SCHED_LIST)
    return SS_ERR_INVALID_ARG;
  if (p->schedule == SS_SCHED_LIST) {
    if (p->n_segments < 1 || p->n_segments > 16) return SS_ERR_INVALID_ARG;
    for (int k = 0; k < p->n_segments; ++k)
      if (p->n_prime_list[k] < 1 || p->n_prime_list[k] > 64) return SS_ERR_INVALID_ARG;
  }
  if (p->n_segments < 0) return SS_ERR_INVALID_ARG;
  if (p->mode < SS_MODE_DP || p->mode > SS_MODE_POINT) return SS_ERR_INVALID_ARG;
  // 0 = default; otherwise at least 1/64 texel so the step count stays bounded
  if (!(p->uniform_step == 0.0 || p->uniform_step >= 1.0 / 64.0) || isinf(p->uniform_step))
    return SS_ERR_INVALID_ARG;
  if (p->prune != 0 && p->prune != 1) return SS_ERR_INVALID_ARG;
  if (p->ray_tile < 0 || p->ray_tile > SS_TILE_32x2) return SS_ERR_INVALID_ARG;
  r->n_prime0 = p->n_prime0 ? p->n_prime0 : 5;
  r->schedule = p->schedule;
  r->n_segments = p->n_segments;
  r->mode = p->mode;
  r->prune = p->prune;
  r->ray_tile = p->ray_tile ? p->ray_tile : SS_TILE_8x8;
  r->uniform_step = p->uniform_step > 0.0 ? p->uniform_step : 1.0;
  for (int k = 0; k < 16; ++k) r->n_prime_list[k] = p->n_prime_list[k];
  r->sphere = !isinf(p->body_radius_m);
  return SS_OK;
}

static int32_t check_tile(const ss_tile* t, int mode) {
  if (!t) return SS_ERR_INVALID_ARG;
  if (t->width < 0 || t->rows < 0) return SS_ERR_INVALID_ARG;
  if (t->width == 0 || t->rows == 0) return SS_OK;
  if (!size_ok(t->width, t->rows) || !t->height) return SS_ERR_INVALID_ARG;
  if (!(t->texel_m > 0.0) || isinf(t->texel_m)) return SS_ERR_INVALID_ARG;
  if (ss_maxmip_floats(t->width, t->rows) > 0 && !t->maxmip) return SS_ERR_INVALID_ARG;
  if (mode == SS_MODE_EXACT && !t->bound) return SS_ERR_INVALID_ARG;
  const int64_t x0 = t->ray_x0, y0 = t->ray_y0, w = t->ray_w, h = t->ray_h;
  if (!(x0 == 0 && y0 == 0 && w == 0 && h == 0) &&
      (x0 < 0 || y0 < 0 || w < 1 || h < 1 || x0 + w > t->width || y0 + h > t->rows))
    return SS_ERR_INVALID_ARG;
  return SS_OK;
}

static int32_t check_sun(const ss_sun* s) {
  if (!s) return SS_ERR_INVALID_ARG;
  if (!(fabs(s->elev_rad) < 0.5 * M_PI)) return SS_ERR_INVALID_ARG;
  if (!isfinite(s->azim_rad)) return SS_ERR_INVALID_ARG;
  if (!(s->ang_radius_rad > 0.0) || !(s->ang_radius_rad < 0.5)) return SS_ERR_INVALID_ARG;
  return SS_OK;
}

// Workgroups of 256 lanes one device holds at once (8 per CU at 8 wavefronts
// per SIMD): the per-tile kernels remap workgroup ids within groups of this
// many.  Cached per device.
static int device_wg_group() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 2048;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 256;
  v = 8 * ncu;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

static int32_t make_tilek(const ss_tile* t, const ss_sun* s, const Resolved& rp, double max_len_m,
                          double radius, TileK* K) {
  memset(K, 0, sizeof(*K));
  K->wg_group = device_wg_group();
  const int W = t->width, H = t->rows;
  const int L = levels_of(W, H);
  if (L > SS_MAXLEV) return SS_ERR_UNSUPPORTED;
  K->h = t->height;
  K->mm = t->maxmip;
  K->bnd = t->bound;
  K->bmm = t->bound ? t->bound + bound_base(W, H) : nullptr;
  K->W = W;
  K->H = H;
  K->L = L;
  const bool whole = t->ray_w == 0 && t->ray_h == 0;
  K->rx0 = whole ? 0 : t->ray_x0;
  K->ry0 = whole ? 0 : t->ray_y0;
  K->RW = whole ? W : t->ray_w;
  K->RH = whole ? H : t->ray_h;
  for (int m = 0; m < L; ++m) {
    dims_of(W, H, m, &K->lw[m], &K->lh[m]);
    K->loff[m] = m == 0 ? 0 : (int)ss_maxmip_level_offset(W, H, m);
  }
  const double e = s->elev_rad, a = s->azim_rad;
  const double ce = cos(e);
  const double Lx = ce * cos(a), Ly = ce * sin(a), Lz = sin(e);
  const double delta = t->texel_m / ce;  // ray length per texel of horizontal travel
  K->texel = (float)t->texel_m;
  K->invR = rp.sphere ? (float)(1.0 / radius) : 0.0f;
  K->Lx = (float)Lx;
  K->Ly = (float)Ly;
  K->Lz = (float)Lz;
  K->half_delta = (float)(0.5 * delta);
  K->two_over_delta = (float)(2.0 / delta);
  K->rL = (float)s->ang_radius_rad;
  K->inv_rL = (float)(1.0 / s->ang_radius_rad);
  K->prune_margin = 1e-5f;
  K->tan_rL = (float)tan(s->ang_radius_rad);
  K->tan_margin = (float)tan(1e-5);
  K->prune = rp.prune;
  K->ustep = (float)(rp.uniform_step * delta);

  // concatenated runs: run j traces N'_j levels (top level N'_j - 1) and
  // covers 2^(N'_j - 1) texels of travel; enough runs to reach the cap, or
  // to span the tile diagonal without one
  // run j starts at half-texel grid index a0_j, i.e. at ray length
  // tau_j = (a0_j + 1) delta/2 (run_start_len)
  const double need = max_len_m > 0.0 ? max_len_m / t->texel_m
                                      : sqrt((double)W * W + (double)H * H) + 2.0;
  const double half_delta = 0.5 * delta;
  double covered = 0.0;
  int j = 0, ga = 0;
  for (;;) {
    if (j >= SS_MAXSEG) return SS_ERR_UNSUPPORTED;
    int np = rp.schedule == SS_SCHED_EQUAL ? rp.n_prime0 : rp.n_prime0 + j;
    if (rp.schedule == SS_SCHED_LIST) np = rp.n_prime_list[j];
    if (np > L) np = L;
    if (np < 1) np = 1;
    K->m0[j] = np - 1;
    K->a0[j] = ga;
    K->tau[j] = run_start_len(ga, half_delta);
    ga += 2 << K->m0[j];
    covered += ldexp(1.0, np - 1);
    j++;
    if (rp.n_segments > 0 ? j >= rp.n_segments : covered >= need) break;
  }
  K->nseg = j;
  K->tau[j] = run_start_len(ga, half_delta);
  const double tau = (double)(ga + 1) * half_delta;
  // uniform steps stop at the cap, or without one at the tile edge and at the
  // latest after the runs' extent (the tile diagonal)
  K->ucap = max_len_m > 0.0 ? (float)(max_len_m / t->texel_m * delta) : (float)tau;
  if (rp.sphere) {
    // the texture-space projection needs 1 + c t > 0 along every ray
    const double half_ext = 0.5 * sqrt((double)W * W + (double)H * H) * t->texel_m;
    const double cmax = fabs(Lz) * sqrt(1.0 + half_ext * half_ext / (radius * radius)) / radius * 1.01;
    const double tmax = fmax(tau, (double)K->ucap);
    if (Lz < 0.0 && isfinite(tmax) && cmax * tmax > 0.5) return SS_ERR_UNSUPPORTED;
  }
  return SS_OK;
}

// ------------------------------------------------------------------------
// Per-tile entry points.
// ------------------------------------------------------------------------

static int32_t cast_common(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                           float* d_shadow, unsigned long long* counter, int32_t* d_sample,
                           void* stream) {
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  if ((rc = check_tile(tile, rp.mode))) return rc;
  if ((rc = check_sun(sun))) return rc;
  if (tile->width == 0 || tile->rows == 0) return SS_OK;
  if (!d_shadow) return SS_ERR_INVALID_ARG;
  TileK K;
  if ((rc = make_tilek(tile, sun, rp, params->max_len_m, params->body_radius_m, &K))) return rc;
  SS_HIP(launch_forward(K, rp.sphere, rp.mode, rp.ray_tile, counter != nullptr, d_shadow, counter,
                        d_sample, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_shadow_cast(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                                  float* d_shadow, void* stream) {
  return cast_common(tile, sun, params, d_shadow, nullptr, nullptr, stream);
}

extern "C" int32_t ss_shadow_cast_counted(const ss_tile* tile, const ss_sun* sun,
                                          const ss_params* params, float* d_shadow,
                                          unsigned long long* d_eval_count, void* stream) {
  if (!d_eval_count) return SS_ERR_INVALID_ARG;
  return cast_common(tile, sun, params, d_shadow, d_eval_count, nullptr, stream);
}

extern "C" int32_t ss_shadow_cast_save(const ss_tile* tile, const ss_sun* sun,
                                       const ss_params* params, float* d_shadow,
                                       int32_t* d_sample, void* stream) {
  if (!d_sample && tile && tile->width > 0 && tile->rows > 0) return SS_ERR_INVALID_ARG;
  return cast_common(tile, sun, params, d_shadow, nullptr, d_sample, stream);
}

static int32_t backward_common(const ss_tile* tile, const ss_sun* sun, const ss_params* params,
                               const int32_t* d_sample, const float* d_shadow,
                               const float* d_grad_shadow, float* d_grad_height,
                               double* d_grad_sun, void* stream) {
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  if ((rc = check_tile(tile, rp.mode))) return rc;
  if ((rc = check_sun(sun))) return rc;
  if (tile->width == 0 || tile->rows == 0) return SS_OK;
  if (!d_grad_shadow || !d_grad_height || !d_grad_sun) return SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_grad_sun) & 7) != 0) return SS_ERR_INVALID_ARG;
  TileK K;
  if ((rc = make_tilek(tile, sun, rp, params->max_len_m, params->body_radius_m, &K))) return rc;
  SS_HIP(launch_adjoint(K, rp.sphere, rp.mode, sun->elev_rad, sun->azim_rad, d_grad_shadow,
                        d_sample, d_shadow, d_grad_height, d_grad_sun, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_shadow_points(const ss_tile* tile, const ss_sun* sun,
                                    const ss_params* params, const float* d_xy, int64_t n,
                                    float* d_shadow, void* stream) {
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  if ((rc = check_tile(tile, rp.mode))) return rc;
  if ((rc = check_sun(sun))) return rc;
  if (n < 0 || n > SS_MAX_POINTS || (n > 0 && (!d_xy || !d_shadow))) return SS_ERR_INVALID_ARG;
  if (n == 0 || tile->width == 0 || tile->rows == 0) return n == 0 ? SS_OK : SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_xy) & 7) != 0) return SS_ERR_INVALID_ARG;
  TileK K;
  if ((rc = make_tilek(tile, sun, rp, params->max_len_m, params->body_radius_m, &K))) return rc;
  SS_HIP(launch_points(K, rp.sphere, rp.mode, d_xy, n, 0, d_shadow, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_shadow_points_backward(const ss_tile* tile, const ss_sun* sun,
                                             const ss_params* params, const float* d_xy,
                                             int64_t n, int32_t width,
                                             const float* d_grad_shadow, float* d_grad_height,
                                             double* d_grad_sun, void* stream) {
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  if ((rc = check_tile(tile, rp.mode))) return rc;
  if ((rc = check_sun(sun))) return rc;
  if (n < 0 || n > SS_MAX_POINTS || width < 0 || width > 16384) return SS_ERR_INVALID_ARG;
  if (n == 0) return SS_OK;
  if (width > 0 && (n % width != 0 || n / width > 16384)) return SS_ERR_INVALID_ARG;
  if (!d_xy || !d_grad_shadow || !d_grad_height || !d_grad_sun) return SS_ERR_INVALID_ARG;
  if (tile->width == 0 || tile->rows == 0) return SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_xy) & 7) != 0) return SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_grad_sun) & 7) != 0) return SS_ERR_INVALID_ARG;
  TileK K;
  if ((rc = make_tilek(tile, sun, rp, params->max_len_m, params->body_radius_m, &K))) return rc;
  SS_HIP(launch_points_adjoint(K, rp.sphere, rp.mode, sun->elev_rad, sun->azim_rad, d_xy, n, width,
                               d_grad_shadow, d_grad_height, d_grad_sun, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_shadow_points_image(const ss_tile* tile, const ss_sun* sun,
                                          const ss_params* params, const float* d_xy,
                                          int32_t width, int32_t height, float* d_shadow,
                                          void* stream) {
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  if ((rc = check_tile(tile, rp.mode))) return rc;
  if ((rc = check_sun(sun))) return rc;
  if (width < 1 || height < 1 || width > 16384 || height > 16384) return SS_ERR_INVALID_ARG;
  if (!d_xy || !d_shadow || tile->width == 0 || tile->rows == 0) return SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_xy) & 7) != 0) return SS_ERR_INVALID_ARG;
  TileK K;
  if ((rc = make_tilek(tile, sun, rp, params->max_len_m, params->body_radius_m, &K))) return rc;
  SS_HIP(launch_points(K, rp.sphere, rp.mode, d_xy, (long long)width * height, width, d_shadow,
                       (hipStream_t)stream));
  return SS_OK;
}

static bool finite3(const double* v) {
  return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
}

extern "C" int32_t ss_view_cast(const ss_tile* tile, double body_radius_m, const ss_camera* cam,
                                float* d_t, float* d_xy, int32_t* d_steps, void* stream) {
  if (!tile || !cam) return SS_ERR_INVALID_ARG;
  // heights and the bound pyramid are read; the max-mip and the ray window are not
  if (!size_ok(tile->width, tile->rows) || !tile->height || !tile->bound) return SS_ERR_INVALID_ARG;
  if (!(tile->texel_m > 0.0) || isinf(tile->texel_m)) return SS_ERR_INVALID_ARG;
  if (!(body_radius_m > 0.0)) return SS_ERR_INVALID_ARG;
  const bool sphere = !isinf(body_radius_m);
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
    return SS_ERR_INVALID_ARG;
  if (!finite3(cam->eye_m) || !finite3(cam->fwd) || !finite3(cam->right) || !finite3(cam->up))
    return SS_ERR_INVALID_ARG;
  if (cam->fwd[0] == 0.0 && cam->fwd[1] == 0.0 && cam->fwd[2] == 0.0) return SS_ERR_INVALID_ARG;
  const double eyen = sqrt(cam->eye_m[0] * cam->eye_m[0] + cam->eye_m[1] * cam->eye_m[1] +
                           cam->eye_m[2] * cam->eye_m[2]);
  if (sphere && !(eyen < 0.25 * body_radius_m)) return SS_ERR_INVALID_ARG;
  if (!(cam->step_m >= tile->texel_m / 64.0) || !isfinite(cam->step_m)) return SS_ERR_INVALID_ARG;
  if (!(cam->far_m <= 0.0) && !(cam->far_m > 0.0 && isfinite(cam->far_m)))
    return SS_ERR_INVALID_ARG;
  if (cam->mode != SS_VIEW_HIER && cam->mode != SS_VIEW_DENSE) return SS_ERR_INVALID_ARG;
  if (!d_t || !d_xy) return SS_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(d_xy) & 7) != 0 ||
      (reinterpret_cast<uintptr_t>(d_steps) & 7) != 0)
    return SS_ERR_INVALID_ARG;
  const int W = tile->width, H = tile->rows, L = levels_of(W, H);
  if (L > SS_MAXLEV) return SS_ERR_UNSUPPORTED;
  ViewK K;
  memset(&K, 0, sizeof(K));
  K.h = tile->height;
  K.bnd = tile->bound;
  K.bmm = tile->bound + bound_base(W, H);
  K.W = W;
  K.H = H;
  K.L = L;
  for (int m = 0; m < L; ++m) {
    dims_of(W, H, m, &K.lw[m], &K.lh[m]);
    K.loff[m] = m == 0 ? 0 : (int)ss_maxmip_level_offset(W, H, m);
    K.inv_pow2[m] = (float)ldexp(1.0, -m);
  }
  K.texel = (float)tile->texel_m;
  K.invT = (float)(1.0 / tile->texel_m);
  K.R = sphere ? (float)body_radius_m : 0.0f;
  K.invR = sphere ? (float)(1.0 / body_radius_m) : 0.0f;
  K.cx0 = (float)(0.5 * W);
  K.cy0 = (float)(0.5 * H);
  K.ex = (float)cam->eye_m[0];
  K.ey = (float)cam->eye_m[1];
  K.ez = (float)cam->eye_m[2];
  K.fx = (float)cam->fwd[0];
  K.fy = (float)cam->fwd[1];
  K.fz = (float)cam->fwd[2];
  K.rx = (float)cam->right[0];
  K.ry = (float)cam->right[1];
  K.rz = (float)cam->right[2];
  K.ux = (float)cam->up[0];
  K.uy = (float)cam->up[1];
  K.uz = (float)cam->up[2];
  K.img_w = cam->width;
  K.img_h = cam->height;
  K.nbx = (cam->width + 15) / 16;
  K.nby = (cam->height + 15) / 16;
  K.inv_w2 = (float)(2.0 / cam->width);
  K.inv_h2 = (float)(2.0 / cam->height);
  K.step = (float)cam->step_m;
  K.inv_step = (float)(1.0 / (double)K.step);
  K.far = cam->far_m > 0.0 ? (float)cam->far_m : INFINITY;
  // The skip test compares the ray's lowest FP32 height over a cell with the
  // cell's bound; the margin covers FP32 rounding of heights (absolute
  // heights of a few km: a few ulps of 1e-3 m), of the ray point (relative
  // 1e-7 of |eye| + t) and of the sample positions against the cell limits.
  K.m_abs = 1e-2f;
  K.m_rel = 2e-6f;
  K.max_iter = 4 * (W + H + 8) * (L + 2) + 64;
  K.max_samples = 1 << 26;
  SS_HIP(launch_view(K, sphere, cam->mode, d_t, d_xy, d_steps, (hipStream_t)stream));
  return SS_OK;
}

static bool frame_ok(const ss_frame* f) {
  if (!f || !size_ok(f->width, f->rows)) return false;
  if (!(f->texel_m > 0.0) || isinf(f->texel_m)) return false;
  if (!finite3(f->centre) || !finite3(f->ex) || !finite3(f->ey)) return false;
  if (!isfinite(f->origin_m[0]) || !isfinite(f->origin_m[1])) return false;
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  const double tol = 1e-9;
  if (fabs(dot(f->centre, f->centre) - 1.0) > tol || fabs(dot(f->ex, f->ex) - 1.0) > tol ||
      fabs(dot(f->ey, f->ey) - 1.0) > tol)
    return false;
  if (fabs(dot(f->centre, f->ex)) > tol || fabs(dot(f->centre, f->ey)) > tol ||
      fabs(dot(f->ex, f->ey)) > tol)
    return false;
  return true;
}

extern "C" int32_t ss_resample(const float* d_src, const ss_frame* src, float* d_dst,
                               const ss_frame* dst, double body_radius_m, void* stream) {
  if (!d_src || !d_dst || !frame_ok(src) || !frame_ok(dst)) return SS_ERR_INVALID_ARG;
  if (!(body_radius_m > 0.0) || isinf(body_radius_m)) return SS_ERR_INVALID_ARG;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(d_src);
  const uintptr_t a1 = a0 + (uintptr_t)src->width * (uintptr_t)src->rows * 4u;
  const uintptr_t b0 = reinterpret_cast<uintptr_t>(d_dst);
  const uintptr_t b1 = b0 + (uintptr_t)dst->width * (uintptr_t)dst->rows * 4u;
  if (a0 < b1 && b0 < a1) return SS_ERR_INVALID_ARG;
  ResampleK K;
  memset(&K, 0, sizeof(K));
  K.src = d_src;
  K.dst = d_dst;
  K.Ws = src->width;
  K.Hs = src->rows;
  K.Wd = dst->width;
  K.Hd = dst->rows;
  K.R = body_radius_m;
  for (int k = 0; k < 3; ++k) {
    K.cd[k] = dst->centre[k];
    K.exd[k] = dst->ex[k];
    K.eyd[k] = dst->ey[k];
    K.cs[k] = src->centre[k];
    K.exs[k] = src->ex[k];
    K.eys[k] = src->ey[k];
  }
  K.oxd = dst->origin_m[0];
  K.oyd = dst->origin_m[1];
  K.Dd = dst->texel_m;
  K.oxs = src->origin_m[0];
  K.oys = src->origin_m[1];
  K.Ds = src->texel_m;
  SS_HIP(launch_resample(K, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_probe_gather(const float* d_src, int64_t n_floats, int64_t window,
                                   int32_t iters, float* d_out, int64_t n_threads, void* stream) {
  if (!d_src || !d_out || n_floats < 1 || n_floats > (1LL << 32) || iters < 1) return SS_ERR_INVALID_ARG;
  if (n_threads < 256 || n_threads % 256 != 0 || n_threads / 256 > 0x7fffffffLL) return SS_ERR_INVALID_ARG;
  if (window < 0 || (window > 0 && ((window & (window - 1)) != 0 || window > n_floats)))
    return SS_ERR_INVALID_ARG;
  SS_HIP(launch_gather_probe(d_src, n_floats, window, iters, d_out, n_threads, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_probe_gather_tiles(const float* d_src, int32_t width, int32_t rows,
                                         int32_t iters, float* d_out, int64_t n_threads,
                                         void* stream) {
  if (!d_src || !d_out || width < 8 || rows < 8 || width > 65536 || rows > 65536 || iters < 1)
    return SS_ERR_INVALID_ARG;
  if (n_threads < 256 || n_threads % 256 != 0 || n_threads / 256 > 0x7fffffffLL) return SS_ERR_INVALID_ARG;
  SS_HIP(launch_gather_tiles_probe(d_src, width, rows, iters, d_out, n_threads, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_probe_valu(int32_t iters, int64_t n_workgroups, float* d_out, void* stream) {
  if (!d_out || iters < 1 || n_workgroups < 1 || n_workgroups > 0x7fffffffLL) return SS_ERR_INVALID_ARG;
  SS_HIP(launch_valu_probe(iters, n_workgroups, d_out, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_shadow_cast_backward(const ss_tile* tile, const ss_sun* sun,
                                           const ss_params* params, const float* d_grad_shadow,
                                           float* d_grad_height, double* d_grad_sun, void* stream) {
  return backward_common(tile, sun, params, nullptr, nullptr, d_grad_shadow, d_grad_height,
                         d_grad_sun, stream);
}

extern "C" int32_t ss_shadow_cast_backward_penumbra(const ss_tile* tile, const ss_sun* sun,
                                                    const ss_params* params, const float* d_shadow,
                                                    const float* d_grad_shadow,
                                                    float* d_grad_height, double* d_grad_sun,
                                                    void* stream) {
  if (!d_shadow && tile && tile->width > 0 && tile->rows > 0) return SS_ERR_INVALID_ARG;
  return backward_common(tile, sun, params, nullptr, d_shadow, d_grad_shadow, d_grad_height,
                         d_grad_sun, stream);
}

extern "C" int32_t ss_shadow_cast_backward_saved(const ss_tile* tile, const ss_sun* sun,
                                                 const ss_params* params, const int32_t* d_sample,
                                                 const float* d_grad_shadow, float* d_grad_height,
                                                 double* d_grad_sun, void* stream) {
  if (!d_sample && tile && tile->width > 0 && tile->rows > 0) return SS_ERR_INVALID_ARG;
  return backward_common(tile, sun, params, d_sample, nullptr, d_grad_shadow, d_grad_height,
                         d_grad_sun, stream);
}

// ------------------------------------------------------------------------
// Batched form.
// ------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: SS_NXCD queue counters, the tables the batched kernels read (pair
// parameter blocks, output pointers, block prefix sums, per-XCD queue prefix
// sums, block-grid widths), then the staged compact image they are expanded
// from (per-tile templates and records, per-pair records).
struct WsLayout {
  size_t counter, pairs, outs, start, xstart, nbx, tmpl, stile, spair, total;
};

static bool ws_layout(int32_t n_tiles, int32_t n_suns, WsLayout* L) {
  if (n_tiles < 0 || n_suns < 0 || (int64_t)n_tiles * n_suns > 1000000) return false;
  const size_t np = (size_t)n_tiles * n_suns;
  L->counter = 0;
  L->pairs = 256;
  L->outs = L->pairs + align256(np * sizeof(TileK));
  L->start = L->outs + align256(np * sizeof(float*));
  L->xstart = L->start + align256((np + 1) * sizeof(long long));
  L->nbx = L->xstart + align256((size_t)SS_NXCD * (np + 1) * sizeof(long long));
  L->tmpl = L->nbx + align256(np * sizeof(int));
  L->stile = L->tmpl + align256((size_t)n_tiles * sizeof(TileK));
  L->spair = L->stile + align256(((size_t)n_tiles + 1) * sizeof(StageTile));
  L->total = L->spair + align256(np * sizeof(StagePair));
  return true;
}

extern "C" int64_t ss_batched_workspace_bytes(int32_t n_tiles, int32_t n_suns) {
  WsLayout L;
  if (!ws_layout(n_tiles, n_suns, &L)) return -1;
  return (int64_t)L.total;
}

// Host side of a batch: its description and the compact image to stage.
struct BatchImage {
  std::vector<TileK> tmpl;       // per tile: the set-up for its first sun
  std::vector<StageTile> stile;  // per tile + totals
  std::vector<StagePair> spair;  // per (tile, sun)
  BatchDesc bd;
  Resolved rp;
};

// Forms the FP64 set-up of every (tile, sun) pair on the host; each pair's
// parameter block equals make_tilek's for that pair (the expand kernel rebuilds
// it from the tile's template, the pair's sun fields and its run starts).
static int32_t build_image(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                           int32_t n_suns, const ss_params* params, float* const* d_shadow,
                           int ray_tile, BatchImage* bi) {
  int32_t rc;
  if ((rc = resolve_params(params, &bi->rp))) return rc;
  if (ray_tile) bi->rp.ray_tile = ray_tile;
  const size_t np = (size_t)n_tiles * n_suns;
  bi->tmpl.assign(n_tiles, TileK());
  bi->stile.assign((size_t)n_tiles + 1, StageTile());
  bi->spair.assign(np, StagePair());
  long long items = 0, xq[SS_NXCD] = {0};
  for (int t = 0; t < n_tiles; ++t) {
    StageTile& st = bi->stile[t];
    st.start = items;
    for (int x = 0; x < SS_NXCD; ++x) st.xt[x] = xq[x];
    for (int k = 0; k < n_suns; ++k) {
      const size_t p = (size_t)t * n_suns + k;
      TileK K;
      if ((rc = make_tilek(&tiles[t], &suns[k], bi->rp, params->max_len_m, params->body_radius_m,
                           &K)))
        return rc;
      if (k == 0) {
        bi->tmpl[t] = K;
        int nbx, nb;
        grid_for(K, bi->rp.ray_tile, &nbx, &nb);
        st.nbx = nbx;
        st.items = (nb + SS_ITEM_BLOCKS - 1) / SS_ITEM_BLOCKS;
      }
      StagePair& sp = bi->spair[p];
      memcpy(sp.sun, &K.Lx, sizeof(sp.sun));
      sp.half_delta = 0.5 * (tiles[t].texel_m / cos(suns[k].elev_rad));
      sp.out = d_shadow[p];
    }
    items += (long long)n_suns * st.items;
    // queue x holds band x of every pair: [x n / SS_NXCD, (x + 1) n / SS_NXCD) of its n items
    for (int x = 0; x < SS_NXCD; ++x)
      xq[x] += (long long)n_suns *
               ((long long)(x + 1) * st.items / SS_NXCD - (long long)x * st.items / SS_NXCD);
  }
  StageTile& tot = bi->stile[n_tiles];
  tot.start = items;
  for (int x = 0; x < SS_NXCD; ++x) tot.xt[x] = xq[x];
  bi->bd.n_pairs = (int)np;
  bi->bd.n_tiles = n_tiles;
  bi->bd.n_suns = n_suns;
  bi->bd.total_items = items;
  return SS_OK;
}

// Enqueues the staging of the image and its expansion into the tables.
static int32_t stage_image(const BatchImage& bi, unsigned char* ws, hipStream_t s) {
  WsLayout L;
  ws_layout(bi.bd.n_tiles, bi.bd.n_suns, &L);
  SS_HIP(launch_stage(ws + L.tmpl, bi.tmpl.data(), bi.tmpl.size() * sizeof(TileK), s));
  SS_HIP(launch_stage(ws + L.stile, bi.stile.data(), bi.stile.size() * sizeof(StageTile), s));
  SS_HIP(launch_stage(ws + L.spair, bi.spair.data(), bi.spair.size() * sizeof(StagePair), s));
  SS_HIP(launch_expand(reinterpret_cast<const TileK*>(ws + L.tmpl),
                       reinterpret_cast<const StageTile*>(ws + L.stile),
                       reinterpret_cast<const StagePair*>(ws + L.spair), bi.bd.n_tiles,
                       bi.bd.n_suns, reinterpret_cast<TileK*>(ws + L.pairs),
                       reinterpret_cast<float**>(ws + L.outs),
                       reinterpret_cast<long long*>(ws + L.start),
                       reinterpret_cast<long long*>(ws + L.xstart),
                       reinterpret_cast<int*>(ws + L.nbx), s));
  return SS_OK;
}

static int32_t check_batch(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns, int32_t n_suns,
                           const ss_params* params, float* const* d_shadow) {
  if (n_tiles < 0 || n_suns < 0) return SS_ERR_INVALID_ARG;
  if (n_tiles == 0 || n_suns == 0) return SS_OK;
  if (!tiles || !suns || !params || !d_shadow) return SS_ERR_INVALID_ARG;
  Resolved rp;
  int32_t rc = resolve_params(params, &rp);
  if (rc) return rc;
  for (int t = 0; t < n_tiles; ++t) {
    if ((rc = check_tile(&tiles[t], rp.mode))) return rc;
    if (tiles[t].width == 0 || tiles[t].rows == 0) return SS_ERR_INVALID_ARG;
  }
  for (int k = 0; k < n_suns; ++k)
    if ((rc = check_sun(&suns[k]))) return rc;
  for (int64_t p = 0; p < (int64_t)n_tiles * n_suns; ++p)
    if (!d_shadow[p]) return SS_ERR_INVALID_ARG;
  if (ss_batched_workspace_bytes(n_tiles, n_suns) < 0) return SS_ERR_INVALID_ARG;
  return SS_OK;
}

static int32_t check_workspace(int32_t n_tiles, int32_t n_suns, const void* d_workspace,
                               int64_t ws_bytes) {
  const int64_t need = ss_batched_workspace_bytes(n_tiles, n_suns);
  if (!d_workspace || ws_bytes < need) return SS_ERR_WORKSPACE;
  if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) return SS_ERR_WORKSPACE;
  return SS_OK;
}

// The batched call's form: flat (one workgroup per ray block of every pair;
// the default) or, with SS_BATCH_FORM=persistent in the environment, the
// persistent kernel with per-XCD queues.  Batches of 2^31 blocks or more always
// take the persistent form.  Both give the same outputs bit for bit.
static bool batch_persistent() {
  const char* e = getenv("SS_BATCH_FORM");
  return e && strcmp(e, "persistent") == 0;
}

// Maximum mipmaps (and, in the exact mode, tap-bound pyramids) of every tile,
// then the batched launch over tables already in the workspace.
static int32_t enqueue_batch(const ss_tile* tiles, int32_t n_tiles, const BatchDesc& bd,
                             const Resolved& rp, unsigned char* ws, int fuse, int n_wg,
                             hipStream_t stream) {
  WsLayout L;
  ws_layout(n_tiles, bd.n_suns, &L);
  for (int t = 0; t < n_tiles; ++t) {
    int32_t rc = maxmip_build(tiles[t].height, tiles[t].width, tiles[t].rows, tiles[t].maxmip,
                              fuse, stream);
    if (rc) return rc;
    // the exact mode also reads each tile's tap-bound pyramid (sun-independent)
    if (rp.mode == SS_MODE_EXACT &&
        (rc = ss_bound_build(tiles[t].height, tiles[t].width, tiles[t].rows, tiles[t].bound,
                             stream)))
      return rc;
  }
  if (!batch_persistent() && bd.total_items < (1LL << 31)) {
    SS_HIP(launch_batched_flat(reinterpret_cast<const TileK*>(ws + L.pairs),
                               reinterpret_cast<float* const*>(ws + L.outs),
                               reinterpret_cast<const long long*>(ws + L.start),
                               reinterpret_cast<const int*>(ws + L.nbx), bd, device_wg_group(),
                               rp.sphere, rp.mode, rp.ray_tile, stream));
    return SS_OK;
  }
  SS_HIP(launch_fill_u32(reinterpret_cast<unsigned int*>(ws + L.counter), 0u, SS_NXCD, stream));
  SS_HIP(launch_batched(reinterpret_cast<const TileK*>(ws + L.pairs),
                        reinterpret_cast<float* const*>(ws + L.outs),
                        reinterpret_cast<const long long*>(ws + L.start),
                        reinterpret_cast<const long long*>(ws + L.xstart),
                        reinterpret_cast<const int*>(ws + L.nbx),
                        reinterpret_cast<unsigned int*>(ws + L.counter), bd, rp.sphere, rp.mode,
                        rp.ray_tile, n_wg, stream));
  return SS_OK;
}

// The whole batched call on a workspace: stage, expand, build, launch; only
// kernel launches, so it runs unchanged under a caller's stream capture.
static int32_t batched_on(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                          int32_t n_suns, const ss_params* params, float* const* d_shadow,
                          unsigned char* ws, hipStream_t s) {
  BatchImage bi;
  int32_t rc = build_image(tiles, n_tiles, suns, n_suns, params, d_shadow, 0, &bi);
  if (rc) return rc;
  if ((rc = stage_image(bi, ws, s))) return rc;
  const bool persistent = batch_persistent() || bi.bd.total_items >= (1LL << 31);
  const int n_wg = persistent ? batched_workgroups(bi.rp.sphere, bi.rp.mode, bi.rp.ray_tile) : 0;
  return enqueue_batch(tiles, n_tiles, bi.bd, bi.rp, ws, 6, n_wg, s);
}

extern "C" int32_t ss_shadow_cast_batched(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                                          int32_t n_suns, const ss_params* params,
                                          float* const* d_shadow, void* d_workspace,
                                          int64_t workspace_bytes, void* stream) {
  int32_t rc = check_batch(tiles, n_tiles, suns, n_suns, params, d_shadow);
  if (rc) return rc;
  if (n_tiles == 0 || n_suns == 0) return SS_OK;
  if ((rc = check_workspace(n_tiles, n_suns, d_workspace, workspace_bytes))) return rc;
  return batched_on(tiles, n_tiles, suns, n_suns, params, d_shadow,
                    static_cast<unsigned char*>(d_workspace), (hipStream_t)stream);
}

// ------------------------------------------------------------------------
// Batched call without a caller workspace: the tables live in a fixed
// library-owned device array (one per GPU, held until the process ends).
// ------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[SS_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each device, looked up once per device with
// that device current (in host code the array's name is only a stand-in).
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static int32_t scratch_on_current_device(unsigned char** out) {
  int dev = 0;
  SS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return SS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    SS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return SS_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return SS_OK;
}

extern "C" int32_t ss_shadow_cast_batched_noalloc(const ss_tile* tiles, int32_t n_tiles,
                                                  const ss_sun* suns, int32_t n_suns,
                                                  const ss_params* params, float* const* d_shadow,
                                                  void* stream) {
  int32_t rc = check_batch(tiles, n_tiles, suns, n_suns, params, d_shadow);
  if (rc) return rc;
  if (n_tiles == 0 || n_suns == 0) return SS_OK;
  if (ss_batched_workspace_bytes(n_tiles, n_suns) > (int64_t)SS_NOALLOC_SCRATCH_BYTES)
    return SS_ERR_WORKSPACE;
  unsigned char* ws = nullptr;
  if ((rc = scratch_on_current_device(&ws))) return rc;
  return batched_on(tiles, n_tiles, suns, n_suns, params, d_shadow, ws, (hipStream_t)stream);
}

// ------------------------------------------------------------------------
// Tuner and captured plan.
// ------------------------------------------------------------------------

struct TuneKey {
  std::string s;
  bool operator<(const TuneKey& o) const { return s < o.s; }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, std::pair<int, int>> g_tune;

// Persistent tuner results: with SS_TUNE_CACHE naming a file, choices are read
// from it once per process and each new one is appended, one JSON object per
// line: {"key": "...", "ray_tile": n, "fuse_depth": f}.  Keys start with the
// device's architecture name.  Unreadable lines and out-of-range choices are
// ignored (the tuner then runs again); the choices never change results.
static std::once_flag g_tune_file_once;

static void tune_file_load() {
  const char* path = getenv("SS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[1024], key[900];
  int rt = 0, fd = 0;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (fgets(line, sizeof line, f)) {
    if (sscanf(line, " {\"key\": \"%899[^\"]\", \"ray_tile\": %d, \"fuse_depth\": %d}", key, &rt,
               &fd) != 3)
      continue;
    if (rt < SS_TILE_8x8 || rt > SS_TILE_32x2 || fd < 1 || fd > 6) continue;
    g_tune.emplace(TuneKey{key}, std::make_pair(rt, fd));
  }
  fclose(f);
}

static void tune_file_append(const std::string& key, int rt, int fd) {
  const char* path = getenv("SS_TUNE_CACHE");
  if (!path || !*path || key.size() >= 900 || key.find('"') != std::string::npos) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"ray_tile\": %d, \"fuse_depth\": %d}\n", key.c_str(), rt, fd);
  fclose(f);
}

static std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  return std::string(prop.gcnArchName);
}

static std::string tune_key(const ss_tile* tiles, int n_tiles, int n_suns, const Resolved& rp,
                            const ss_params* p) {
  char buf[128];
  std::string k = arch_name() + "|";
  snprintf(buf, sizeof buf, "m%d s%d n%d g%d q%d r%.3g c%.3g|", rp.mode, rp.sphere, rp.n_prime0,
           rp.schedule, rp.prune, p->body_radius_m, p->max_len_m);
  k += buf;
  for (int t = 0; t < n_tiles; ++t) {
    snprintf(buf, sizeof buf, "%dx%d@%.4g,", tiles[t].width, tiles[t].rows, tiles[t].texel_m);
    k += buf;
  }
  snprintf(buf, sizeof buf, "|%d|%s", n_suns, batch_persistent() ? "persistent" : "flat");
  return k + buf;
}

// Milliseconds between two recorded events; a HIP error comes back as such.
static hipError_t time_ms(hipEvent_t a, hipEvent_t b, double* out) {
  float ms = 0.0f;
  hipError_t e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  *out = ms;
  return e;
}

// Two timing events, released on every path out of the tuner (a destructor
// cannot report the release's own status, so that one is dropped).
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Times each fusion depth on the largest tile's mipmap, and each ray-tile shape
// with the batched kernel itself on the largest tile and up to 8 of the suns
// (spread over the list); the choices never change results.
static int32_t tune(const ss_tile* tiles, int n_tiles, const ss_sun* suns, int n_suns,
                    const ss_params* params, float* const* d_shadow, unsigned char* ws,
                    hipStream_t s, int* best_tile, int* best_fuse) {
  int big = 0;
  for (int t = 1; t < n_tiles; ++t)
    if ((int64_t)tiles[t].width * tiles[t].rows > (int64_t)tiles[big].width * tiles[big].rows) big = t;
  EventPair ev;
  SS_HIP(hipEventCreate(&ev.a));
  SS_HIP(hipEventCreate(&ev.b));
  const hipEvent_t a = ev.a, b = ev.b;
  // fusion depth
  double best = 1e30;
  *best_fuse = 6;
  const int fuses[4] = {6, 5, 4, 3};
  for (int f : fuses) {
    for (int rep = 0; rep < 3; ++rep) {
      SS_HIP(hipEventRecord(a, s));
      int32_t rc = maxmip_build(tiles[big].height, tiles[big].width, tiles[big].rows,
                                tiles[big].maxmip, f, s);
      if (rc) return rc;
      SS_HIP(hipEventRecord(b, s));
      double ms = 0.0;
      SS_HIP(time_ms(a, b, &ms));
      if (rep > 0 && ms < best) {
        best = ms;
        *best_fuse = f;
      }
    }
  }
  // ray-tile shape: the batched launch (in the selected form) over (largest tile) x
  // (sun subset); the sub-batch's workspace fits in the caller's (fewer pairs)
  const int ns = n_suns < 8 ? n_suns : 8;
  std::vector<ss_sun> sub(ns);
  std::vector<float*> sub_out(ns);
  for (int k = 0; k < ns; ++k) {
    const int idx = (int)(((int64_t)k * n_suns) / ns);
    sub[k] = suns[idx];
    sub_out[k] = d_shadow[(size_t)big * n_suns + idx];
  }
  best = 1e30;
  *best_tile = SS_TILE_8x8;
  const int shapes[4] = {SS_TILE_8x8, SS_TILE_16x4, SS_TILE_4x16, SS_TILE_32x2};
  for (int sh : shapes) {
    BatchImage bi;
    int32_t rc = build_image(&tiles[big], 1, sub.data(), ns, params, sub_out.data(), sh, &bi);
    if (rc) return rc;
    if ((rc = stage_image(bi, ws, s))) return rc;
    const int n_wg = batched_workgroups(bi.rp.sphere, bi.rp.mode, bi.rp.ray_tile);
    for (int rep = 0; rep < 3; ++rep) {
      SS_HIP(hipEventRecord(a, s));
      if ((rc = enqueue_batch(&tiles[big], 1, bi.bd, bi.rp, ws, *best_fuse, n_wg, s))) return rc;
      SS_HIP(hipEventRecord(b, s));
      double ms = 0.0;
      SS_HIP(time_ms(a, b, &ms));
      if (rep > 0 && ms < best) {
        best = ms;
        *best_tile = sh;
      }
    }
  }
  return SS_OK;
}

struct ss_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int ray_tile = 0, fuse = 0;
};

extern "C" int32_t ss_batched_plan_create(const ss_tile* tiles, int32_t n_tiles, const ss_sun* suns,
                                          int32_t n_suns, const ss_params* params,
                                          float* const* d_shadow, void* d_workspace,
                                          int64_t workspace_bytes, void* stream,
                                          ss_plan** plan_out) {
  if (!plan_out) return SS_ERR_INVALID_ARG;
  *plan_out = nullptr;
  int32_t rc = check_batch(tiles, n_tiles, suns, n_suns, params, d_shadow);
  if (rc) return rc;
  if (n_tiles == 0 || n_suns == 0) return SS_ERR_INVALID_ARG;
  if ((rc = check_workspace(n_tiles, n_suns, d_workspace, workspace_bytes))) return rc;
  hipStream_t s = (hipStream_t)stream;
  Resolved rp;
  resolve_params(params, &rp);
  // tune (mipmaps and tap-bound pyramids first: the ray kernels read them)
  for (int t = 0; t < n_tiles; ++t) {
    rc = maxmip_build(tiles[t].height, tiles[t].width, tiles[t].rows, tiles[t].maxmip, 6, s);
    if (rc) return rc;
    if (rp.mode == SS_MODE_EXACT &&
        (rc = ss_bound_build(tiles[t].height, tiles[t].width, tiles[t].rows, tiles[t].bound, s)))
      return rc;
  }
  int tile_code = params->ray_tile, fuse = 6;
  const std::string key = tune_key(tiles, n_tiles, n_suns, rp, params);
  bool cached = false;
  std::call_once(g_tune_file_once, tune_file_load);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{key});
    if (it != g_tune.end()) {
      if (!tile_code) tile_code = it->second.first;
      fuse = it->second.second;
      cached = true;
    }
  }
  if (!cached) {
    int bt_code = 0, bf = 6;
    rc = tune(tiles, n_tiles, suns, n_suns, params, d_shadow,
              static_cast<unsigned char*>(d_workspace), s, &bt_code, &bf);
    if (rc) return rc;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[TuneKey{key}] = {bt_code, bf};
      tune_file_append(key, bt_code, bf);
    }
    if (!tile_code) tile_code = bt_code;
    fuse = bf;
  }
  BatchImage bi;
  if ((rc = build_image(tiles, n_tiles, suns, n_suns, params, d_shadow, tile_code, &bi))) return rc;
  unsigned char* ws = static_cast<unsigned char*>(d_workspace);
  // the tables are expanded once, outside the graph; the graph holds the builds and the launch
  if ((rc = stage_image(bi, ws, s))) return rc;
  SS_HIP(hipStreamSynchronize(s));
  const int n_wg = batched_workgroups(bi.rp.sphere, bi.rp.mode, bi.rp.ray_tile);
  ss_plan* plan = new ss_plan();
  plan->ray_tile = tile_code;
  plan->fuse = fuse;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete plan;
    return hip_fail(e);
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = enqueue_batch(tiles, n_tiles, bi.bd, bi.rp, ws, fuse, n_wg, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (rc == SS_OK && e2 != hipSuccess) rc = hip_fail(e2);
    plan->graph = g;
    if (rc == SS_OK) {
      e2 = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
      if (e2 != hipSuccess) rc = hip_fail(e2);
    }
  } else {
    rc = hip_fail(e);
  }
  const hipError_t ed = hipStreamDestroy(cs);
  if (rc == SS_OK && ed != hipSuccess) rc = hip_fail(ed);
  if (rc != SS_OK) {
    ss_batched_plan_destroy(plan);
    return rc;
  }
  *plan_out = plan;
  return SS_OK;
}

extern "C" int32_t ss_batched_plan_launch(ss_plan* plan, void* stream) {
  if (!plan || !plan->exec) return SS_ERR_INVALID_ARG;
  SS_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
  return SS_OK;
}

extern "C" int32_t ss_batched_plan_config(const ss_plan* plan, int32_t* ray_tile, int32_t* fuse_depth) {
  if (!plan) return SS_ERR_INVALID_ARG;
  if (ray_tile) *ray_tile = plan->ray_tile;
  if (fuse_depth) *fuse_depth = plan->fuse;
  return SS_OK;
}

extern "C" int32_t ss_batched_plan_destroy(ss_plan* plan) {
  if (!plan) return SS_OK;
  hipError_t e = hipSuccess, e2 = hipSuccess;
  if (plan->exec) e = hipGraphExecDestroy(plan->exec);
  if (plan->graph) e2 = hipGraphDestroy(plan->graph);
  delete plan;  // released either way: a failed destroy leaves nothing to retry with
  if (e != hipSuccess) return hip_fail(e);
  if (e2 != hipSuccess) return hip_fail(e2);
  return SS_OK;
}

extern "C" const char* ss_status_string(int32_t status) {
  switch (status) {
    case SS_OK: return "ok";
    case SS_ERR_INVALID_ARG: return "invalid argument";
    case SS_ERR_HIP: return g_last_hip == hipSuccess ? "HIP error" : hipGetErrorString(g_last_hip);
    case SS_ERR_WORKSPACE: return "workspace missing or too small";
    case SS_ERR_UNSUPPORTED: return "unsupported parameter combination";
    default: return "unknown status";
  }
}
