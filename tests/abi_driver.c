/* Host-only driver of the C ABI for the sanitizer build (tests/test_abi_sanitized.py).
 *
 * Calls every entry point with arguments that its validation must reject
 * before anything is enqueued, and the layout and status helpers over many
 * shapes, so AddressSanitizer and UBSan watch the host code of libsoftshadow
 * (validation, parameter resolution, layout arithmetic).  No device memory is
 * touched: every pointer is either NULL or a fake address that a rejected call
 * never dereferences.  Prints "ok" and returns 0 when every status is as
 * expected.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "softshadow.h"

static int fails = 0;

#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
      fails++;                                                    \
    }                                                             \
  } while (0)

#define FAKE(a) ((float*)(uintptr_t)(a))

static ss_tile tile(int w, int h) {
  ss_tile t;
  memset(&t, 0, sizeof t);
  t.height = FAKE(0x100000);
  t.maxmip = FAKE(0x200000);
  t.bound = FAKE(0x300000);
  t.width = w;
  t.rows = h;
  t.texel_m = 10.0;
  return t;
}

static ss_params params(void) {
  ss_params p;
  memset(&p, 0, sizeof p);
  p.body_radius_m = 1737400.0;
  return p;
}

int main(void) {
  /* layout helpers over many shapes, including the limits */
  const int32_t sizes[] = {1, 2, 3, 7, 64, 255, 256, 257, 1000, 4096, 65535, 65536, 65537, 0, -1};
  for (unsigned a = 0; a < sizeof sizes / sizeof sizes[0]; ++a) {
    for (unsigned b = 0; b < sizeof sizes / sizeof sizes[0]; ++b) {
      const int32_t w = sizes[a], h = sizes[b];
      const int ok = w >= 1 && h >= 1 && w <= 65536 && h <= 65536 && (int64_t)w * h < (1LL << 30);
      const int32_t L = ss_maxmip_levels(w, h);
      EXPECT(ok ? L >= 1 : L == 0);
      const int64_t n = ss_maxmip_floats(w, h);
      EXPECT(ok ? n >= 0 : n == -1);
      const int64_t nb = ss_bound_floats(w, h);
      EXPECT(ok ? nb >= (int64_t)w * h : nb == -1);
      for (int32_t m = -1; m <= L + 1 && ok; ++m) {
        const int64_t off = ss_maxmip_level_offset(w, h, m);
        EXPECT(m >= 1 && m <= L ? (off >= 0 && off % 64 == 0 && off <= n) : off == -1);
        const int64_t ob = ss_bound_level_offset(w, h, m);
        EXPECT(m >= 1 && m <= L ? ob >= off : 1);
      }
    }
  }
  for (int32_t s = -6; s <= 1; ++s) EXPECT(ss_status_string(s) != NULL);

  /* maximum mipmap and tap-bound builds */
  EXPECT(ss_maxmip_build(NULL, 64, 64, FAKE(0x200000), 0, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_maxmip_build(FAKE(0x100000), 64, 64, NULL, 0, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_maxmip_build(FAKE(0x100000), 64, 64, FAKE(0x200000), 7, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_maxmip_build(FAKE(0x100000), -3, 64, FAKE(0x200000), 0, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_bound_build(NULL, 64, 64, FAKE(0x300000), NULL) == SS_ERR_INVALID_ARG);

  /* per-tile shadow calls */
  ss_sun sun = {0.03, 1.0, 0.00466};
  ss_sun bad_sun[3] = {{2.0, 0.0, 0.00466}, {0.03, NAN, 0.00466}, {0.03, 0.0, 0.0}};
  ss_tile t = tile(64, 64);
  ss_params p = params();
  for (int k = 0; k < 3; ++k)
    EXPECT(ss_shadow_cast(&t, &bad_sun[k], &p, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast(NULL, &sun, &p, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast(&t, &sun, NULL, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast(&t, &sun, &p, NULL, NULL) == SS_ERR_INVALID_ARG);
  ss_params q = p;
  q.body_radius_m = 0.0;
  EXPECT(ss_shadow_cast(&t, &sun, &q, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  q = p;
  q.mode = 9;
  EXPECT(ss_shadow_cast(&t, &sun, &q, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  q = p;
  q.schedule = SS_SCHED_LIST;
  q.n_segments = 17;
  EXPECT(ss_shadow_cast(&t, &sun, &q, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  q.n_segments = 2;
  q.n_prime_list[0] = 5;
  q.n_prime_list[1] = 0;
  EXPECT(ss_shadow_cast(&t, &sun, &q, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  ss_tile tw = tile(64, 64);
  tw.ray_x0 = 60;
  tw.ray_w = 8;
  tw.ray_h = 4;
  EXPECT(ss_shadow_cast(&tw, &sun, &p, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  ss_tile tb = tile(64, 64);
  tb.bound = NULL;
  q = p;
  q.mode = SS_MODE_EXACT;
  EXPECT(ss_shadow_cast(&tb, &sun, &q, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  ss_tile big = tile(32768, 32768);
  EXPECT(ss_shadow_cast(&big, &sun, &p, FAKE(0x400000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_counted(&t, &sun, &p, FAKE(0x400000), NULL, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_save(&t, &sun, &p, FAKE(0x400000), NULL, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_backward(&t, &sun, &p, NULL, FAKE(0x500000), (double*)FAKE(0x600000), NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_backward_saved(&t, &sun, &p, NULL, FAKE(0x400000), FAKE(0x500000),
                                       (double*)FAKE(0x600000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_backward_penumbra(&t, &sun, &p, NULL, FAKE(0x400000), FAKE(0x500000),
                                          (double*)FAKE(0x600000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_backward_penumbra(&t, &sun, &p, FAKE(0x400000), FAKE(0x400000),
                                          FAKE(0x500000), (double*)FAKE(0x600004), NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points(&t, &sun, &p, FAKE(0x400004), 10, FAKE(0x500000), NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points(&t, &sun, &p, NULL, 10, FAKE(0x500000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points(&t, &sun, &p, FAKE(0x400000), -1, FAKE(0x500000), NULL) ==
         SS_ERR_INVALID_ARG);

  EXPECT(ss_shadow_points(&t, &sun, &p, FAKE(0x400000), SS_MAX_POINTS + 1, FAKE(0x500000), NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points_backward(&t, &sun, &p, FAKE(0x400000), 65, 8, FAKE(0x500000),
                                   FAKE(0x600000), (double*)FAKE(0x700000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points_backward(&t, &sun, &p, FAKE(0x400000), 64, 0, FAKE(0x500000),
                                   FAKE(0x600000), (double*)FAKE(0x700004), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points_backward(&t, &sun, &p, NULL, 0, 0, NULL, NULL, NULL, NULL) == SS_OK);

  EXPECT(ss_shadow_points_image(&t, &sun, &p, FAKE(0x400000), 0, 8, FAKE(0x500000), NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_points_image(&t, &sun, &p, FAKE(0x400004), 8, 8, FAKE(0x500000), NULL) ==
         SS_ERR_INVALID_ARG);

  /* batched */
  ss_tile tiles[2] = {tile(64, 64), tile(128, 32)};
  ss_sun suns[2] = {sun, sun};
  float* outs[4] = {FAKE(0x700000), FAKE(0x710000), FAKE(0x720000), FAKE(0x730000)};
  const int64_t ws = ss_batched_workspace_bytes(2, 2);
  EXPECT(ws > 0);
  EXPECT(ss_batched_workspace_bytes(-1, 2) < 0);
  EXPECT(ss_shadow_cast_batched(tiles, 2, suns, 2, &p, (float* const*)outs, FAKE(0x800000), ws - 1,
                                NULL) == SS_ERR_WORKSPACE);
  EXPECT(ss_shadow_cast_batched(tiles, 2, suns, 2, &p, NULL, FAKE(0x800000), ws, NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_batched_noalloc(tiles, -1, suns, 2, &p, (float* const*)outs, NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_batched_noalloc(tiles, 2, suns, 2, &p, NULL, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_shadow_cast_batched_noalloc(tiles, 0, suns, 2, &p, NULL, NULL) == SS_OK);
  q = p;
  q.mode = SS_MODE_EXACT;
  tiles[1].bound = NULL;  /* the exact mode needs every tile's tap-bound buffer */
  EXPECT(ss_shadow_cast_batched(tiles, 2, suns, 2, &q, (float* const*)outs, FAKE(0x800000), ws,
                                NULL) == SS_ERR_INVALID_ARG);
  tiles[1].bound = FAKE(0x300000);
  ss_plan* plan = NULL;
  EXPECT(ss_batched_plan_create(tiles, 2, suns, 2, &p, (float* const*)outs, FAKE(0x800000), ws - 1,
                                NULL, &plan) == SS_ERR_WORKSPACE);
  EXPECT(plan == NULL);
  EXPECT(ss_batched_plan_destroy(NULL) == SS_OK);

  /* view rays */
  ss_camera cam;
  memset(&cam, 0, sizeof cam);
  cam.width = 64;
  cam.height = 32;
  cam.eye_m[2] = 500.0;
  cam.fwd[1] = 1.0;
  cam.fwd[2] = -0.5;
  cam.right[0] = 0.5;
  cam.up[2] = 0.4;
  cam.step_m = 5.0;
  ss_tile tv = tile(64, 64);
  EXPECT(ss_view_cast(&tv, 1737400.0, &cam, NULL, FAKE(0x900000), NULL, NULL) == SS_ERR_INVALID_ARG);
  ss_camera c2 = cam;
  c2.step_m = 0.01;
  EXPECT(ss_view_cast(&tv, 1737400.0, &c2, FAKE(0x900000), FAKE(0xA00000), NULL, NULL) ==
         SS_ERR_INVALID_ARG);
  c2 = cam;
  c2.mode = 5;
  EXPECT(ss_view_cast(&tv, 1737400.0, &c2, FAKE(0x900000), FAKE(0xA00000), NULL, NULL) ==
         SS_ERR_INVALID_ARG);
  tv.bound = NULL;
  EXPECT(ss_view_cast(&tv, 1737400.0, &cam, FAKE(0x900000), FAKE(0xA00000), NULL, NULL) ==
         SS_ERR_INVALID_ARG);

  /* resampling */
  ss_frame f;
  memset(&f, 0, sizeof f);
  f.width = 64;
  f.rows = 64;
  f.texel_m = 10.0;
  f.centre[2] = 1.0;
  f.ex[0] = 1.0;
  f.ey[1] = 1.0;
  ss_frame g = f;
  g.ex[0] = 0.9;
  EXPECT(ss_resample(FAKE(0x100000), &f, FAKE(0x200000), &g, 1737400.0, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_resample(FAKE(0x100000), &f, FAKE(0x100100), &f, 1737400.0, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_resample(FAKE(0x100000), &f, FAKE(0x200000), &f, INFINITY, NULL) == SS_ERR_INVALID_ARG);

  /* probe */
  EXPECT(ss_probe_gather(NULL, 1024, 0, 8, FAKE(0x200000), 256, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_probe_gather_tiles(NULL, 64, 64, 8, FAKE(0x200000), 256, NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_probe_gather_tiles(FAKE(0x100000), 7, 64, 8, FAKE(0x200000), 256, NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_probe_gather_tiles(FAKE(0x100000), 64, 64, 8, FAKE(0x200000), 255, NULL) ==
         SS_ERR_INVALID_ARG);
  EXPECT(ss_probe_valu(0, 8, FAKE(0x200000), NULL) == SS_ERR_INVALID_ARG);
  EXPECT(ss_probe_valu(16, 8, NULL, NULL) == SS_ERR_INVALID_ARG);

  if (fails) return 1;
  printf("ok\n");
  return 0;
}
