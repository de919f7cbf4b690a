"""Host-only checks of the C ABI: the library loads without a GPU, exports
every symbol include/softshadow.h declares, computes the mipmap layout, and
rejects bad arguments before anything is enqueued (no device call is made)."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2005_06671_amd import _lib
    _lib.lib()
    return _lib


def declared():
    src = open(os.path.join(ROOT, "include", "softshadow.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L.lib(), n), n
    assert set(names) == set(L.SIGNATURES)


def test_layout(L):
    lib = L.lib()
    assert lib.ss_maxmip_levels(256, 256) == 9
    assert lib.ss_maxmip_levels(16384, 16384) == 15
    assert lib.ss_maxmip_levels(1, 1) == 1
    assert lib.ss_maxmip_levels(0, 5) == 0
    assert lib.ss_maxmip_floats(1, 1) == 0
    for W, H in [(256, 256), (1536, 1536), (37, 53), (4096, 2048)]:
        nl = lib.ss_maxmip_levels(W, H)
        prev = 0
        w, h = W, H
        for m in range(1, nl):
            off = lib.ss_maxmip_level_offset(W, H, m)
            assert off % 64 == 0 and off >= prev
            w, h = (w + 1) // 2, (h + 1) // 2
            prev = off + w * h
        assert lib.ss_maxmip_floats(W, H) >= prev
    assert lib.ss_maxmip_level_offset(256, 256, 0) == -1
    assert lib.ss_maxmip_level_offset(256, 256, 10) == -1
    assert lib.ss_maxmip_floats(-1, 4) == -1


def good(L):
    fake = 0x100000
    t = L.SSTile(fake, fake, 64, 64, 10.0)
    s = L.SSSun(math.radians(1.5), 0.3, math.radians(0.267))
    p = L.SSParams(1737400.0, 0.0, 5, 0, 0, 0, 1.0, 1, 0)
    return t, s, p


def cast(L, t, s, p, out=0x200000):
    return L.lib().ss_shadow_cast(C.byref(t), C.byref(s), C.byref(p), out, None)


def test_rejects_bad_arguments(L):
    lib = L.lib()
    t, s, p = good(L)
    assert lib.ss_shadow_cast(None, C.byref(s), C.byref(p), 0x200000, None) == L.SS_ERR_INVALID_ARG
    for field, val in [("width", -3), ("texel_m", 0.0), ("texel_m", float("nan"))]:
        t2, _, _ = good(L)
        setattr(t2, field, val)
        assert cast(L, t2, s, p) == L.SS_ERR_INVALID_ARG, field
    t2, _, _ = good(L)
    t2.height = 0
    assert cast(L, t2, s, p) == L.SS_ERR_INVALID_ARG
    t2, _, _ = good(L)
    t2.maxmip = 0
    assert cast(L, t2, s, p) == L.SS_ERR_INVALID_ARG
    for field, val in [("elev_rad", math.pi / 2), ("ang_radius_rad", 0.0), ("azim_rad", math.inf)]:
        _, s2, _ = good(L)
        setattr(s2, field, val)
        assert cast(L, t, s2, p) == L.SS_ERR_INVALID_ARG, field
    for field, val in [("body_radius_m", -1.0), ("mode", 7), ("schedule", 3), ("prune", 2),
                       ("ray_tile", 9), ("n_segments", -1), ("uniform_step", -1.0)]:
        _, _, p2 = good(L)
        setattr(p2, field, val)
        assert cast(L, t, s, p2) == L.SS_ERR_INVALID_ARG, field
    assert cast(L, t, s, p, out=0) == L.SS_ERR_INVALID_ARG
    # a schedule with more runs than supported
    _, _, p2 = good(L)
    p2.schedule = 1
    p2.n_prime0 = 1
    p2.max_len_m = 1e6
    assert cast(L, t, s, p2) == L.SS_ERR_UNSUPPORTED
    # an explicit run schedule needs 1..16 runs of >= 1 level
    for nseg, lst in [(0, (5,)), (17, (5,) * 16), (2, (5, 0))]:
        _, _, p4 = good(L)
        p4.schedule = 2
        p4.n_segments = nseg
        for k, v in enumerate(lst):
            p4.n_prime_list[k] = v
        assert cast(L, t, s, p4) == L.SS_ERR_INVALID_ARG, (nseg, lst)
    # the exact mode needs the tap-bound pyramid, forward and backward
    _, _, p3 = good(L)
    p3.mode = L.SS_MODE_EXACT
    assert cast(L, t, s, p3) == L.SS_ERR_INVALID_ARG
    assert lib.ss_shadow_cast_backward(C.byref(t), C.byref(s), C.byref(p3), 0x300000, 0x400000,
                                       0x500000, None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_shadow_cast_counted(C.byref(t), C.byref(s), C.byref(p), 0x200000, None,
                                      None) == L.SS_ERR_INVALID_ARG
    # the recorded forward and its adjoint need the record
    assert lib.ss_shadow_cast_save(C.byref(t), C.byref(s), C.byref(p), 0x200000, None,
                                   None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_shadow_cast_backward_saved(C.byref(t), C.byref(s), C.byref(p), None, 0x300000,
                                             0x400000, 0x500000, None) == L.SS_ERR_INVALID_ARG


def test_batched_validation(L):
    lib = L.lib()
    t, s, p = good(L)
    tiles = (L.SSTile * 2)(t, t)
    suns = (L.SSSun * 3)(s, s, s)
    outs = (C.c_void_p * 6)(*([0x600000] * 6))
    need = lib.ss_batched_workspace_bytes(2, 3)
    assert need > 0 and lib.ss_batched_workspace_bytes(-1, 3) == -1
    assert lib.ss_shadow_cast_batched(tiles, 2, suns, 3, C.byref(p), outs, 0x700000, need - 1,
                                      None) == L.SS_ERR_WORKSPACE
    assert lib.ss_shadow_cast_batched(tiles, 2, suns, 3, C.byref(p), outs, 0x700001, need,
                                      None) == L.SS_ERR_WORKSPACE
    outs[4] = None
    assert lib.ss_shadow_cast_batched(tiles, 2, suns, 3, C.byref(p), outs, 0x700000, need,
                                      None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_shadow_cast_batched(tiles, 0, suns, 3, C.byref(p), outs, 0, 0, None) == 0
    plan = C.c_void_p()
    assert lib.ss_batched_plan_create(tiles, 2, suns, 3, C.byref(p), outs, 0x700000, need, None,
                                      None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_batched_plan_launch(None, None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_batched_plan_destroy(None) == 0
    # the exact mode needs every tile's tap-bound buffer
    outs[4] = 0x600000
    p.mode = L.SS_MODE_EXACT
    t2 = L.SSTile.from_buffer_copy(t)
    t2.bound = 0x800000
    tiles = (L.SSTile * 2)(t2, t)
    assert lib.ss_shadow_cast_batched(tiles, 2, suns, 3, C.byref(p), outs, 0x700000, need,
                                      None) == L.SS_ERR_INVALID_ARG
    assert lib.ss_batched_plan_create(tiles, 2, suns, 3, C.byref(p), outs, 0x700000, need, None,
                                      C.byref(plan)) == L.SS_ERR_INVALID_ARG


def test_probe_validation(L):
    lib = L.lib()
    ok = (0x100000, 1024, 0, 8, 0x200000, 256, None)
    for k, bad in [(0, None), (1, 0), (2, 3), (2, 2048), (3, 0), (4, None), (5, 100)]:
        args = list(ok)
        args[k] = bad
        assert lib.ss_probe_gather(*args) == L.SS_ERR_INVALID_ARG, (k, bad)


def test_ray_window_validation(L):
    lib = L.lib()
    t, s, p = good(L)
    for win in [(0, 0, 0, 5), (-1, 0, 4, 4), (0, 0, 65, 4), (60, 0, 5, 4), (0, 61, 4, 4),
                (3, 3, 0, 2)]:
        t2, _, _ = good(L)
        t2.ray_x0, t2.ray_y0, t2.ray_w, t2.ray_h = win
        assert cast(L, t2, s, p) == L.SS_ERR_INVALID_ARG, win


def test_size_limits(L):
    """Each side <= 65536 and fewer than 2^30 texels (32-bit byte offsets)."""
    lib = L.lib()
    assert lib.ss_maxmip_levels(65536, 16383) == 17
    assert lib.ss_maxmip_levels(32768, 32768) == 0
    assert lib.ss_maxmip_floats(65536, 16384) == -1
    assert lib.ss_bound_floats(65537, 1) == -1
    t, s, p = good(L)
    t.width, t.rows = 32768, 32768
    assert cast(L, t, s, p) == L.SS_ERR_INVALID_ARG
    assert lib.ss_maxmip_build(0x100000, 32768, 32768, 0x200000, 0, None) == L.SS_ERR_INVALID_ARG


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 3), (100, 37), (4096, 4096), (65536, 3)])
def test_bound_layout(L, shape):
    """Tap-bound pyramid: level 0 [rows][width] first, then the maximum-mipmap
    levels of it at a 64-float aligned base."""
    lib = L.lib()
    W, H = shape
    base = (W * H + 63) // 64 * 64
    assert lib.ss_bound_level_offset(W, H, 0) == 0
    for m in range(1, lib.ss_maxmip_levels(W, H)):
        assert lib.ss_bound_level_offset(W, H, m) == base + lib.ss_maxmip_level_offset(W, H, m)
    assert lib.ss_bound_floats(W, H) == base + lib.ss_maxmip_floats(W, H)
    assert lib.ss_bound_floats(0, 5) == -1 and lib.ss_bound_level_offset(W, H, 99) == -1
    assert lib.ss_bound_build(None, 0, 0, None, None) == 0
    assert lib.ss_bound_build(None, W, H, 0x100000, None) == L.SS_ERR_INVALID_ARG


def test_status_strings(L):
    lib = L.lib()
    for code in (0, -1, -2, -3, -4, -99):
        assert isinstance(lib.ss_status_string(code), bytes)


def test_product_fails_loudly_without_library(monkeypatch):
    from paper_2005_06671_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libsoftshadow.so")
    with pytest.raises(ImportError):
        _lib.lib()


def test_view_validation(L):
    """ss_view_cast checks the tile, the camera and the buffers before any launch."""
    lib = L.lib()
    fake = 0x100000
    v3 = C.c_double * 3

    def cam(**kw):
        c = L.SSCamera(64, 32, v3(0.0, 0.0, 500.0), v3(0.0, 1.0, -0.5), v3(0.5, 0.0, 0.0),
                       v3(0.0, 0.2, 0.4), 5.0, 0.0, L.SS_VIEW_HIER)
        for k, v in kw.items():
            setattr(c, k, v)
        return c

    def call(t=None, radius=1737400.0, c=None, out_t=fake, out_xy=fake, steps=None):
        t = t or L.SSTile(fake, fake, 64, 64, 10.0, fake, 0, 0, 0, 0)
        c = c or cam()
        return lib.ss_view_cast(C.byref(t), radius, C.byref(c), out_t, out_xy, steps, None)

    assert call(t=L.SSTile(fake, fake, 64, 64, 10.0, None, 0, 0, 0, 0)) == L.SS_ERR_INVALID_ARG
    assert call(t=L.SSTile(fake, fake, 0, 64, 10.0, fake, 0, 0, 0, 0)) == L.SS_ERR_INVALID_ARG
    assert call(t=L.SSTile(None, fake, 64, 64, 10.0, fake, 0, 0, 0, 0)) == L.SS_ERR_INVALID_ARG
    assert call(t=L.SSTile(fake, fake, 64, 64, 0.0, fake, 0, 0, 0, 0)) == L.SS_ERR_INVALID_ARG
    assert call(radius=0.0) == L.SS_ERR_INVALID_ARG
    assert call(radius=-math.inf) == L.SS_ERR_INVALID_ARG
    for bad in [dict(width=0), dict(height=-1), dict(width=16385), dict(step_m=0.1),
                dict(step_m=math.nan), dict(far_m=math.nan), dict(far_m=math.inf), dict(mode=2),
                dict(fwd=v3(0.0, 0.0, 0.0)), dict(right=v3(math.nan, 0.0, 0.0)),
                dict(eye_m=v3(0.0, 0.0, 1737400.0 / 4))]:
        assert call(c=cam(**bad)) == L.SS_ERR_INVALID_ARG, bad
    # the eye limit applies on the sphere only
    assert call(radius=math.inf, c=cam(eye_m=v3(0.0, 0.0, 1e6)), out_t=None) == L.SS_ERR_INVALID_ARG
    assert call(out_t=None) == L.SS_ERR_INVALID_ARG
    assert call(out_xy=None) == L.SS_ERR_INVALID_ARG
    assert call(out_xy=fake + 4) == L.SS_ERR_INVALID_ARG
    assert call(steps=fake + 4) == L.SS_ERR_INVALID_ARG


def test_resample_validation(L):
    """ss_resample checks both frames (orthonormal, finite, sizes) and the buffers."""
    lib = L.lib()
    v3, v2 = C.c_double * 3, C.c_double * 2

    def fr(**kw):
        f = L.SSFrame(64, 32, 10.0, v3(0.0, 0.0, 1.0), v3(1.0, 0.0, 0.0), v3(0.0, 1.0, 0.0),
                      v2(0.0, 0.0))
        for k, v in kw.items():
            setattr(f, k, v)
        return f

    src, dst = 0x100000, 0x800000

    def call(fs=None, fd=None, s=src, d=dst, radius=1737400.0):
        a, b = fs or fr(), fd or fr()
        return lib.ss_resample(s, C.byref(a), d, C.byref(b), radius, None)

    for bad in [dict(width=0), dict(rows=70000), dict(texel_m=0.0), dict(texel_m=math.inf),
                dict(centre=v3(0.0, 0.0, 2.0)), dict(ex=v3(1.0, 0.0, 0.1)),
                dict(ey=v3(1.0, 0.0, 0.0)), dict(centre=v3(math.nan, 0.0, 1.0)),
                dict(origin_m=v2(math.inf, 0.0))]:
        assert call(fs=fr(**bad)) == L.SS_ERR_INVALID_ARG, bad
        assert call(fd=fr(**bad)) == L.SS_ERR_INVALID_ARG, bad
    assert call(s=None) == L.SS_ERR_INVALID_ARG
    assert call(d=None) == L.SS_ERR_INVALID_ARG
    assert call(radius=0.0) == L.SS_ERR_INVALID_ARG
    assert call(radius=math.inf) == L.SS_ERR_INVALID_ARG
    # overlapping buffers (64 x 32 floats = 8 KiB)
    assert call(d=src + 4096) == L.SS_ERR_INVALID_ARG
    assert call(s=dst + 8188) == L.SS_ERR_INVALID_ARG


def test_points_image_validation(L):
    lib = L.lib()
    t, s, p = good(L)
    f = lambda xy=0x400000, w=64, h=32, out=0x500000: lib.ss_shadow_points_image(  # noqa: E731
        C.byref(t), C.byref(s), C.byref(p), xy, w, h, out, None)
    for args in [dict(w=0), dict(h=0), dict(w=16385), dict(xy=None), dict(out=None),
                 dict(xy=0x400004)]:
        assert f(**args) == L.SS_ERR_INVALID_ARG, args


def test_points_backward_validation(L):
    lib = L.lib()
    t, s, p = good(L)
    f = lambda xy=0x400000, n=64, w=0, g=0x500000, gh=0x600000, gs=0x700000: (  # noqa: E731
        lib.ss_shadow_points_backward(C.byref(t), C.byref(s), C.byref(p), xy, n, w, g, gh, gs,
                                      None))
    for args in [dict(n=-1), dict(w=-1), dict(w=16385), dict(n=65, w=8), dict(n=16385 * 2, w=2),
                 dict(xy=None), dict(g=None), dict(gh=None), dict(gs=None), dict(xy=0x400004),
                 dict(gs=0x700004), dict(n=(1 << 36) + 1)]:
        assert f(**args) == L.SS_ERR_INVALID_ARG, args
    assert f(n=0, xy=None) == L.SS_OK  # nothing to do, nothing touched
    assert lib.ss_shadow_points(C.byref(t), C.byref(s), C.byref(p), 0x400000, (1 << 36) + 1,
                                0x500000, None) == L.SS_ERR_INVALID_ARG


def test_valu_probe_validation(L):
    lib = L.lib()
    for args in [(0, 8, 0x400000), (16, 0, 0x400000), (16, 1 << 31, 0x400000), (16, 8, None)]:
        assert lib.ss_probe_valu(*args, None) == L.SS_ERR_INVALID_ARG, args


def test_cap_far_beyond_a_small_tile_is_unsupported(L):
    """A run spans at most the tile's top mip level, so a cap of many tile widths needs more
    than the 48 runs a ray may take: rejected before anything is enqueued."""
    t, s, p = good(L)  # 64 x 64 texels of 10 m
    p.max_len_m = 100000.0
    assert cast(L, t, s, p) == L.SS_ERR_UNSUPPORTED
    p.max_len_m = 640.0
    t.height = 0  # a call that gets past the schedule fails on the missing buffer instead
    assert cast(L, t, s, p) == L.SS_ERR_INVALID_ARG
