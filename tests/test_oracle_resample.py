"""Pins of the oracle's resampling between gnomonic tile frames (Sec. 3.3 stitched
virtual texture, Sec. 4 cube-sphere faces).

Fixed by geometry: the identity frame copies bit for bit; a frame shifted by
whole texels in the same plane crops or shifts exactly (so a sub-tile of a face
is a crop); half a texel gives the mean of two neighbours; an in-plane rotation
of the axes maps a linear height field to the rotated linear field; and heights
given as a smooth function of the surface direction, sampled on one cube face
and resampled into a tile on another face across the seam, reproduce that
function at the new texels' directions within the bilinear interpolation error.
"""
import math

import numpy as np
import pytest

import oracle

R = 1737400.0


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def face(w, rows, texel, centre=(0, 0, 1), ex=(1, 0, 0), ey=(0, 1, 0), origin=(0.0, 0.0)):
    return oracle.Frame(w, rows, texel, tuple(map(float, centre)), tuple(map(float, ex)),
                        tuple(map(float, ey)), tuple(map(float, origin)))


def texel_dirs(f: oracle.Frame):
    """Unit directions of a frame's texel centres, from the frame's definition."""
    i = np.arange(f.width) + 0.5 - f.width / 2
    j = np.arange(f.rows) + 0.5 - f.rows / 2
    X = f.origin[0] + i[None, :] * f.texel_m
    Y = f.origin[1] + j[:, None] * f.texel_m
    P = (R * np.array(f.centre)[None, None, :] + X[..., None] * np.array(f.ex)[None, None, :]
         + Y[..., None] * np.array(f.ey)[None, None, :])
    return P / np.linalg.norm(P, axis=-1, keepdims=True)


def test_identity_copies_bitwise():
    rng = np.random.default_rng(1)
    h = rng.uniform(-3000, 3000, size=(37, 53)).astype(np.float32)
    f = face(53, 37, 10.0)
    out, _, cov, _ = oracle.resample(h, f, f, R)
    assert cov.all()
    assert np.array_equal(out.view(np.uint32), h.view(np.uint32))


@pytest.mark.parametrize("dx,dy", [(3, 0), (-5, 2), (0, -7)])
def test_whole_texel_shift_and_crop(dx, dy):
    """A destination grid shifted by whole texels in the same plane: an exact crop."""
    rng = np.random.default_rng(2)
    h = rng.uniform(-1000, 1000, size=(40, 50)).astype(np.float32)
    D = 8.0
    src = face(50, 40, D)
    dst = face(20, 16, D, origin=(dx * D, dy * D))
    out, _, cov, _ = oracle.resample(h, src, dst, R)
    # destination texel (i, j) is source texel (i + 15 + dx, j + 12 + dy)
    i0, j0 = (50 - 20) // 2 + dx, (40 - 16) // 2 + dy
    assert cov.all()
    assert np.array_equal(out, h[j0:j0 + 16, i0:i0 + 20])


def test_half_texel_is_mean():
    rng = np.random.default_rng(3)
    h = rng.uniform(-1000, 1000, size=(20, 30)).astype(np.float32)
    D = 4.0
    src = face(30, 20, D)
    dst = face(10, 10, D, origin=(0.5 * D, 0.0))
    out, o64, cov, _ = oracle.resample(h, src, dst, R)
    i0, j0 = 10, 5
    ref = 0.5 * (h[j0:j0 + 10, i0:i0 + 10].astype(np.float64) +
                 h[j0:j0 + 10, i0 + 1:i0 + 11].astype(np.float64))
    assert cov.all()
    assert np.allclose(o64, ref, rtol=0, atol=1e-9)


def test_in_plane_rotation_of_a_linear_field():
    """Same tangent point, axes turned by theta: a field linear in the source plane
    coordinates arrives as the rotated linear field."""
    D = 5.0
    W = 64
    a, bx, by = 120.0, 0.3, -0.2
    xs = (np.arange(W) + 0.5 - W / 2) * D
    h = (a + bx * xs[None, :] + by * xs[:, None]).astype(np.float32)
    src = face(W, W, D)
    th = math.radians(30.0)
    ex = (math.cos(th), math.sin(th), 0.0)
    ey = (-math.sin(th), math.cos(th), 0.0)
    dst = face(24, 24, D, ex=ex, ey=ey)
    out, o64, cov, _ = oracle.resample(h, src, dst, R)
    u = (np.arange(24) + 0.5 - 12) * D
    X = u[None, :] * ex[0] + u[:, None] * ey[0]
    Y = u[None, :] * ex[1] + u[:, None] * ey[1]
    ref = a + bx * X + by * Y
    assert cov.all()
    # the float32 field is linear up to half an ulp per texel (~1e-5 m here)
    assert np.abs(o64 - ref).max() < 1e-4


def test_cube_face_seam_reproduces_a_function_of_direction():
    """Heights h = 900 (d . u) + 300 (d . v)^2 over the sphere, sampled on the +z cube face
    near its +x edge, resampled into a tile tangent at the seam direction: the values equal
    the function at the new texels' directions within the bilinear error."""
    u, v = unit((0.3, -0.5, 0.8)), unit((0.9, 0.1, 0.4))
    g = lambda d: 900.0 * (d @ u) + 300.0 * (d @ v) ** 2  # noqa: E731
    D = 10.0
    # +z face sub-tile whose grid reaches the face edge x/z = 1 (plane coordinate X = R)
    Ws = 300
    src = face(Ws, 200, D, origin=(R - 0.5 * Ws * D, 0.0))
    h = g(texel_dirs(src)).astype(np.float32)
    seam = unit((1.0, 0.0, 1.0))
    ex = unit(np.cross((0.0, 1.0, 0.0), seam))
    dst = face(100, 80, D * 0.8, centre=seam, ex=ex, ey=(0.0, 1.0, 0.0))
    out, o64, cov, mar = oracle.resample(h, src, dst, R)
    dd = texel_dirs(dst)
    # covered exactly where the direction lies on the +z side of the seam (x < z)
    side = (dd[..., 0] < dd[..., 2])
    sure = mar > 1e-6
    assert np.array_equal(cov[sure], side[sure])
    assert 0.3 < cov.mean() < 0.7
    # float32 storage (half an ulp of ~900 m: 3e-5 m) plus second differences of g over
    # one texel (10 m on a 1737 km sphere: ~1e-8 m)
    err = np.abs(o64[cov] - g(dd[cov]))
    assert err.max() < 1e-4


def test_source_behind_and_outside():
    """Directions behind the source plane or beyond its edges are not covered."""
    h = np.ones((10, 10), dtype=np.float32)
    src = face(10, 10, 10.0)
    far = face(10, 10, 10.0, centre=(0, 0, -1), ex=(1, 0, 0), ey=(0, -1, 0))
    dst = face(10, 10, 10.0, origin=(500.0, 0.0))
    assert not oracle.resample(h, src, far, R)[2].any()
    assert not oracle.resample(h, src, dst, R)[2].any()
    qx, qy, front = oracle.frame_source_coords(src, far, R, 0, 0)
    assert front < 0
