"""Pins of the view-ray oracle (Sec. 4, view ray casting) against closed forms.

Each case has an answer fixed by geometry alone: a flat or tilted plane (the
view ray's height above a linear terrain is linear in t, so the straight-line
refinement is exact), a bare or raised sphere (a quadratic root), a ramp
between two texel centres (pins the bilinear offsets), the radial line above a
texel centre (central projection maps it to one texel position), mirror
symmetry, and the admissible-set rules for near ties, the far limit, an eye
inside the terrain and rays that never meet the tile.
"""
import math

import numpy as np
import pytest

import oracle

R_MOON = 1737.4e3


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def direction(cam, px, py):
    """The camera's pixel ray, from its definition."""
    sx = 2.0 * (px + 0.5) / cam.width - 1.0
    sy = 1.0 - 2.0 * (py + 0.5) / cam.height
    return unit(np.array(cam.fwd) + sx * np.array(cam.right) + sy * np.array(cam.up))


def oblique_camera(w=24, h=16, eye=(-300.0, -200.0, 900.0), step=5.0, far=0.0):
    fwd = unit((0.5, 0.35, -1.0))
    right = 0.45 * unit(np.cross(fwd, (0, 0, 1)))
    up = 0.3 * unit(np.cross(right, fwd))
    return oracle.Camera(w, h, tuple(eye), tuple(fwd), tuple(right), tuple(up), step, far)


def test_direction_matches_definition():
    cam = oblique_camera()
    for px, py in [(0, 0), (23, 15), (7, 9)]:
        assert np.allclose(oracle.view_direction(cam, px, py), direction(cam, px, py),
                           atol=1e-15)


@pytest.mark.parametrize("c", [0.0, 37.25, -120.0])
def test_flat_plane_closed_form(c):
    W = H = 128
    D = 10.0
    h = np.full((H, W), c, dtype=np.float32)
    cam = oblique_camera()
    res = oracle.view(h, math.inf, D, cam)
    E = np.array(cam.eye)
    hits = 0
    for py in range(cam.height):
        for px in range(cam.width):
            V = direction(cam, px, py)
            t = (E[2] - c) / -V[2]
            P = E + t * V
            qx, qy = P[0] / D + W / 2, P[1] / D + H / 2
            r = res[py, px]
            if 0.5 < qx < W - 0.5 and 0.5 < qy < H - 0.5:
                hits += 1
                assert r["n_hit"] == math.ceil(t / cam.step_m)
                assert abs(r["t_hit"] - t) < 1e-9 * t
                assert abs(r["qx"] - qx) < 1e-9 and abs(r["qy"] - qy) < 1e-9
                assert r["n_adm"] == 1
    assert hits > 100


def test_tilted_plane_closed_form():
    """h = a + g X (X the tangent-plane coordinate): bilinear sampling reproduces it."""
    W = H = 160
    D = 8.0
    a, g = 50.0, 0.21
    X = ((np.arange(W) + 0.5) - W / 2) * D
    h = np.broadcast_to(a + g * X, (H, W)).astype(np.float64)
    h32 = h.astype(np.float32)
    cam = oblique_camera(eye=(-250.0, -180.0, 700.0), step=4.0)
    res = oracle.view(h32, math.inf, D, cam)
    E = np.array(cam.eye)
    hits = 0
    for py in range(cam.height):
        for px in range(cam.width):
            V = direction(cam, px, py)
            # E_z + t V_z = a + g (E_x + t V_x)
            t = (E[2] - a - g * E[0]) / (g * V[0] - V[2])
            P = E + t * V
            qx, qy = P[0] / D + W / 2, P[1] / D + H / 2
            r = res[py, px]
            if 1.0 < qx < W - 1.0 and 1.0 < qy < H - 1.0:
                hits += 1
                # float32 storage of the plane: at most half an ulp per texel height
                assert r["n_hit"] == math.ceil(t / cam.step_m)
                assert abs(r["t_hit"] - t) < 1e-4
    assert hits > 100


def test_ramp_between_texel_centres():
    """A block of height Hw from column i0 on: the terrain ramps linearly from 0 at
    x = i0 - 1/2 to Hw at x = i0 + 1/2; a ray along +x meets it in closed form."""
    W, H = 64, 32
    D = 10.0
    i0, Hw = 40, 200.0
    h = np.zeros((H, W), dtype=np.float32)
    h[:, i0:] = Hw
    # eye on the row y = 16.5 texels (tile centre row + 0.5), ray along +x and slightly down
    ey = 0.5 * D
    E = np.array([(-10.0) * D, ey, 120.0])
    fwd = unit((1.0, 0.0, -0.05))
    cam = oracle.Camera(1, 1, tuple(E), tuple(fwd), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 2.5)
    r = oracle.view(h, math.inf, D, cam)[0, 0]
    V = fwd
    # world x of the ramp foot: (i0 - 1/2 - W/2) D; height on the ramp: Hw (x - foot)/D
    foot = (i0 - 0.5 - W / 2) * D
    t = (E[2] - Hw * (E[0] - foot) / D) / (Hw / D * V[0] - V[2])
    x = E[0] + t * V[0]
    assert foot < x < foot + D
    assert abs(r["t_hit"] - t) < 1e-9 * t
    assert r["n_hit"] == math.ceil(t / cam.step_m)


@pytest.mark.parametrize("c", [0.0, 850.0])
def test_sphere_quadratic_root(c):
    W = H = 256
    D = 20.0
    h = np.full((H, W), c, dtype=np.float32)
    cam = oblique_camera(w=12, h=8, eye=(-900.0, -600.0, 3000.0), step=5.0)
    res = oracle.view(h, R_MOON, D, cam)
    E = np.array(cam.eye) + np.array([0.0, 0.0, R_MOON])  # from the sphere centre
    hits = 0
    for py in range(cam.height):
        for px in range(cam.width):
            V = direction(cam, px, py)
            b = E @ V
            cc = E @ E - (R_MOON + c) ** 2
            t = -b - math.sqrt(b * b - cc)
            P = E + t * V
            qx = R_MOON * P[0] / (P[2] * D) + W / 2
            qy = R_MOON * P[1] / (P[2] * D) + H / 2
            r = res[py, px]
            if 0.5 < qx < W - 0.5 and 0.5 < qy < H - 0.5:
                hits += 1
                assert r["n_hit"] == math.ceil(t / cam.step_m)
                # secant root of a convex f: off by at most step^2 f''/(8 f') ~ 1e-5 m
                assert abs(r["t_hit"] - t) < 1e-4
                assert abs(r["qx"] - qx) < 1e-5 and abs(r["qy"] - qy) < 1e-5
    assert hits > 50


def test_radial_line_maps_to_texel_centre():
    """Looking straight down the local vertical above texel (i, j): central projection
    keeps q fixed, the height drops linearly, so the hit is at distance d exactly."""
    W = H = 128
    D = 20.0
    rng = np.random.default_rng(3)
    h = rng.uniform(-300, 300, size=(H, W)).astype(np.float32)
    for i, j in [(10, 20), (64, 64), (120, 3)]:
        X, Y = (i + 0.5 - W / 2) * D, (j + 0.5 - H / 2) * D
        n = unit((X, Y, R_MOON))
        d = 1234.5
        P = (R_MOON + float(h[j, i]) + d) * n
        E = P - np.array([0.0, 0.0, R_MOON])
        cam = oracle.Camera(1, 1, tuple(E), tuple(-n), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 7.0)
        r = oracle.view(h, R_MOON, D, cam)[0, 0]
        assert abs(r["qx"] - (i + 0.5)) < 1e-6 and abs(r["qy"] - (j + 0.5)) < 1e-6
        assert abs(r["t_hit"] - d) < 1e-6
        assert r["n_hit"] == math.ceil(d / 7.0)


def test_mirror_symmetry():
    """Mirroring the terrain and the camera across the tile's x = W/2 line mirrors hits."""
    W = H = 96
    D = 10.0
    rng = np.random.default_rng(7)
    h = rng.uniform(0, 150, size=(H, W)).astype(np.float32)
    cam = oblique_camera(w=16, h=12, eye=(-120.0, -150.0, 500.0), step=3.0)
    m = lambda v: (-v[0], v[1], v[2])
    cam_m = oracle.Camera(cam.width, cam.height, m(cam.eye), m(cam.fwd),
                          tuple(-np.array(m(cam.right))), m(cam.up), cam.step_m)
    a = oracle.view(h, math.inf, D, cam)
    # the mirrored camera's right vector is flipped too, so pixel columns swap
    b = oracle.view(np.ascontiguousarray(h[:, ::-1]), math.inf, D, cam_m)[:, ::-1]
    assert np.array_equal(a["n_hit"], b["n_hit"])
    ok = a["n_hit"] >= 0
    assert ok.sum() > 50
    assert np.allclose(a["t_hit"][ok], b["t_hit"][ok], rtol=1e-12)
    assert np.allclose(a["qx"][ok], W - b["qx"][ok], atol=1e-9)


def test_admissible_set_near_tie():
    """A sample exactly on a flat plateau is a tie: it and the next sample are admissible."""
    D = 10.0
    c = 40.0
    h = np.full((64, 64), c, dtype=np.float32)
    V = unit((0.6, 0.1, -0.5))
    step = 4.0
    n_tie = 57
    E = np.array([-150.0, -40.0, 0.0])
    E[2] = c - n_tie * step * V[2]  # sample n_tie lands on the plateau (up to rounding)
    cam = oracle.Camera(1, 1, tuple(E), tuple(V), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), step)
    r = oracle.view(h, math.inf, D, cam, tol=oracle.ViewTol(eh_abs=1e-6))[0, 0]
    assert r["n_hit"] == n_tie + 1
    assert list(r["adm"][:r["n_adm"]]) == [n_tie, n_tie + 1]
    # without tolerance the tie is decided by its sign alone
    r0 = oracle.view(h, math.inf, D, cam)[0, 0]
    assert r0["n_hit"] in (n_tie, n_tie + 1) and r0["n_adm"] == 1


def test_far_limit_eye_inside_and_misses():
    D = 10.0
    h = np.full((64, 64), 20.0, dtype=np.float32)
    V = unit((0.3, 0.2, -0.6))
    E = np.array([-100.0, -80.0, 300.0])
    t = (E[2] - 20.0) / -V[2]
    mk = lambda eye, fwd, far=0.0: oracle.Camera(1, 1, tuple(eye), tuple(fwd), (0, 0, 0),
                                                 (0, 0, 0), 2.0, far)
    assert abs(oracle.view(h, math.inf, D, mk(E, V))[0, 0]["t_hit"] - t) < 1e-9
    assert oracle.view(h, math.inf, D, mk(E, V, far=t - 5.0))[0, 0]["n_hit"] == -1
    assert oracle.view(h, math.inf, D, mk(E, V, far=t + 5.0))[0, 0]["n_hit"] >= 0
    # eye below the terrain: hit at once
    r = oracle.view(h, math.inf, D, mk((0.0, 0.0, 5.0), V))[0, 0]
    assert r["n_hit"] == 0 and r["t_hit"] == 0.0
    # looking up, and looking away from the tile from outside it
    assert oracle.view(h, math.inf, D, mk((0, 0, 100.0), unit((0.2, 0.1, 0.5))))[0, 0]["n_hit"] == -1
    assert oracle.view(h, math.inf, D, mk((-500.0, 0, 100.0), unit((-1, 0, -0.1))))[0, 0]["n_hit"] == -1
    # sphere: the same looking up
    assert oracle.view(h, R_MOON, D, mk((0, 0, 100.0), unit((0.2, 0.1, 0.5))))[0, 0]["n_hit"] == -1


def test_side_entry_below_terrain():
    """A ray entering the tile through its side below the terrain hits at the first
    sample inside; the refinement uses the clamped terrain just outside."""
    D = 10.0
    h = np.full((32, 32), 100.0, dtype=np.float32)
    V = unit((1.0, 0.0, -0.01))
    E = np.array([-16 * D - 12.3, 0.0, 50.0])  # 12.3 m outside the x = 0 edge, 50 m up
    cam = oracle.Camera(1, 1, tuple(E), tuple(V), (0, 0, 0), (0, 0, 0), 5.0)
    r = oracle.view(h, math.inf, D, cam)[0, 0]
    t_edge = 12.3 / V[0]
    assert r["n_hit"] == math.ceil(t_edge / 5.0)
    # both samples are below the (clamped) terrain: no crossing, the hit is t_{n-1}
    assert r["t_hit"] == (r["n_hit"] - 1) * 5.0
