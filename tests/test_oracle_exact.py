"""Pins of the exact mode in the oracle and of the tap-bound pyramid.

The exact mode is defined as the smallest clearance over every sample of the
half-texel grid t_n = (n + 1) delta/2 (the grid of the descent's final samples,
Alg. 1), up to the cap or the tile edge.  Its closed-form pins (flat ground, a
sun half below the horizon, a straight ridge) sit with the other modes in
test_oracle_method.py.  Here: it bounds the descent from below everywhere and
equals it where the descent visits the occluder; an occluder moved anywhere
along the ray is always found; and the tap-bound pyramid bounds every tap of
every bilinear sample, checked by enumerating sample positions with the
sampling rule written out.
"""
import math

import numpy as np
import pytest

from test_oracle_method import RL, R, S, fbm_like

SHAPES = [(1, 1), (1, 7), (5, 1), (6, 9), (17, 13), (32, 32), (33, 64)]


def taps_of(q, n):
    """Texel indices read by a bilinear sample at continuous coordinate q
    (texel i covers [i, i+1)): floor(q - 1/2) and the next one, clamped."""
    a = math.floor(q - 0.5)
    return {min(max(a, 0), n - 1), min(max(a + 1, 0), n - 1)}


@pytest.mark.parametrize("shape", SHAPES)
def test_tap_bound_level0_is_block_maximum(orc, shape):
    rows, W = shape
    rng = np.random.default_rng(rows * 100 + W)
    h = rng.standard_normal(shape).astype(np.float32) * 50
    h[rng.random(shape) < 0.1] = -0.0
    d = orc.tap_bound(h)
    for y in range(rows):
        for x in range(W):
            m = -math.inf
            for yy in range(y - 1, y + 2):
                for xx in range(x - 1, x + 2):
                    if 0 <= yy < rows and 0 <= xx < W:
                        m = max(m, float(h[yy, xx]))
            assert d[0][y, x] == np.float32(m)
            assert not (d[0][y, x] == 0 and math.copysign(1.0, d[0][y, x]) < 0)
    assert len(d) == orc.maxmip_levels(W, rows)


@pytest.mark.parametrize("shape", SHAPES)
def test_tap_bound_covers_every_sample_in_a_cell(orc, shape):
    """Every tap of a sample at most half a texel outside a level-m cell is
    bounded by that cell's entry, and some sample inside the cell attains the
    level-0 entry."""
    rows, W = shape
    rng = np.random.default_rng(7 + rows * 31 + W)
    h = (rng.standard_normal(shape) * 100).astype(np.float32)
    d = orc.tap_bound(h)
    for _ in range(400):
        m = int(rng.integers(0, len(d)))
        ly, lx = d[m].shape
        cy, cx = int(rng.integers(0, ly)), int(rng.integers(0, lx))
        # a point in the cell's box (level-0 coordinates), clipped to the tile,
        # pushed up to half a texel outside it
        x0, x1 = cx << m, min((cx + 1) << m, W)
        y0, y1 = cy << m, min((cy + 1) << m, rows)
        qx = rng.uniform(x0 - 0.499, x1 + 0.499)
        qy = rng.uniform(y0 - 0.499, y1 + 0.499)
        hmax = max(float(h[j, i]) for j in taps_of(qy, rows) for i in taps_of(qx, W))
        assert hmax <= float(d[m][cy, cx])
    # attained: the level-0 entry is the largest tap over the texel's samples
    for y in range(rows):
        for x in range(W):
            best = -math.inf
            for qy in (y + 0.0, y + 0.5, y + 0.999):
                for qx in (x + 0.0, x + 0.5, x + 0.999):
                    best = max(best, max(float(h[j, i]) for j in taps_of(qy, rows)
                                         for i in taps_of(qx, W)))
            assert best == float(d[0][y, x])


CASES = [((16, 16), 20.0, R), ((32, 32), 10.0, math.inf), ((40, 48), 15.0, R),
         ((64, 64), 5.0, math.inf)]


@pytest.mark.parametrize("shape,D,radius", CASES)
def test_exact_bounds_descent_and_equals_dense_stepping(orc, shape, D, radius):
    rows, W = shape
    h = fbm_like(shape, 57 + W, 150.0)
    for e, a in [(0.5, 0.3), (1.5, 2.0), (4.0, 4.4)]:
        p = orc.Params(W, rows, D, radius, math.radians(e), a, RL)
        _, a_x, tr = orc.shadow(h, p.replace(mode=2), trace=True)
        _, a_u = orc.shadow(h, p.replace(mode=1, uniform_step=0.5))
        _, a_dp = orc.shadow(h, p)
        assert np.array_equal(a_x, a_u)
        assert np.all(a_dp >= a_x)
        # the deciding sample sits on the half-texel grid
        m0, tau, delta = orc.schedule(p)
        hit = np.isfinite(a_x)
        assert np.allclose(tr["t"][hit], (tr["n"][hit] + 1) * delta / 2, rtol=0, atol=1e-9 * D)


@pytest.mark.parametrize("radius", [math.inf, R])
def test_exact_finds_a_pillar_anywhere_on_the_ray(orc, radius):
    """A one-texel pillar on the ray's row at every distance: the exact mode's
    clearance is the pillar's (its crest texel centre is on the grid when the
    sun is along +column and delta/2 = half a texel), on the plane in closed form."""
    W, rows, D, hr = 96, 3, 20.0, 60.0
    e = math.radians(2.0)
    for ip in range(3, W, 7):
        h = np.zeros((rows, W), np.float32)
        h[:, ip] = hr
        p = orc.Params(W, rows, D, radius, e, 0.0, RL, mode=2)
        s, alpha = orc.shadow(h, p)
        for i in range(0, ip):
            x = (ip - i) * D
            if radius == math.inf:
                # the crest is the tap at the pillar's centre; bilinear on the
                # half-texel grid reaches it exactly
                want = e - math.atan(hr / x)
                assert abs(alpha[1, i] - want) < 1e-12
            else:
                # found, up to the curvature terms: the local verticals at the
                # origin and at the pillar tilt by X/R from the tile's (X the
                # offset from the tile centre) and the pillar sits about
                # x^2/(2R) below the origin's horizon plane; missing the pillar
                # would leave alpha near e instead
                xi, xp = abs((i + 0.5 - W / 2) * D), abs((ip + 0.5 - W / 2) * D)
                assert abs(alpha[1, i] - (e - math.atan(hr / x))) < (xi + xp + x) / R + 1e-6
        assert np.all(s[:, ip:] == 1.0) or radius != math.inf
