"""Pins of shadow rays from arbitrary surface points in the oracle (the
origin is the bilinear terrain at continuous texel coordinates): texel
centres reproduce the texel-grid results exactly in every mode; flat ground
is lit and a sun half below a flat horizon gives alpha = e exactly from any
point; the descent from a point is never below dense stepping from it."""
import math

import numpy as np
import pytest

from test_oracle_method import RL, R, S, fbm_like


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("radius", [R, math.inf])
def test_centres_equal_texel_grid(orc, mode, radius):
    h = fbm_like((40, 48), 5, 150.0)
    p = orc.Params(48, 40, 15.0, radius, math.radians(1.2), 2.0, RL, mode=mode)
    s, a = orc.shadow(h, p)
    jj, ii = np.mgrid[0:40, 0:48]
    xy = np.stack([ii.reshape(-1) + 0.5, jj.reshape(-1) + 0.5], axis=1)
    sp, ap = orc.shadow_points(h, p, xy)
    assert np.array_equal(sp, s.reshape(-1))
    assert np.array_equal(ap, a.reshape(-1))


def test_flat_and_half_set_sun_from_any_point(orc):
    rng = np.random.default_rng(2)
    h = np.zeros((48, 40), np.float32)
    xy = np.stack([rng.uniform(0, 40, 300), rng.uniform(0, 48, 300)], axis=1)
    for radius in (R, math.inf):
        p = orc.Params(40, 48, 10.0, radius, math.radians(2.0), 0.9, RL)
        s, _ = orc.shadow_points(h, p, xy)
        assert np.all(s == 1.0)
    e = math.radians(0.2)
    for mode in (0, 2, 3):
        p = orc.Params(40, 48, 10.0, math.inf, e, 0.9, RL, mode=mode)
        s, a = orc.shadow_points(h, p, xy)
        seen = np.isfinite(a)
        assert seen.mean() > 0.9
        assert np.all(np.abs(a[seen] - e) < 1e-13)
        assert np.all(np.abs(s[seen] - S(e / RL)) < 1e-12)


@pytest.mark.parametrize("radius", [R, math.inf])
def test_point_origin_descent_never_below_dense(orc, radius):
    h = fbm_like((64, 64), 9, 150.0)
    rng = np.random.default_rng(3)
    xy = np.stack([rng.uniform(0, 64, 500), rng.uniform(0, 64, 500)], axis=1)
    for e, a in [(0.5, 0.3), (2.0, 4.0)]:
        p = orc.Params(64, 64, 10.0, radius, math.radians(e), a, RL)
        m0, tau, delta = orc.schedule(p)
        _, a_dp = orc.shadow_points(h, p, xy)
        _, a_u = orc.shadow_points(h, p.replace(mode=1, uniform_step=0.5,
                                                uniform_tmax_m=tau[-1] + delta), xy)
        assert np.all(a_dp >= a_u)
    with pytest.raises(ValueError):
        orc.shadow_points(h, p, [[64.0, 3.0]])
