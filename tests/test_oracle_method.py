"""Pins of the whole method in the oracle (Sec. 3.1-3.4, Alg. 1).

Special cases with closed forms (flat ground, a sun half below the horizon, a
straight ridge), the exact invariant that the descent's final samples are a
subset of dense half-texel stepping, equality with dense stepping behind a
single occluder, the descent's texel walk against dense sampling of the path,
and the near-tie enumerator against the plain path at zero tolerance.
"""
import math
import os

import numpy as np
import pytest

R = 1737400.0
RL = math.radians(0.267)
HERE = os.path.dirname(os.path.abspath(__file__))


def S(d):
    d = max(-1.0, min(1.0, d))
    return (math.pi - math.acos(d) + d * math.sqrt(1 - d * d)) / math.pi


def fbm_like(shape, seed, amp):
    """Small rough test terrain: sum of a few random sinusoids plus noise."""
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(6):
        f = rng.uniform(0.02, 0.4)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    h += rng.standard_normal(shape) * amp * 0.05
    return h.astype(np.float32)


@pytest.mark.parametrize("radius,elev", [(math.inf, RL * 1.001), (math.inf, math.radians(3)),
                                         (R, math.radians(0.3)), (R, math.radians(2.0))])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_flat_ground_is_lit(orc, radius, elev, mode):
    h = np.zeros((64, 64), np.float32)
    for a in (0.0, 0.7, 2.5, 4.0):
        p = orc.Params(64, 64, 20.0, radius, elev, a, RL, mode=mode)
        s, _ = orc.shadow(h, p)
        assert np.all(s == 1.0)


@pytest.mark.parametrize("mode,step", [(0, 1.0), (1, 1.0), (1, 0.5), (2, 1.0), (3, 1.0)])
def test_half_set_sun(orc, mode, step):
    """Plane, h = 0, e = 0.2 deg < r_L: every sample's clearance is exactly e."""
    e = math.radians(0.2)
    h = np.zeros((48, 40), np.float32)
    p = orc.Params(40, 48, 10.0, math.inf, e, 0.9, RL, mode=mode, uniform_step=step)
    s, alpha, tr = orc.shadow(h, p, trace=True)
    first_inside = np.array([[orc.probe(h, p, i, j, 0.5 * orc.schedule(p)[2])["inside"]
                              for i in range(40)] for j in range(48)]) == 1.0
    assert np.all(np.abs(alpha[first_inside] - e) < 1e-13)
    assert np.all(np.abs(s[first_inside] - S(e / RL)) < 1e-12)
    assert np.all(s[~first_inside] == 1.0)
    assert abs(S(0.2 / 0.267) - 0.927459) < 1e-6


def ridge_case(e_deg):
    W, rows, D, ir, hr = 256, 6, 20.0, 250, 100.0
    h = np.zeros((rows, W), np.float32)
    h[:, ir] = hr
    return h, W, rows, D, ir, hr, math.radians(e_deg)


@pytest.mark.parametrize("e_deg", [1.5, 3.0])
@pytest.mark.parametrize("mode,step", [(0, 1.0), (1, 0.5), (2, 1.0)])
def test_straight_ridge_penumbra(orc, e_deg, mode, step):
    """Plane, sun along +column, one-texel ridge: s(x) = S((e - atan(h_r/x))/r_L)."""
    h, W, rows, D, ir, hr, e = ridge_case(e_deg)
    p = orc.Params(W, rows, D, math.inf, e, 0.0, RL, mode=mode, uniform_step=step)
    s, _ = orc.shadow(h, p)
    for i in range(ir):
        x = (ir - i) * D
        want = S((e - math.atan(hr / x)) / RL)
        assert np.all(np.abs(s[:, i] - want) < 1e-12), (i, s[0, i], want)
    assert np.all(s[:, ir:] == 1.0)
    # extents of umbra and penumbra against the golden closed form
    gold = {float(a): (float(c), float(d)) for a, b, c, d, _ in
            (l.split() for l in open(os.path.join(HERE, "golden", "ridge_penumbra.txt"))
             if not l.startswith("#"))}
    umbra_end, light_begin = gold[e_deg]
    xs = (ir - np.arange(ir)) * D
    assert np.all(s[0, :ir][xs < umbra_end - 1e-6] == 0.0)
    assert np.all(s[0, :ir][xs > light_begin + 1e-6] == 1.0)
    pen = (xs > umbra_end + 1e-6) & (xs < light_begin - 1e-6)
    assert np.all((s[0, :ir][pen] > 0) & (s[0, :ir][pen] < 1))


CASES = [((16, 16), 20.0, R), ((32, 32), 10.0, math.inf), ((40, 48), 15.0, R),
         ((64, 64), 20.0, R), ((64, 64), 5.0, math.inf)]


@pytest.mark.parametrize("shape,D,radius", CASES)
def test_descent_never_below_dense_half_texel_stepping(orc, shape, D, radius):
    """Every final sample of the descent lies on the grid t_n of dense stepping
    at half a texel, so the descent's clearance can only be larger (exactly)."""
    rows, W = shape
    h = fbm_like(shape, 31 + W, 150.0)
    for k, (e, a) in enumerate([(0.5, 0.3), (1.5, 2.0), (4.0, 4.4), (0.25, 5.9)]):
        p = orc.Params(W, rows, D, radius, math.radians(e), a, RL)
        m0, tau, delta = orc.schedule(p)
        _, a_dp = orc.shadow(h, p)
        _, a_u = orc.shadow(h, p.replace(mode=1, uniform_step=0.5, uniform_tmax_m=tau[-1] + delta))
        assert np.all(a_dp >= a_u)
        assert np.any(a_dp == a_u)


@pytest.mark.parametrize("radius", [math.inf, R])
def test_single_occluder_matches_dense_stepping(orc, radius):
    """A cone lit along its row: beyond the first segment the descent finds the
    crest, which lies on the half-texel grid, so it equals dense stepping."""
    W, rows, D = 200, 9, 20.0
    ic, jc = 180, 4
    y, x = np.mgrid[0:rows, 0:W]
    h = np.maximum(0.0, 120.0 - 6.0 * np.hypot(x - ic, y - jc)).astype(np.float32)
    p = orc.Params(W, rows, D, radius, math.radians(1.5), 0.0, RL)
    _, a_dp = orc.shadow(h, p)
    m0, tau, delta = orc.schedule(p)
    _, a_u = orc.shadow(h, p.replace(mode=1, uniform_step=0.5, uniform_tmax_m=tau[-1] + delta))
    far = np.arange(W) < ic - 2 ** (m0[0] + 1)
    assert np.all(np.abs(a_dp[jc, far] - a_u[jc, far]) < 1e-9)


@pytest.mark.parametrize("radius", [math.inf, R])
def test_texel_walk_matches_dense_sampling(orc, radius):
    """The cells the descent walks (Fig. 3b: all texels under the footprint)
    are the cells dense sampling of the path visits, with matching spans."""
    rng = np.random.default_rng(5)
    W, rows, D = 96, 80, 10.0
    h = fbm_like((rows, W), 2, 80.0)
    for trial in range(30):
        e = math.radians(rng.uniform(0.3, 5))
        a = rng.uniform(0, 2 * math.pi)
        p = orc.Params(W, rows, D, radius, e, a, RL)
        i, j = int(rng.integers(0, W)), int(rng.integers(0, rows))
        te = orc.ray_consts(h, p, i, j)["texit"]
        m = int(rng.integers(0, 5))
        ta = rng.uniform(0.0, 0.6) * min(te, 2000.0)
        tb = min(te, ta + rng.uniform(0.2, 2.5) * D * 2 ** m)
        cells = orc.path_cells(h, p, i, j, m, ta, tb)
        ts = np.linspace(ta, tb, 1501)[1:-1]
        step = ts[1] - ts[0]
        seen = {}
        for t in ts:
            pr = orc.probe(h, p, i, j, t)
            c = (int(math.floor(pr["qx"] / 2 ** m)), int(math.floor(pr["qy"] / 2 ** m)))
            seen.setdefault(c, []).append(t)
        got = {c: span for c, span in cells}
        assert set(seen) <= set(got)
        for c, (t0, t1) in got.items():
            if t1 - t0 > 3 * step:
                assert c in seen
            if c in seen:
                assert min(seen[c]) >= t0 - 1e-9 and max(seen[c]) <= t1 + 1e-9
        spans = [span for _, span in cells]
        assert abs(spans[0][0] - ta) < 1e-12 and abs(spans[-1][1] - tb) < 1e-12
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 == b0


@pytest.mark.parametrize("shape,D,radius", CASES[:4])
def test_tie_enumeration_reduces_to_plain_path(orc, shape, D, radius):
    rows, W = shape
    h = fbm_like(shape, 77 + W, 200.0)
    p = orc.Params(W, rows, D, radius, math.radians(1.0), 2.2, RL)
    _, alpha = orc.shadow(h, p)
    for lin in range(0, W * rows, 7):
        alts = orc.alternatives(h, p, lin, 0.0, 0.0, 0.0, 0.0)
        assert alts is not None and len(alts) == 1
        assert alts[0] == alpha.flat[lin] or (np.isinf(alts[0]) and np.isinf(alpha.flat[lin]))


def test_tie_enumeration_contains_plain_path(orc):
    h = fbm_like((48, 48), 9, 200.0)
    p = orc.Params(48, 48, 10.0, R, math.radians(1.0), 2.2, RL)
    _, alpha = orc.shadow(h, p)
    for lin in range(0, 48 * 48, 5):
        alts = orc.alternatives(h, p, lin, 1e-2, 1e-7, 1e-3, 1e-6)
        assert alts is not None
        a = alpha.flat[lin]
        assert np.any(alts == a) or (np.isinf(a) and np.any(np.isinf(alts)))


@pytest.mark.parametrize("mode,step", [(1, 1.0), (1, 0.5), (2, 1.0)])
def test_uniform_tie_enumeration(orc, mode, step):
    """Uniform stepping's near-tie set: at zero tolerance exactly the plain
    loop's minimum; with tolerance it always holds that minimum, and for a ray
    whose last step sits at the tile edge also the minimum without that step
    (computed independently by capping the plain loop just before it)."""
    rows, W = 40, 56
    h = fbm_like((rows, W), 31, 200.0)
    p = orc.Params(W, rows, 10.0, R, math.radians(1.0), 0.0, RL, mode=mode, uniform_step=step)
    _, alpha = orc.shadow(h, p)
    for lin in range(0, W * rows, 11):
        a0 = orc.alternatives(h, p, lin, 0.0, 0.0, 0.0, 0.0)
        assert a0 is not None and len(a0) == 1
        assert a0[0] == alpha.flat[lin] or (np.isinf(a0[0]) and np.isinf(alpha.flat[lin]))
        a1 = orc.alternatives(h, p, lin, 1e-2, 1e-7, 1e-3, 1e-6)
        assert np.any(a1 == alpha.flat[lin]) or np.isinf(alpha.flat[lin])
    # a ray on the plane, nearly along +x, whose last step lands 1e-7 texel inside the
    # edge x = W, where a wall raises the terrain: the plain loop counts that step and it
    # decides; the enumeration must also offer the minimum without it, which the plain
    # loop gives when capped just before that step
    hp = fbm_like((rows, W), 32, 150.0)
    hp[:, -1] += 600.0
    i, j = 30, 20
    k_edge = W - i - 1  # step k sits at x = i + 1/2 + (k + 1/2) cos(a)
    cos_a = (W - 1e-7 - (i + 0.5)) / (k_edge + 0.5)
    pp = orc.Params(W, rows, 10.0, math.inf, math.radians(1.0), math.acos(cos_a), RL, mode=1,
                    uniform_step=1.0)
    lin = j * W + i
    _, a_plain, tr = orc.shadow(hp, pp, np.array([lin]), trace=True)
    assert tr["n"][0] == k_edge
    delta = 10.0 / math.cos(math.radians(1.0))
    _, a_short = orc.shadow(hp, pp.replace(uniform_tmax_m=k_edge * delta), np.array([lin]))
    assert a_short[0] > a_plain[0]
    alts = orc.alternatives(hp, pp, lin, 1e-2, 1e-7, 1e-3, 1e-6)
    assert np.any(alts == a_plain[0]) and np.any(alts == a_short[0])
    assert orc.alternatives(hp, pp, lin, 0.0, 0.0, 0.0, 0.0).tolist() == [a_plain[0]]
