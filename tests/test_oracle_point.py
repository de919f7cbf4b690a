"""Pins of Alg. 1 read literally (the point-sample descent, mode 3) in the
oracle, and of the explicit run schedule.

Closed forms (flat ground, a sun half below the horizon) run with the other
modes in test_oracle_method.py.  Here: its final samples lie on the half-texel
grid, so its clearance is never below dense stepping over the same extent; and
on the plane its control flow (sample order, re-centring behind the choice,
strict far-first tie rule, per-level reset) is checked against a second
formulation written in the algorithm's normalised ray parameter t in [0, 1],
with the paper's sentinels, instead of grid indices.
"""
import math

import numpy as np
import pytest

from test_oracle_method import RL, R, fbm_like


def test_schedule_list(orc):
    p = orc.Params(4096, 4096, 5.0, R, math.radians(1.0), 0.3, RL, schedule=2, n_segments=4,
                   n_prime_list=(5, 5, 5, 3))
    m0, tau, delta = orc.schedule(p)
    assert list(m0) == [4, 4, 4, 2]
    assert np.allclose(np.diff(tau), [16 * delta, 16 * delta, 16 * delta, 4 * delta], rtol=0,
                       atol=1e-9)
    assert abs(tau[0] - delta / 2) < 1e-12


CASES = [((48, 48), 20.0, R), ((40, 64), 10.0, math.inf), ((64, 64), 5.0, R)]


@pytest.mark.parametrize("shape,D,radius", CASES)
def test_point_descent_never_below_dense_stepping(orc, shape, D, radius):
    rows, W = shape
    h = fbm_like(shape, 71 + W, 150.0)
    for e, a in [(0.5, 0.3), (1.5, 2.0), (4.0, 4.4)]:
        for sched in [dict(), dict(schedule=2, n_segments=4, n_prime_list=(5, 5, 5, 3))]:
            p = orc.Params(W, rows, D, radius, math.radians(e), a, RL, mode=3, **sched)
            m0, tau, delta = orc.schedule(p)
            _, a_pt, tr = orc.shadow(h, p, trace=True)
            # the last run's samples reach at most one top-level texel past its end
            far = tau[-1] + 2.0 ** (m0[-1] + 1) * delta
            _, a_u = orc.shadow(h, p.replace(mode=1, uniform_step=0.5, uniform_tmax_m=far))
            assert np.all(a_pt >= a_u)
            assert np.any(a_pt == a_u)
            hit = np.isfinite(a_pt)
            assert np.allclose(tr["t"][hit], (tr["n"][hit] + 1) * delta / 2, rtol=0, atol=1e-9 * D)


def alg1_normalised(h, W, rows, D, e, az, i, j, m0s, mips, RLv):
    """Alg. 1 in its own terms on the plane (sun at azimuth az): per run
    of length T = 2^m0 delta, t runs over [0, 1]; level k samples t_k,
    t_k - 2^-(k+1), t_k - 2^-k at mip m = m0 - k (nearest texel; m = 0
    bilinear); t* takes the smallest H - max h with strict '<' in that order;
    the next level starts from t* + 2^-(k+1); the sentinel resets each level."""
    delta = D / math.cos(e)
    hp = float(h[j, i])
    alpha = math.inf
    start = delta / 2
    for m0 in m0s:
        T = 2.0 ** m0 * delta
        tk = 1.0
        choice = None
        for k in range(m0 + 1):
            m = m0 - k
            best, tstar = math.inf, -1.0
            for q in range(3):
                tq = tk - q * 2.0 ** (-k - 1)
                t = start + tq * T
                qx = i + 0.5 + t * math.cos(e) * math.cos(az) / D
                qy = j + 0.5 + t * math.cos(e) * math.sin(az) / D
                if not (0 <= qx < W and 0 <= qy < rows):
                    continue
                H = hp + t * math.sin(e)
                if m > 0:
                    hv = float(mips[m - 1][int(math.floor(qy)) >> m, int(math.floor(qx)) >> m])
                else:
                    x, y = qx - 0.5, qy - 0.5
                    x0, y0 = math.floor(x), math.floor(y)
                    fx, fy = x - x0, y - y0
                    cx = [min(max(x0 + d, 0), W - 1) for d in (0, 1)]
                    cy = [min(max(y0 + d, 0), rows - 1) for d in (0, 1)]
                    hv = ((1 - fy) * ((1 - fx) * float(h[cy[0], cx[0]]) + fx * float(h[cy[0], cx[1]]))
                          + fy * ((1 - fx) * float(h[cy[1], cx[0]]) + fx * float(h[cy[1], cx[1]])))
                if H - hv < best:
                    best, tstar = H - hv, tq
            if tstar < 0:
                choice = None
                break
            choice = (best, start + tstar * T)
            tk = tstar + 2.0 ** (-k - 1)
        if choice is not None:
            dh, t = choice
            alpha = min(alpha, math.atan2(dh * math.cos(e), t - dh * math.sin(e)))
        start += T
    return alpha


@pytest.mark.parametrize("e_deg", [0.7, 2.0, 6.0])
@pytest.mark.parametrize("lst", [(3,), (5, 5, 5), (5, 5, 5, 3), (1, 2, 3, 4)])
def test_point_descent_matches_normalised_form(orc, e_deg, lst):
    # off-axis sun: with it along a texel axis, half the grid samples sit
    # exactly on texel lines and either side is a correct reading
    W, rows, D, az = 80, 9, 10.0, 0.013
    rng = np.random.default_rng(len(lst) * 10 + int(e_deg * 10))
    h = (rng.standard_normal((rows, W)).cumsum(axis=1) * 3.0
         + rng.standard_normal((rows, W)) * 4.0).astype(np.float32)
    e = math.radians(e_deg)
    p = orc.Params(W, rows, D, math.inf, e, az, RL, mode=3, schedule=2, n_segments=len(lst),
                   n_prime_list=lst)
    m0, tau, delta = orc.schedule(p)
    _, alpha = orc.shadow(h, p)
    mips = orc.maxmip(h)
    for j in (2, 4):
        for i in range(W):
            want = alg1_normalised(h, W, rows, D, e, az, i, j, list(m0), mips, RL)
            got = alpha[j, i]
            assert (got == want) or abs(got - want) < 1e-12, (i, j, got, want)
