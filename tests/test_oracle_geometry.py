"""Pins of the oracle's ray geometry against closed forms.

Gnomonic tile (texture-space ray of Sec. 3.2 and the cube-sphere faces of
Sec. 4): texel centres project back onto themselves, the straight ray maps to
a straight texture-space line with the projective form t K / (1 + c t), the
tip height is |p + tL| - R on the sphere and h_p + t sin e on the plane, and
the segment schedule follows Sec. 3.3 (one level-m0 texel of travel per run).
"""
import math

import numpy as np
import pytest

R = 1737400.0


def rand_h(shape, seed, amp=400.0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) * amp).astype(np.float32)


@pytest.mark.parametrize("radius", [R, math.inf])
def test_texel_centre_round_trip(orc, radius):
    h = rand_h((40, 56), 1)
    p = orc.Params(56, 40, 7.5, radius, math.radians(2.0), 1.1)
    for i, j in [(0, 0), (55, 39), (17, 23), (28, 20)]:
        pr = orc.probe(h, p, i, j, 0.0)
        assert abs(pr["qx"] - (i + 0.5)) < 1e-9 and abs(pr["qy"] - (j + 0.5)) < 1e-9
        assert abs(pr["H"] - float(h[j, i])) < 1e-7


def test_planar_tip_height(orc):
    h = rand_h((32, 32), 2)
    e = math.radians(3.3)
    p = orc.Params(32, 32, 10.0, math.inf, e, 0.4)
    for t in (1.0, 17.0, 150.0):
        pr = orc.probe(h, p, 5, 9, t)
        assert abs(pr["H"] - (float(h[9, 5]) + t * math.sin(e))) < 1e-9


def test_sphere_tip_height_and_projection(orc):
    """H(t) = sqrt(rho^2 + 2 t rho s + t^2) - R and q(t) - q_p = t K/(1 + c t)."""
    W, Hh, D = 64, 48, 25.0
    h = rand_h((Hh, W), 3)
    e, a = math.radians(1.2), 2.3
    p = orc.Params(W, Hh, D, R, e, a)
    L = np.array([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)])
    for i, j in [(0, 0), (63, 47), (10, 30), (40, 5)]:
        X = (i + 0.5 - W / 2) * D
        Y = (j + 0.5 - Hh / 2) * D
        ell = math.sqrt(X * X + Y * Y + R * R)
        n = np.array([X, Y, R]) / ell
        rho = R + float(h[j, i])
        s = float(n @ L)
        K = (ell / rho) * (L[:2] - np.array([X, Y]) * L[2] / R) / D
        c = L[2] * ell / (rho * R)
        for t in (3.0, 400.0, 9000.0):
            pr = orc.probe(h, p, i, j, t)
            Ht = math.sqrt(rho * rho + 2 * t * rho * s + t * t) - R
            assert abs(pr["H"] - Ht) < 1e-6
            dq = t * K / (1 + c * t)
            assert abs(pr["qx"] - (i + 0.5) - dq[0]) < 1e-9
            assert abs(pr["qy"] - (j + 0.5) - dq[1]) < 1e-9


@pytest.mark.parametrize("radius", [R, math.inf])
def test_exit_on_boundary(orc, radius):
    h = rand_h((30, 50), 4)
    for a in (0.3, 1.9, 3.5, 5.0, 0.0, math.pi / 2):
        p = orc.Params(50, 30, 12.0, radius, math.radians(1.0), a)
        for i, j in [(3, 4), (45, 25), (25, 15)]:
            te = orc.ray_consts(h, p, i, j)["texit"]
            pr = orc.probe(h, p, i, j, te)
            on = min(abs(pr["qx"]), abs(pr["qx"] - 50), abs(pr["qy"]), abs(pr["qy"] - 30))
            assert on < 1e-9
            assert orc.probe(h, p, i, j, te * (1 - 1e-9))["inside"] == 1.0


def test_schedules(orc):
    def p(W, D, L):
        return orc.Params(W, W, D, R, math.radians(1.0), 0.0, max_len_m=L)
    m0, tau, delta = orc.schedule(p(4096, 5.0, 30000.0))
    assert m0 == list(range(4, 13))
    m0, tau, delta = orc.schedule(p(16384, 2.0, 60000.0))
    assert m0 == list(range(4, 15))
    m0, tau, delta = orc.schedule(p(256, 20.0, 0.0))
    assert m0 == [4, 5, 6, 7, 8]
    assert abs(delta - 20.0 / math.cos(math.radians(1.0))) < 1e-12
    assert tau[0] == 0.5 * delta
    for k in range(len(m0)):
        assert abs(tau[k + 1] - tau[k] - delta * 2 ** m0[k]) < 1e-9
    m0, _, _ = orc.schedule(p(2048, 10.0, 0.0).replace(schedule=1, n_segments=3))
    assert m0 == [4, 4, 4]
