"""Pins of the angular clearance and the disc-occlusion fraction.

The oracle's closed-form clearance (Sec. 3.4: J*(N.N_L) to first order) is
checked against the signed 3-D angle between the sun direction and the
terrain point below the ray tip, computed here with plain vector algebra.
The disc fraction (Sec. 3.4, Eq. 6 first term) is checked against circular
segment geometry tabulated in tests/golden/disc_fraction.txt.
"""
import math
import os

import numpy as np
import pytest

R = 1737400.0
HERE = os.path.dirname(os.path.abspath(__file__))


def signed_angle(p, L, O):
    v = O - p
    # sky direction perpendicular to L in the plane of L and the local vertical at the tip
    return v, L


@pytest.mark.parametrize("radius", [R, math.inf])
def test_clearance_is_3d_angle(orc, radius):
    rng = np.random.default_rng(11)
    W, Hh, D = 40, 40, 30.0
    h = (rng.standard_normal((Hh, W)) * 200).astype(np.float32)
    for trial in range(40):
        e = math.radians(rng.uniform(0.3, 6.0))
        a = rng.uniform(0, 2 * math.pi)
        p = orc.Params(W, Hh, D, radius, e, a)
        i, j = int(rng.integers(0, W)), int(rng.integers(0, Hh))
        c = orc.ray_consts(h, p, i, j)
        t = rng.uniform(1.0, 0.9 * c["texit"]) if math.isfinite(c["texit"]) else 50.0
        pr = orc.probe(h, p, i, j, t)
        if pr["inside"] != 1.0:
            continue
        L = np.array([c["Lx"], c["Ly"], c["Lz"]])
        P0 = np.array([c["px"], c["py"], c["pz"]])
        tip = P0 + t * L
        if math.isinf(radius):
            up = np.array([0.0, 0.0, 1.0])
            O = tip - pr["dh"] * up
            sky = up - (up @ L) * L
        else:
            rh = tip / np.linalg.norm(tip)
            O = tip - pr["dh"] * rh
            sky = rh - (rh @ L) * L
        sky /= np.linalg.norm(sky)
        v = O - P0
        ang = math.atan2(-(v @ sky), v @ L)
        assert abs(ang - pr["alpha"]) < 1e-11


def test_disc_fraction_special_values(orc):
    assert orc.disc_fraction(-1.0) == 0.0
    assert orc.disc_fraction(1.0) == 1.0
    assert abs(orc.disc_fraction(0.0) - 0.5) < 1e-15
    for d in np.linspace(-1, 1, 41):
        assert abs(orc.disc_fraction(d) + orc.disc_fraction(-d) - 1.0) < 1e-14
        if abs(d) < 0.99:
            g = (orc.disc_fraction(d + 1e-6) - orc.disc_fraction(d - 1e-6)) / 2e-6
            assert abs(g - 2 * math.sqrt(1 - d * d) / math.pi) < 1e-7


def test_disc_fraction_against_segment_areas(orc):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "disc_fraction.txt"))
            if not l.startswith("#")]
    for d, v in rows:
        assert abs(orc.disc_fraction(float(d)) - float(v)) < 1e-11
