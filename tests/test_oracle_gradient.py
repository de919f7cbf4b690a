"""Pins of the reference gradient (torch float64 autograd along the oracle's
branch) against central finite differences of the FP64 oracle forward.

Texels whose +/- perturbation changes any ray's decision record (segment,
final sample, base texel) are skipped: there the shadow factor is not
differentiable.  The forward values along the branch must equal the oracle's.
"""
import math

import numpy as np
import pytest

from oracle import grad_ref

R = 1737400.0
RL = math.radians(0.267)


def terrain(shape, seed, amp):
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(5):
        f = rng.uniform(0.05, 0.3)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    return h.astype(np.float32)


def off_corner(alpha):
    """Rays whose d = alpha / r_L is away from +-1, where the disc fraction's slope has
    a square-root corner (a difference quotient straddling it is not a derivative)."""
    d = np.abs(np.asarray(alpha) / RL)
    return (d < 0.98) | (d > 1.02)


def key(tr):
    return np.stack([tr["seg"], tr["n"], tr["base_i"], tr["base_j"]], axis=-1)


@pytest.mark.parametrize("radius", [R, math.inf])
def test_branch_forward_equals_oracle(orc, radius):
    h = terrain((32, 40), 3, 60.0)
    p = orc.Params(40, 32, 10.0, radius, math.radians(1.5), 0.8, RL)
    s, _, tr = orc.shadow(h, p, trace=True)
    _, _, _, s_b = grad_ref.reference_gradient(h, p, tr, np.zeros(s.size))
    # |p + tL| - R cancels about 2e-10 m in FP64 on the Moon's radius, which is
    # ~1e-8 in s for the first samples (t of a few metres); the plane is exact.
    tol = 1e-12 if math.isinf(radius) else 1e-7
    assert np.max(np.abs(s_b - s.reshape(-1))) < tol


@pytest.mark.parametrize("radius", [R, math.inf])
def test_height_gradient_matches_finite_differences(orc, radius):
    rng = np.random.default_rng(4)
    # low relief: about a fifth of the rays end in the penumbra, where s has a gradient
    h = terrain((28, 28), 23, 3.0)
    p = orc.Params(28, 28, 10.0, radius, math.radians(1.5), 2.1, RL)
    s0, al0, tr0 = orc.shadow(h, p, trace=True)
    assert ((s0 > 0) & (s0 < 1)).sum() > 100
    w = rng.standard_normal(s0.shape) * off_corner(al0)
    g_h, _, _, _ = grad_ref.reference_gradient(h, p, tr0, w)
    checked = nonzero = 0
    live = np.flatnonzero(g_h.reshape(-1))
    eps = 1e-4  # the error of central differences falls as eps^2 (checked down to 3e-5)
    for lin in np.concatenate([rng.permutation(live)[:25], rng.permutation(h.size)[:15]]):
        j, i = divmod(int(lin), h.shape[1])
        hp = h.copy()
        hm = h.copy()
        hp[j, i] += np.float32(eps)
        hm[j, i] -= np.float32(eps)
        dp_ = float(hp[j, i]) - float(h[j, i])
        dm_ = float(h[j, i]) - float(hm[j, i])
        sp, _, trp = orc.shadow(hp, p, trace=True)
        sm, _, trm = orc.shadow(hm, p, trace=True)
        if not (np.array_equal(key(trp), key(tr0)) and np.array_equal(key(trm), key(tr0))):
            continue
        fd = (np.sum(w * sp) - np.sum(w * sm)) / (dp_ + dm_)
        assert abs(fd - g_h[j, i]) <= 1e-4 * max(1.0, abs(fd)), (i, j, fd, g_h[j, i])
        checked += 1
        nonzero += int(abs(fd) > 1e-3)
    assert checked >= 20 and nonzero >= 10


@pytest.mark.parametrize("radius", [R, math.inf])
def test_sun_gradient_matches_finite_differences(orc, radius):
    rng = np.random.default_rng(6)
    h = terrain((28, 28), 7, 3.0)
    e0, a0 = math.radians(1.5), 2.1
    p = orc.Params(28, 28, 10.0, radius, e0, a0, RL)
    s0, al0, tr0 = orc.shadow(h, p, trace=True)
    w = rng.standard_normal(s0.shape) * off_corner(al0)
    _, g_e, g_a, _ = grad_ref.reference_gradient(h, p, tr0, w)
    # the FP64 forward carries ~1e-8 of rounding in s (see above), so the step
    # must be large enough for the difference quotient to rise above it
    eps = 1e-5
    for name, g in (("elev", g_e), ("azim", g_a)):
        pp = p.replace(**{"elev" if name == "elev" else "azim": (e0 if name == "elev" else a0) + eps})
        pm = p.replace(**{"elev" if name == "elev" else "azim": (e0 if name == "elev" else a0) - eps})
        sp, _, trp = orc.shadow(h, pp, trace=True)
        sm, _, trm = orc.shadow(h, pm, trace=True)
        same = np.all(key(trp) == key(tr0), axis=-1) & np.all(key(trm) == key(tr0), axis=-1)
        # rays whose decisions moved do not have a derivative; compare on the rest
        ww = np.where(same, w, 0.0)
        _, g_e2, g_a2, _ = grad_ref.reference_gradient(h, p, tr0, ww)
        g = g_e2 if name == "elev" else g_a2
        fd = (np.sum(ww * sp) - np.sum(ww * sm)) / (2 * eps)
        assert abs(fd) > 1.0, (name, fd)  # penumbra rays make s depend on the sun
        assert abs(fd - g) <= 2e-4 * max(1.0, abs(fd)), (name, fd, g)
        assert same.mean() > 0.8


def points_case(orc, radius, seed):
    rng = np.random.default_rng(seed)
    h = terrain((28, 28), 23, 3.0)
    p = orc.Params(28, 28, 10.0, radius, math.radians(1.5), 2.1, RL)
    xy = rng.uniform(0.0, 28.0, size=(300, 2))
    f = np.mod(xy - 0.5, 1.0)
    xy = xy[((f > 0.05) & (f < 0.95)).all(axis=1)]  # origins off the bilinear kinks
    return rng, h, p, xy


@pytest.mark.parametrize("radius", [R, math.inf])
def test_points_branch_forward_equals_oracle(orc, radius):
    """Rays from surface points: the origin height is the bilinear terrain (Sec. 3.4)."""
    _, h, p, xy = points_case(orc, radius, 11)
    s, _, tr = orc.shadow_points(h, p, xy, trace=True)
    _, _, _, s_b = grad_ref.reference_gradient(h, p, tr, np.zeros(s.size), points=xy)
    tol = 1e-12 if math.isinf(radius) else 1e-7
    assert np.max(np.abs(s_b - s)) < tol


@pytest.mark.parametrize("radius", [R, math.inf])
def test_points_height_gradient_matches_finite_differences(orc, radius):
    """dL/dh through the points' rays, the origin's four bilinear taps included,
    against central differences of the oracle's forward from the same points."""
    rng, h, p, xy = points_case(orc, radius, 13)
    s0, al0, tr0 = orc.shadow_points(h, p, xy, trace=True)
    w = rng.standard_normal(s0.shape) * off_corner(al0)
    g_h, _, _, _ = grad_ref.reference_gradient(h, p, tr0, w, points=xy)
    # the lower-left origin taps of penumbra points, texels with a gradient, and others
    pen = (s0 > 0) & (s0 < 1)
    assert pen.sum() > 30
    taps = np.unique((np.floor(xy[pen, 1] - 0.5).astype(int).clip(0, 27) * 28
                      + np.floor(xy[pen, 0] - 0.5).astype(int).clip(0, 27)))
    live = np.flatnonzero(g_h.reshape(-1))
    cand = np.concatenate([rng.permutation(taps)[:20], rng.permutation(live)[:15],
                           rng.permutation(h.size)[:10]])
    eps = 1e-4
    checked = origin = 0
    for lin in cand:
        j, i = divmod(int(lin), h.shape[1])
        hp = h.copy()
        hm = h.copy()
        hp[j, i] += np.float32(eps)
        hm[j, i] -= np.float32(eps)
        dp_ = float(hp[j, i]) - float(h[j, i])
        dm_ = float(h[j, i]) - float(hm[j, i])
        sp, _, trp = orc.shadow_points(hp, p, xy, trace=True)
        sm, _, trm = orc.shadow_points(hm, p, xy, trace=True)
        if not (np.array_equal(key(trp), key(tr0)) and np.array_equal(key(trm), key(tr0))):
            continue
        fd = (np.sum(w * sp) - np.sum(w * sm)) / (dp_ + dm_)
        assert abs(fd - g_h[j, i]) <= 1e-4 * max(1.0, abs(fd)), (i, j, fd, g_h[j, i])
        checked += 1
        origin += int(int(lin) in taps and abs(fd) > 1e-3)
    assert checked >= 25 and origin >= 8


def test_sun_term_scale_bounds_the_sum(orc):
    """The absolute sums of the per-ray sun terms bound the sun gradient itself, and equal
    it when every upstream gradient has the sign of its ray's derivative."""
    import math as m
    from oracle import grad_ref
    from parity import well_conditioned
    rng = np.random.default_rng(4)
    h = (rng.standard_normal((40, 48)) * 60.0).astype(np.float32)
    p = orc.Params(48, 40, 20.0, 1737400.0, m.radians(1.2), 0.7, m.radians(0.267))
    s, _, tr = orc.shadow(h, p, trace=True)
    mask = (well_conditioned(tr) & (s.reshape(-1) > 0) & (s.reshape(-1) < 1)).astype(float)
    g = rng.standard_normal(s.size) * mask
    _, ge, ga, _ = grad_ref.reference_gradient(h, p, tr, g)
    se, sa = grad_ref.sun_term_scale(h, p, tr, g)
    assert abs(ge) <= se * (1 + 1e-12) and abs(ga) <= sa * (1 + 1e-12) and se > 0
    # with g_r = sign(ds_r/de) the elevation sum is its own absolute sum
    import torch
    from torch.func import jvp
    ht = torch.tensor(h.astype(np.float64))
    a0 = torch.tensor(0.7, dtype=torch.float64)
    _, dse = jvp(lambda e: grad_ref.shadow_on_branch(ht, e, a0, p, tr), (torch.tensor(m.radians(1.2), dtype=torch.float64),),
                 (torch.tensor(1.0, dtype=torch.float64),))
    g2 = np.sign(dse.numpy()) * mask
    _, ge2, _, _ = grad_ref.reference_gradient(h, p, tr, g2)
    se2, _ = grad_ref.sun_term_scale(h, p, tr, g2)
    assert abs(ge2 - se2) <= 1e-9 * se2
