"""Determinism on the GPU: every forward path writes each output once, so two runs
give the same bits; the adjoint accumulates with atomics, so two runs agree to
rounding of the summation order."""
import math

import numpy as np
import pytest
import torch

import synth
from synth.configs import view_scene

pytestmark = pytest.mark.gpu

R = synth.R_MOON


@pytest.fixture(scope="module")
def ss():
    import paper_2005_06671_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def h():
    return synth.dem_for("small", device="cuda")


def same(a, b):
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_forward_repeats_bitwise(ss, h, mode):
    e, a, r = synth.sun_list("small")[0]
    p = ss.Params(radius_m=R, mode=mode)
    s1 = ss.shadow_cast(h, 20.0, e, a, r, p).clone()
    s2 = ss.shadow_cast(h, 20.0, e, a, r, p)
    torch.cuda.synchronize()
    assert same(s1, s2)


def test_view_and_resample_repeat_bitwise(ss, h):
    cam = view_scene("oblique", 96, 64, 256, 256, 20.0)
    t1, xy1 = (x.clone() for x in ss.view_cast(h, 20.0, ss.Camera(**cam), R))
    t2, xy2 = ss.view_cast(h, 20.0, ss.Camera(**cam), R)
    fs = ss.Frame(256, 256, 20.0, (0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    c, s = math.cos(0.3), math.sin(0.3)
    fd = ss.Frame(120, 90, 13.0, (0.0, 0.0, 1.0), (c, s, 0.0), (-s, c, 0.0), (33.0, -12.0))
    d1 = torch.full((90, 120), float("nan"), device="cuda")
    d2 = torch.full((90, 120), float("nan"), device="cuda")
    ss.resample(h, fs, d1, fd, R)
    ss.resample(h, fs, d2, fd, R)
    torch.cuda.synchronize()
    assert same(t1, t2) and same(xy1, xy2) and same(d1, d2)


@pytest.mark.parametrize("saved", [False, True])
def test_adjoint_repeats_to_rounding(ss, h, saved):
    e, a, r = synth.sun_list("small")[0]
    p = ss.Params(radius_m=R)
    g = torch.randn(h.shape, generator=torch.Generator().manual_seed(3)).cuda()
    outs = []
    for _ in range(2):
        if saved:
            s, smp = ss.shadow_cast_save(h, 20.0, e, a, r, p)
            gh, gs = ss.shadow_cast_backward_saved(h, 20.0, e, a, smp, g, r, p)
        else:
            gh, gs = ss.shadow_cast_backward(h, 20.0, e, a, g, r, p)
        torch.cuda.synchronize()
        outs.append((gh.clone(), gs.clone()))
    (g1, s1), (g2, s2) = outs
    assert float((g1 - g2).norm()) <= 1e-6 * float(g1.norm()) + 1e-12
    assert torch.allclose(s1, s2, rtol=1e-9, atol=0.0)
