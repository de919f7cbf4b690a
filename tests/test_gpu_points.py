"""GPU tests of shadow rays from arbitrary surface points (ss_shadow_points):
texel centres give ss_shadow_cast's values bit for bit in every mode, and
random points match the oracle's rays from the same points."""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

R = 1737400.0
RL = math.radians(0.267)


@pytest.fixture(scope="module")
def ss():
    import paper_2005_06671_amd as m
    m.lib()
    return m


def rough(shape, seed, amp):
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(6):
        f = rng.uniform(0.01, 0.2)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    h += rng.standard_normal(shape) * amp * 0.02
    return h.astype(np.float32)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("radius", [R, math.inf])
def test_centres_equal_grid(ss, mode, radius):
    h = rough((136, 200), 61, 120.0)
    hd = torch.from_numpy(h).cuda()
    p = ss.Params(radius_m=radius, mode=mode)
    grid = ss.shadow_cast(hd, 15.0, math.radians(1.1), 0.8, RL, p)
    jj, ii = torch.meshgrid(torch.arange(136, device="cuda"), torch.arange(200, device="cuda"),
                            indexing="ij")
    xy = torch.stack([ii.reshape(-1) + 0.5, jj.reshape(-1) + 0.5], dim=1).float().contiguous()
    pts = ss.shadow_points(hd, 15.0, math.radians(1.1), 0.8, xy, RL, p)
    torch.cuda.synchronize()
    assert torch.equal(pts.view(torch.int32), grid.reshape(-1).view(torch.int32))


@pytest.mark.parametrize("mode", [0, 2, 3])
@pytest.mark.parametrize("radius,e_deg,az", [(R, 1.5, 2.2), (math.inf, 0.7, 4.0), (R, 3.0, 0.3)])
def test_random_points_match_oracle(ss, mode, radius, e_deg, az):
    h = rough((160, 176), 67, 150.0)
    hd = torch.from_numpy(h).cuda()
    rng = np.random.default_rng(int(e_deg * 10) + mode)
    xy = np.stack([rng.uniform(0, 176, 20000), rng.uniform(0, 160, 20000)], axis=1).astype(np.float32)
    p = ss.Params(radius_m=radius, mode=mode)
    got = ss.shadow_points(hd, 10.0, math.radians(e_deg), az, torch.from_numpy(xy).cuda(), RL, p)
    torch.cuda.synchronize()
    po = oracle.Params(176, 160, 10.0, radius, math.radians(e_deg), az, RL, mode=mode)
    ref, _ = oracle.shadow_points(h, po, xy.astype(np.float64))
    d = np.abs(got.cpu().numpy() - ref)
    print("points", mode, radius, e_deg, "max", d.max(), "n>1e-4", int((d > 1e-4).sum()))
    # the exact mode has no discrete choice that FP32 could flip; the descents
    # may at FP64 near-ties (same allowance as the texel-grid protocol)
    assert (d > 1e-4).mean() <= (0.0 if mode == 2 else 2e-3)
