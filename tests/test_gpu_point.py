"""GPU tests of Alg. 1 read literally (SS_MODE_POINT) through the C ABI:
parity with the oracle's point-sample descent on small, ragged and full-size
tiles, with the geometric schedule and the paper's {5,5,5} and {5,5,5,3};
bitwise invariance under prune and ray-tile settings; the batched path."""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

R = 1737400.0
RL = math.radians(0.267)
SCHEDULES = {"geometric": dict(),
             "555": dict(schedule=1, n_segments=3),
             "5553": dict(schedule=2, n_segments=4, n_prime_list=(5, 5, 5, 3))}


@pytest.fixture(scope="module")
def ss():
    import paper_2005_06671_amd as m
    m.lib()
    return m


def dev():
    return torch.device("cuda:0")


def rough(shape, seed, amp):
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(7):
        f = rng.uniform(0.01, 0.3)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    h += rng.standard_normal(shape) * amp * 0.02
    return h.astype(np.float32)


def run(ss, hd, p: oracle.Params, prune=1, ray_tile=0, mm=None):
    params = ss.Params(radius_m=p.radius_m, max_len_m=p.max_len_m, n_prime0=p.n_prime0,
                       schedule=p.schedule, n_segments=p.n_segments, mode=p.mode, prune=prune,
                       ray_tile=ray_tile, n_prime_list=tuple(p.n_prime_list))
    s = ss.shadow_cast(hd, p.texel_m, p.elev, p.azim, p.ang_radius, params, mm=mm)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("sched", list(SCHEDULES))
def test_small_workload_point_full_grid(ss, sched):
    from synth import dem_for, sun_list
    h = dem_for("small").numpy()
    hd = torch.from_numpy(h).to(dev())
    e, a, r = sun_list("small")[0]
    p = oracle.Params(256, 256, 20.0, R, e, a, r, mode=3, **SCHEDULES[sched])
    assert_parity(compare(h, p, run(ss, hd, p), label=f"small point {sched}"))


RAGGED = [((136, 200), 20.0, R, 1.5, 0.4), ((136, 200), 20.0, math.inf, 1.5, 2.8),
          ((77, 301), 10.0, R, 0.6, 4.0), ((250, 61), 30.0, R, 3.5, 5.6),
          ((129, 129), 5.0, math.inf, 0.25, 1.2)]


@pytest.mark.parametrize("shape,D,radius,e_deg,az", RAGGED)
def test_point_ragged_and_invariant(ss, shape, D, radius, e_deg, az):
    print("point", shape, D, radius, e_deg, az, flush=True)
    h = rough(shape, shape[0] * 7 + shape[1], 150.0)
    hd = torch.from_numpy(h).to(dev())
    for sched in ("geometric", "5553"):
        p = oracle.Params(shape[1], shape[0], D, radius, math.radians(e_deg), az, RL, mode=3,
                          **SCHEDULES[sched])
        base = run(ss, hd, p, prune=0)
        for prune in (0, 1):
            for tile in (1, 2, 3, 4):
                assert np.array_equal(bits(run(ss, hd, p, prune=prune, ray_tile=tile)), bits(base))
        assert_parity(compare(h, p, base, label=f"point ragged {shape} {sched}"))


def test_point_full_size_sampled(ss):
    from synth import config, dem_for, sun_list
    c = config("tile")
    W, H, D = c["tiles"][0]
    hd = dem_for("tile", device=dev())
    h = hd.cpu().numpy()
    mm = ss.maxmip(hd)
    rng = np.random.default_rng(17)
    rays = np.sort(rng.choice(W * H, size=10000, replace=False)).astype(np.int64)
    for si, (e, a, r) in enumerate(sun_list("tile")[:2]):
        for sched in ("geometric", "5553"):
            p = oracle.Params(W, H, D, R, e, a, r, max_len_m=c["max_len"], mode=3,
                              **SCHEDULES[sched])
            got = run(ss, hd, p, mm=mm)
            assert_parity(compare(h, p, got, rays, label=f"tile sun{si} point {sched}"))


def test_point_batched_equals_per_tile(ss):
    shapes = [(96, 128, 20.0), (200, 136, 10.0)]
    heights = [torch.from_numpy(rough((r, w), w + r, 120.0)).to(dev()) for (w, r, _) in shapes]
    texels = [t for (_, _, t) in shapes]
    suns = [(math.radians(0.8), 0.3, RL), (math.radians(2.5), 4.0, RL)]
    params = ss.Params(radius_m=R, mode=ss.SS_MODE_POINT, schedule=ss.SS_SCHED_LIST,
                       n_segments=4, n_prime_list=(5, 5, 5, 3))
    outs = ss.shadow_cast_batched(heights, texels, suns, params)
    torch.cuda.synchronize()
    for t, h in enumerate(heights):
        for k, (e, a, r) in enumerate(suns):
            ref = ss.shadow_cast(h, texels[t], e, a, r, params)
            torch.cuda.synchronize()
            assert torch.equal(outs[t][k].view(torch.int32), ref.view(torch.int32)), (t, k)
