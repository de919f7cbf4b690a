"""Batched form: one persistent launch over (tile, sun, ray block) items and its
captured HIP graph.  Outputs must be bit-identical to the per-tile kernel, on
replays too, and within 1e-4 of the oracle on sampled rays of the full
8-tile x 64-sun workload."""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

R = 1737400.0


@pytest.fixture(scope="module")
def ss():
    import paper_2005_06671_amd as m
    m.lib()
    return m


def dev():
    return torch.device("cuda:0")


def small_batch():
    from synth import make_dem
    shapes = [(96, 96, 20.0), (70, 130, 15.0), (256, 256, 10.0)]
    hs = [make_dem(w, r, D, 800.0, 50 + k, craters=30, device=dev()) for k, (w, r, D) in enumerate(shapes)]
    texels = [D for _, _, D in shapes]
    suns = [(math.radians(0.4 + 0.7 * k), 0.3 + 1.1 * k, math.radians(0.267)) for k in range(5)]
    return hs, texels, suns


def per_tile(ss, hs, texels, suns, params):
    out = []
    for h, D in zip(hs, texels):
        mm = ss.maxmip(h)
        out.append([ss.shadow_cast(h, D, e, a, r, params, mm=mm).clone() for e, a, r in suns])
    torch.cuda.synchronize()
    return out


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("mode", [0, 1])
def test_batched_equals_per_tile(ss, mode):
    hs, texels, suns = small_batch()
    params = ss.Params(radius_m=R, max_len_m=2500.0, mode=mode)
    ref = per_tile(ss, hs, texels, suns, params)
    for tile in (1, 2, 3, 4):
        params.ray_tile = tile
        got = ss.shadow_cast_batched(hs, texels, suns, params)
        torch.cuda.synchronize()
        for t in range(len(hs)):
            for k in range(len(suns)):
                assert same(got[t][k], ref[t][k]), (mode, tile, t, k)


def test_graph_plan_replays(ss):
    hs, texels, suns = small_batch()
    params = ss.Params(radius_m=R, max_len_m=2500.0)
    ref = per_tile(ss, hs, texels, suns, params)
    plan = ss.BatchedPlan(hs, texels, suns, params)
    rt, fd = plan.config()
    assert rt in (1, 2, 3, 4) and 1 <= fd <= 6
    for rep in range(4):
        for row in plan.outs:
            for o in row:
                o.fill_(-1.0)
        torch.cuda.synchronize()
        # eager work between replays on the same stream
        _ = ss.shadow_cast(hs[0], texels[0], *suns[0], params)
        plan.launch()
        torch.cuda.synchronize()
        for t in range(len(hs)):
            for k in range(len(suns)):
                assert same(plan.outs[t][k], ref[t][k]), (rep, t, k)
    plan.close()


def test_full_batched_workload(ss):
    """8 tiles of 512^2 .. 4096^2 x 64 suns (3.52 G rays) in one graph replay."""
    from synth import config, dem_for, sun_list
    c = config("batched")
    hs = [dem_for("batched", t, device=dev()) for t in range(len(c["tiles"]))]
    texels = [D for _, _, D in c["tiles"]]
    suns = sun_list("batched")
    params = ss.Params(radius_m=R, max_len_m=c["max_len"])
    print("creating plan", flush=True)
    plan = ss.BatchedPlan(hs, texels, suns, params)
    print("plan config", plan.config(), flush=True)
    plan.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for t in (0, 2, 6):
        for k in (0, 31, 63):
            mm = ss.maxmip(hs[t])
            one = ss.shadow_cast(hs[t], texels[t], *suns[k], params, mm=mm)
            torch.cuda.synchronize()
            assert same(plan.outs[t][k], one), (t, k)
    for t, k in ((1, 5), (7, 60)):
        W, H, D = c["tiles"][t]
        e, a, r = suns[k]
        p = oracle.Params(W, H, D, R, e, a, r, max_len_m=c["max_len"])
        rays = np.sort(rng.choice(W * H, size=3000, replace=False)).astype(np.int64)
        st = compare(hs[t].cpu().numpy(), p, plan.outs[t][k].cpu().numpy(), rays,
                     label=f"batched tile{t} sun{k}")
        assert_parity(st)
    plan.close()
