"""GPU tests of the exact mode (the minimum over the whole half-texel sample
grid, by branch and bound over the tap-bound pyramid) and of the tap-bound
pyramid itself, through the C ABI: the pyramid bit-exact against the oracle's
definition; the exact mode bit-identical to uniform stepping at half a texel
(the same sample set) with every prune and ray-tile setting; and parity with
the oracle's dense stepping on small, ragged, degenerate and full-size tiles."""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

R = 1737400.0
RL = math.radians(0.267)


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


def run(ss, hd, p: oracle.Params, mode, step=1.0, prune=1, ray_tile=0, mm=None, bound=None):
    params = ss.Params(radius_m=p.radius_m, max_len_m=p.max_len_m, mode=mode, uniform_step=step,
                       prune=prune, ray_tile=ray_tile)
    s = ss.shadow_cast(hd, p.texel_m, p.elev, p.azim, p.ang_radius, params, mm=mm, bound=bound)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


BOUND_SHAPES = [(1, 1), (1, 9), (7, 1), (2, 3), (37, 53), (64, 64), (200, 136), (130, 1030),
                (1536, 1536), (4096, 4096)]


@pytest.mark.parametrize("shape", BOUND_SHAPES)
def test_bound_pyramid_bit_exact(ss, shape):
    print("bound", shape, flush=True)
    rng = np.random.default_rng(shape[0] * 5 + shape[1])
    h = (rng.standard_normal(shape) * 300).astype(np.float32)
    h.flat[::53] = -0.0
    hd = torch.from_numpy(h).to(dev())
    got = ss.bound_unpack(ss.bound_build(hd), shape[1], shape[0])
    ref = oracle.tap_bound(h)
    assert len(got) == len(ref)
    for m, (g, r) in enumerate(zip(got, ref)):
        assert np.array_equal(bits(g.cpu().numpy()), bits(r)), (shape, m)


CASES = [((256, 256), 20.0, R, 1.5, 2.2, 0.0), ((136, 200), 20.0, R, 1.5, 0.4, 0.0),
         ((136, 200), 20.0, math.inf, 1.5, 2.8, 0.0), ((77, 301), 10.0, R, 0.6, 4.0, 0.0),
         ((250, 61), 30.0, R, 3.5, 5.6, 0.0), ((129, 129), 5.0, math.inf, 0.25, 1.2, 0.0),
         ((256, 240), 15.0, R, 1.0, 4.1, 1500.0), ((200, 200), 10.0, R, 0.2, 0.9, 0.0)]


@pytest.mark.parametrize("shape,D,radius,e_deg,az,cap", CASES)
def test_exact_is_half_texel_stepping_and_matches_oracle(ss, shape, D, radius, e_deg, az, cap):
    print("exact", shape, D, radius, e_deg, az, cap, flush=True)
    h = rough(shape, shape[0] * 3 + shape[1], 150.0)
    hd = torch.from_numpy(h).to(dev())
    p = oracle.Params(shape[1], shape[0], D, radius, math.radians(e_deg), az, RL, max_len_m=cap,
                      mode=2)
    base = run(ss, hd, p, mode=1, step=0.5, prune=0)
    for prune in (1, 0):
        for tile in (1, 2, 3, 4):
            got = run(ss, hd, p, mode=2, prune=prune, ray_tile=tile)
            assert np.array_equal(bits(got), bits(base)), (prune, tile)
    assert np.array_equal(bits(run(ss, hd, p, mode=1, step=0.5, prune=1)), bits(base))
    assert_parity(compare(h, p, base, label=f"exact {shape}"))


def test_small_workload_exact_full_grid(ss):
    from synth import dem_for, sun_list
    h = dem_for("small").numpy()
    hd = torch.from_numpy(h).to(dev())
    e, a, r = sun_list("small")[0]
    p = oracle.Params(256, 256, 20.0, R, e, a, r, mode=2)
    got = run(ss, hd, p, mode=2)
    assert_parity(compare(h, p, got, label="small exact"))
    # never lit where the descent is dark: the descent's samples are a subset
    dp = run(ss, hd, p, mode=0)
    assert np.all(got <= dp + 2e-6)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 3)])
def test_exact_degenerate_tiles(ss, shape):
    h = rough(shape, 5, 50.0)
    hd = torch.from_numpy(h).to(dev())
    for radius in (R, math.inf):
        p = oracle.Params(shape[1], shape[0], 10.0, radius, math.radians(1.0), 0.3, RL, mode=2)
        got = run(ss, hd, p, mode=2)
        assert np.array_equal(bits(got), bits(run(ss, hd, p, mode=1, step=0.5)))
        assert_parity(compare(h, p, got, label=f"exact degenerate {shape}"))


def sampled(n_texels, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_texels, size=k, replace=False)).astype(np.int64)


@pytest.mark.parametrize("name,suns,k", [("tile", 2, 4000), ("polar", 1, 1500)])
def test_exact_full_size(ss, name, suns, k):
    """Full-size tiles: bit-identical to half-texel stepping over the whole
    image, and the oracle's dense stepping on sampled rays."""
    from synth import config, dem_for, sun_list
    c = config(name)
    W, H, D = c["tiles"][0]
    print("exact full size", name, flush=True)
    hd = dem_for(name, device=dev())
    mm = ss.maxmip(hd)
    bound = ss.bound_build(hd)
    h = hd.cpu().numpy()
    for si, (e, a, r) in enumerate(sun_list(name)[:suns]):
        p = oracle.Params(W, H, D, R, e, a, r, max_len_m=c["max_len"], mode=2)
        got = run(ss, hd, p, mode=2, mm=mm, bound=bound)
        ref = run(ss, hd, p, mode=1, step=0.5, mm=mm)
        assert np.array_equal(bits(got), bits(ref)), (name, si)
        st = compare(h, p, got, sampled(W * H, k, 21 + si), label=f"{name} sun{si} exact")
        assert_parity(st)
