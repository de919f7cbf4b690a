"""GPU parity of the maximum mipmap and the forward shadow kernels against the
FP64 oracle, closed forms, result invariance of the tuning knobs and early
exits, and edge cases.  Every call goes through the C ABI (libsoftshadow.so)."""
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


# ---------------------------------------------------------------- max-mip

MIP_SHAPES = [(1, 1), (1, 9), (7, 1), (37, 53), (64, 64), (200, 136), (256, 256), (130, 1030),
              (1536, 1536), (3072, 3072), (4096, 4096)]


@pytest.mark.parametrize("shape", MIP_SHAPES)
def test_maxmip_bit_exact(ss, shape):
    print("maxmip", shape, flush=True)
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    h = (rng.standard_normal(shape) * 500).astype(np.float32)
    h.flat[::97] = -0.0
    hd = torch.from_numpy(h).to(dev())
    ref = oracle.maxmip(h)
    for fuse in (6, 4, 1):
        mm = ss.maxmip(hd, fuse_depth=fuse)
        got = ss.maxmip_unpack(mm, shape[1], shape[0])
        assert len(got) == len(ref)
        for m, (g, r) in enumerate(zip(got, ref), start=1):
            assert np.array_equal(g.cpu().numpy().view(np.uint32), r.view(np.uint32)), (fuse, m)


def test_maxmip_unaligned_source(ss):
    rng = np.random.default_rng(3)
    base = (rng.standard_normal(1 + 96 * 96) * 100).astype(np.float32)
    h = base[1:].reshape(96, 96)
    hd_base = torch.from_numpy(base).to(dev())
    hd = hd_base[1:].view(96, 96)  # 4-byte aligned only: scalar load path
    mm = ss.maxmip(hd)
    for g, r in zip(ss.maxmip_unpack(mm, 96, 96), oracle.maxmip(np.ascontiguousarray(h))):
        assert np.array_equal(g.cpu().numpy(), r)


def test_maxmip_polar_size(ss):
    """16384^2 (the large polar workload): 15 levels, bit-exact."""
    from synth import dem_for
    print("maxmip polar", flush=True)
    hd = dem_for("polar", device=dev())
    mm = ss.maxmip(hd)
    torch.cuda.synchronize()
    h = hd.cpu().numpy()
    ref = oracle.maxmip(h)
    got = ss.maxmip_unpack(mm, 16384, 16384)
    assert len(got) == 14
    for g, r in zip(got, ref):
        assert np.array_equal(g.cpu().numpy(), r)


# ---------------------------------------------------------------- forward parity

def run(ss, h, p: oracle.Params, prune=1, ray_tile=0, mm=None):
    hd = torch.from_numpy(h).to(dev())
    params = ss.Params(radius_m=p.radius_m, max_len_m=p.max_len_m, n_prime0=p.n_prime0,
                       schedule=p.schedule, n_segments=p.n_segments, mode=p.mode,
                       uniform_step=p.uniform_step, prune=prune, ray_tile=ray_tile)
    s = ss.shadow_cast(hd, p.texel_m, p.elev, p.azim, p.ang_radius, params, mm=mm)
    torch.cuda.synchronize()
    return s.cpu().numpy()


def test_small_workload_dp_full_grid(ss):
    from synth import dem_for, sun_list
    h = dem_for("small").numpy()
    e, a, r = sun_list("small")[0]
    p = oracle.Params(256, 256, 20.0, R, e, a, r)
    st = compare(h, p, run(ss, h, p), label="small dp")
    assert_parity(st)


def test_small_workload_uniform_full_grid(ss):
    from synth import dem_for, sun_list
    h = dem_for("small").numpy()
    e, a, r = sun_list("small")[0]
    for step in (1.0, 0.5):
        p = oracle.Params(256, 256, 20.0, R, e, a, r, mode=1, uniform_step=step)
        st = compare(h, p, run(ss, h, p), label=f"small uniform {step}")
        assert_parity(st)


RAGGED = [((136, 200), 20.0, R, 1.5, 0.4), ((136, 200), 20.0, math.inf, 1.5, 2.8),
          ((77, 301), 10.0, R, 0.6, 4.0), ((250, 61), 30.0, R, 3.5, 5.6),
          ((129, 129), 5.0, math.inf, 0.25, 1.2)]


@pytest.mark.parametrize("shape,D,radius,e_deg,az", RAGGED)
def test_ragged_tiles_dp_and_uniform(ss, shape, D, radius, e_deg, az):
    h = rough(shape, shape[0] + shape[1], 150.0)
    p = oracle.Params(shape[1], shape[0], D, radius, math.radians(e_deg), az, RL)
    assert_parity(compare(h, p, run(ss, h, p), label=f"ragged dp {shape}"))
    pu = p.replace(mode=1)
    assert_parity(compare(h, pu, run(ss, h, pu), label=f"ragged uniform {shape}"))


def test_equal_schedule_and_caps(ss):
    """The paper's {5,5,5} runs and a horizontal cap shorter than the tile."""
    h = rough((160, 160), 5, 120.0)
    p = oracle.Params(160, 160, 10.0, R, math.radians(1.0), 0.9, RL, schedule=1, n_segments=3)
    assert_parity(compare(h, p, run(ss, h, p), label="equal 5,5,5"))
    p2 = oracle.Params(160, 160, 10.0, R, math.radians(1.0), 0.9, RL, max_len_m=700.0)
    assert_parity(compare(h, p2, run(ss, h, p2), label="cap 700 m"))
    p3 = p2.replace(mode=1)
    assert_parity(compare(h, p3, run(ss, h, p3), label="uniform cap 700 m"))


# ---------------------------------------------------------------- closed forms

def S(d):
    d = max(-1.0, min(1.0, d))
    return (math.pi - math.acos(d) + d * math.sqrt(1 - d * d)) / math.pi


@pytest.mark.parametrize("e_deg", [1.5, 3.0])
def test_straight_ridge_closed_form(ss, e_deg):
    W, rows, D, ir, hr = 256, 6, 20.0, 250, 100.0
    h = np.zeros((rows, W), np.float32)
    h[:, ir] = hr
    e = math.radians(e_deg)
    for mode, step in ((0, 1.0), (1, 0.5)):
        p = oracle.Params(W, rows, D, math.inf, e, 0.0, RL, mode=mode, uniform_step=step)
        s = run(ss, h, p)
        want = np.array([S((e - math.atan(hr / ((ir - i) * D))) / RL) for i in range(ir)])
        assert np.max(np.abs(s[:, :ir] - want[None, :])) < 1e-4
        assert np.all(s[:, ir:] == 1.0)


@pytest.mark.parametrize("radius", [R, math.inf])
def test_flat_ground_lit_and_half_set_sun(ss, radius):
    h = np.zeros((64, 64), np.float32)
    for mode in (0, 1):
        p = oracle.Params(64, 64, 20.0, radius, math.radians(0.3), 0.7, RL, mode=mode)
        assert np.all(run(ss, h, p) == 1.0)
    if math.isinf(radius):
        e = math.radians(0.2)
        p = oracle.Params(64, 64, 20.0, radius, e, 0.7, RL)
        s = run(ss, h, p)
        s_ref, _ = oracle.shadow(h, p)
        inner = s_ref < 1.0
        assert inner.mean() > 0.9
        assert np.max(np.abs(s[inner] - S(e / RL))) < 1e-5


# ---------------------------------------------------------------- invariance

def test_prune_and_ray_tiles_do_not_change_results(ss):
    from synth import dem_for, sun_list
    h = dem_for("small").numpy()
    e, a, r = sun_list("small")[0]
    for radius in (R, math.inf):
        for mode in (0, 1):
            p = oracle.Params(256, 256, 20.0, radius, e, a, r, mode=mode)
            base = run(ss, h, p, prune=0)
            for tile in (1, 2, 3, 4):
                for prune in (0, 1):
                    got = run(ss, h, p, prune=prune, ray_tile=tile)
                    assert np.array_equal(got.view(np.uint32), base.view(np.uint32)), (radius, mode, tile, prune)


# ---------------------------------------------------------------- full-size workloads

def sampled(n_texels, k, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_texels, size=k, replace=False)).astype(np.int64)


@pytest.mark.parametrize("name,k", [("tile", 20000), ("diff", 20000)])
def test_full_size_sampled_parity(ss, name, k):
    from synth import config, dem_for, sun_list
    c = config(name)
    W, Hh, D = c["tiles"][0]
    print("full size", name, flush=True)
    hd = dem_for(name, device=dev())
    h = hd.cpu().numpy()
    mm = ss.maxmip(hd)
    suns = sun_list(name)
    for si, (e, a, r) in enumerate(suns[:3]):
        for mode in (0, 1):
            p = oracle.Params(W, Hh, D, R, e, a, r, max_len_m=c["max_len"], mode=mode)
            params = ss.Params(radius_m=R, max_len_m=c["max_len"], mode=mode)
            s = ss.shadow_cast(hd, D, e, a, r, params, mm=mm)
            torch.cuda.synchronize()
            rays = sampled(W * Hh, k // (4 if mode else 1), 11 + si)
            st = compare(h, p, s.cpu().numpy(), rays, label=f"{name} sun{si} mode{mode}")
            assert_parity(st)


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 3)])
def test_degenerate_tiles(ss, shape):
    h = rough(shape, 3, 50.0)
    for radius in (R, math.inf):
        for mode in (0, 1):
            p = oracle.Params(shape[1], shape[0], 10.0, radius, math.radians(1.0), 0.3, RL, mode=mode)
            s = run(ss, h, p)
            s_ref, _ = oracle.shadow(h, p)
            assert np.max(np.abs(s - s_ref)) <= 1e-4


def test_empty_tile_is_a_noop(ss):
    import ctypes as C
    from paper_2005_06671_amd import _lib as L
    t = L.SSTile(0, 0, 0, 5, 1.0)
    s = L.SSSun(0.1, 0.2, RL)
    p = L.SSParams(R, 0.0, 5, 0, 0, 0, 1.0, 1, 0)
    assert L.lib().ss_shadow_cast(C.byref(t), C.byref(s), C.byref(p), 0, 0) == 0
    assert L.lib().ss_maxmip_build(0, 0, 7, 0, 0, 0) == 0


def test_sun_below_local_horizon(ss):
    """Elevation 0.2 deg on a 33 km tile: the local horizon tilts by more than
    the sun's elevation near the edges, so tip heights first decrease."""
    h = rough((256, 256), 8, 30.0)
    p = oracle.Params(256, 256, 128.0, R, math.radians(0.2), 1.0, RL, max_len_m=20000.0)
    assert_parity(compare(h, p, run(ss, h, p), label="low sun big texels"))


def test_gather_tiles_probe_reads_its_patches(ss):
    """The coherent gather probe reads exactly the 8 x 8 patches its definition names: lane
    k of a wavefront sums src[(py + k // 8) * width + px + k % 8] over its steps, with the
    patch origins drawn from the wavefront's xorshift sequence (recomputed here)."""
    width, rows, iters, n_threads = 40, 24, 8, 512
    src = torch.arange(width * rows, dtype=torch.float32, device=dev()).view(rows, width) * 0.25
    out = ss.probe_gather_tiles(src, iters, n_threads)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    s_np = src.cpu().numpy().reshape(-1).astype(np.float64)
    M = 0xFFFFFFFF
    for tid in range(n_threads):
        lane, wave = tid & 63, tid >> 6
        x = (wave * 2654435761 + 97) & M
        x ^= x >> 16
        acc = [0.0] * 8
        for k in range(0, iters, 8):
            for q in range(8):
                x ^= (x << 13) & M
                x ^= x >> 17
                x ^= (x << 5) & M
                px, py = (x & 0xFFFF) % (width - 7), (x >> 16) % (rows - 7)
                acc[q] += s_np[(py + (lane >> 3)) * width + px + (lane & 7)]
        ref = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]))
        assert abs(got[tid] - ref) <= 1e-3, (tid, got[tid], ref)
