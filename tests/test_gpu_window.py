"""GPU tests of the ray window (rays start in a sub-rectangle, terrain is the
whole tile) through the C ABI: bit-identical to the same texels of a
whole-tile launch in every mode and ray-tile shape; a core inside a halo sees
the halo's terrain (and the oracle agrees on those rays) where the cropped
core alone does not; the recorded adjoint over a window equals the
whole-tile adjoint with the upstream gradient zero outside it; batched
windows equal per-tile windows."""
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


def rough(shape, seed, amp):
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(6):
        f = rng.uniform(0.01, 0.2)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    return h.astype(np.float32)


WINDOWS = [(0, 0, 200, 136), (17, 9, 61, 45), (150, 100, 50, 36), (0, 135, 200, 1), (199, 0, 1, 136)]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_window_equals_whole_tile(ss, mode):
    h = rough((136, 200), 41, 120.0)
    hd = torch.from_numpy(h).cuda()
    for radius in (R, math.inf):
        p = ss.Params(radius_m=radius, mode=mode)
        full = ss.shadow_cast(hd, 15.0, math.radians(1.3), 2.1, RL, p)
        for (x0, y0, w, hh) in WINDOWS:
            for tile in (1, 3):
                pw = ss.Params(radius_m=radius, mode=mode, ray_tile=tile)
                got = ss.shadow_cast(hd, 15.0, math.radians(1.3), 2.1, RL, pw,
                                     window=(x0, y0, w, hh))
                torch.cuda.synchronize()
                assert got.shape == (hh, w)
                ref = full[y0:y0 + hh, x0:x0 + w].contiguous()
                assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), (radius, x0, y0)


def test_core_sees_its_halo(ss):
    """Plane geometry: a 64 x 64 core at the centre of a 192 x 192 tile whose
    halo holds a ridge toward the sun; the core's shadows follow the oracle over
    the whole tile, and differ from the cropped core's."""
    W = 192
    h = rough((W, W), 7, 30.0)
    h[:, 150:154] += 400.0  # ridge beyond the core, toward the sun (+column)
    hd = torch.from_numpy(h).cuda()
    e, a, D = math.radians(2.0), 0.05, 10.0
    win = (64, 64, 64, 64)
    p = ss.Params(radius_m=math.inf)
    got = ss.shadow_cast(hd, D, e, a, RL, p, window=win)
    torch.cuda.synchronize()
    rays = np.array([(64 + y) * W + 64 + x for y in range(64) for x in range(64)], dtype=np.int64)
    po = oracle.Params(W, W, D, math.inf, e, a, RL)
    s_full = np.zeros(W * W, dtype=np.float32)
    s_full[rays] = got.cpu().numpy().reshape(-1)
    assert_parity(compare(h, po, s_full, rays, label="core in halo"))
    core = torch.from_numpy(np.ascontiguousarray(h[64:128, 64:128])).cuda()
    alone = ss.shadow_cast(core, D, e, a, RL, p)
    torch.cuda.synchronize()
    assert float((alone - got).abs().max()) > 0.5  # the ridge shades part of the core


def test_window_adjoint(ss):
    h = rough((136, 200), 43, 80.0)
    hd = torch.from_numpy(h).cuda()
    e, a = math.radians(1.5), 0.7
    p = ss.Params(radius_m=R)
    win = (31, 17, 97, 70)
    rng = np.random.default_rng(3)
    gw = torch.from_numpy(rng.standard_normal((70, 97)).astype(np.float32)).cuda()
    s_w, smp = ss.shadow_cast_save(hd, 20.0, e, a, RL, p, window=win)
    gh_w, gs_w = ss.shadow_cast_backward_saved(hd, 20.0, e, a, smp, gw, RL, p, window=win)
    g_full = torch.zeros_like(hd)
    g_full[17:87, 31:128] = gw
    gh_f, gs_f = ss.shadow_cast_backward(hd, 20.0, e, a, g_full, RL, p)
    torch.cuda.synchronize()
    assert float((gh_w - gh_f).double().norm()) <= 1e-5 * float(gh_f.double().norm())
    assert torch.allclose(gs_w, gs_f, rtol=1e-6, atol=1e-12)


def test_batched_windows(ss, form):
    hs = [torch.from_numpy(rough(s, s[0], 100.0)).cuda() for s in [(96, 128), (136, 200)]]
    texels = [20.0, 10.0]
    wins = [(5, 7, 100, 50), None]
    suns = [(math.radians(0.9), 0.4, RL), (math.radians(2.2), 3.3, RL)]
    for mode in (0, 3):
        p = ss.Params(radius_m=R, mode=mode)
        outs = ss.shadow_cast_batched(hs, texels, suns, p, windows=wins)
        torch.cuda.synchronize()
        for t in range(2):
            for k, (e, a, r) in enumerate(suns):
                ref = ss.shadow_cast(hs[t], texels[t], e, a, r, p, window=wins[t])
                torch.cuda.synchronize()
                assert torch.equal(outs[t][k].view(torch.int32), ref.view(torch.int32)), (mode, t, k)


def test_gather_probe_sums(ss):
    """The memory probe reads only inside its buffer or window: over ones, every
    lane sums exactly its rounded-up iteration count."""
    src = torch.ones(1 << 20, device="cuda")
    for win in (0, 1 << 12, 1 << 20):
        out = ss.probe_gather(src, win, iters=12, n_threads=1 << 14)
        torch.cuda.synchronize()
        assert torch.all(out == 16.0), win


def test_valu_probe_runs_its_chains(ss):
    """The FP32 VALU probe: every lane's eight chains x -> a x + b (a = 0.999, b = 0.001 in
    FP32), 4 * iters steps each (float64 reference of the same recurrence)."""
    iters = 64
    out = ss.probe_valu(iters, 16)
    torch.cuda.synchronize()
    a, b = float(np.float32(0.999)), float(np.float32(0.001))  # the kernel's FP32 constants
    x0 = torch.arange(256, dtype=torch.float64) * 1e-3
    ref = torch.zeros(256, dtype=torch.float64)
    for c in range(8):
        v = x0 + c
        for _ in range(4 * iters):
            v = v * a + b
        ref += v
    got = out.view(16, 256).double().cpu()
    assert torch.allclose(got, ref.expand(16, 256), rtol=1e-5, atol=1e-5)
