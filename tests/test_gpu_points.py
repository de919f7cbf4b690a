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


# ---------------------------------------------------------------------------
# Adjoint at fixed points (ss_shadow_points_backward)
# ---------------------------------------------------------------------------

def smooth(shape, seed, amp):
    """Sums of plane waves (no texel noise): many rays with well-conditioned decisions."""
    rng = np.random.default_rng(seed)
    rows, width = shape
    y, x = np.mgrid[0:rows, 0:width].astype(np.float64)
    h = np.zeros(shape)
    for k in range(6):
        f = rng.uniform(0.01, 0.2)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    return h.astype(np.float32)


def centres(rows, width):
    jj, ii = torch.meshgrid(torch.arange(rows, device="cuda"), torch.arange(width, device="cuda"),
                            indexing="ij")
    return torch.stack([ii + 0.5, jj + 0.5], dim=-1).float().contiguous()


@pytest.mark.parametrize("mode", [0, 2, 3])
@pytest.mark.parametrize("radius", [R, math.inf])
def test_backward_centres_equal_grid(ss, mode, radius):
    """At texel centres the bilinear origin is the texel itself: the points adjoint
    (list and image form) equals the tile adjoint up to the order of the atomic sums."""
    h = smooth((136, 200), 71, 100.0)
    hd = torch.from_numpy(h).cuda()
    p = ss.Params(radius_m=radius, mode=mode)
    e, a = math.radians(1.4), 2.0
    g = torch.randn(136, 200, generator=torch.Generator().manual_seed(mode)).cuda()
    gh_t, gs_t = ss.shadow_cast_backward(hd, 15.0, e, a, g, RL, p)
    img = centres(136, 200)
    gh_l, gs_l = ss.shadow_points_backward(hd, 15.0, e, a, img.reshape(-1, 2), g.reshape(-1), RL, p)
    gh_i, gs_i = ss.shadow_points_backward(hd, 15.0, e, a, img, g, RL, p)
    torch.cuda.synchronize()
    nt = float(gh_t.norm())
    assert nt > 0
    for gh, gs in ((gh_l, gs_l), (gh_i, gs_i)):
        assert float((gh - gh_t).norm()) <= 1e-5 * nt
        assert torch.allclose(gs, gs_t, rtol=1e-7, atol=1e-12 * float(gs_t.abs().max()))


def test_backward_image_skips_nan_and_ragged(ss):
    """An image of points with misses (NaN) and ragged 8 x 8 tiles: the same gradient
    as the list of its finite points; zero upstream gradient adds nothing."""
    h = smooth((150, 170), 73, 100.0)
    hd = torch.from_numpy(h).cuda()
    p = ss.Params(radius_m=R)
    e, a = math.radians(1.2), 0.9
    rng = np.random.default_rng(7)
    H, W = 61, 77
    xy = np.stack([rng.uniform(0, 170, (H, W)), rng.uniform(0, 150, (H, W))], axis=-1).astype(np.float32)
    miss = rng.random((H, W)) < 0.2
    xy[miss] = np.nan
    g = rng.standard_normal((H, W)).astype(np.float32)
    img = torch.from_numpy(xy).cuda()
    gi = torch.from_numpy(g).cuda()
    gh_i, gs_i = ss.shadow_points_backward(hd, 10.0, e, a, img, gi, RL, p)
    keep = ~miss.reshape(-1)
    lst = torch.from_numpy(np.ascontiguousarray(xy.reshape(-1, 2)[keep])).cuda()
    gh_l, gs_l = ss.shadow_points_backward(hd, 10.0, e, a, lst,
                                           torch.from_numpy(g.reshape(-1)[keep]).cuda(), RL, p)
    z = torch.zeros_like(gi)
    gh_z, gs_z = ss.shadow_points_backward(hd, 10.0, e, a, img, z, RL, p)
    torch.cuda.synchronize()
    assert float(gh_l.norm()) > 0
    assert float((gh_i - gh_l).norm()) <= 1e-5 * float(gh_l.norm())
    assert torch.allclose(gs_i, gs_l, rtol=1e-7)
    assert not bool(gh_z.any()) and not bool(gs_z.any())


def off_lines(xy, margin=0.05):
    """Points whose bilinear origin is away from the lines through texel centres
    (the origin height's slope, hence its gradient, jumps there)."""
    f = np.mod(np.asarray(xy, dtype=np.float64) - 0.5, 1.0)
    return ((f > margin) & (f < 1.0 - margin)).all(axis=1)


@pytest.mark.parametrize("mode", [0, 2, 3])
@pytest.mark.parametrize("radius,e_deg,az", [(R, 1.5, 0.7), (math.inf, 2.0, 2.3), (R, 1.0, 4.1)])
def test_points_backward_matches_reference_gradient(ss, mode, radius, e_deg, az):
    """Against the float64 reference gradient along the oracle's branch from the same
    points (origin height the differentiable bilinear terrain), on rays whose every
    decision has a wide FP64 margin and whose origin is off the bilinear kinks."""
    from oracle import grad_ref
    from parity import well_conditioned
    shape = (192, 224)
    h = smooth(shape, 79 + mode, 80.0)
    rng = np.random.default_rng(int(e_deg * 10) + 3 * mode)
    n = 30000
    xy = np.stack([rng.uniform(0, shape[1], n), rng.uniform(0, shape[0], n)], axis=1).astype(np.float32)
    xy64 = xy.astype(np.float64)
    po = oracle.Params(shape[1], shape[0], 20.0, radius, math.radians(e_deg), az, RL, mode=mode)
    s, _, tr = oracle.shadow_points(h, po, xy64, trace=True)
    mask = well_conditioned(tr) & off_lines(xy64) & (s > 0.0) & (s < 1.0)
    print("well-conditioned penumbra points", int(mask.sum()))
    assert mask.sum() > 200
    g = rng.standard_normal(n) * mask
    ref_h, ref_e, ref_a, _ = grad_ref.reference_gradient(h, po, tr, g, points=xy64)
    hd = torch.from_numpy(h).cuda()
    gh, gsun = ss.shadow_points_backward(hd, 20.0, po.elev, az, torch.from_numpy(xy).cuda(),
                                         torch.from_numpy(g.astype(np.float32)).cuda(), RL,
                                         ss.Params(radius_m=radius, mode=mode))
    torch.cuda.synchronize()
    gh = gh.cpu().numpy().astype(np.float64)
    gsun = gsun.cpu().numpy()
    rel = np.linalg.norm(gh - ref_h) / np.linalg.norm(ref_h)
    print("rel err dL/dh", rel, "sun", gsun, ref_e, ref_a)
    assert rel <= 1e-3
    assert abs(gsun[0] - ref_e) <= 1e-3 * abs(ref_e) + 1e-9
    assert abs(gsun[1] - ref_a) <= 1e-3 * max(abs(ref_a), 1e-3 * abs(ref_e))


def test_shadow_at_autograd_through_frame(ss):
    """A frame's view hits as fixed points: autograd through shadow_at gives the points
    adjoint's gradients in h and in the sun direction; misses give NaN and no gradient."""
    from synth.configs import view_scene
    import synth
    h = synth.dem_for("small", device="cuda")
    cam = ss.Camera(**view_scene("oblique", 96, 64, 256, 256, 20.0))
    _, xy = ss.view_cast(h, 20.0, cam, R)
    e = torch.tensor(math.radians(1.3), dtype=torch.float64, requires_grad=True)
    a = torch.tensor(0.6, dtype=torch.float64, requires_grad=True)
    hh = h.clone().requires_grad_(True)
    p = ss.Params(radius_m=R)
    s = ss.shadow_at(hh, e, a, xy, 20.0, RL, p)
    fin = torch.isfinite(s)
    assert bool(fin.any())
    assert torch.equal(fin, torch.isfinite(xy[..., 0]))
    w = torch.randn(s.shape, generator=torch.Generator().manual_seed(5)).cuda()
    (torch.where(fin, s, torch.zeros_like(s)) * w).sum().backward()
    g = torch.where(fin, w, torch.zeros_like(w)).contiguous()
    gh, gsun = ss.shadow_points_backward(h, 20.0, float(e), float(a), xy, g, RL, p)
    torch.cuda.synchronize()
    assert float(gh.norm()) > 0
    assert float((hh.grad - gh).norm()) <= 1e-5 * float(gh.norm())
    assert abs(float(e.grad) - float(gsun[0])) <= 1e-7 * abs(float(gsun[0])) + 1e-12
    assert abs(float(a.grad) - float(gsun[1])) <= 1e-7 * abs(float(gsun[1])) + 1e-12
