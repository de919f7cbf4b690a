"""GPU adjoint (hand-written backward kernel) against the torch float64
reference gradient along the oracle's branch, on rays whose every decision has
an FP64 margin well above single-precision resolution (the others get zero
upstream gradient on both sides), and against finite differences of the GPU
forward on the 2048^2 differentiable workload."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import grad_ref
from parity import well_conditioned

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
    for k in range(6):
        f = rng.uniform(0.01, 0.2)
        th = rng.uniform(0, 2 * math.pi)
        h += amp / (k + 1) * np.sin(f * (x * math.cos(th) + y * math.sin(th)) + rng.uniform(0, 6))
    return h.astype(np.float32)


def gpu_backward(ss, h, p, g):
    hd = torch.from_numpy(h).to(dev())
    gd = torch.from_numpy(g.astype(np.float32).reshape(h.shape)).to(dev())
    params = ss.Params(radius_m=p.radius_m, max_len_m=p.max_len_m, mode=p.mode)
    gh, gsun = ss.shadow_cast_backward(hd, p.texel_m, p.elev, p.azim, gd, p.ang_radius, params)
    torch.cuda.synchronize()
    return gh.cpu().numpy().astype(np.float64), gsun.cpu().numpy()


CASES = [((256, 256), 20.0, R, 1.5, 0.7, 0.0), ((192, 256), 20.0, math.inf, 2.0, 2.3, 0.0),
         ((256, 240), 15.0, R, 1.0, 4.1, 1500.0)]


@pytest.mark.parametrize("mode", [0, 2, 3])
@pytest.mark.parametrize("shape,D,radius,e_deg,az,cap", CASES)
def test_adjoint_matches_reference_gradient(ss, shape, D, radius, e_deg, az, cap, mode):
    """Descent (mode 0), exact mode (2) and point descent (3): in each the
    deciding sample sits at t = (n + 1) delta/2, the chain the reference
    differentiates."""
    h = rough(shape, shape[0] + 3, 80.0)
    p = oracle.Params(shape[1], shape[0], D, radius, math.radians(e_deg), az, RL, max_len_m=cap,
                      mode=mode)
    s, _, tr = oracle.shadow(h, p, trace=True)
    mask = well_conditioned(tr)
    inside = (s.reshape(-1) > 0.0) & (s.reshape(-1) < 1.0)
    print("well-conditioned", mask.mean(), "penumbra", inside.mean(), (mask & inside).sum())
    assert (mask & inside).sum() > 100
    rng = np.random.default_rng(1)
    g = rng.standard_normal(s.size) * mask
    ref_h, ref_e, ref_a, _ = grad_ref.reference_gradient(h, p, tr, g)
    gh, gsun = gpu_backward(ss, h, p, g)
    rel = np.linalg.norm(gh - ref_h) / np.linalg.norm(ref_h)
    print("rel err dL/dh", rel, "sun", gsun, ref_e, ref_a)
    assert rel <= 1e-3
    assert abs(gsun[0] - ref_e) <= 1e-3 * abs(ref_e) + 1e-9
    assert abs(gsun[1] - ref_a) <= 1e-3 * max(abs(ref_a), 1e-3 * abs(ref_e))


def test_adjoint_full_size_sampled(ss):
    """2048^2 differentiable workload: upstream gradient on the well-conditioned
    rays of a 200000-ray random sample; the reference runs on exactly those rays."""
    from synth import config, dem_for, sun_list
    c = config("diff")
    W, H, D = c["tiles"][0]
    hd = dem_for("diff", device=dev())
    h = hd.cpu().numpy()
    e, a, r = sun_list("diff")[0]
    p = oracle.Params(W, H, D, R, e, a, r, max_len_m=c["max_len"])
    rng = np.random.default_rng(3)
    rays = np.sort(rng.choice(W * H, size=200000, replace=False)).astype(np.int64)
    s, _, tr = oracle.shadow_threaded(h, p, rays, trace=True)
    mask = well_conditioned(tr) & (s > 0) & (s < 1)
    print("sampled well-conditioned penumbra rays", int(mask.sum()))
    assert mask.sum() > 300
    g_r = rng.standard_normal(rays.size) * mask
    ref_h, ref_e, ref_a, _ = grad_ref.reference_gradient(h, p, tr, g_r, rays=rays)
    g = np.zeros(W * H)
    g[rays] = g_r
    gh, gsun = gpu_backward(ss, h, p, g)
    rel = np.linalg.norm(gh - ref_h) / np.linalg.norm(ref_h)
    print("rel err dL/dh", rel, "sun", gsun, ref_e, ref_a)
    assert rel <= 1e-3
    assert abs(gsun[0] - ref_e) <= 1e-3 * abs(ref_e)
    assert abs(gsun[1] - ref_a) <= 1e-3 * max(abs(ref_a), 1e-3 * abs(ref_e))


def lambert_loss(ss, h, e, a, r, D, params, target):
    """Shaded image I = s * max(0, n_t . L) with the normal from central
    differences of h; L = sum (I - target)^2 (float64)."""
    L = torch.tensor([math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), math.sin(e)],
                     dtype=torch.float64, device=h.device)
    s = ss.shadow(h, torch.tensor(e, dtype=torch.float64), torch.tensor(a, dtype=torch.float64),
                  D, r, params)
    hp = torch.nn.functional.pad(h[None, None].double(), (1, 1, 1, 1), mode="replicate")[0, 0]
    dx = (hp[1:-1, 2:] - hp[1:-1, :-2]) / (2 * D)
    dy = (hp[2:, 1:-1] - hp[:-2, 1:-1]) / (2 * D)
    nrm = torch.stack([-dx, -dy, torch.ones_like(dx)])
    nrm = nrm / torch.sqrt((nrm * nrm).sum(0))
    lam = torch.clamp((nrm * L.view(3, 1, 1)).sum(0), min=0.0)
    img = s.double() * lam
    return ((img - target) ** 2).sum(), img


def test_differentiable_workload_finite_differences(ss):
    """2048^2 DEM, forward shadow + Lambert shading, loss against a target
    rendered from heights perturbed by N(0, 5 m); dL/dh from the adjoint vs
    central differences of the GPU forward (step 1e-2 m) at 64 texels."""
    from synth import config, dem_for, sun_list
    c = config("diff")
    W, H, D = c["tiles"][0]
    h0 = dem_for("diff", device=dev())
    e, a, r = sun_list("diff")[0]
    params = ss.Params(radius_m=R, max_len_m=c["max_len"])
    gen = torch.Generator(device="cpu").manual_seed(99)
    noisy = (h0 + (torch.randn(H, W, generator=gen) * 5.0).to(dev())).contiguous()
    with torch.no_grad():
        _, target = lambert_loss(ss, noisy, e, a, r, D, params, 0.0)
    h = h0.clone().requires_grad_(True)
    loss, img0 = lambert_loss(ss, h, e, a, r, D, params, target)
    loss.backward()
    g = h.grad.detach()
    # texels where the loss is sensitive, spread over the tile
    rng = np.random.default_rng(5)
    cand = torch.nonzero(g.abs() > g.abs().mean()).cpu().numpy()
    pick = cand[rng.choice(len(cand), size=min(len(cand), 256), replace=False)]
    eps = 1e-2
    checked = 0
    with torch.no_grad():
        for j, i in pick:
            if checked >= 64:
                break
            vals = []
            for sgn in (1.0, -1.0, 0.0):
                hh = h0.clone()
                hh[j, i] += sgn * eps
                # rounding of the perturbed float32 height
                step = float(hh[j, i] - h0[j, i])
                lv, _ = lambert_loss(ss, hh, e, a, r, D, params, target)
                vals.append((float(lv), step))
            (lp, sp), (lm, sm), (l0, _) = vals
            fwd = (lp - l0) / sp
            bwd = (l0 - lm) / (-sm)
            if abs(fwd - bwd) > 0.05 * max(abs(fwd), abs(bwd)) + 1e-6:
                continue  # a decision flipped inside +-eps: not differentiable here
            fd = (lp - lm) / (sp - sm)
            gk = float(g[j, i])
            assert abs(fd - gk) <= 1e-2 * abs(fd) + 1e-4 * float(g.abs().max()), (i, j, fd, gk)
            checked += 1
    assert checked >= 40
