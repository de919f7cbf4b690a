"""GPU tests of the recorded forward (ss_shadow_cast_save) and the adjoint
that reads the record (ss_shadow_cast_backward_saved), in every mode: the
forward is bit-identical to ss_shadow_cast, the recorded sample index equals
the oracle's deciding sample on penumbra rays whose decisions are well clear of
FP32 resolution, and the gradients equal the replaying adjoint's up to the
order of the atomic sums."""
import math

import numpy as np
import pytest
import torch

import oracle
from parity import well_conditioned

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


MODES = [(0, 1.0), (1, 1.0), (1, 0.5), (2, 1.0), (3, 1.0)]
CASES = [((200, 256), 20.0, R, 1.5, 0.7, 0.0), ((160, 176), 20.0, math.inf, 2.0, 2.3, 0.0),
         ((256, 240), 15.0, R, 1.0, 4.1, 1500.0)]


@pytest.mark.parametrize("mode,step", MODES)
@pytest.mark.parametrize("shape,D,radius,e_deg,az,cap", CASES)
def test_saved_forward_and_backward(ss, shape, D, radius, e_deg, az, cap, mode, step):
    print("saved", shape, mode, step, flush=True)
    h = rough(shape, shape[0] + 11, 80.0)
    hd = torch.from_numpy(h).cuda()
    e = math.radians(e_deg)
    params = ss.Params(radius_m=radius, max_len_m=cap, mode=mode, uniform_step=step)
    s_plain = ss.shadow_cast(hd, D, e, az, RL, params)
    s_save, sample = ss.shadow_cast_save(hd, D, e, az, RL, params)
    torch.cuda.synchronize()
    assert torch.equal(s_plain.view(torch.int32), s_save.view(torch.int32))
    # the recorded sample is the oracle's deciding sample on penumbra rays
    # whose every decision is well conditioned
    p = oracle.Params(shape[1], shape[0], D, radius, e, az, RL, max_len_m=cap, mode=mode,
                      uniform_step=step)
    s_or, _, tr = oracle.shadow(h, p, trace=True)
    pen = (s_or.reshape(-1) > 0) & (s_or.reshape(-1) < 1)
    mask = well_conditioned(tr) & pen
    got = sample.cpu().numpy().reshape(-1)
    assert mask.sum() > 100
    bad = np.nonzero(got[mask] != tr.reshape(-1)["n"][mask])[0]
    assert bad.size == 0, (bad.size, got[mask][bad[:5]], tr.reshape(-1)["n"][mask][bad[:5]])
    assert np.all(got[s_or.reshape(-1) == 1.0] >= -1)
    # gradients: recorded vs replayed
    g = torch.from_numpy(np.random.default_rng(5).standard_normal(shape).astype(np.float32)).cuda()
    gh1, gs1 = ss.shadow_cast_backward(hd, D, e, az, g, RL, params)
    gh2, gs2 = ss.shadow_cast_backward_saved(hd, D, e, az, sample, g, RL, params)
    torch.cuda.synchronize()
    a, b = gh1.double(), gh2.double()
    assert float((a - b).norm()) <= 1e-5 * max(float(a.norm()), 1e-30)
    assert torch.allclose(gs1, gs2, rtol=1e-6, atol=1e-9 * float(gs1.abs().max()) + 1e-12)


@pytest.mark.parametrize("mode", [0, 2])
def test_autograd_replays_by_default(ss, mode):
    """shadow() recomputes the decisions in its backward unless record=True; the two give
    the same gradients up to the order of the atomic sums, and the default path equals a
    direct call of the replaying adjoint."""
    shape, D = (192, 224), 20.0
    h = torch.from_numpy(rough(shape, 77, 80.0)).cuda()
    params = ss.Params(radius_m=R, mode=mode)
    g = torch.from_numpy(np.random.default_rng(9).standard_normal(shape).astype(np.float32)).cuda()
    grads = []
    for record in (False, True):
        hh = h.clone().requires_grad_(True)
        et = torch.tensor(math.radians(1.2), dtype=torch.float64, requires_grad=True)
        at = torch.tensor(0.9, dtype=torch.float64, requires_grad=True)
        s = ss.shadow(hh, et, at, D, RL, params, record=record)
        (s * g).sum().backward()
        torch.cuda.synchronize()
        grads.append((hh.grad.double(), float(et.grad), float(at.grad)))
    gh_direct, gs_direct = ss.shadow_cast_backward(h, D, math.radians(1.2), 0.9, g, RL, params)
    torch.cuda.synchronize()
    (a, ea, aa), (b, eb, ab) = grads
    assert float(a.norm()) > 0
    assert float((a - b).norm()) <= 1e-5 * float(a.norm())
    assert float((a - gh_direct.double()).norm()) <= 1e-5 * float(a.norm())
    assert abs(ea - eb) <= 1e-6 * abs(ea) + 1e-12 and abs(aa - ab) <= 1e-6 * abs(aa) + 1e-12
    assert abs(ea - float(gs_direct[0])) <= 1e-6 * abs(ea) + 1e-12


@pytest.mark.parametrize("mode,step", MODES)
def test_penumbra_backward_equals_full_replay(ss, mode, step):
    """ss_shadow_cast_backward_penumbra (rays at s = 0 or 1 not replayed) accumulates the
    same gradients as the full replay, to the order of the atomic sums; the forward's
    values are 0 or 1 only at |d| >= 1, so umbra and fully lit rays are the ones skipped."""
    shape, D = (176, 200), 20.0
    h = torch.from_numpy(rough(shape, 41, 90.0)).cuda()
    e, az = math.radians(1.1), 2.9
    params = ss.Params(radius_m=R, mode=mode, uniform_step=step)
    s = ss.shadow_cast(h, D, e, az, RL, params)
    g = torch.from_numpy(np.random.default_rng(13).standard_normal(shape).astype(np.float32)).cuda()
    gh1, gs1 = ss.shadow_cast_backward(h, D, e, az, g, RL, params)
    gh2, gs2 = ss.shadow_cast_backward_penumbra(h, D, e, az, s, g, RL, params)
    torch.cuda.synchronize()
    frac_skip = float(((s == 0) | (s == 1)).float().mean())
    print("rays skipped", frac_skip)
    assert 0.05 < frac_skip < 0.999
    a, b = gh1.double(), gh2.double()
    assert float(a.norm()) > 0
    assert float((a - b).norm()) <= 1e-5 * float(a.norm())
    assert torch.allclose(gs1, gs2, rtol=1e-6, atol=1e-9 * float(gs1.abs().max()) + 1e-12)


def test_penumbra_backward_compacting_form_on_a_large_tile(ss):
    """On launches of 2^18 ray blocks or more (an 8192^2 tile) the penumbra adjoint lists the
    contributing rays of each workgroup's blocks and replays only those; the gradients still
    equal the full replay's to the order of the atomic sums."""
    n, D = 8192, 4.0
    dev = torch.device("cuda:0")
    y, x = torch.meshgrid(torch.arange(n, device=dev, dtype=torch.float32),
                          torch.arange(n, device=dev, dtype=torch.float32), indexing="ij")
    gen = np.random.default_rng(17)
    h = torch.zeros((n, n), device=dev)
    for k in range(6):
        f, th, ph = gen.uniform(0.002, 0.05), gen.uniform(0, 2 * math.pi), gen.uniform(0, 6)
        h += 300.0 / (k + 1) * torch.sin(f * (x * math.cos(th) + y * math.sin(th)) + ph)
    del x, y
    e, az = math.radians(0.9), 1.3
    params = ss.Params(radius_m=R, max_len_m=8000.0)
    mm = ss.maxmip(h)
    s = ss.shadow_cast(h, D, e, az, RL, params, mm=mm)
    g = torch.randn((n, n), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
    gh1, gs1 = ss.shadow_cast_backward(h, D, e, az, g, RL, params, mm=mm)
    gh2, gs2 = ss.shadow_cast_backward_penumbra(h, D, e, az, s, g, RL, params, mm=mm)
    torch.cuda.synchronize()
    pen = float(((s > 0) & (s < 1)).float().mean())
    print("penumbra fraction", pen)
    assert 0.005 < pen < 0.9
    a, b = gh1.double(), gh2.double()
    assert float(a.norm()) > 0
    assert float((a - b).norm()) <= 1e-5 * float(a.norm())
    assert torch.allclose(gs1, gs2, rtol=1e-6, atol=1e-9 * float(gs1.abs().max()) + 1e-12)
