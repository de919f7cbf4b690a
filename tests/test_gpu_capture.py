"""Every per-call entry point of the boundary recorded into a caller's HIP graph
(torch.cuda.graph stream capture): the max-mip build, the forward, the
replaying adjoint and the batched call (both forms).  Each replay must equal the
eager calls on the same inputs -- bit for bit for the mipmap and the shadow
factors, to the order of the atomic sums for the gradients -- with eager work
and synchronisations between replays, and a replay after the heights change
must follow them (the graph rebuilds the mipmap)."""
import math

import numpy as np
import pytest
import torch

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


def bits(t):
    return t.view(torch.int32)


def levels(ss, mm):
    """The mipmap's levels (the padding between them is never written)."""
    return torch.cat([v.reshape(-1) for v in ss.maxmip_unpack(mm, 264, 200)])


def close(a, b, rel):
    a, b = a.double(), b.double()
    return float((a - b).norm()) <= rel * max(float(a.norm()), 1e-300)


@pytest.mark.parametrize("form", ["flat", "persistent"])
def test_graph_capture_matches_eager(ss, form, monkeypatch):
    monkeypatch.setenv("SS_BATCH_FORM", form)
    dev = torch.device("cuda:0")
    D = 20.0
    h0 = torch.from_numpy(rough((200, 264), 5, 90.0)).to(dev)
    h1 = torch.from_numpy(rough((128, 96), 6, 60.0)).to(dev)
    params = ss.Params(radius_m=R)
    e, a = math.radians(1.3), 0.8
    suns = [(math.radians(0.9), 0.3, RL), (math.radians(2.2), 4.0, RL), (math.radians(1.5), 2.5, RL)]
    g = torch.from_numpy(np.random.default_rng(3).standard_normal((200, 264)).astype(np.float32)).to(dev)

    # buffers the graph writes
    mm = torch.empty(ss.maxmip_floats(264, 200), dtype=torch.float32, device=dev)
    out = torch.empty_like(h0)
    gh = torch.empty_like(h0)
    gs = torch.empty(2, dtype=torch.float64, device=dev)
    mms_b = [torch.empty(ss.maxmip_floats(h.shape[1], h.shape[0]), dtype=torch.float32, device=dev)
             for h in (h0, h1)]
    outs_b = [[torch.empty_like(h) for _ in suns] for h in (h0, h1)]
    ws = torch.empty(ss.batched_workspace_bytes(2, len(suns)), dtype=torch.uint8, device=dev)

    def work():
        ss.maxmip(h0, out=mm)
        ss.shadow_cast(h0, D, e, a, RL, params, mm=mm, out=out)
        gh.zero_()
        gs.zero_()
        ss.shadow_cast_backward(h0, D, e, a, g, RL, params, mm=mm, grad_h=gh, grad_sun=gs)
        ss.shadow_cast_batched([h0, h1], [D, 15.0], suns, params, outs=outs_b, mms=mms_b, ws=ws)

    def eager_reference():
        work()
        torch.cuda.synchronize()
        return (mm.clone(), out.clone(), gh.clone(), gs.clone(),
                [[o.clone() for o in row] for row in outs_b])

    def check(ref):
        mm_r, out_r, gh_r, gs_r, ob_r = ref
        assert torch.equal(levels(ss, mm), levels(ss, mm_r))
        assert torch.equal(bits(out), bits(out_r))
        assert close(gh, gh_r, 1e-5) and close(gs, gs_r, 1e-9)
        for row, row_r in zip(outs_b, ob_r):
            for o, o_r in zip(row, row_r):
                assert torch.equal(bits(o), bits(o_r))

    ref = eager_reference()
    # the batched outputs equal per-sun launches (sanity of the eager reference itself)
    for t, (h, D_t) in enumerate(((h0, D), (h1, 15.0))):
        for k, (se, sa, sr) in enumerate(suns):
            s1 = ss.shadow_cast(h, D_t, se, sa, sr, params)
            assert torch.equal(bits(s1), bits(ref[4][t][k]))

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        work()
    torch.cuda.synchronize()
    for rep in range(3):
        # scribble over every output eagerly, then replay
        for t in (mm, out, gh, gs):
            t.fill_(float("nan"))
        for row in outs_b:
            for o in row:
                o.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check(ref)
        _ = ss.shadow_cast(h1, 15.0, e, a, RL, params)  # unrelated eager work between replays
    # new heights: the replay rebuilds the mipmap and follows them
    h0.add_(torch.linspace(0, 300.0, 264, device=dev).view(1, -1))
    h1.mul_(1.5)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    got = (mm.clone(), out.clone(), gh.clone(), gs.clone(), [[o.clone() for o in row] for row in outs_b])
    ref2 = eager_reference()
    assert not torch.equal(bits(ref2[1]), bits(ref[1]))
    assert torch.equal(levels(ss, got[0]), levels(ss, ref2[0]))
    assert torch.equal(bits(got[1]), bits(ref2[1]))
    assert close(got[2], ref2[2], 1e-5) and close(got[3], ref2[3], 1e-9)
    for row, row_r in zip(got[4], ref2[4]):
        for o, o_r in zip(row, row_r):
            assert torch.equal(bits(o), bits(o_r))
