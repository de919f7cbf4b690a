"""The allocation-free batched entry point (ss_shadow_cast_batched_noalloc),
called through the C ABI: its outputs equal ss_shadow_cast_batched's bit for
bit on two calls in a row, the second with a smaller batch, in both batched
forms and two modes; a batch too large for its fixed device array is refused
before anything runs."""
import ctypes as C
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


def run_both(ss, heights, texels, suns, params):
    """(outputs of ss_shadow_cast_batched, outputs of ss_shadow_cast_batched_noalloc)."""
    from paper_2005_06671_amd import _lib as L
    from paper_2005_06671_amd.api import _alloc_batch, _batch_structs, _stream
    res = []
    for noalloc in (False, True):
        mms, outs, ptrs, ws = _alloc_batch(heights, suns, None, None)
        for row in outs:
            for o in row:
                o.fill_(float("nan"))
        tiles, sn = _batch_structs(heights, mms, texels, suns)
        p = params.c()
        st = _stream(heights[0].device)
        if noalloc:
            rc = L.lib().ss_shadow_cast_batched_noalloc(tiles, len(heights), sn, len(suns),
                                                        C.byref(p), ptrs, st)
        else:
            rc = L.lib().ss_shadow_cast_batched(tiles, len(heights), sn, len(suns), C.byref(p),
                                                ptrs, ws.data_ptr(), ws.numel(), st)
        assert rc == 0, rc
        torch.cuda.synchronize()
        res.append(outs)
    return res


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("form", ["flat", "persistent"])
def test_noalloc_matches_batched(ss, form, mode, monkeypatch):
    monkeypatch.setenv("SS_BATCH_FORM", form)
    print("noalloc", form, mode, flush=True)
    dev = torch.device("cuda:0")
    params = ss.Params(radius_m=R, max_len_m=2500.0, mode=mode)
    big = [torch.from_numpy(rough((160, 200), 1, 80.0)).to(dev),
           torch.from_numpy(rough((96, 72), 2, 60.0)).to(dev)]
    suns_big = [(math.radians(0.8), 0.4, RL), (math.radians(2.0), 3.9, RL),
                (math.radians(1.4), 5.5, RL)]
    small = [torch.from_numpy(rough((40, 56), 3, 50.0)).to(dev)]
    suns_small = [(math.radians(1.1), 1.7, RL), (math.radians(2.6), 0.2, RL)]
    for heights, texels, suns in ((big, [20.0, 15.0], suns_big), (small, [10.0], suns_small)):
        ref, got = run_both(ss, heights, texels, suns, params)
        for row_r, row_g in zip(ref, got):
            for o_r, o_g in zip(row_r, row_g):
                assert not torch.isnan(o_r).any()
                assert torch.equal(o_r.view(torch.int32), o_g.view(torch.int32))


def test_noalloc_refuses_oversized_batch(ss):
    from paper_2005_06671_amd import _lib as L
    from paper_2005_06671_amd.api import _batch_structs, _stream
    dev = torch.device("cuda:0")
    h = torch.from_numpy(rough((32, 32), 4, 40.0)).to(dev)
    n_suns = 4000
    assert L.lib().ss_batched_workspace_bytes(1, n_suns) > L.SS_NOALLOC_SCRATCH_BYTES
    mm = ss.maxmip(h)
    out = torch.full_like(h, 7.0)
    suns = [(math.radians(1.0), 0.001 * k, RL) for k in range(n_suns)]
    tiles, sn = _batch_structs([h], [mm], [10.0], suns)
    ptrs = (C.c_void_p * n_suns)(*([out.data_ptr()] * n_suns))
    p = ss.Params(radius_m=R).c()
    rc = L.lib().ss_shadow_cast_batched_noalloc(tiles, 1, sn, n_suns, C.byref(p), ptrs,
                                                _stream(dev))
    torch.cuda.synchronize()
    assert rc == L.SS_ERR_WORKSPACE
    assert torch.all(out == 7.0)
