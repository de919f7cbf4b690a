"""Pins of the oracle's maximum mipmap (Sec. 3.2, "Maximum mipmaps").

A level-m texel holds the largest height of the level-0 block it covers; the
oracle builds it recursively from 2x2 children, this test from the direct
block definition.  Plus the structural invariants.
"""
import numpy as np
import pytest


def block_max(h, m):
    S = 1 << m
    rows, width = h.shape
    R = -(-rows // S) * S
    W = -(-width // S) * S
    pad = np.full((R, W), -np.inf, dtype=np.float32)
    pad[:rows, :width] = h + np.float32(0.0)
    return pad.reshape(R // S, S, W // S, S).max(axis=(1, 3))


@pytest.mark.parametrize("size,levels", [((1, 1), 1), ((2, 2), 2), ((3, 1), 3), ((256, 256), 9),
                                         ((1536, 1536), 12), ((4096, 4096), 13),
                                         ((16384, 16384), 15), ((512, 3072), 13)])
def test_level_count(orc, size, levels):
    assert orc.maxmip_levels(*size) == levels


@pytest.mark.parametrize("shape", [(1, 7), (5, 3), (37, 53), (64, 64), (96, 160), (256, 256),
                                   (129, 1)])
def test_block_definition_bitwise(orc, shape):
    rng = np.random.default_rng(sum(shape))
    h = (rng.standard_normal(shape) * 300).astype(np.float32)
    lv = orc.maxmip(h)
    assert len(lv) == orc.maxmip_levels(shape[1], shape[0]) - 1
    for m, M in enumerate(lv, start=1):
        ref = block_max(h, m)
        assert M.shape == ref.shape
        assert np.array_equal(M.view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_invariants(orc):
    rng = np.random.default_rng(7)
    h = (rng.standard_normal((200, 136)) * 50).astype(np.float32)
    lv = [h] + orc.maxmip(h)
    for m in range(1, len(lv)):
        P, Cc = lv[m], lv[m - 1]
        assert P.shape == ((Cc.shape[0] + 1) // 2, (Cc.shape[1] + 1) // 2)
        for dj in (0, 1):
            for di in (0, 1):
                ch = Cc[dj::2, di::2]
                assert np.all(P[:ch.shape[0], :ch.shape[1]] >= ch)
    assert lv[-1].shape == (1, 1) and lv[-1][0, 0] == h.max()


def test_negative_zero_canonical(orc):
    h = np.full((8, 8), -0.0, dtype=np.float32)
    for M in orc.maxmip(h):
        assert not np.any(np.signbit(M))
