"""Seeded terrain defined on the sphere, for tiles in several gnomonic frames.

Heights are a function of the surface direction only, so every tile frame
(cube-face sub-tiles, tiles across a face seam, a working tile tangent
anywhere) samples the same planet.  Recipe: smooth Gaussian bumps of random
angular width and sign, plus one straight ridge along a great-circle arc.
"""
from __future__ import annotations

import math

import numpy as np

R_MOON = 1737400.0


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def frame_dirs(width: int, rows: int, texel_m: float, centre, ex, ey, origin=(0.0, 0.0),
               radius_m: float = R_MOON) -> np.ndarray:
    """Unit directions [rows, width, 3] of a frame's texel centres."""
    i = np.arange(width) + 0.5 - width / 2
    j = np.arange(rows) + 0.5 - rows / 2
    X = origin[0] + i[None, :] * texel_m
    Y = origin[1] + j[:, None] * texel_m
    P = (radius_m * np.asarray(centre, dtype=np.float64)[None, None, :]
         + X[..., None] * np.asarray(ex, dtype=np.float64)[None, None, :]
         + Y[..., None] * np.asarray(ey, dtype=np.float64)[None, None, :])
    return unit(P)


def planet_height(dirs: np.ndarray, seed: int, centre, n_bumps: int = 60, extent_m: float = 20e3,
                  ridge=None, radius_m: float = R_MOON) -> np.ndarray:
    """Heights (float32, metres) at unit directions near ``centre``: n_bumps Gaussian bumps
    (width 200 m - 3 km, height -600..+900 m) within extent_m of centre, and an optional
    ridge = (start dir, end dir, height m, half-width m) along the great-circle arc."""
    rng = np.random.default_rng(seed)
    c = unit(centre)
    a = unit(np.cross(c, (0.0, 1.0, 0.0)) if abs(c[1]) < 0.9 else np.cross(c, (1.0, 0.0, 0.0)))
    b = np.cross(c, a)
    h = np.zeros(dirs.shape[:-1])
    for _ in range(n_bumps):
        u, v = rng.uniform(-1, 1, 2) * extent_m / radius_m
        p = unit(c + u * a + v * b)
        w = rng.uniform(200.0, 3000.0) / radius_m
        amp = rng.uniform(-600.0, 900.0)
        ang = np.arccos(np.clip(dirs @ p, -1.0, 1.0))
        h += amp * np.exp(-0.5 * (ang / w) ** 2)
    if ridge is not None:
        s, e, height, half = ridge
        s, e = unit(s), unit(e)
        n = unit(np.cross(s, e))
        off = np.abs(np.arcsin(np.clip(dirs @ n, -1.0, 1.0))) * radius_m  # distance from the circle
        # along the arc: between s and e
        t_s = np.einsum("...k,k->...", dirs, np.cross(n, s))
        t_e = np.einsum("...k,k->...", dirs, np.cross(e, n))
        inside = (t_s >= 0) & (t_e >= 0)
        h += np.where(inside, height * np.clip(1.0 - off / half, 0.0, 1.0), 0.0)
    return h.astype(np.float32)


def seam_frames(core: int = 256, halo: int = 256, texel_m: float = 10.0, n_src: int = 1536,
                offset_m: float = 1.2e3):
    """Frames of two cube-face sub-tiles (n_src^2 texels) meeting at the +z/+x face seam, and
    of a working tile (core + 2 halo texels a side) tangent on the +z side, offset_m (surface)
    from the seam.  The sources reach the seam; the face plane stretches ~1.4x there."""
    R = R_MOON
    plane = n_src * texel_m
    fa = dict(width=n_src, rows=n_src, texel_m=texel_m, centre=(0.0, 0.0, 1.0),
              ex=(1.0, 0.0, 0.0), ey=(0.0, 1.0, 0.0), origin=(R - 0.5 * plane, 0.0))
    fb = dict(width=n_src, rows=n_src, texel_m=texel_m, centre=(1.0, 0.0, 0.0),
              ex=(0.0, 0.0, -1.0), ey=(0.0, 1.0, 0.0), origin=(-R + 0.5 * plane, 0.0))
    rot = offset_m / R
    wc = unit((math.cos(math.pi / 4 + rot), 0.0, math.sin(math.pi / 4 + rot)))
    wx = unit(np.cross((0.0, 1.0, 0.0), wc))
    W = core + 2 * halo
    fw = dict(width=W, rows=W, texel_m=texel_m, centre=tuple(wc), ex=tuple(wx),
              ey=(0.0, 1.0, 0.0), origin=(0.0, 0.0))
    return fa, fb, fw


def seam_scene(core: int = 256, halo: int = 256, texel_m: float = 10.0, seed: int = 20050699):
    """The seam frames with heights from planet_height: a ridge runs along the +x face
    1.5-3 km beyond the seam, so a sun from +x shades the core across the seam.  Returns
    dict(sources=[(heights, frame dict)], work=frame dict, window=(x0, y0, w, h))."""
    R = R_MOON
    fa, fb, fw = seam_frames(core, halo, texel_m)
    seam = unit((1.0, 0.0, 1.0))
    d0 = 2.2e3 / R
    rs = unit((math.cos(math.pi / 4 - d0), -3e3 / R, math.sin(math.pi / 4 - d0)))
    re = unit((math.cos(math.pi / 4 - d0), 3e3 / R, math.sin(math.pi / 4 - d0)))
    ridge = (rs, re, 1400.0, 700.0)
    srcs = []
    for f in (fa, fb):
        d = frame_dirs(f["width"], f["rows"], texel_m, f["centre"], f["ex"], f["ey"], f["origin"])
        srcs.append((planet_height(d, seed, seam, n_bumps=40, ridge=ridge), f))
    return dict(sources=srcs, work=fw, window=(halo, halo, core, core), seam=tuple(seam))
