"""The five workloads: tile sizes, spacings, DEM recipes and sun directions.

Sun directions are given in each tile's centre frame: elevation above the
tangent plane and azimuth measured from +column toward +row.  The sun's
apparent radius is 0.267 degrees throughout (the solar disc seen from the Moon).
"""
from __future__ import annotations

import math

import torch

R_MOON = 1737400.0
SUN_RADIUS_RAD = math.radians(0.267)
BASE_SEED = 20050667

CONFIGS = {
    # small: 256^2 fBm only, 20 m/texel, rays run to the tile edge
    "small": dict(index=0, tiles=[(256, 256, 20.0)], amplitude=2000.0, craters=0,
                  max_len=0.0),
    # tile: 4096^2, 5 m/texel, fBm + 2000 craters, 30 km rays
    "tile": dict(index=1, tiles=[(4096, 4096, 5.0)], amplitude=2000.0, craters=2000,
                 max_len=30000.0),
    # differentiable: 2048^2, 10 m/texel, fBm + craters
    "diff": dict(index=2, tiles=[(2048, 2048, 10.0)], amplitude=2000.0, craters=2000,
                 max_len=30000.0),
    # batched: 8 uneven tiles x 64 suns
    "batched": dict(index=3,
                    tiles=[(512, 512, 20.0), (1024, 1024, 17.5), (1536, 1536, 15.0),
                           (2048, 2048, 12.5), (2048, 2048, 10.0), (3072, 3072, 7.5),
                           (4096, 4096, 5.0), (4096, 4096, 5.0)],
                    amplitude=2000.0, craters=2000, max_len=30000.0),
    # large polar: 16384^2, 2 m/texel, fBm 4 km + 20000 craters, 60 km rays
    "polar": dict(index=4, tiles=[(16384, 16384, 2.0)], amplitude=4000.0, craters=20000,
                  max_len=60000.0),
}


def config(name: str) -> dict:
    return CONFIGS[name]


def seed_of(name: str, tile: int = 0) -> int:
    return BASE_SEED + CONFIGS[name]["index"] + 1000 * tile


def sun_list(name: str, tile: int = 0):
    """List of (elevation_rad, azimuth_rad, angular_radius_rad) for a workload."""
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed_of(name, tile) + 77)
    u = lambda n: torch.rand(n, generator=gen, dtype=torch.float64).tolist()  # noqa: E731
    if name == "small":
        return [(math.radians(1.5), 2.0 * math.pi * u(1)[0], SUN_RADIUS_RAD)]
    if name == "tile":
        es = u(8)
        az = u(8)
        return [(math.radians(0.5 + 2.5 * e), 2.0 * math.pi * a, SUN_RADIUS_RAD)
                for e, a in zip(es, az)]
    if name == "diff":
        return [(math.radians(1.5), 2.0 * math.pi * u(1)[0], SUN_RADIUS_RAD)]
    if name == "batched":
        a0 = 2.0 * math.pi * u(1)[0]
        out = []
        for k in range(64):
            e = 0.3 + 3.7 * (1.0 - math.cos(math.pi * k / 63.0)) / 2.0
            out.append((math.radians(e), a0 + math.radians(10.0 * k / 63.0), SUN_RADIUS_RAD))
        return out
    if name == "polar":
        # two azimuths at the same low elevation (the second drawn after the first)
        a0 = u(1)[0]
        a1 = u(1)[0]
        return [(math.radians(0.2), 2.0 * math.pi * a, SUN_RADIUS_RAD) for a in (a0, a1)]
    raise KeyError(name)


def dem_for(name: str, tile: int = 0, device="cpu"):
    """Heightfield for tile ``tile`` of workload ``name`` as float32 [rows, width]."""
    from .dem import make_dem
    c = CONFIGS[name]
    w, r, texel = c["tiles"][tile]
    return make_dem(w, r, texel, c["amplitude"], seed_of(name, tile), craters=c["craters"],
                    device=device)


def look_at(eye, target, hfov_deg: float, width: int, height: int, step_m: float,
            far_m: float = 0.0) -> dict:
    """Pinhole camera fields (eye, fwd, right, up, ...) looking from eye to target, both in
    the tile frame relative to the tile-centre surface point; square pixels."""
    import numpy as np
    e = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - e
    f /= np.linalg.norm(f)
    z = np.array([0.0, 0.0, 1.0]) if abs(f[2]) < 0.999 else np.array([0.0, 1.0, 0.0])
    r = np.cross(f, z)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(hfov_deg) / 2.0)
    tv = th * height / width
    return dict(width=int(width), height=int(height), eye=tuple(e.tolist()),
                fwd=tuple(f.tolist()), right=tuple((th * r).tolist()), up=tuple((tv * u).tolist()),
                step_m=float(step_m), far_m=float(far_m))


def view_scene(kind: str, width_px: int, height_px: int, tile_w: int, tile_h: int,
               texel_m: float, step_m: float | None = None) -> dict:
    """Camera recipes over a tile of tile_w x tile_h texels (side S = tile_w * texel_m):
    oblique   -- 0.35 S back from a corner, 0.5 S up, looking at the tile centre;
    grazing   -- low over one edge, looking across the tile toward the horizon (sky,
                 long rays, far misses);
    nadir     -- 0.4 S above the centre looking straight down (rays along the local
                 vertical, where the texture path barely moves);
    outside   -- beyond the tile's -x edge at 400 m, looking inward (side entries);
    flyover   -- the frame workload: 8 km up over the tile's south-west quarter,
                 heading north-east, 25 degrees below the horizon, 60 degree field of view
                 (a spacecraft passing over mountains)."""
    S = tile_w * texel_m
    step = step_m if step_m is not None else 0.5 * texel_m
    if kind == "oblique":
        return look_at((-0.35 * S, -0.3 * S, 0.5 * S), (0.0, 0.0, 0.0), 60.0, width_px,
                       height_px, step)
    if kind == "grazing":
        return look_at((-0.45 * S, 0.05 * S, 2600.0), (0.5 * S, 0.1 * S, 1800.0), 70.0,
                       width_px, height_px, step)
    if kind == "nadir":
        return look_at((0.02 * S, -0.01 * S, 0.4 * S), (0.02 * S, -0.01 * S, 0.0), 40.0,
                       width_px, height_px, step)
    if kind == "outside":
        return look_at((-0.6 * S, 0.1 * S, 400.0), (0.2 * S, 0.0, -300.0), 60.0, width_px,
                       height_px, step)
    if kind == "flyover":
        eye = (-0.3 * S, -0.3 * S, 8000.0)
        d = 8000.0 / math.tan(math.radians(25.0))
        tgt = (eye[0] + d / math.sqrt(2.0), eye[1] + d / math.sqrt(2.0), 0.0)
        return look_at(eye, tgt, 60.0, width_px, height_px, step)
    raise KeyError(kind)
