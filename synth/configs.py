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
        return [(math.radians(0.2), 2.0 * math.pi * u(1)[0], SUN_RADIUS_RAD)]
    raise KeyError(name)


def dem_for(name: str, tile: int = 0, device="cpu"):
    """Heightfield for tile ``tile`` of workload ``name`` as float32 [rows, width]."""
    from .dem import make_dem
    c = CONFIGS[name]
    w, r, texel = c["tiles"][tile]
    return make_dem(w, r, texel, c["amplitude"], seed_of(name, tile), craters=c["craters"],
                    device=device)
