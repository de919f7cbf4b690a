"""Seeded synthetic digital elevation models: fBm gradient noise plus craters.

These stand in for the lunar polar DEMs the paper renders (Sec. 3.1 quotes
30 m/texel LOLA-class data; Sec. 6.3 uses stitched fields of 1024-2048 texels).
The recipe: 8 octaves of gradient noise with persistence 0.5 and lacunarity 2
over the tile extent, plus bowl craters (depth 0.2 D, rim 0.04 D) whose
diameters follow a cumulative D^-2 law on [50 m, 5 km].

Everything runs in torch float64 on the requested device and is rounded to
float32 at the end.  The same seed gives the same array on the same device.
Rows are the slow axis: ``h[row, column]``; texel (column i, row j) covers
[i, i+1) x [j, j+1) in texel units.
"""
from __future__ import annotations

import math

import torch

_F64 = torch.float64


def _gradient_noise(xs: torch.Tensor, ys: torch.Tensor, grad: torch.Tensor) -> torch.Tensor:
    """2-D gradient (Perlin-style) noise on an integer lattice with quintic fade.

    ``xs`` is a row vector of lattice x coordinates, ``ys`` a column vector of
    lattice y coordinates, ``grad[gy, gx, 2]`` holds unit gradients.  Returns a
    grid ``[len(ys), len(xs)]`` scaled by sqrt(2) so values lie in [-1, 1].
    """
    x0 = torch.floor(xs)
    y0 = torch.floor(ys)
    fx = xs - x0
    fy = ys - y0
    ix = x0.long()
    iy = y0.long()

    def corner(dx: int, dy: int) -> torch.Tensor:
        g = grad[(iy + dy).view(-1, 1), (ix + dx).view(1, -1)]  # [ny, nx, 2]
        ox = (fx - dx).view(1, -1)
        oy = (fy - dy).view(-1, 1)
        return g[..., 0] * ox + g[..., 1] * oy

    def fade(f: torch.Tensor) -> torch.Tensor:
        return f * f * f * (f * (f * 6.0 - 15.0) + 10.0)

    ux = fade(fx).view(1, -1)
    uy = fade(fy).view(-1, 1)
    n00 = corner(0, 0)
    n10 = corner(1, 0)
    n01 = corner(0, 1)
    n11 = corner(1, 1)
    nx0 = n00 + ux * (n10 - n00)
    nx1 = n01 + ux * (n11 - n01)
    return (nx0 + uy * (nx1 - nx0)) * math.sqrt(2.0)


def fbm(width: int, rows: int, texel_m: float, amplitude_m: float, seed: int,
        octaves: int = 8, persistence: float = 0.5, lacunarity: float = 2.0,
        device: str | torch.device = "cpu", chunk_rows: int = 1024) -> torch.Tensor:
    """Fractional Brownian motion heights in metres, |h| <= amplitude_m.

    The base wavelength is the tile extent max(width, rows) * texel_m.  Octave o
    has frequency lacunarity**o / extent and weight persistence**o; the sum is
    divided by the total weight.  Each octave draws its own lattice gradients
    and lattice offset from a CPU generator seeded with ``seed``.
    """
    extent = max(width, rows) * texel_m
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(seed))
    lattices = []
    total_w = 0.0
    for o in range(octaves):
        freq = lacunarity ** o / extent
        n = int(math.ceil(freq * extent)) + 3
        theta = torch.rand((n, n), generator=gen, dtype=_F64) * (2.0 * math.pi)
        g = torch.stack([torch.cos(theta), torch.sin(theta)], dim=-1)
        off = torch.rand(2, generator=gen, dtype=_F64)
        w = persistence ** o
        total_w += w
        lattices.append((freq, g.to(device), float(off[0]), float(off[1]), w))

    out = torch.empty((rows, width), dtype=torch.float32, device=device)
    cx = (torch.arange(width, dtype=_F64, device=device) + 0.5) * texel_m
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        cy = (torch.arange(r0, r1, dtype=_F64, device=device) + 0.5) * texel_m
        acc = torch.zeros((r1 - r0, width), dtype=_F64, device=device)
        for freq, g, ox, oy, w in lattices:
            acc += w * _gradient_noise(cx * freq + ox, cy * freq + oy, g)
        out[r0:r1] = (acc * (amplitude_m / total_w)).to(torch.float32)
    return out


def crater_table(count: int, width: int, rows: int, texel_m: float, seed: int,
                 d_min: float = 50.0, d_max: float = 5000.0, exponent: float = 2.0):
    """Crater centres (metres) and diameters from a truncated power law.

    Cumulative count N(>D) is proportional to D**-exponent on [d_min, d_max];
    diameters are drawn by inverting that distribution.  Centres are uniform
    over the tile extent.
    """
    gen = torch.Generator(device="cpu")
    gen.manual_seed(int(seed) ^ 0x5EED)
    u = torch.rand(count, generator=gen, dtype=_F64)
    a = d_min ** (-exponent)
    b = d_max ** (-exponent)
    diam = (a - u * (a - b)) ** (-1.0 / exponent)
    cxm = torch.rand(count, generator=gen, dtype=_F64) * (width * texel_m)
    cym = torch.rand(count, generator=gen, dtype=_F64) * (rows * texel_m)
    return cxm, cym, diam


def add_craters(h: torch.Tensor, texel_m: float, count: int, seed: int,
                d_min: float = 50.0, d_max: float = 5000.0,
                depth_ratio: float = 0.2, rim_ratio: float = 0.04) -> torch.Tensor:
    """Add ``count`` bowl craters with raised rims to ``h`` in place.

    Profile for radius R = D/2 at distance r from the centre:
    bowl  h_rim - depth_ratio*D + depth_ratio*D*(r/R)**2  for r <= R;
    flank h_rim*((R/r)**3 - 1/27)/(1 - 1/27)              for R < r <= 3R;
    zero beyond 3R, with h_rim = rim_ratio*D.
    """
    rows, width = h.shape
    cxm, cym, diam = crater_table(count, width, rows, texel_m, seed, d_min, d_max)
    dev = h.device
    for k in range(count):
        R = float(diam[k]) * 0.5
        D = 2.0 * R
        xc = float(cxm[k])
        yc = float(cym[k])
        reach = 3.0 * R
        i0 = max(0, int(math.floor((xc - reach) / texel_m - 0.5)))
        i1 = min(width, int(math.ceil((xc + reach) / texel_m + 0.5)) + 1)
        j0 = max(0, int(math.floor((yc - reach) / texel_m - 0.5)))
        j1 = min(rows, int(math.ceil((yc + reach) / texel_m + 0.5)) + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        xs = (torch.arange(i0, i1, dtype=_F64, device=dev) + 0.5) * texel_m - xc
        ys = (torch.arange(j0, j1, dtype=_F64, device=dev) + 0.5) * texel_m - yc
        r = torch.sqrt(xs.view(1, -1) ** 2 + ys.view(-1, 1) ** 2)
        h_rim = rim_ratio * D
        bowl = h_rim - depth_ratio * D + depth_ratio * D * (r / R) ** 2
        rr = torch.clamp(r, min=R)
        flank = h_rim * ((R / rr) ** 3 - 1.0 / 27.0) / (1.0 - 1.0 / 27.0)
        prof = torch.where(r <= R, bowl, torch.where(r <= reach, flank, torch.zeros_like(r)))
        h[j0:j1, i0:i1] += prof.to(h.dtype)
    return h


def make_dem(width: int, rows: int, texel_m: float, amplitude_m: float, seed: int,
             craters: int = 0, device: str | torch.device = "cpu") -> torch.Tensor:
    """fBm heightfield plus ``craters`` power-law craters, float32 [rows, width]."""
    h = fbm(width, rows, texel_m, amplitude_m, seed, device=device)
    if craters > 0:
        h64 = h.to(_F64)
        add_craters(h64, texel_m, craters, seed)
        h = h64.to(torch.float32)
    return h.contiguous()
