"""Reference gradient of the shadow factor (TEST INFRASTRUCTURE).

Once the descent's discrete choices are fixed (the segment that gave the
smallest clearance and its final sample index n*), the shadow factor is a
smooth function of the heightfield and the sun direction:

* the ray origin p = (R + h_p) n (Sec. 3.1) moves with the origin height h_p;
* the sample sits at t* = tau0 + n* delta/2 with delta = texel/cos(e)
  (Appendix, one texel of travel per step);
* the clearance height is dh = |p + t* L| - R - h_bil(q(t*)) with the bilinear
  height of the four texels around the projected tip;
* the angular clearance and the disc fraction follow Sec. 3.4.

This module evaluates that chain in torch float64 so autograd yields dL/dh and
dL/d(elevation, azimuth).  The discrete choices come from the C oracle's own
trace, never from the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64


def _bilinear(h: torch.Tensor, qx: torch.Tensor, qy: torch.Tensor) -> torch.Tensor:
    """Bilinear height over texel centres, taps clamped to the tile (Sec. 3.4 sampling)."""
    rows, width = h.shape
    x, y = qx - 0.5, qy - 0.5
    x0, y0 = torch.floor(x.detach()), torch.floor(y.detach())
    fx, fy = x - x0, y - y0
    i0 = x0.long().clamp(0, width - 1)
    i1 = (x0.long() + 1).clamp(0, width - 1)
    j0 = y0.long().clamp(0, rows - 1)
    j1 = (y0.long() + 1).clamp(0, rows - 1)
    return (1 - fy) * ((1 - fx) * h[j0, i0] + fx * h[j0, i1]) + fy * ((1 - fx) * h[j1, i0] + fx * h[j1, i1])


def shadow_on_branch(h: torch.Tensor, elev: torch.Tensor, azim: torch.Tensor, p, trace,
                     rays=None, points=None) -> torch.Tensor:
    """s for the given rays along the oracle's branch, differentiable in h, elev, azim.

    h: float64 [rows, width] (may require grad); elev, azim: 0-d float64 tensors.
    p: oracle.Params (its elev/azim are ignored in favour of the tensors).
    trace: oracle trace records for the same rays (structured numpy array).
    rays: linear texel indices, or None for every texel in order.
    points: instead of texel centres, rays from these surface points ([n, 2] continuous
    texel coordinates); the origin height is then the bilinear terrain there, so it
    depends on the four texels around the point.
    """
    rows, width = h.shape
    tr = np.asarray(trace).reshape(-1)
    seg = torch.as_tensor(tr["seg"].astype(np.int64))
    n = torch.as_tensor(tr["n"].astype(np.float64), dtype=F64)
    if points is None:
        lin = np.arange(rows * width) if rays is None else np.asarray(rays).reshape(-1)
        i = torch.as_tensor(lin % width)
        j = torch.as_tensor(lin // width)
        ox = torch.zeros(len(lin), dtype=F64)
        oy = torch.zeros(len(lin), dtype=F64)
    else:
        pts = np.asarray(points, dtype=np.float64).reshape(-1, 2)
        i = torch.as_tensor(np.floor(pts[:, 0]).astype(np.int64))
        j = torch.as_tensor(np.floor(pts[:, 1]).astype(np.int64))
        ox = torch.as_tensor(pts[:, 0] - (np.floor(pts[:, 0]) + 0.5))
        oy = torch.as_tensor(pts[:, 1] - (np.floor(pts[:, 1]) + 0.5))
    lit = seg == -2
    D = float(p.texel_m)
    planar = math.isinf(p.radius_m)
    R = float(p.radius_m)

    ce = torch.cos(elev)
    L = torch.stack([ce * torch.cos(azim), ce * torch.sin(azim), torch.sin(elev)])
    delta = D / ce
    t = 0.5 * delta + n * (0.5 * delta)

    X = (i.to(F64) + 0.5 + ox - 0.5 * width) * D
    Y = (j.to(F64) + 0.5 + oy - 0.5 * rows) * D
    if points is None:
        hp = h[j, i]
    else:
        hp = _bilinear(h, i.to(F64) + 0.5 + ox, j.to(F64) + 0.5 + oy)
    if planar:
        nrm = torch.stack([torch.zeros_like(X), torch.zeros_like(X), torch.ones_like(X)])
        P = torch.stack([X + t * L[0], Y + t * L[1], hp + t * L[2]])
        qx = P[0] / D + 0.5 * width
        qy = P[1] / D + 0.5 * rows
        Ht = P[2]
    else:
        ell = torch.sqrt(X * X + Y * Y + R * R)
        nrm = torch.stack([X / ell, Y / ell, R / ell])
        rho = R + hp
        P = rho * nrm + t * L.view(3, 1)
        qx = R * P[0] / (P[2] * D) + 0.5 * width
        qy = R * P[1] / (P[2] * D) + 0.5 * rows
        Plen = torch.sqrt(P[0] * P[0] + P[1] * P[1] + P[2] * P[2])
        Ht = Plen - R

    x = qx - 0.5
    y = qy - 0.5
    x0 = torch.floor(x.detach())
    y0 = torch.floor(y.detach())
    fx = x - x0
    fy = y - y0
    i0 = x0.long().clamp(0, width - 1)
    i1 = (x0.long() + 1).clamp(0, width - 1)
    j0 = y0.long().clamp(0, rows - 1)
    j1 = (y0.long() + 1).clamp(0, rows - 1)
    # rays lit by default have no sample; park their indices on a valid texel
    i0 = torch.where(lit, torch.zeros_like(i0), i0)
    i1 = torch.where(lit, torch.zeros_like(i1), i1)
    j0 = torch.where(lit, torch.zeros_like(j0), j0)
    j1 = torch.where(lit, torch.zeros_like(j1), j1)
    hb = (1 - fy) * ((1 - fx) * h[j0, i0] + fx * h[j0, i1]) + fy * ((1 - fx) * h[j1, i0] + fx * h[j1, i1])
    dh = Ht - hb

    Lc = L.view(3, 1)
    sp = (nrm * Lc).sum(0)
    cr = torch.stack([nrm[1] * L[2] - nrm[2] * L[1], nrm[2] * L[0] - nrm[0] * L[2],
                      nrm[0] * L[1] - nrm[1] * L[0]])
    cp = torch.sqrt((cr * cr).sum(0))
    if planar:
        alpha = torch.atan2(dh * cp, t - dh * sp)
    else:
        alpha = torch.atan2(dh * rho * cp, t * Plen - dh * (rho * sp + t))

    rL = float(p.ang_radius)
    dd = alpha / rL
    inside = (dd.abs() < 1.0) & ~lit
    d = torch.where(inside, dd, torch.zeros_like(dd))
    sv = (math.pi - torch.acos(d) + d * torch.sqrt(1.0 - d * d)) / math.pi
    out = torch.where(inside, sv, torch.where(dd > 0, torch.ones_like(dd), torch.zeros_like(dd)))
    return torch.where(lit, torch.ones_like(out), out)


def reference_gradient(h_np: np.ndarray, p, trace, grad_s: np.ndarray, rays=None, points=None):
    """(dL/dh [rows,width] float64, dL/delev, dL/dazim) for L = sum(grad_s * s)."""
    h = torch.tensor(np.asarray(h_np, dtype=np.float64), dtype=F64, requires_grad=True)
    e = torch.tensor(float(p.elev), dtype=F64, requires_grad=True)
    a = torch.tensor(float(p.azim), dtype=F64, requires_grad=True)
    s = shadow_on_branch(h, e, a, p, trace, rays, points)
    g = torch.as_tensor(np.asarray(grad_s, dtype=np.float64).reshape(-1))
    (s * g).sum().backward()
    return h.grad.numpy(), float(e.grad), float(a.grad), s.detach().numpy()


def sun_term_scale(h_np: np.ndarray, p, trace, grad_s: np.ndarray, rays=None):
    """(sum_r |g_r ds_r/delev|, sum_r |g_r ds_r/dazim|) along the oracle's branch.

    dL/d(elev, azim) = sum_r g_r ds_r/d(elev, azim) can cancel heavily (random
    upstream gradients, rays on both sides of a ridge); the rounding error of
    any evaluation of such a sum scales with the sum of the absolute terms, not
    with the result.  Per-ray derivatives by forward-mode differentiation."""
    from torch.func import jvp
    h = torch.tensor(np.asarray(h_np, dtype=np.float64), dtype=F64)
    e0 = torch.tensor(float(p.elev), dtype=F64)
    a0 = torch.tensor(float(p.azim), dtype=F64)
    one = torch.tensor(1.0, dtype=F64)
    _, dse = jvp(lambda e: shadow_on_branch(h, e, a0, p, trace, rays), (e0,), (one,))
    _, dsa = jvp(lambda a: shadow_on_branch(h, e0, a, p, trace, rays), (a0,), (one,))
    g = torch.as_tensor(np.asarray(grad_s, dtype=np.float64).reshape(-1))
    return float((g * dse).abs().sum()), float((g * dsa).abs().sum())
