"""GPU-vs-oracle comparison used by the GPU tests (test helper, not a test).

A texel passes when |s_gpu - s_oracle| <= TOL.  A texel that differs by more
passes only if the oracle's near-tie enumeration (decisions whose FP64 margin
is below single-precision resolution may go either way: for the descent its
crossings, lower bounds and samples, for uniform stepping whether a step at the
tile edge or the cap counts) yields a valid result within TOL of the GPU value;
everything else is a failure.  The enumeration
runs in the oracle alone and never reads GPU output.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

import oracle

TOL = 1e-4
# FP32 resolution of the kernels' decisions: heights eh_abs + eh_rel * t (m),
# positions et_abs + et_rel * (t / delta) (texels).  An FP32 lower bound or
# clearance carries a few ulps of the tip rise (<= ~2.5 km) plus the position
# error times the slope; positions carry ~3e-7 relative error of the offset
# from the origin (K u), i.e. ~1e-6 texel per texel travelled with margin.
EH = (4e-3, 2e-7)
ET = (2e-3, 1e-6)


def disc(alpha, rL):
    """Visible disc fraction for angular clearances (+inf lit, -inf umbra)."""
    a = np.asarray(alpha, dtype=np.float64)
    d = np.clip(np.nan_to_num(a / rL, posinf=1.0, neginf=-1.0), -1.0, 1.0)
    return (math.pi - np.arccos(d) + d * np.sqrt(1.0 - d * d)) / math.pi


def compare(h: np.ndarray, p: oracle.Params, s_gpu: np.ndarray, rays=None, tol: float = TOL,
            max_alt: int = 4000, label: str = "") -> dict:
    """Statistics of the comparison; raises AssertionError on unexplained texels."""
    t0 = time.time()
    s_or, _ = oracle.shadow_threaded(h, p, rays)
    s_or = np.asarray(s_or).reshape(-1)
    g = np.asarray(s_gpu, dtype=np.float64).reshape(-1)
    if rays is not None:
        g = g[np.asarray(rays)]
        idx = np.asarray(rays)
    else:
        idx = np.arange(g.size)
    d = np.abs(g - s_or)
    bad = np.nonzero(d > tol)[0]
    explained = 0
    unexplained = []
    capped = 0
    for k in bad[:max_alt]:
        alts = None
        if p.mode in (0, 1, 2):
            alts = oracle.alternatives(h, p, int(idx[k]), EH[0], EH[1], ET[0], ET[1])
        if alts is None:
            capped += 1 if p.mode in (0, 1, 2) else 0
            unexplained.append((int(idx[k]), float(g[k]), float(s_or[k])))
            continue
        sv = disc(alts, p.ang_radius)
        if np.any(np.abs(sv - g[k]) <= tol):
            explained += 1
        else:
            unexplained.append((int(idx[k]), float(g[k]), float(s_or[k])))
    stats = dict(label=label, n=int(g.size), max_abs=float(d.max()) if d.size else 0.0,
                 mean_abs=float(d.mean()) if d.size else 0.0, n_over=int(bad.size),
                 frac_over=float(bad.size / max(1, g.size)), explained=explained,
                 unexplained=len(unexplained), capped=capped, seconds=time.time() - t0,
                 examples=unexplained[:5])
    print("parity", stats, flush=True)
    log = os.environ.get("SS_PARITY_LOG")
    if log:
        with open(log, "a") as f:
            f.write(json.dumps(stats) + "\n")
    return stats


def assert_parity(stats: dict, max_frac_over: float = 2e-3) -> None:
    assert stats["n_over"] <= 4000, stats
    assert stats["unexplained"] == 0, stats
    assert stats["frac_over"] <= max_frac_over, stats


def well_conditioned(tr):
    """Rays whose every oracle decision clears FP32 resolution by a wide margin:
    lower-bound and clearance gaps (m), rounding of the sample index (half
    texels), clearance gap between runs (rad), crossing spacing relative to
    the distance travelled (FP32 offsets carry ~3e-7 relative error), and the
    deciding sample's distance from a line through texel centres (the bilinear
    slope, hence the gradient, jumps there).  Used to pick the rays whose
    gradients the adjoint tests compare."""
    t = tr.reshape(-1)
    return ((t["margin_lb"] > 0.05) & (t["margin_dh"] > 0.05) & (t["margin_round"] > 0.01)
            & (t["margin_seg"] > 2e-5) & (t["margin_geo"] > 2e-5) & (t["margin_tap"] > 2e-5))
