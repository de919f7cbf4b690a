"""View-ray comparison against the oracle (test helper, not a test).

A pixel passes when the GPU's hit lies in the step of one of the oracle's
admissible first-hit samples, or both report no hit where a miss is admissible.
Where the GPU chose the oracle's certain hit, the refined ray length must also
agree: the straight-line refinement moves by at most step * 2 eps / (f_{n-1} -
f_n) when each f carries an error eps, plus FP32 rounding of t itself.  The
admissible sets come from the oracle alone and never read GPU output.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

# FP32 resolution of the kernel's f = H - b: heights carry a few ulps of
# |eye| + t (the ray point) and of the terrain (a few km: ~2e-4 m per ulp);
# positions carry ~1e-7 relative error of |eye| + t from the direction and
# the ray point; the margin takes a few of each.
TOL = oracle.ViewTol(eh_abs=5e-3, eh_rel=5e-7, ep_abs=1e-3, ep_rel=5e-7)


def check(h: np.ndarray, radius_m: float, texel_m: float, cam: oracle.Camera, t_gpu, xy_gpu,
          pixels=None, label: str = "") -> dict:
    """Compare GPU hits ([H, W] t and [H, W, 2] xy, or per listed pixel) with the oracle."""
    ref = oracle.view(h, radius_m, texel_m, cam, pixels, TOL) if pixels is not None else \
        oracle.view_threaded(h, radius_m, texel_m, cam, TOL)
    ref = ref.reshape(-1)
    tg = np.asarray(t_gpu, dtype=np.float64).reshape(-1)
    xyg = np.asarray(xy_gpu, dtype=np.float64).reshape(-1, 2)
    if pixels is not None:
        pix = np.asarray(pixels).reshape(-1, 2)
        lin = pix[:, 1] * cam.width + pix[:, 0]
        tg, xyg = tg[lin], xyg[lin]
    eyen = float(np.linalg.norm(cam.eye))
    step = cam.step_m
    n_exact = n_alt = n_miss = 0
    bad = []
    for k in range(ref.size):
        r = ref[k]
        assert r["status"] == 0 and r["adm_overflow"] == 0, (label, k, "oracle cap")
        g_hit = math.isfinite(tg[k])
        if not g_hit:
            if r["n_hit"] < 0 and not np.isfinite(xyg[k]).any():
                n_miss += 1
            else:
                bad.append((k, "gpu miss", int(r["n_hit"]), float(r["t_hit"])))
            continue
        if r["n_hit"] >= 0:
            fp, fh = float(r["f_prev"]), float(r["f_hit"])
            if math.isnan(fp):
                tol_t = 1e-6 * (eyen + r["t_hit"])
            else:
                tol_t = step * min(1.0, 2.0 * r["eps"] / max(fp - fh, 1e-300)) + \
                    2e-7 * (eyen + r["t_hit"]) + 1e-4
            if abs(tg[k] - r["t_hit"]) <= tol_t:
                tol_q = r["dqdt"] * tol_t + 1e-4 + 2e-7 * (eyen + r["t_hit"]) / texel_m
                if np.all(np.abs(xyg[k] - (r["qx"], r["qy"])) <= tol_q):
                    n_exact += 1
                    continue
                bad.append((k, "xy", tuple(xyg[k]), (float(r["qx"]), float(r["qy"]))))
                continue
        # another admissible sample: the hit must lie in that sample's step
        adm = [int(a) for a in r["adm"][:r["n_adm"]]]
        slack = 2e-7 * (eyen + tg[k]) + 1e-4
        if any((n - 1) * step - slack <= tg[k] <= n * step + slack for n in adm):
            n_alt += 1
            continue
        bad.append((k, "gpu hit", float(tg[k]), int(r["n_hit"]), float(r["t_hit"]), adm))
    stats = dict(label=label, pixels=int(ref.size), exact=n_exact, alternative=n_alt,
                 miss=n_miss, bad=len(bad))
    assert not bad, (stats, bad[:8])
    return stats
