#!/usr/bin/env python
"""Benchmark of the soft-shadow hot path on one MI355X.

Workload (the 4096^2 tile configuration): a 4096 x 4096 fp32 DEM at 5 m/texel
(seeded fBm, 2 km amplitude, plus 2000 power-law craters) on a sphere of radius
1737.4 km, 8 seeded suns with elevation uniform in [0.5, 3] degrees and disc
radius 0.267 degrees, shadow rays capped at 30 km of horizontal travel.

One step = build the maximum mipmap + run the descent forward for all 8 suns
(8 x 16.8 M rays), as one replay of the batched plan's HIP graph (the build,
then one launch over every ray block of the 8 suns).  `value` is rays per
second of the whole step, inputs resident in HBM.  The same work as eight
per-sun launches of the per-tile kernel is timed beside it (bit-identical
outputs).  Beside it the JSON line reports uniform stepping on the same
suns (the paper's baseline), forward+backward throughput, the roofline of the
dominant kernel, and the FP64 CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s DP+max-mip vs uniform stepping (fwd, fwd+bwd) at |Δ|≤1e-4 on 1 GPU"
WORKLOAD = ("tile: 4096x4096 fp32 DEM, 5 m/texel, fBm 2 km + 2000 craters, sphere R=1737.4 km, "
            "8 suns elev U[0.5,3] deg, r_L=0.267 deg, 30 km rays")

# Algorithmic VALU work per unit, in lane operations, fixed from the kernel
# formulas before tuning: one max-mip lower-bound evaluation (top-level DDA step
# or child piece: t(u), the tip's lowest height over the piece, crossings,
# index, compare) 35; one bilinear clearance sample (four taps, tip height,
# clearance, argmin) 45; one uniform step 40.  Achieved = units x ops / kernel
# time; the peak is the non-packed FP32 lane rate of the chip.
OPS_LB = 35
OPS_SAMPLE = 45
OPS_USTEP = 40
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz VALU lane-slots (FP32 not packed)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def src_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


DP_SOURCES = ["paper_2005_06671_amd/csrc/ray.h", "paper_2005_06671_amd/csrc/batched.hip",
              "paper_2005_06671_amd/csrc/common.h"]
TRAFFIC_FILE = "descent_tile_traffic.json"
COUNTERS_FILE = "descent_tile_counters.txt"
COUNTERS_JSON = "descent_tile_counters.json"


def traffic_from_profile():
    """HBM bytes per launch of the descent kernel from the committed counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != src_hash(DP_SOURCES):
        return None
    return d.get("hbm_bytes_per_launch")


def counters_from_profile():
    """VALU counters of the descent kernel (one batched launch over the 8 suns) from the
    committed summary, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", COUNTERS_JSON)
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != src_hash(DP_SOURCES):
        return None
    return d.get("flat_descent")


def cpu_baseline(h_np, params_or, seconds=15.0):
    """The FP64 oracle on a bounded random sample of the workload's rays."""
    import numpy as np
    import oracle
    threads = max(1, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(1234)
    n_all = h_np.size
    oracle.shadow(h_np, params_or, np.arange(1, dtype=np.int64))  # builds the oracle's mipmap
    # grow the sample until it takes about `seconds` of wall time
    n = 4096 * threads
    while True:
        rays = rng.choice(n_all, size=min(n_all, n), replace=False)
        t0 = time.perf_counter()
        oracle.shadow_threaded(h_np, params_or, rays, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * seconds or rays.size >= n_all:
            break
        n = int(rays.size * min(8.0, max(1.5, seconds / max(dt, 1e-3))))
    n = rays.size
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} random texels of the 4096^2 tile, first sun, descent, FP64 C oracle on "
                      f"{threads} host threads ({cpu}), {dt:.1f} s"}


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_profiles(trace_dir, fetch_dir, write_dir, counters_dir, out_dir):
    """Turns rocprofv3 CSV output of this benchmark into the committed summaries:
    per-kernel durations, HBM bytes per launch (FETCH_SIZE/WRITE_SIZE scaled by
    the same counters on the 512 MiB calibration copy) and VALU counters."""
    import collections
    os.makedirs(out_dir, exist_ok=True)
    lines = []
    stats = _csv_rows(os.path.join(trace_dir, "bench_kernel_stats.csv"))
    lines.append("kernel | calls | avg us | total ms")
    for r in stats[:12]:
        lines.append(f"{r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f}")
    with open(os.path.join(out_dir, "bench_tile_kernel_stats.txt"), "w") as f:
        f.write("# rocprofv3 --kernel-trace --stats summary of the tile benchmark (the timed step: "
                "20 graph replays after 5 warm-up ones; the plan's choices come from the tuner "
                "cache a previous run wrote, so no tuning launch is traced)\n")
        f.write("# command: SS_TUNE_CACHE=/tmp/ss_tune.jsonl python bench.py --steps 2 --warmup 1 "
                "--no-cpu --no-extras --dem-cache /tmp/dem_tile.npy; SS_TUNE_CACHE=/tmp/ss_tune.jsonl "
                "rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o bench -- "
                "python bench.py --steps 20 --warmup 5 --no-cpu --no-extras --dem-cache "
                "/tmp/dem_tile.npy\n")
        f.write("\n".join(lines) + "\n")

    def per_kernel(d, counter):
        acc = collections.defaultdict(list)
        for r in _csv_rows(os.path.join(d, "bench_counter_collection.csv")):
            if r["Counter_Name"] == counter:
                acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return acc

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = 512 * 1024 * 1024 / 1024.0  # KiB moved each way by the calibration copy
    cal_f = copy_bytes / max(fetch["__amd_rocclr_copyBuffer"])
    cal_w = copy_bytes / max(write["__amd_rocclr_copyBuffer"])
    out = {"kernel_src_sha": src_hash(DP_SOURCES), "fetch_scale": cal_f, "write_scale": cal_w,
           "kernels": {}}
    for name in fetch:
        if not name.startswith("void ss::"):
            continue
        fb = sum(fetch[name]) / len(fetch[name]) * 1024 * cal_f
        wb = sum(write.get(name, [0.0])) / max(1, len(write.get(name, []))) * 1024 * cal_w
        out["kernels"][name] = {"launches": len(fetch[name]), "fetch_bytes": fb,
                                "write_bytes": wb}
    dp = [k for k in out["kernels"] if "flat_kernel<true, 8, 0>" in k]
    if dp:
        k = out["kernels"][dp[0]]
        out["hbm_bytes_per_launch"] = k["fetch_bytes"] + k["write_bytes"]
        out["kernel"] = dp[0]
    out["command"] = ("SS_TUNE_CACHE=/tmp/ss_tune.jsonl rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) "
                      "--kernel-include-regex 'ss::|copy' --output-format csv -d <dir> -o bench -- "
                      "python bench.py --steps 1 --warmup 0 --no-cpu --no-extras --calibrate-copy "
                      "--dem-cache /tmp/dem_tile.npy")
    with open(os.path.join(out_dir, TRAFFIC_FILE), "w") as f:
        json.dump(out, f, indent=1)
    if counters_dir:
        summarize_counters(os.path.join(counters_dir, "bench_counter_collection.csv"), out_dir)


def summarize_counters(csv_path, out_dir):
    """VALU and L2 counters per kernel (averaged over its dispatches).  A persistent
    kernel's waves each run many ray blocks, so compare its total, not per-wave, counts."""
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in _csv_rows(csv_path):
        acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["kernel | VALU instr per dispatch | waves | VALU instr per wave | "
             "active lanes per VALU instr | trans per wave | L2 hit rate"]
    for name, d in acc.items():
        v = {c: sum(x) / len(x) for c, x in d.items()}
        waves = v.get("SQ_WAVES", 1.0)
        hit = v.get("TCC_HIT_sum")
        miss = v.get("TCC_MISS_sum")
        hr = f"{hit / (hit + miss):.3f}" if hit is not None and miss is not None else "-"
        lines.append(f"{name[:70]} | {v.get('SQ_INSTS_VALU', 0):.4g} | {waves:.0f} | "
                     f"{v.get('SQ_INSTS_VALU', 0) / waves:.0f} | "
                     f"{v.get('SQ_THREAD_CYCLES_VALU', 0) / max(1.0, v.get('SQ_ACTIVE_INST_VALU', 1)):.1f} | "
                     f"{v.get('SQ_INSTS_VALU_TRANS_F32', 0) / waves:.0f} | {hr}")
    flat = [n for n in acc if "flat_kernel<true, 8, 0>" in n]
    if flat:
        v = {c: sum(x) / len(x) for c, x in acc[flat[0]].items()}
        with open(os.path.join(out_dir, COUNTERS_JSON), "w") as f:
            json.dump({"kernel_src_sha": src_hash(DP_SOURCES), "kernel": flat[0],
                       "flat_descent": {
                           "SQ_INSTS_VALU": v.get("SQ_INSTS_VALU", 0.0),
                           "SQ_WAVES": v.get("SQ_WAVES", 0.0),
                           "active_lanes": v.get("SQ_THREAD_CYCLES_VALU", 0.0)
                           / max(1.0, v.get("SQ_ACTIVE_INST_VALU", 1.0)),
                           "L2_hit_rate": (v["TCC_HIT_sum"] / (v["TCC_HIT_sum"] + v["TCC_MISS_sum"])
                                           if "TCC_HIT_sum" in v and "TCC_MISS_sum" in v
                                           else None)}}, f, indent=1)
    with open(os.path.join(out_dir, COUNTERS_FILE), "w") as f:
        f.write("# SS_TUNE_CACHE=/tmp/ss_tune.jsonl rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU "
                "SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_INSTS_VALU_TRANS_F32 TCC_HIT_sum "
                "TCC_MISS_sum --kernel-include-regex 'flat_kernel|shadow_kernel' --output-format csv "
                "-d <dir> -o bench -- python bench.py --steps 1 --warmup 0 --no-cpu --no-extras "
                "--dem-cache /tmp/dem_tile.npy\n")
        f.write("\n".join(lines) + "\n")


def _pct(xs):
    import numpy as np
    return [float(v) for v in np.percentile(np.asarray(xs, dtype=np.float64), [10, 50, 90])]


def _timed(fn, reps):
    """Per-repetition milliseconds of fn() between events on the current stream."""
    import torch
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return ts


def _timed_busy(fn, reps, spin_cycles=400000):
    """As _timed, with the GPU kept busy (a spin kernel) while the start event and fn's
    launches are enqueued, so the events time the GPU work alone, not host launch latency
    (for launches of a few microseconds)."""
    import torch
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(spin_cycles)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return ts


def _err_stats(x, ref):
    """mean, 99th percentile and fraction above 0.05 of |x - ref|."""
    d = (x - ref).abs().flatten()
    ds, _ = d.sort()
    p99 = float(ds[min(ds.numel() - 1, int(0.99 * ds.numel()))])
    return {"mean_abs": float(d.mean()), "p99_abs": p99, "frac_gt_0.05": float((d > 0.05).float().mean())}


def leg_accuracy(ss, h, mm, D, suns, c):
    """Image error of the descent and of one-texel uniform stepping against
    dense stepping on the half-texel grid (the grid the descent's final samples
    use), over every sun of the workload; and the exact mode (the same grid's
    minimum by branch and bound), timed against dense stepping and checked
    bit-identical to it."""
    import torch
    from synth import R_MOON
    W, H = h.shape[1], h.shape[0]
    pd = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"])
    pu1 = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_UNIFORM)
    pu2 = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_UNIFORM,
                    uniform_step=0.5)
    px = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_EXACT)
    pp = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_POINT)
    bound = ss.bound_build(h)
    t_bound = _timed(lambda: ss.bound_build(h, out=bound), 3)
    dp, u1, u2, ex, pt = [], [], [], [], []
    t_u2, t_ex, cnt = [], [], []
    for (e, a, r) in suns:
        dp.append(ss.shadow_cast(h, D, e, a, r, pd, mm=mm))
        pt.append(ss.shadow_cast(h, D, e, a, r, pp, mm=mm))
        u1.append(ss.shadow_cast(h, D, e, a, r, pu1, mm=mm))
        o2 = torch.empty_like(h)
        ox = torch.empty_like(h)
        t_u2 += _timed(lambda: ss.shadow_cast(h, D, e, a, r, pu2, mm=mm, out=o2), 1)
        ss.shadow_cast(h, D, e, a, r, px, mm=mm, out=ox, bound=bound)
        t_ex += _timed(lambda: ss.shadow_cast(h, D, e, a, r, px, mm=mm, out=ox, bound=bound), 2)[1:]
        u2.append(o2)
        ex.append(ox)
        _, k = ss.shadow_cast_counted(h, D, e, a, r, px, mm=mm, bound=bound)
        cnt.append([int(v) for v in k.cpu().tolist()])
    dp, u1, u2, ex = torch.stack(dp), torch.stack(u1), torch.stack(u2), torch.stack(ex)
    pt = torch.stack(pt)
    rays = W * H * len(suns)
    exact = {"mrays_s": rays / (sum(t_ex) / 1e3) / 1e6,
             "dense_mrays_s": rays / (sum(t_u2) / 1e3) / 1e6,
             "speedup_vs_dense": sum(t_u2) / sum(t_ex),
             "bit_identical_to_dense": bool(torch.equal(ex.view(torch.int32), u2.view(torch.int32))),
             "bound_build_ms": min(t_bound),
             "tests_per_ray": sum(k[0] for k in cnt) / rays,
             "samples_per_ray": sum(k[1] for k in cnt) / rays,
             "launch_ms": t_ex}
    # the same 8 suns as one persistent batched launch (tap-bound pyramid and max-mip
    # rebuilt inside the call), outputs checked against the per-sun launches
    outs_b = [torch.empty_like(h) for _ in suns]
    ss.shadow_cast_batched([h], [D], suns, px, outs=[outs_b], mms=[mm], bounds=[bound])
    t_b = min(_timed(lambda: ss.shadow_cast_batched([h], [D], suns, px, outs=[outs_b], mms=[mm],
                                                     bounds=[bound]), 2))
    exact["batched_mrays_s"] = rays / (t_b / 1e3) / 1e6
    exact["batched_equal_per_sun"] = all(torch.equal(outs_b[k].view(torch.int32),
                                                     ex[k].view(torch.int32)) for k in range(len(suns)))
    del outs_b
    desc = _err_stats(dp, u2)
    point = _err_stats(pt, u2)
    uni1 = _err_stats(u1, u2)
    del dp, pt, u1, ex
    # equal-error sweep: coarser uniform steps until the error passes the
    # descent's, with their cost (the "same accuracy" comparison)
    sweep = []
    for step in (2.0, 4.0, 8.0, 16.0, 32.0, 64.0, 128.0):
        pu = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_UNIFORM,
                       uniform_step=step)
        ts, outs_u = [], []
        for k, (e, a, r) in enumerate(suns):
            o = ss.shadow_cast(h, D, e, a, r, pu, mm=mm)
            ts += _timed(lambda: ss.shadow_cast(h, D, e, a, r, pu, mm=mm, out=o), 1)
            outs_u.append(o)
        st = _err_stats(torch.stack(outs_u), u2)
        del outs_u
        st.update({"step_texels": step, "launch_ms": sum(ts) / len(ts)})
        sweep.append(st)
        if st["mean_abs"] > desc["mean_abs"] and st["frac_gt_0.05"] > desc["frac_gt_0.05"]:
            break
    return {"reference": "uniform stepping at delta/2 (dense half-texel grid), all suns",
            "descent": desc, "point_descent": point, "uniform_1_texel": uni1,
            "mean_s_dense": float(u2.mean()), "uniform_step_sweep": sweep}, exact


def equal_error_speedup(err, sweep, descent_ms):
    """Per-sun time of uniform stepping at the step whose mean |s - s_dense| equals err,
    interpolated log-linearly in (step, error) and (step, time) between the sweep's
    points, divided by the descent's per-sun time (> 1: the descent is faster at equal
    mean error).  None if the sweep does not bracket err."""
    pts = sorted((p["step_texels"], p["mean_abs"], p["launch_ms"]) for p in sweep)
    for (s0, e0, t0), (s1, e1, t1) in zip(pts, pts[1:]):
        if e0 <= err <= e1 and e0 > 0 and e1 > e0:
            f = (math.log(err) - math.log(e0)) / (math.log(e1) - math.log(e0))
            t = math.exp(math.log(t0) + f * (math.log(t1) - math.log(t0)))
            step = math.exp(math.log(s0) + f * (math.log(s1) - math.log(s0)))
            return {"uniform_step_texels": step, "uniform_ms_per_sun": t,
                    "descent_ms_per_sun": descent_ms, "speedup": t / descent_ms}
    return None


def leg_schedules(ss, h, mm, D, suns):
    """The paper's step-count study (Sec. 6.3) on the tile DEM: runs {5,5,5}
    against {5,5,5,3} for the point-sample descent (Alg. 1 as printed) and the
    texel descent, and uniform stepping with 100 one-texel steps; per-launch
    time averaged over the suns, and grid samples evaluated per ray."""
    from synth import R_MOON
    W, H = h.shape[1], h.shape[0]
    cfg = {"555": dict(schedule=ss.SS_SCHED_EQUAL, n_segments=3),
           "5553": dict(schedule=ss.SS_SCHED_LIST, n_segments=4, n_prime_list=(5, 5, 5, 3))}
    res = {}
    for mode_name, mode in (("point", ss.SS_MODE_POINT), ("descent", ss.SS_MODE_DP)):
        for k, kw in cfg.items():
            p = ss.Params(radius_m=R_MOON, mode=mode, **kw)
            ts, ev = [], []
            for (e, a, r) in suns:
                ss.shadow_cast(h, D, e, a, r, p, mm=mm)
                ts += _timed(lambda: ss.shadow_cast(h, D, e, a, r, p, mm=mm), 1)
                _, c = ss.shadow_cast_counted(h, D, e, a, r, p, mm=mm)
                ev.append(sum(int(v) for v in c.cpu().tolist()))
            res[f"{mode_name}_{k}"] = {"launch_ms": sum(ts) / len(ts),
                                       "evals_per_ray": sum(ev) / len(ev) / (W * H)}
    pu = ss.Params(radius_m=R_MOON, mode=ss.SS_MODE_UNIFORM, max_len_m=100.0 * D)
    ts = []
    for (e, a, r) in suns:
        ss.shadow_cast(h, D, e, a, r, pu, mm=mm)
        ts += _timed(lambda: ss.shadow_cast(h, D, e, a, r, pu, mm=mm), 1)
    res["uniform_100_steps"] = {"launch_ms": sum(ts) / len(ts)}
    for m in ("point", "descent"):
        res[f"{m}_time_ratio_5553_over_555"] = res[f"{m}_5553"]["launch_ms"] / res[f"{m}_555"]["launch_ms"]
    res["uniform_100_over_point_555"] = res["uniform_100_steps"]["launch_ms"] / res["point_555"]["launch_ms"]
    return res


def leg_gather(ss, dev, n_rays, src_floats, roof, iters=64, n_threads=1 << 21):
    """Rate of incoherent 4-byte gathers (every lane of a wavefront on its own
    cache line), from the library's gather probe (indices generated in the
    kernel, eight loads in flight per lane) over a buffer the size of the
    tile's heightfield plus mipmap, inside 1 MiB windows (L2-resident) and
    16 KiB windows (L1-resident); the rate of coherent gathers (each wavefront
    reads an 8 x 8 patch of a tile-sized image per step, the pattern of the
    descent's 8 x 8 ray tiles); and the descent's own gather rate (one per lower
    bound, four per bilinear sample) against both."""
    import torch
    src = torch.rand(src_floats, device=dev)
    out = torch.empty(n_threads, dtype=torch.float32, device=dev)
    res = {}
    for name, win in (("whole_buffer", 0), ("window_1MiB", 1 << 18), ("window_16KiB", 1 << 12)):
        ss.probe_gather(src, win, iters, n_threads, out)
        t = min(_timed(lambda: ss.probe_gather(src, win, iters, n_threads, out), 3))
        res["incoherent_" + name + "_gathers_per_s"] = n_threads * iters / (t / 1e3)
    # coherent: a wavefront reads one 8 x 8 patch of a tile-sized image per step, as the
    # descent's 8 x 8 ray tiles read neighbouring texels (the measured L2-side ceiling for
    # that pattern)
    side = int(math.isqrt(src_floats))
    img = src[:side * side].view(side, side)
    ss.probe_gather_tiles(img, iters, n_threads, out)
    t = min(_timed(lambda: ss.probe_gather_tiles(img, iters, n_threads, out), 3))
    res["coherent_8x8_patch_gathers_per_s"] = n_threads * iters / (t / 1e3)
    res["descent_gathers_per_s"] = ((roof["lb_evals_per_ray"] + 4.0 * roof["samples_per_ray"])
                                    * n_rays / (roof["avg_launch_ms"] / 1e3))
    res["descent_over_incoherent_1MiB"] = (res["descent_gathers_per_s"]
                                           / res["incoherent_window_1MiB_gathers_per_s"])
    res["descent_over_coherent_8x8"] = (res["descent_gathers_per_s"]
                                        / res["coherent_8x8_patch_gathers_per_s"])
    return res


def leg_valu(ss, dev, iters=4096, n_workgroups=8192):
    """The FP32 VALU rate the roofline divides by, measured: eight independent non-packed FMA
    chains per lane at full occupancy (ss_probe_valu)."""
    out = ss.probe_valu(iters, n_workgroups, device=dev)
    t = min(_timed(lambda: ss.probe_valu(iters, n_workgroups, out=out), 3))
    rate = 32.0 * iters * n_workgroups * 256 / (t / 1e3) / 1e12
    return {"fma_lane_tops": rate, "of_peak": rate / PEAK_VALU_TOPS, "ms": t}


def cpu_uniform_baseline(h_np, params_or, seconds=5.0):
    """The FP64 oracle's uniform stepping (1 texel) on a bounded random sample."""
    import numpy as np
    import oracle
    threads = max(1, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(4321)
    n = 256 * threads
    while True:
        rays = rng.choice(h_np.size, size=min(h_np.size, n), replace=False)
        t0 = time.perf_counter()
        oracle.shadow_threaded(h_np, params_or, rays, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.6 * seconds or rays.size >= h_np.size:
            break
        n = int(rays.size * min(8.0, max(1.5, seconds / max(dt, 1e-3))))
    return {"value": rays.size / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{rays.size} random texels, first sun, uniform stepping at 1 texel, "
                      f"{dt:.1f} s"}


def leg_cold_maxmip(ss, h, mm, mm_bytes, reps=5):
    """Mipmap build after reading 1 GiB through the caches: L2 and MALL then hold none of the
    tile, and (a read leaves clean lines) nothing of the flush is written back inside the timed
    build.  Flushing by writing instead charges the build with that write-back (about twice the
    time at 4096^2)."""
    import torch
    scratch = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=h.device)
    ts = []
    for _ in range(reps):
        scratch.sum()
        ts += _timed(lambda: ss.maxmip(h, out=mm), 1)
    del scratch
    ms = float(sum(ts) / len(ts))
    return {"avg_launch_ms": ms, "achieved_GBs": mm_bytes / (ms / 1e3) / 1e9,
            "frac": mm_bytes / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, "flush": "read 1 GiB"}


def maxmip_bytes(ss, W, H):
    """Algorithmic HBM bytes of one build: the tile read once, levels >= 1 written once."""
    return 4 * W * H + 4 * sum(((W + (1 << m) - 1) >> m) * ((H + (1 << m) - 1) >> m)
                               for m in range(1, ss.maxmip_levels(W, H)))


def leg_diff(ss, reps=5):
    """The 2048^2 differentiable workload: forward and forward+adjoint rays/s."""
    import torch
    from synth import config, dem_for, sun_list, R_MOON
    c = config("diff")
    W, H, D = c["tiles"][0]
    e, a, r = sun_list("diff")[0]
    h = dem_for("diff", device="cuda")
    mm = ss.maxmip(h)
    p = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"])
    out = torch.empty_like(h)
    g = torch.randn(H, W, generator=torch.Generator(device="cpu").manual_seed(11)).to(h.device)
    gh = torch.zeros_like(h)
    gs = torch.zeros(2, dtype=torch.float64, device=h.device)

    sample = torch.empty(h.shape, dtype=torch.int32, device=h.device)

    def fwd():
        ss.maxmip(h, out=mm)
        ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out)

    def fwd_bwd():
        # recorded forward, adjoint from the record
        ss.maxmip(h, out=mm)
        ss.shadow_cast_save(h, D, e, a, r, p, mm=mm, out=out, sample=sample)
        ss.shadow_cast_backward_saved(h, D, e, a, sample, g, r, p, mm=mm, grad_h=gh, grad_sun=gs)

    def fwd_bwd_replay():
        fwd()
        ss.shadow_cast_backward_penumbra(h, D, e, a, out, g, r, p, mm=mm, grad_h=gh, grad_sun=gs)

    fwd_bwd()
    fwd_bwd_replay()
    tf = _timed(fwd, reps)
    tb = _timed(fwd_bwd, reps)
    tr = _timed(fwd_bwd_replay, reps)
    n = W * H
    return {"fwd_mrays_s": n / (min(tf) / 1e3) / 1e6,
            "fwd_bwd_mrays_s": n / (min(tr) / 1e3) / 1e6,
            "fwd_bwd_record_mrays_s": n / (min(tb) / 1e3) / 1e6,
            "fwd_ms": min(tf), "fwd_bwd_ms": min(tr), "fwd_bwd_record_ms": min(tb),
            "backward": "replaying adjoint (decisions recomputed for rays with s strictly inside "
                        "(0, 1)); record: 4 B/ray from the forward"}


def leg_frame(ss, reps=10):
    """Whole frames as Sec. 4 and 6.3 run them, on the 2048^2 tile (10 m/texel; the
    paper's stitched fields are 1024-2048 texels): view rays from a camera 8 km up
    heading across the tile (25 degrees down, 60 degree field of view), then one
    shadow ray from every visible point (shaded in 8 x 8 pixel tiles), in each shadow mode.
    Per image size: view
    rays by the pyramid walk and by the dense march (identical output), grid samples
    and pyramid cells per pixel, shadow rays per mode, the frame time and rate (view
    walk + shadows), and the adjoint of the descent's shadow rays at the hits.  Terrain set-up (max-mip, tap-bound pyramid) runs once per
    terrain change, not per frame, and is reported apart."""
    import torch
    from synth import config, dem_for, sun_list, R_MOON
    from synth.configs import view_scene
    c = config("diff")
    W, H, D = c["tiles"][0]
    e, a, r = sun_list("diff")[0]
    h = dem_for("diff", device="cuda")
    mm = ss.maxmip(h)
    bound = ss.bound_build(h)
    setup_ms = min(_timed(lambda: (ss.maxmip(h, out=mm), ss.bound_build(h, out=bound)), 5))
    modes = {
        "descent": ss.Params(radius_m=R_MOON, max_len_m=c["max_len"]),
        "point_555": ss.Params(radius_m=R_MOON, mode=ss.SS_MODE_POINT,
                               schedule=ss.SS_SCHED_EQUAL, n_segments=3),
        "point_5553": ss.Params(radius_m=R_MOON, mode=ss.SS_MODE_POINT,
                                schedule=ss.SS_SCHED_LIST, n_segments=4,
                                n_prime_list=(5, 5, 5, 3)),
        "uniform_100_steps": ss.Params(radius_m=R_MOON, mode=ss.SS_MODE_UNIFORM,
                                       max_len_m=100.0 * D),
    }
    out = {"tile": f"{W}x{H} at {D} m/texel", "terrain_setup_ms": setup_ms}
    for (pw, ph) in ((1920, 1080), (512, 512)):
        cam = view_scene("flyover", pw, ph, W, H, D)
        ch = ss.Camera(**cam, mode=ss.SS_VIEW_HIER)
        cd = ss.Camera(**cam, mode=ss.SS_VIEW_DENSE)
        t = torch.empty((ph, pw), dtype=torch.float32, device=h.device)
        xy = torch.empty((ph, pw, 2), dtype=torch.float32, device=h.device)
        s = torch.empty((ph, pw), dtype=torch.float32, device=h.device)
        _, _, st = ss.view_cast(h, D, ch, R_MOON, bound, steps=True)
        _, _, sd = ss.view_cast(h, D, cd, R_MOON, bound, steps=True)
        vh = min(_timed(lambda: ss.view_cast(h, D, ch, R_MOON, bound, out_t=t, out_xy=xy), reps))
        vd = min(_timed(lambda: ss.view_cast(h, D, cd, R_MOON, bound, out_t=t, out_xy=xy), reps))
        ss.view_cast(h, D, ch, R_MOON, bound, out_t=t, out_xy=xy)
        res = {"view_walk_ms": vh, "view_dense_ms": vd,
               "visible_frac": float(torch.isfinite(t).float().mean()),
               "walk_samples_per_pixel": float(st[..., 0].float().mean()),
               "walk_cells_per_pixel": float(st[..., 1].float().mean()),
               "dense_samples_per_pixel": float(sd[..., 0].float().mean())}
        res["steps_ratio_dense_over_walk"] = res["dense_samples_per_pixel"] / (
            res["walk_samples_per_pixel"] + res["walk_cells_per_pixel"])
        for name, p in modes.items():
            ss.shadow_points_image(h, D, e, a, xy, r, p, mm, out=s, bound=bound)
            ms = min(_timed(lambda: ss.shadow_points_image(h, D, e, a, xy, r, p, mm, out=s,
                                                           bound=bound), reps))
            res[f"shadow_{name}_ms"] = ms
            res[f"frame_{name}_ms"] = vh + ms
            res[f"frame_{name}_hz"] = 1e3 / (vh + ms)
        # the adjoint at the frame's hits (points held fixed): dL/dh and dL/d(sun) for a
        # seeded upstream gradient over the visible pixels
        g = torch.randn((ph, pw), generator=torch.Generator().manual_seed(11)).to(h.device)
        g = torch.where(torch.isfinite(t), g, torch.zeros_like(g)).contiguous()
        gh = torch.zeros_like(h)
        gsun = torch.zeros(2, dtype=torch.float64, device=h.device)
        pd = modes["descent"]
        ss.shadow_points_backward(h, D, e, a, xy, g, r, pd, mm=mm, grad_h=gh, grad_sun=gsun)
        res["shadow_adjoint_descent_ms"] = min(_timed(
            lambda: ss.shadow_points_backward(h, D, e, a, xy, g, r, pd, mm=mm, grad_h=gh,
                                              grad_sun=gsun), reps))
        out[f"{pw}x{ph}"] = res
    out["paper_context"] = ("GTX 970M, whole frame with shading: 1920x1080 5.4 ms (185 Hz) "
                            "{5,5,5}, 6.2 ms {5,5,5,3}, 18.2 ms uniform 100 steps; 512^2 402 Hz")
    return out


def leg_stitch(ss, reps=10):
    """Building a working tile from tiles in other frames (Sec. 3.3 stitched virtual texture,
    Sec. 4 cube faces): a 4096^2 tile at 5 m/texel tangent 1.2 km from the +z/+x face seam,
    resampled from two 6144^2 cube-face sub-tiles meeting there (two launches), then its
    2048^2 core shaded through a ray window (descent, 30 km cap, e = 1.5 deg from across the
    seam).  Stitch rate in destination texels/s and in bytes/s against HBM, counting the
    algorithmic 4 bytes written plus 4 read per destination texel (neighbouring texels share
    their source taps)."""
    import math
    import torch
    from synth import R_MOON
    from synth.planet import seam_frames
    fa, fb, fw = seam_frames(core=2048, halo=1024, texel_m=5.0, n_src=6144)
    dev = "cuda"
    gen = torch.Generator(device=dev).manual_seed(7)
    srcs = [(torch.rand((f["rows"], f["width"]), generator=gen, device=dev) * 2000.0 - 500.0,
             ss.Frame(**f)) for f in (fa, fb)]
    W = fw["width"]
    out = torch.empty((W, W), dtype=torch.float32, device=dev)
    fr = ss.Frame(**fw)
    ss.stitch(srcs, fr, R_MOON, out=out)
    ts = _timed(lambda: ss.stitch(srcs, fr, R_MOON, out=out), reps)
    ms = min(ts)
    nan = int(torch.isnan(out).sum())
    win = (1024, 1024, 2048, 2048)
    p = ss.Params(radius_m=R_MOON, max_len_m=30000.0)
    mm = ss.maxmip(out)
    s = torch.empty((2048, 2048), dtype=torch.float32, device=dev)
    e, a, r = math.radians(1.5), 0.0, math.radians(0.267)
    ss.shadow_cast(out, 5.0, e, a, r, p, mm=mm, out=s, window=win)
    tsh = min(_timed(lambda: ss.shadow_cast(out, 5.0, e, a, r, p, mm=mm, out=s, window=win), reps))
    n = W * W
    return {"work_tile": f"{W}x{W} at 5 m/texel", "sources": "2 x 6144^2 cube-face sub-tiles",
            "stitch_ms": ms, "uncovered_texels": nan,
            "stitch_gtexels_s": n / (ms / 1e3) / 1e9,
            "stitch_gb_s": 8.0 * n / (ms / 1e3) / 1e9,
            "stitch_frac_of_hbm": 8.0 * n / (ms / 1e3) / 8.0e12,
            "core_shadow_ms": tsh, "core_mrays_s": 2048 * 2048 / (tsh / 1e3) / 1e6}


def leg_batched(ss, reps=3):
    """8 uneven tiles x 64 suns through one captured graph (mipmaps + persistent kernel)."""
    from synth import config, dem_for, sun_list, R_MOON
    c = config("batched")
    heights = [dem_for("batched", t, device="cuda") for t in range(len(c["tiles"]))]
    texels = [tx for (_, _, tx) in c["tiles"]]
    suns = sun_list("batched")
    plan = ss.BatchedPlan(heights, texels, suns, ss.Params(radius_m=R_MOON, max_len_m=c["max_len"]))
    plan.launch()
    ts = _timed(plan.launch, reps)
    rays = sum(w * r for (w, r, _) in c["tiles"]) * len(suns)
    rt, fd = plan.config()
    plan.close()
    del plan
    # the exact mode over the same batch (tap-bound pyramids rebuilt in the graph)
    plan = ss.BatchedPlan(heights, texels, suns,
                          ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_EXACT))
    plan.launch()
    tx = _timed(plan.launch, 1)
    plan.close()
    del plan, heights
    return {"rays": rays, "graph_launch_ms": min(ts), "mrays_s": rays / (min(ts) / 1e3) / 1e6,
            "ray_tile": rt, "fuse_depth": fd, "exact_graph_launch_ms": min(tx),
            "exact_mrays_s": rays / (min(tx) / 1e3) / 1e6}


def leg_polar(ss, reps=3):
    """16384^2 at 2 m/texel, sun at 0.2 degrees, 60 km rays: forward and forward+adjoint."""
    import torch
    from synth import config, dem_for, sun_list, R_MOON
    c = config("polar")
    W, H, D = c["tiles"][0]
    e, a, r = sun_list("polar")[0]
    h = dem_for("polar", device="cuda")
    mm = ss.maxmip(h)
    p = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"])
    out = torch.empty_like(h)

    def fwd():
        ss.maxmip(h, out=mm)
        ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out)

    fwd()
    tf = _timed(fwd, reps)
    mm_b = maxmip_bytes(ss, W, H)
    t_mm = min(_timed_busy(lambda: ss.maxmip(h, out=mm), 3))
    mm_res = {"warm_ms": t_mm, "warm_frac": mm_b / (t_mm / 1e3) / 1e9 / PEAK_HBM_GBS,
              "cold": leg_cold_maxmip(ss, h, mm, mm_b, reps=3)}
    g = torch.ones_like(h)
    gh = torch.zeros_like(h)
    gs = torch.zeros(2, dtype=torch.float64, device=h.device)

    def fwd_bwd():
        ss.maxmip(h, out=mm)
        ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out)
        ss.shadow_cast_backward_penumbra(h, D, e, a, out, g, r, p, mm=mm, grad_h=gh, grad_sun=gs)

    fwd_bwd()
    tb = _timed(fwd_bwd, 2)
    n = W * H
    ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out)
    mean_s = float(out.mean())
    # uniform stepping at one texel (the paper's baseline), same cap and exits
    pu = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_UNIFORM)
    ss.shadow_cast(h, D, e, a, r, pu, mm=mm, out=out)
    tu = _timed(lambda: ss.shadow_cast(h, D, e, a, r, pu, mm=mm, out=out), 2)
    bound = ss.bound_build(h)
    px = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_EXACT)
    tx = _timed(lambda: ss.shadow_cast(h, D, e, a, r, px, mm=mm, out=out, bound=bound), 1)
    res = {"fwd_mrays_s": n / (min(tf) / 1e3) / 1e6, "fwd_bwd_mrays_s": n / (min(tb) / 1e3) / 1e6,
           "fwd_ms": min(tf), "fwd_bwd_ms": min(tb), "mean_s": mean_s,
           "backward": "replaying adjoint (decisions recomputed for rays with s in (0, 1))",
           "uniform_1_texel_mrays_s": n / (min(tu) / 1e3) / 1e6, "uniform_1_texel_ms": min(tu),
           "speedup_vs_uniform": min(tu) / min(tf),
           "exact_mrays_s": n / (min(tx) / 1e3) / 1e6, "exact_ms": min(tx), "maxmip": mm_res}
    del bound
    del h, mm, out, g, gh
    return res


def leg_small(ss, reps=50):
    """The 256^2 small configuration (20 m/texel, rays to the tile edge, e = 1.5 deg): descent
    and one-texel uniform stepping, forward, per launch (launch-bound: 65536 rays)."""
    from synth import config, dem_for, sun_list, R_MOON
    c = config("small")
    W, H, D = c["tiles"][0]
    e, a, r = sun_list("small")[0]
    h = dem_for("small", device="cuda")
    mm = ss.maxmip(h)
    out = torch_empty_like(h)
    res = {}
    for name, p in (("descent", ss.Params(radius_m=R_MOON)),
                    ("uniform_1_texel", ss.Params(radius_m=R_MOON, mode=ss.SS_MODE_UNIFORM))):
        ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out)
        t = float(sorted(_timed(lambda: ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out),
                                reps))[reps // 2])
        res[f"{name}_launch_ms"] = t
        res[f"{name}_mrays_s"] = W * H / (t / 1e3) / 1e6
    res["speedup_vs_uniform"] = res["uniform_1_texel_launch_ms"] / res["descent_launch_ms"]
    return res


def torch_empty_like(h):
    import torch
    return torch.empty_like(h)


def cpu_oracle_configs(seconds_each=4.0):
    """The FP64 oracle (descent and one-texel uniform stepping) on the small tile in full and
    on 2^16 random rays of the differentiable and polar tiles, extrapolated linearly to
    their full ray counts (the oracle's cost is per ray)."""
    import numpy as np
    import oracle
    from synth import config, dem_for, sun_list, R_MOON
    threads = max(1, len(os.sched_getaffinity(0)))
    out = {"cores": threads}
    for name in ("small", "diff", "polar"):
        c = config(name)
        W, H, D = c["tiles"][0]
        e, a, r = sun_list(name)[0]
        h = dem_for(name, device="cuda").cpu().numpy()
        rays = None if name == "small" else np.sort(
            np.random.default_rng(99).choice(W * H, size=1 << 16, replace=False)).astype(np.int64)
        n = W * H if rays is None else rays.size
        po = oracle.Params(W, H, D, R_MOON, e, a, r, max_len_m=c["max_len"])
        oracle.shadow(h, po, np.arange(1, dtype=np.int64))  # the oracle's mipmap, untimed
        row = {"rays_timed": n, "extrapolated": rays is not None}
        for mname, mode in (("descent", 0), ("uniform_1_texel", 1)):
            t0 = time.perf_counter()
            oracle.shadow_threaded(h, po.replace(mode=mode), rays, threads=threads)
            dt = time.perf_counter() - t0
            row[f"{mname}_mrays_s"] = n / dt / 1e6
            row[f"{mname}_full_tile_s"] = dt * (W * H) / n
        out[name] = row
        del h
    return out


def leg_exact(ss, reps=2):
    """The exact mode alone on the 4096^2 tile, all 8 suns: launch times, rays/s and the
    units per ray (for profiling its kernel)."""
    import torch
    from synth import config, dem_for, sun_list, R_MOON
    c = config("tile")
    W, H, D = c["tiles"][0]
    h = dem_for("tile", device="cuda")
    mm = ss.maxmip(h)
    bound = ss.bound_build(h)
    out = torch.empty_like(h)
    p = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_EXACT)
    ts = []
    for (e, a, r) in sun_list("tile"):
        ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out, bound=bound)
        ts.append(min(_timed(lambda: ss.shadow_cast(h, D, e, a, r, p, mm=mm, out=out,
                                                    bound=bound), reps)))
    return {"launch_ms": ts, "mrays_s": W * H * len(ts) / (sum(ts) / 1e3) / 1e6}


LEGS = {"small": lambda ss: leg_small(ss),
        "frame": lambda ss: leg_frame(ss), "stitch": lambda ss: leg_stitch(ss),
        "diff": lambda ss: leg_diff(ss), "exact": lambda ss: leg_exact(ss)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every leg beside the headline step (uniform, accuracy, backward, "
                         "cold mipmap, batched, polar, differentiable)")
    ap.add_argument("--no-big", action="store_true",
                    help="skip the batched (8 tiles x 64 suns) and polar (16384^2) legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB device copy first (counter calibration)")
    ap.add_argument("--dem-cache", default="",
                    help="load the DEM from this .npy if present, else generate and save it")
    ap.add_argument("--summarize", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "COUNTERS", "OUT"),
                    help="write profile summaries from rocprofv3 CSV directories and exit")
    ap.add_argument("--leg", action="append", choices=sorted(LEGS),
                    help="run only this extra leg (repeatable) and print its JSON; for profiling")
    args = ap.parse_args()
    if args.summarize:
        summarize_profiles(*args.summarize)
        return
    if args.leg:
        import paper_2005_06671_amd as ss
        print(json.dumps({name: LEGS[name](ss) for name in args.leg}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the path would "
              "shard by replicating the DEM and its mipmap and splitting ray blocks across GPUs, "
              "which this single-GPU build does not implement", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2005_06671_amd as ss
    from synth import config, dem_for, sun_list, seed_of, R_MOON

    dev = torch.device("cuda:0")
    c = config("tile")
    W, H, D = c["tiles"][0]
    suns = sun_list("tile")
    if args.dem_cache and os.path.exists(args.dem_cache):
        h = torch.from_numpy(np.load(args.dem_cache)).to(dev)
    else:
        h = dem_for("tile", device=dev)
        if args.dem_cache:
            np.save(args.dem_cache, h.cpu().numpy())
    mm = torch.empty(ss.maxmip_floats(W, H), dtype=torch.float32, device=dev)
    outs = [torch.empty_like(h) for _ in suns]
    params = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"])
    rays_per_step = W * H * len(suns)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def pair():
        return (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    # The step: one replay of the batched plan's graph (max-mip build, then one launch over
    # every ray block of the 8 suns).  Outputs equal the per-sun launches below bit for bit.
    plan = ss.BatchedPlan([h], [D], suns, params, outs=[outs], mms=[mm])
    plan_cfg = plan.config()
    ev_step = [pair() for _ in range(args.steps)]
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev_step[i][0].record(stream)
        plan.launch()
        ev_step[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / max(1, args.steps)
    value = rays_per_step / (ms_per_step / 1e3) / 1e6
    step_ms = [a.elapsed_time(b) for a, b in ev_step]
    avg_step_ms = float(np.mean(step_ms))
    plan.close()

    # the same work as eight per-sun launches of the per-tile kernel (after the timed region)
    reps = max(2, min(args.steps, 5))
    ev_dp = [[pair() for _ in suns] for _ in range(reps)]
    ev_mm = [pair() for _ in range(reps)]
    outs_ps = [torch.empty_like(h) for _ in suns]

    def per_sun_step(i=None):
        if i is not None:
            ev_mm[i][0].record(stream)
        ss.maxmip(h, out=mm)
        if i is not None:
            ev_mm[i][1].record(stream)
        for k, (e, a, r) in enumerate(suns):
            if i is not None:
                ev_dp[i][k][0].record(stream)
            ss.shadow_cast(h, D, e, a, r, params, mm=mm, out=outs_ps[k])
            if i is not None:
                ev_dp[i][k][1].record(stream)

    per_sun_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(reps):
        per_sun_step(i)
    torch.cuda.synchronize()
    ps_ms = (time.perf_counter() - t0) * 1e3 / reps
    launch_ms = [a.elapsed_time(b) for row in ev_dp for a, b in row]
    maxmip_ms = [a.elapsed_time(b) for a, b in ev_mm]
    avg_dp_ms = float(np.mean(launch_ms))
    avg_mm_ms = float(np.mean(maxmip_ms))
    same = all(torch.equal(outs[k].view(torch.int32), outs_ps[k].view(torch.int32))
               for k in range(len(suns)))
    if not same:
        raise RuntimeError("batched and per-sun launches disagree")
    del outs_ps

    # algorithmic units of the step (instrumented twin of the same per-ray code, untimed)
    units = []
    for k, (e, a, r) in enumerate(suns):
        _, cnt = ss.shadow_cast_counted(h, D, e, a, r, params, mm=mm)
        units.append([int(x) for x in cnt.cpu().tolist()])
    n_lb = float(np.sum([u[0] for u in units]))
    n_smp = float(np.sum([u[1] for u in units]))
    ops_per_step = OPS_LB * n_lb + OPS_SAMPLE * n_smp
    # the events bracket the whole graph, so the max-mip build (0.2% of it) counts as
    # kernel time and the figure errs low
    achieved = ops_per_step / (avg_step_ms / 1e3) / 1e12
    traffic = traffic_from_profile()
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                "frac": achieved / PEAK_VALU_TOPS, "traffic": traffic,
                "kernel": "flat_kernel<sphere, 8x8, descent> (one launch over every ray block "
                          "of the 8 suns)",
                "avg_launch_ms": avg_step_ms, "timed_span": "graph replay incl. max-mip build",
                "lb_evals_per_ray": n_lb / rays_per_step, "samples_per_ray": n_smp / rays_per_step,
                "ops_per_unit": {"lower_bound": OPS_LB, "bilinear_sample": OPS_SAMPLE},
                "plan_ray_tile_fuse_depth": list(plan_cfg)}
    cnt = counters_from_profile()
    if cnt:
        # issued VALU wavefront instructions against one per SIMD per 4 cycles (the full-rate
        # issue of a 64-lane wavefront on a 16-lane SIMD), from the committed counters
        simd_slots = 256 * 4 * 2.4e9 * (avg_step_ms / 1e3) / 4.0
        roofline["issue_frac"] = cnt["SQ_INSTS_VALU"] / simd_slots
        roofline["valu_instr_per_unit"] = cnt["SQ_INSTS_VALU"] * 64.0 / (n_lb + n_smp)
        roofline["active_lanes_per_valu_instr"] = cnt["active_lanes"]
    mm_bytes = float(maxmip_bytes(ss, W, H))
    # the build's two launches timed on the GPU alone (the stream kept busy while they are
    # enqueued); the per-sun loop's events above also hold host launch latency
    t_mm = float(np.mean(_timed_busy(lambda: ss.maxmip(h, out=mm), 10)))
    maxmip = {"bound": "hbm", "avg_launch_ms": t_mm,
              "achieved_GBs": mm_bytes / (t_mm / 1e3) / 1e9, "peak_GBs": PEAK_HBM_GBS,
              "frac": mm_bytes / (t_mm / 1e3) / 1e9 / PEAK_HBM_GBS,
              "per_sun_loop_ms": avg_mm_ms,
              "note": "64 MiB source is L2/MALL resident between builds (warm)"}
    ps_ops = ops_per_step / len(suns)  # the per-sun launches do the same units
    extras = {"step_ms_p10_p50_p90": _pct(step_ms),
              "per_sun_launches": {
                  "ms_per_step": ps_ms, "mrays_s": rays_per_step / (ps_ms / 1e3) / 1e6,
                  "kernel": "shadow_kernel<sphere, 8x8, descent, plain>",
                  "avg_launch_ms": avg_dp_ms, "launch_ms_p10_p50_p90": _pct(launch_ms),
                  "launch_ms_per_sun": [float(np.mean([ev_dp[i][k][0].elapsed_time(ev_dp[i][k][1])
                                                       for i in range(reps)]))
                                        for k in range(len(suns))],
                  "roofline_frac": ps_ops / (avg_dp_ms / 1e3) / 1e12 / PEAK_VALU_TOPS,
                  "outputs_equal_batched": same}}
    if not args.no_extras:
        extras["accuracy_vs_dense"], extras["exact_mode"] = leg_accuracy(ss, h, mm, D, suns, c)
        maxmip["cold"] = leg_cold_maxmip(ss, h, mm, mm_bytes)
        extras["schedule_study"] = leg_schedules(ss, h, mm, D, suns)
        extras["gather_ceiling"] = leg_gather(ss, dev, rays_per_step,
                                              W * H + ss.maxmip_floats(W, H), roofline)
        extras["valu_ceiling"] = leg_valu(ss, dev)
        roofline["peak_measured_fma_tops"] = extras["valu_ceiling"]["fma_lane_tops"]
        # uniform stepping, one texel per step, same suns, cap and exits, timed like the
        # step: the batched call over the 8 suns (max-mip build + one launch) after a
        # warm-up, 5 event-timed repetitions; and as per-sun launches
        pu = ss.Params(radius_m=R_MOON, max_len_m=c["max_len"], mode=ss.SS_MODE_UNIFORM)
        ws_u = torch.empty(ss.batched_workspace_bytes(1, len(suns)), dtype=torch.uint8,
                           device=dev)

        def uniform_batched():
            ss.shadow_cast_batched([h], [D], suns, pu, outs=[outs], mms=[mm], ws=ws_u)

        def uniform_per_sun():
            ss.maxmip(h, out=mm)
            for k, (e, a, r) in enumerate(suns):
                ss.shadow_cast(h, D, e, a, r, pu, mm=mm, out=outs[k])

        uniform_batched()
        t_ub = _timed(uniform_batched, 5)
        uniform_per_sun()
        t_ups = _timed(uniform_per_sun, 3)
        uniform = rays_per_step / (float(np.median(t_ub)) / 1e3) / 1e6
        extras["uniform_mrays_s"] = uniform
        extras["uniform_ms_per_step_p10_p50_p90"] = _pct(t_ub)
        extras["speedup_vs_uniform"] = value / uniform
        u_ps = rays_per_step / (float(np.median(t_ups)) / 1e3) / 1e6
        extras["per_sun_launches"]["uniform_mrays_s"] = u_ps
        extras["per_sun_launches"]["speedup_vs_uniform"] = extras["per_sun_launches"]["mrays_s"] / u_ps
        ucnt = []
        for k, (e, a, r) in enumerate(suns[:2]):
            _, cnt_u = ss.shadow_cast_counted(h, D, e, a, r, pu, mm=mm)
            ucnt.append(int(cnt_u[1].item()))
        extras["uniform_steps_per_ray"] = float(np.mean(ucnt)) / (W * H)
        u_ops = OPS_USTEP * extras["uniform_steps_per_ray"] * rays_per_step
        extras["uniform_roofline_frac"] = (u_ops / (float(np.median(t_ub)) / 1e3) / 1e12
                                           / PEAK_VALU_TOPS)
        # equal-error comparison: the uniform step whose image error against dense stepping
        # equals the descent's (log-linear between the sweep's steps), and its per-sun time
        acc = extras["accuracy_vs_dense"]
        extras["speedup_vs_uniform_equal_error"] = equal_error_speedup(
            acc["descent"]["mean_abs"], acc["uniform_step_sweep"], avg_dp_ms)
        # the same-accuracy comparison: the exact mode (descent as incumbent, then
        # branch and bound over the max-mip tap-bound pyramid) returns the dense
        # half-texel stepping result bit for bit; one-texel stepping is coarser
        # than both (its error against dense is in accuracy_vs_dense)
        ex = extras["exact_mode"]
        extras["equal_accuracy"] = {
            "exact_over_dense_uniform_identical_output": ex["speedup_vs_dense"],
            # the exact mode is timed as per-sun launches: against uniform stepping launched alike
            "exact_over_uniform_1_texel": ex["mrays_s"] / extras["per_sun_launches"]["uniform_mrays_s"],
            "exact_bit_identical_to_dense": ex["bit_identical_to_dense"],
            "uniform_1_texel_mean_abs_error": extras["accuracy_vs_dense"]["uniform_1_texel"]["mean_abs"]}
        extras["equal_accuracy"]["same_accuracy_figure"] = (
            "exact mode (branch and bound over the max-mip tap bounds, output identical to "
            "dense half-texel stepping): exact_over_dense_uniform_identical_output")
        # forward + backward (hand-written adjoint) for every sun: the forward, then the
        # adjoint recomputing the decisions of the rays with s strictly inside (0, 1) (the
        # autograd default; the others have no derivative), and the recorded form
        # (4-byte deciding sample per ray written by the forward, read by the adjoint)
        g = torch.randn(H, W, generator=torch.Generator(device="cpu").manual_seed(7)).to(dev)
        gh = torch.zeros_like(h)
        gsun = torch.zeros(2, dtype=torch.float64, device=dev)
        samples = [torch.empty(h.shape, dtype=torch.int32, device=dev) for _ in suns]

        def fb_replay():
            ss.maxmip(h, out=mm)
            for k, (e, a, r) in enumerate(suns):
                ss.shadow_cast(h, D, e, a, r, params, mm=mm, out=outs[k])
                ss.shadow_cast_backward_penumbra(h, D, e, a, outs[k], g, r, params, mm=mm,
                                                 grad_h=gh, grad_sun=gsun)

        def fb_record():
            ss.maxmip(h, out=mm)
            for k, (e, a, r) in enumerate(suns):
                ss.shadow_cast_save(h, D, e, a, r, params, mm=mm, out=outs[k], sample=samples[k])
                ss.shadow_cast_backward_saved(h, D, e, a, samples[k], g, r, params, mm=mm,
                                              grad_h=gh, grad_sun=gsun)

        fb_replay()
        fb_record()
        t_fr = float(np.median(_timed(fb_replay, 3)))
        t_fs = float(np.median(_timed(fb_record, 3)))
        extras["fwd_bwd_mrays_s"] = rays_per_step / (t_fr / 1e3) / 1e6
        extras["fwd_bwd_record_mrays_s"] = rays_per_step / (t_fs / 1e3) / 1e6
        del samples
        extras["small_256"] = leg_small(ss)
        extras["differentiable_2048"] = leg_diff(ss)
        extras["frame"] = leg_frame(ss)
        extras["stitch_across_seam"] = leg_stitch(ss)
        if not args.no_big:
            extras["batched_8x64"] = leg_batched(ss)
            extras["polar_16384"] = leg_polar(ss)

    cpu = None
    if not args.no_cpu:
        import oracle
        e, a, r = suns[0]
        po = oracle.Params(W, H, D, R_MOON, e, a, r, max_len_m=c["max_len"])
        cpu = cpu_baseline(h.cpu().numpy(), po)
        if not args.no_extras:
            extras["cpu_uniform_oracle"] = cpu_uniform_baseline(h.cpu().numpy(),
                                                                po.replace(mode=1))
            extras["cpu_oracle_configs"] = cpu_oracle_configs()

    line = {"metric": METRIC, "value": value, "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": WORKLOAD, "rays_per_step": rays_per_step, "suns": len(suns),
                       "seed": seed_of("tile"), "mode": "descent (geometric runs from N'=5)"},
            "roofline": roofline, "cpu_baseline": cpu, "maxmip": maxmip}
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
