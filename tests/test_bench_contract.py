"""bench.py's command-line contract on the CPU (no GPU is touched): more than one
GPU is refused with a message and status 2; the options the harness and the
profiling commands use exist; profile summaries parse the committed format."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_options_exist():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--no-cpu", "--no-extras", "--leg",
                "--summarize", "--dem-cache", "--calibrate-copy"):
        assert opt in r.stdout, opt


def test_committed_traffic_record_is_well_formed():
    with open(os.path.join(ROOT, "profiles", "descent_tile_traffic.json")) as f:
        d = json.load(f)
    assert len(d["kernel_src_sha"]) == 16 and d["hbm_bytes_per_launch"] > 0
    assert "flat_kernel<true, 8, 0>" in d["kernel"]
    assert d["fetch_scale"] > 0 and d["write_scale"] > 0 and "rocprofv3" in d["command"]


def test_committed_counters_record_is_well_formed():
    """The counters the bench's issue fraction comes from, taken on the kernel source the
    traffic record names."""
    with open(os.path.join(ROOT, "profiles", "descent_tile_counters.json")) as f:
        d = json.load(f)
    with open(os.path.join(ROOT, "profiles", "descent_tile_traffic.json")) as f:
        t = json.load(f)
    assert d["kernel_src_sha"] == t["kernel_src_sha"]
    c = d["flat_descent"]
    assert c["SQ_INSTS_VALU"] > 0 and c["SQ_WAVES"] > 0 and 0 < c["active_lanes"] <= 64


def test_equal_error_speedup_interpolates():
    """Log-linear interpolation between the sweep's two bracketing steps."""
    sys.path.insert(0, ROOT)
    import bench
    sweep = [{"step_texels": 16.0, "mean_abs": 0.01, "launch_ms": 2.0},
             {"step_texels": 32.0, "mean_abs": 0.04, "launch_ms": 0.5}]
    r = bench.equal_error_speedup(0.02, sweep, 1.0)
    # error doubles halfway (in log) between 0.01 and 0.04: step 16*sqrt(2), time 2/sqrt(4)=1
    assert abs(r["uniform_step_texels"] - 16.0 * 2 ** 0.5) < 1e-9
    assert abs(r["uniform_ms_per_sun"] - 1.0) < 1e-9 and abs(r["speedup"] - 1.0) < 1e-9
    assert bench.equal_error_speedup(0.5, sweep, 1.0) is None


def test_loader_refuses_a_stale_library(tmp_path):
    """A library whose recorded source hash differs from the sources beside it is refused
    (ImportError), so a GPU run never loads a binary built from other sources."""
    import shutil
    pkg = os.path.join(ROOT, "paper_2005_06671_amd")
    if not os.path.exists(os.path.join(pkg, "libsoftshadow.so")):
        import pytest
        pytest.skip("library not built")
    dst = tmp_path / "repo"
    shutil.copytree(pkg, dst / "paper_2005_06671_amd", ignore=shutil.ignore_patterns("_build"))
    shutil.copytree(os.path.join(ROOT, "include"), dst / "include")
    with open(dst / "paper_2005_06671_amd" / "csrc" / "common.h", "a") as f:
        f.write("\n// edited after the build\n")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2005_06671_amd import _lib\n"
            "try:\n    _lib.lib()\nexcept ImportError as e:\n    print('refused', 'stale' in str(e))\n"
            "else:\n    print('loaded')\n") % str(dst)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.stdout.strip() == "refused True", r.stdout + r.stderr
