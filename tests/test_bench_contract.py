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
