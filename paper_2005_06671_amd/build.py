"""Builds libsoftshadow.so for gfx950 with hipcc (in-tree, next to this file).

Each HIP source compiles to an object in parallel (under _build/, not
committed), then hipcc links the shared library.  Beside the library goes
libsoftshadow.so.srchash, the hash of every source, header and flag it was
built from; the loader refuses a library whose hash no longer matches the
sources next to it.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsoftshadow.so")
HASH_FILE = LIB + ".srchash"
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HEADERS = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [
    os.path.join(ROOT, "include", "softshadow.h")]

# Packed FP32 instructions are kept out of the device code on purpose; FMA
# contraction stays within single expressions so the forward, adjoint and
# batched kernels, which inline the same device code, round identically.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


def source_hash() -> str:
    """Hash of the sources, headers and flags the library is built from."""
    h = hashlib.sha256()
    for p in SOURCES + HEADERS:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    # the flags without the include path, which differs between checkouts
    h.update(" ".join(f for f in FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    digest = source_hash()

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o")
        cmd = [hipcc] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        return obj, subprocess.run(cmd, capture_output=True, text=True)

    jobs = min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(o, r) for o, r in results if r.returncode != 0]
    for _, r in failed:
        sys.stderr.write(r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed compiling " + ", ".join(o for o, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libsoftshadow.so")
    os.replace(tmp, LIB)
    with open(HASH_FILE, "w") as f:
        f.write(digest + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
