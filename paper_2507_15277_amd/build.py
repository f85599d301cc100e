"""Ahead-of-time build of libfewfit.so and the variant code objects.

Sec. III-B: recompiling a kernel at run time costs many runs' worth of time,
so every variant is compiled ahead of time, here into one gfx950 code object
per variant (``variants/<name>.co``) with a manifest listing their
descriptors.  Compile time and code-object size are recorded per variant
(the paper's Tables II and III report the same two costs).

Run ``python -m paper_2507_15277_amd.build`` (or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

from . import space

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
VARIANT_DIR = os.path.join(PKG, "variants")
LIB = os.path.join(PKG, "libfewfit.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instructions are kept out of every device build.
DEVICE_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(verbose=False) -> str:
    srcs = [os.path.join(CSRC, "runtime.hip"), os.path.join(CSRC, "noalloc.hip"), os.path.join(CSRC, "ptune.cpp"),
            os.path.join(CSRC, "setfile.cpp")]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *DEVICE_FLAGS, "-fPIC", "-shared", "-fvisibility=hidden", "-Wall",
           "-Wl,-Bsymbolic", "-o", tmp, *srcs]
    _run(cmd, verbose)
    os.replace(tmp, LIB)
    return LIB


def _compile_variant(v: space.Variant, outdir: str):
    out = os.path.join(outdir, v.name + ".co")
    tmp = out + ".tmp"
    cmd = [HIPCC, *DEVICE_FLAGS, "--cuda-device-only", "--no-gpu-bundle-output", "-c",
           os.path.join(CSRC, v.source), "-o", tmp]
    cmd += [f"-D{k}={val}" for k, val in v.defines().items()]
    t0 = time.perf_counter()
    _run(cmd, False)
    dt = time.perf_counter() - t0
    os.replace(tmp, out)
    return v, dt, os.path.getsize(out)


def build_variants(variants=None, outdir=VARIANT_DIR, jobs=None, verbose=False):
    """Compile every variant in parallel; write manifest.txt and build_stats.txt."""
    variants = space.full_family() if variants is None else variants
    os.makedirs(outdir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    results = {}
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile_variant, v, outdir): v for v in variants}
        for f in cf.as_completed(futs):
            v, dt, size = f.result()
            results[v] = (dt, size)
            if verbose:
                print(f"  built {v.name} ({dt:.1f} s, {size} B)", flush=True)
    with open(os.path.join(outdir, "manifest.txt"), "w") as f:
        f.write("# id name MWG NWG KWG MI WM WN SK VW LDS GM SG PREC PD\n")
        for vid, v in enumerate(variants):
            f.write(v.descriptor(vid) + "\n")
    with open(os.path.join(outdir, "build_stats.txt"), "w") as f:
        f.write("# id name compile_s code_object_bytes\n")
        for vid, v in enumerate(variants):
            dt, size = results[v]
            f.write(f"{vid} {v.name} {dt:.3f} {size}\n")
    return [(v, *results[v]) for v in variants]


def build_all(verbose=False):
    t0 = time.perf_counter()
    build_library(verbose)
    res = build_variants(verbose=verbose)
    if verbose:
        print(f"built libfewfit.so and {len(res)} variants in {time.perf_counter() - t0:.1f} s",
              flush=True)
    return res


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature;
    # anything else in the output is shown.
    lines = [ln for ln in p.stdout.splitlines()
             if "packed-fp32-ops" not in ln and "hip-link" not in ln and ln.strip()]
    if p.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + "\n".join(lines))
    if lines and verbose:
        print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    build_all(verbose=True)
