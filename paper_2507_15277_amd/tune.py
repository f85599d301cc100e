"""Autotuner: screen and time every variant on every shape (Sec. V-C).

For each (M, N, K, beta) the driver generates seeded inputs, computes the
FP64 screening reference once on the GPU, then for every variant:

1. runs it once on poisoned output (C filled with NaN when beta == 0, so a
   kernel that reads C is caught) and screens the result against the
   reference (Sec. V-C: kernels producing wrong results are dropped);
2. if correct, times it with HIP events: warm-up launches, then several
   trials of back-to-back launches; the table keeps the median, mean, minimum
   and maximum of the per-trial means (the paper keeps the mean of two runs;
   the median of several trials is less sensitive to noise).

Each result is one JSON line appended to the table file, so an interrupted
run resumes where it stopped (keys already present are skipped).  Rows
carry a hash of the kernel source; rows from another source are ignored.

Usage: python -m paper_2507_15277_amd.tune --out table.jsonl [--sets grid,extra,square]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

from . import abi, datagen

PKG = os.path.dirname(os.path.abspath(__file__))
VARIANT_DIR = os.path.join(PKG, "variants")
KERNEL_SRC = os.path.join(PKG, "csrc", "sgemm_variant.hip")

# Seed tags of the workloads (first element of every seed tuple).
CFG_SQUARE, CFG_GRID = 2, 3


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def read_manifest(directory=VARIANT_DIR):
    out = []
    with open(os.path.join(directory, "manifest.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                out.append((int(p[0]), p[1]))
    return out


def workload(sets):
    """[(cfg, M, N, K, beta)] for the requested shape sets."""
    jobs = []
    if "grid" in sets:
        jobs += [(CFG_GRID, M, N, K, 0.0) for (M, N, K) in datagen.grid27()]
    if "extra" in sets:
        jobs += [(CFG_GRID, M, N, K, 0.0) for (M, N, K) in datagen.SKEWED_EXTRA]
    if "square" in sets:
        for beta in (0.0, 0.5):
            jobs += [(CFG_SQUARE, M, N, K, beta) for (M, N, K) in datagen.square_shapes()]
    # A shape shared by two sets is timed once (the first set's inputs).
    seen, out = set(), []
    for j in jobs:
        if j[1:] not in seen:
            seen.add(j[1:])
            out.append(j)
    return out


def key(row):
    return (row["M"], row["N"], row["K"], row["beta"], row["variant"])


def load_rows(path, khash=None):
    """Complete rows of a table file (a truncated last line is skipped)."""
    rows = []
    if not os.path.exists(path):
        return rows
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if khash is None or r.get("build") == khash:
                rows.append(r)
    return rows


def _median(xs):
    s = sorted(xs)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def tune(out, sets=("grid", "extra", "square"), variants=None, target_ms=2.0, trials=5,
         warmup=2, log=print):
    import torch

    khash = kernel_hash()
    manifest = read_manifest()
    n = abi.variant_manifest_load(VARIANT_DIR)
    if n != len(manifest):
        raise RuntimeError("manifest and loaded variant count differ")
    if variants is not None:
        manifest = [m for m in manifest if m[0] in set(variants)]
    done = {key(r) for r in load_rows(out, khash)}
    dev = torch.cuda.get_device_properties(0)
    device = f"{dev.name} {dev.gcnArchName.split(':')[0]}"
    f = open(out, "a")
    t_start = time.time()
    for (cfg, M, N, K, beta) in workload(sets):
        todo = [(vid, name) for vid, name in manifest if (M, N, K, beta, vid) not in done]
        if not todo:
            continue
        t0 = time.time()
        A, B, C0 = datagen.gemm_operands(cfg, M, N, K, beta=beta)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        dC0 = torch.from_numpy(C0).cuda() if C0 is not None else None
        dC = torch.empty(M, N, dtype=torch.float32, device="cuda")
        ref = torch.empty(M * N, dtype=torch.float64, device="cuda")
        tol = torch.empty(M * N, dtype=torch.float64, device="cuda")
        abi.screen_reference(M, N, K, 1.0, dA, K, dB, N, beta, dC0, N, ref, tol)
        best = math.inf
        flops = 2.0 * M * N * K
        n_ok = 0
        for vid, name in todo:
            if beta == 0.0:
                dC.fill_(float("nan"))
            else:
                dC.copy_(dC0)
            row = {"device": device, "M": M, "N": N, "K": K, "beta": beta, "variant": vid,
                   "name": name, "build": khash}
            try:
                abi.sgemm_variant(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N)
                nbad, ratio = abi.screen_compare(M, N, dC, N, ref, tol)
            except abi.FewfitError as e:
                row.update(status="launch_fail", error=str(e))
                f.write(json.dumps(row) + "\n")
                continue
            row["err_ratio"] = ratio if math.isfinite(ratio) else None
            if nbad:
                row.update(status="wrong", nbad=nbad)
                f.write(json.dumps(row) + "\n")
                continue
            if beta != 0.0:
                dC.copy_(dC0)
            # One probe trial sizes the repetition count.
            probe = abi.sgemm_time(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N,
                                   warmup=1, reps=1, trials=1)[0]
            if probe > 20.0 * best:
                ms_list = [probe]       # far off the best: not worth more time
                reps, ntr = 1, 1
            else:
                reps = max(1, min(500, int(math.ceil(target_ms / max(probe, 1e-4)))))
                ntr = trials
                ms_list = abi.sgemm_time(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N,
                                         warmup=warmup, reps=reps, trials=ntr)
            med = _median(ms_list)
            best = min(best, med)
            n_ok += 1
            row.update(status="ok", ms=med, ms_mean=sum(ms_list) / len(ms_list),
                       ms_min=min(ms_list), ms_max=max(ms_list), reps=reps, trials=ntr,
                       tflops=flops / med / 1e9)
            f.write(json.dumps(row) + "\n")
        f.flush()
        del dA, dB, dC0, dC, ref, tol
        torch.cuda.empty_cache()
        log(f"[tune] {M}x{N}x{K} beta={beta}: {n_ok}/{len(todo)} ok, best "
            f"{flops / best / 1e9 if best < math.inf else 0:.2f} TFLOP/s, {time.time() - t0:.1f} s "
            f"(total {time.time() - t_start:.0f} s)")
        sys.stdout.flush()
    f.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--sets", default="grid,extra,square")
    ap.add_argument("--target-ms", type=float, default=2.0)
    ap.add_argument("--trials", type=int, default=5)
    args = ap.parse_args(argv)
    tune(args.out, sets=tuple(args.sets.split(",")), target_ms=args.target_ms, trials=args.trials,
         log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
