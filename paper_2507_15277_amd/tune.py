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

The "precision" set times every variant, FP32 and split-precision forms,
on the 27 grid shapes with lognormal operands, and records each result's
normwise relative error and largest componentwise error against the FP64
screening reference.

Usage: python -m paper_2507_15277_amd.tune --out table.jsonl [--sets grid,extra,square,precision]
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
SPLIT_SRC = os.path.join(PKG, "csrc", "sgemm_split.hip")

# Seed tags of the workloads (first element of every seed tuple).
CFG_SQUARE, CFG_GRID, CFG_PRECISION, CFG_FRESH, CFG_RAGGED, CFG_FRESH_LOGNORMAL = 2, 3, 5, 6, 7, 8

# Per-product truncation error of each 16-bit form, as a multiple of |a||b|,
# and its number of term products.  Round-to-nearest bf16 keeps 8 bits
# (|x - hi| <= 2^-8 |x|), fp16 keeps 11; the dropped terms of bf16x3 are
# hi*d + d*hi + lo*lo + smaller (3.03 * 2^-16), those of bf16x6 mid*lo +
# lo*mid + hi*d + d*hi + smaller (4.03 * 2^-24), fp16s rounds both
# operands once (2 * 2^-11), and fp16x3 drops hi*d + d*hi + lo*lo + smaller
# of its 11-bit pieces (3.01 * 2^-22, for entries within 2^18 of the
# matrix's largest magnitude).
FORM_TRUNCATION = {1: 3.1 * 2.0 ** -16, 2: 4.2 * 2.0 ** -24, 3: 2.1 * 2.0 ** -11, 4: 3.1 * 2.0 ** -22}
FORM_PRODUCTS = {0: 1, 1: 3, 2: 6, 3: 1, 4: 3}


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def kernel_hash() -> str:
    """Build hash of the FP32 variant kernel source."""
    return _sha(KERNEL_SRC)


def split_hash() -> str:
    """Build hash of the split-precision kernel source."""
    return _sha(SPLIT_SRC)


def current_hashes():
    return {kernel_hash(), split_hash()}


def screen_scale(prec, K):
    """Factor applied to the FP32 bound 4*K*2^-24*|A||B| for a form: its
    truncation error plus FP32 accumulation of all its term products."""
    if prec == 0 or K == 0:
        return 1.0
    u = 2.0 ** -24
    return FORM_TRUNCATION[prec] / (4.0 * K * u) + 1.05 * FORM_PRODUCTS[prec]


def read_manifest(directory=VARIANT_DIR, with_prec=False):
    out = []
    with open(os.path.join(directory, "manifest.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                p = line.split()
                out.append((int(p[0]), p[1], int(p[13])) if with_prec else (int(p[0]), p[1]))
    return out


def workload(sets):
    """[(cfg, M, N, K, beta, data)] for the requested shape sets; data is
    "uniform" (entries on [-1, 1)) or "lognormal" (the precision workload)."""
    jobs = []
    if "grid" in sets:
        jobs += [(CFG_GRID, M, N, K, 0.0, "uniform") for (M, N, K) in datagen.grid27()]
    if "extra" in sets:
        jobs += [(CFG_GRID, M, N, K, 0.0, "uniform") for (M, N, K) in datagen.SKEWED_EXTRA]
    if "square" in sets:
        for beta in (0.0, 0.5):
            jobs += [(CFG_SQUARE, M, N, K, beta, "uniform") for (M, N, K) in datagen.square_shapes()]
    if "precision" in sets:
        jobs += [(CFG_PRECISION, M, N, K, 0.0, "lognormal") for (M, N, K) in datagen.grid27()]
    if "ragged" in sets:
        # The grid moved off every multiple of 4 (scalar-load kernels only).
        jobs += [(CFG_RAGGED, M, N, K, 0.0, "uniform") for (M, N, K) in datagen.ragged_grid()]
    if "fresh" in sets:
        # Shapes that chose nothing: timed after the sets and the dispatch
        # rule are frozen, to measure how the sets generalise.
        jobs += [(CFG_FRESH, M, N, K, 0.0, "uniform") for (M, N, K) in datagen.fresh_shapes()]
    if "fresh_lognormal" in sets:
        # The same shapes on the precision workload (every form): how the
        # accuracy-targeted set generalises, in speed and in error.
        jobs += [(CFG_FRESH_LOGNORMAL, M, N, K, 0.0, "lognormal") for (M, N, K) in datagen.fresh_shapes()]
    # A shape shared by two sets is timed once (the first set's inputs).
    seen, out = set(), []
    for j in jobs:
        if j[1:] not in seen:
            seen.add(j[1:])
            out.append(j)
    return out


def key(row):
    return (row["M"], row["N"], row["K"], row["beta"], row.get("data", "uniform"), row["variant"])


def operands(cfg, M, N, K, beta, data):
    if data == "lognormal":
        A = datagen.lognormal((cfg, M, N, K, datagen.OP_A), M, K)
        B = datagen.lognormal((cfg, M, N, K, datagen.OP_B), K, N)
        C0 = datagen.uniform((cfg, M, N, K, datagen.OP_C), M, N) if beta != 0.0 else None
        return A, B, C0
    return datagen.gemm_operands(cfg, M, N, K, beta=beta)


def load_rows(path, khash=None, directory=VARIANT_DIR):
    """Complete rows of a table file (a truncated last line is skipped).
    ``khash``: a build hash or a set of them; rows of other builds are
    dropped.  Rows whose variant id names another variant in the current
    manifest (ids move when the family changes) are dropped too."""
    rows = []
    if not os.path.exists(path):
        return rows
    names = dict(read_manifest(directory)) if os.path.exists(os.path.join(directory, "manifest.txt")) else None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            try:
                r = json.loads(line)
            except json.JSONDecodeError:
                continue
            if names is not None and names.get(r.get("variant")) != r.get("name"):
                continue
            if khash is None or r.get("build") in ({khash} if isinstance(khash, str) else khash):
                rows.append(r)
    return rows


def gpu_clock_mhz():
    """Current shader clock of the first GPU in MHz, from the driver's DPM
    table in sysfs (the level marked '*'), or None where it is not readable."""
    import glob
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as f:
                for line in f:
                    if line.rstrip().endswith("*"):
                        mhz = line.split(":", 1)[1].strip().rstrip("*").strip()
                        return float(mhz.lower().replace("mhz", ""))
        except (OSError, ValueError, IndexError):
            continue
    return None


def _median(xs):
    s = sorted(xs)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def tune(out, sets=("grid", "extra", "square"), variants=None, target_ms=2.0, trials=5,
         warmup=2, log=print):
    import torch

    hashes = {0: kernel_hash(), 1: split_hash()}
    manifest = read_manifest(with_prec=True)
    n = abi.variant_manifest_load(VARIANT_DIR)
    if n != len(manifest):
        raise RuntimeError("manifest and loaded variant count differ")
    if variants is not None:
        manifest = [m for m in manifest if m[0] in set(variants)]
    done = {key(r) for r in load_rows(out, current_hashes())}
    dev = torch.cuda.get_device_properties(0)
    device = f"{dev.name} {dev.gcnArchName.split(':')[0]}"
    f = open(out, "a")
    t_start = time.time()
    for (cfg, M, N, K, beta, data) in workload(sets):
        # The split-precision forms are timed on the precision workload only.
        todo = [(vid, name, prec) for vid, name, prec in manifest
                if (M, N, K, beta, data, vid) not in done and (prec == 0 or data == "lognormal")]
        if not todo:
            continue
        t0 = time.time()
        A, B, C0 = operands(cfg, M, N, K, beta, data)
        dA = torch.from_numpy(A).cuda()
        dB = torch.from_numpy(B).cuda()
        dC0 = torch.from_numpy(C0).cuda() if C0 is not None else None
        dC = torch.empty(M, N, dtype=torch.float32, device="cuda")
        ref = torch.empty(M * N, dtype=torch.float64, device="cuda")
        tol = torch.empty(M * N, dtype=torch.float64, device="cuda")
        abi.screen_reference(M, N, K, 1.0, dA, K, dB, N, beta, dC0, N, ref, tol)
        clk_start = gpu_clock_mhz()
        best = {}
        flops = 2.0 * M * N * K
        n_ok = 0
        for vid, name, prec in todo:
            if beta == 0.0:
                dC.fill_(float("nan"))
            else:
                dC.copy_(dC0)
            row = {"device": device, "M": M, "N": N, "K": K, "beta": beta, "data": data, "variant": vid,
                   "name": name, "prec": prec, "build": hashes[min(prec, 1)]}
            scale = screen_scale(prec, K)
            try:
                abi.sgemm_variant(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N)
                nbad, ratio, rel = abi.screen_compare(M, N, dC, N, ref, tol, tol_scale=scale, norms=True)
            except abi.FewfitError as e:
                row.update(status="launch_fail", error=str(e))
                f.write(json.dumps(row) + "\n")
                continue
            row["err_ratio"] = ratio if math.isfinite(ratio) else None
            row["err_norm"] = rel
            if beta == 0.0 and math.isfinite(ratio):
                # tol = 4*K*u*|A||B| exactly when alpha = 1 and beta = 0.
                row["err_comp"] = ratio * scale * 4.0 * K * 2.0 ** -24
            if nbad:
                row.update(status="wrong", nbad=nbad)
                f.write(json.dumps(row) + "\n")
                continue
            if beta != 0.0:
                dC.copy_(dC0)
            # One probe trial sizes the repetition count.
            probe = abi.sgemm_time(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N,
                                   warmup=1, reps=1, trials=1)[0]
            if probe > 20.0 * best.get(prec, math.inf):
                ms_list = [probe]       # far off the best: not worth more time
                reps, ntr = 1, 1
            else:
                reps = max(1, min(500, int(math.ceil(target_ms / max(probe, 1e-4)))))
                ntr = trials
                ms_list = abi.sgemm_time(vid, M, N, K, 1.0, dA, K, dB, N, beta, dC, N,
                                         warmup=warmup, reps=reps, trials=ntr)
            med = _median(ms_list)
            best[prec] = min(best.get(prec, math.inf), med)
            n_ok += 1
            row.update(status="ok", ms=med, ms_mean=sum(ms_list) / len(ms_list),
                       ms_min=min(ms_list), ms_max=max(ms_list), reps=reps, trials=ntr,
                       tflops=flops / med / 1e9, sclk_mhz=gpu_clock_mhz(), sclk_shape_start_mhz=clk_start)
            f.write(json.dumps(row) + "\n")
        f.flush()
        del dA, dB, dC0, dC, ref, tol
        torch.cuda.empty_cache()
        bests = " ".join(f"{abi.FORM_NAMES[p]} {flops / b / 1e9:.2f}" for p, b in sorted(best.items()))
        clk_end = gpu_clock_mhz()
        log(f"[tune] {M}x{N}x{K} beta={beta} {data}: {n_ok}/{len(todo)} ok, best TFLOP/s {bests}, "
            f"{time.time() - t0:.1f} s (total {time.time() - t_start:.0f} s), shader clock "
            f"{clk_start} -> {clk_end} MHz")
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
