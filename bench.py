#!/usr/bin/env python3
"""Benchmark: SGEMM TFLOP/s geomean over the (M,N,K) grid with a k-variant set.

Workload: the 27 shapes (M, N, K) in {256, 1024, 4096}^3, FP32 row-major,
A and B uniform on [-1, 1) (seeded), alpha = 1, beta = 0, all inputs resident
in HBM.  One step runs every shape through ``sgemm()`` (runtime dispatch to
the member of the portability-tuned set chosen for it), each shape as a loop
of back-to-back launches bracketed by HIP events on the launch stream (the
loop length is fixed per shape so that each shape takes about 1 ms; small
shapes are launch-bound and a single launch would mostly time the events).

Reported: the geometric mean over the 27 shapes of 2MNK / time, the
fraction of the per-shape best variant (the per-shape best from the tuning
table, timed live beside the dispatched one), the roofline of the dominant
kernel, and the FP64 oracle on the host cores as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--k 4] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SGEMM TFLOP/s geomean over (M,N,K) grid; % of per-shape best with k variants"
FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak (256 CU x 2.4 GHz x 256 flop/clk)
TARGET_MS_PER_SHAPE = 1.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def geomean(xs):
    xs = list(xs)
    return math.exp(sum(math.log(x) for x in xs) / len(xs))


def cpu_baseline(shapes, budget_s=15.0):
    """The FP64 oracle on the host cores over a bounded sample of the grid:
    shapes in increasing flop order until the time budget is spent."""
    import oracle
    from paper_2507_15277_amd import datagen

    order = sorted(shapes, key=lambda s: s[0] * s[1] * s[2])
    done, t_total = [], 0.0
    for (M, N, K) in order:
        est = 2.0 * M * N * K / (done[-1][1] if done else 2e9)
        if done and t_total + est > budget_s:
            break
        A, B, _ = datagen.gemm_operands(3, M, N, K)
        t0 = time.perf_counter()
        oracle.ref_gemm(A, B)
        dt = time.perf_counter() - t0
        t_total += dt
        done.append(((M, N, K), 2.0 * M * N * K / dt))
        log(f"[cpu] oracle {M}x{N}x{K}: {2.0 * M * N * K / dt / 1e9:.2f} GFLOP/s")
    return {"value": geomean(r for _, r in done) / 1e12, "unit": "TFLOP/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": (f"{len(done)} of the 27 grid shapes, smallest flop count first "
                       f"({', '.join('x'.join(map(str, s)) for s, _ in done)}), one run each, "
                       f"{t_total:.1f} s total; FP64 triple loop with |A||B|, OpenMP over rows")}


def measured_traffic(kernel, k, khash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None if there is none for this kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__grid27_k{k}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                key, _, val = line.partition(":")
                vals[key.strip().strip("`- ")] = val.strip().strip("`")
    if vals.get("kernel_build") != khash or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser(description="fewfit SGEMM grid benchmark")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phase", choices=("all", "dispatch"), default="all",
                    help="dispatch: only the timed dispatch steps (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_15277_amd import abi, datagen, tuned
    from paper_2507_15277_amd.portability import TABLE, matrix
    from paper_2507_15277_amd.tune import kernel_hash, load_rows

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    shapes = datagen.grid27()
    set_file = tuned.set_path(args.k)
    if not os.path.exists(set_file):
        raise SystemExit(f"{set_file} missing: run the tuner and portability selection first")
    k_loaded = abi.variant_set_load(set_file)
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    rows = load_rows(TABLE, kernel_hash())
    t_table = matrix(rows, shapes, 0.0)
    best_ids = [int(np.argmin(t_table[:, j])) for j in range(len(shapes))]

    # Inputs resident in HBM before timing.
    ops = []
    for (M, N, K) in shapes:
        A, B, _ = datagen.gemm_operands(3, M, N, K)
        ops.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    torch.empty(M, N, dtype=torch.float32, device="cuda")))
    torch.cuda.synchronize()
    picks = [abi.variant_select(*s) for s in shapes]
    reps = []
    for j, s in enumerate(shapes):
        est = float(t_table[picks[j], j]) if np.isfinite(t_table[picks[j], j]) else 1.0
        reps.append(max(1, min(1000, int(round(TARGET_MS_PER_SHAPE / est)))))

    def run_step(vids, ev):
        for j, (M, N, K) in enumerate(shapes):
            dA, dB, dC = ops[j]
            ev[j][0].record(stream)
            for _ in range(reps[j]):
                if vids is None:
                    abi.sgemm(M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, stream)
                else:
                    abi.sgemm_variant(vids[j], M, N, K, 1.0, dA, K, dB, N, 0.0, dC, N, stream)
            ev[j][1].record(stream)

    def timed(vids, steps, warmup):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in shapes]
        for _ in range(warmup):
            run_step(vids, ev)
        torch.cuda.synchronize()
        per = np.zeros(len(shapes))
        t0 = time.perf_counter()
        for _ in range(steps):
            run_step(vids, ev)
            torch.cuda.synchronize()      # read this step's events
            per += [ev[j][0].elapsed_time(ev[j][1]) / reps[j] for j in range(len(shapes))]
        wall = time.perf_counter() - t0
        return per / steps, wall

    # Timed region: the dispatch path, exactly --steps steps.
    torch.cuda.synchronize()
    ms_shape, wall = timed(None, args.steps, args.warmup)
    torch.cuda.synchronize()
    tf = [2.0 * M * N * K / ms / 1e9 for (M, N, K), ms in zip(shapes, ms_shape)]
    value = geomean(tf)

    if args.phase == "all":
        # Per-shape best variant, same protocol, for the fraction of best.
        ms_best, _ = timed(best_ids, max(2, args.steps // 2), 1)
        frac = geomean(min(b, d) / d for b, d in zip(ms_best, ms_shape))
        frac_raw = geomean(b / d for b, d in zip(ms_best, ms_shape))
    else:
        ms_best = np.array([t_table[best_ids[j], j] for j in range(len(shapes))])
        frac = frac_raw = geomean(min(b, d) / d for b, d in zip(ms_best, ms_shape))

    # Dominant kernel: the set member with the most time in a step.
    # Algorithmic work per launch: 2MNK flops; bytes 4(MK + KN + MN) with
    # beta = 0 (A and B read once, C written once).
    share = {}
    for j, (M, N, K) in enumerate(shapes):
        v = picks[j]
        fl, tm, by = share.get(v, (0.0, 0.0, 0.0))
        share[v] = (fl + reps[j] * 2.0 * M * N * K, tm + reps[j] * ms_shape[j],
                    by + reps[j] * 4.0 * (M * K + K * N + M * N))
    dom = max(share, key=lambda v: share[v][1])
    fl, tm, by = share[dom]
    launches = sum(reps[j] for j in range(len(shapes)) if picks[j] == dom)
    achieved = fl / tm / 1e9
    dom_name = abi.variant_info(dom).split()[1]
    roofline = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                "traffic": measured_traffic(dom_name, args.k, kernel_hash()), "kernel": dom_name,
                "launches_per_step": launches, "flop_per_launch": fl / launches,
                "algorithmic_bytes_per_launch": by / launches, "ms_per_launch": tm / launches,
                "shapes": ["x".join(map(str, s)) for j, s in enumerate(shapes) if picks[j] == dom]}

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "pct_of_per_shape_best": 100.0 * frac,
        "config": {"workload": "27-shape grid {256,1024,4096}^3 FP32 SGEMM, alpha=1 beta=0, "
                               f"dispatched over a k={k_loaded} portability-tuned variant set",
                   "k": k_loaded, "set_file": os.path.relpath(set_file, ROOT),
                   "launches_per_shape_per_step": reps,
                   "pct_of_best_uncapped": 100.0 * frac_raw,
                   "per_shape_tflops": {"x".join(map(str, s)): round(x, 3) for s, x in zip(shapes, tf)}},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and args.phase == "all":
        out["cpu_baseline"] = cpu_baseline(shapes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
