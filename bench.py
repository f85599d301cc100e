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
                    [--form fp32|bf16x3|bf16x6|fp16s|fp16x3|mixed] [--cold]

``--cold`` times every call on its own after writing a 512 MB scrub buffer
(more than the 256 MB memory-side cache and the L2s together), so operands
come from HBM; the default is warm, back-to-back calls.

``--form`` other than fp32 runs the same protocol for a split-precision form
(its own k-variant set, ``sgemm_form``) on the precision workload: the 27
grid shapes with lognormal operands.  Its roofline is priced against the
16-bit dense MFMA peak with the MFMA work the form issues (its number of
term products times 2MNK); no CPU baseline is taken for it.  ``--form
mixed`` runs the set chosen over every form's variants for a normwise error
of at most 1e-6 (FF_FORM_MIXED): each shape in its dispatched member's form,
against the fastest variant of any form that meets the target there, and
each member priced against its own form's peak.
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
MFMA16_PEAK_TFLOPS = 2500.0       # MI355X dense bf16 / fp16 matrix peak
FORMS = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16s": 3, "fp16x3": 4, "mixed": 5}
FORM_PRODUCTS = {"fp32": 1, "bf16x3": 3, "bf16x6": 6, "fp16s": 1, "fp16x3": 3}   # MFMA term products per GEMM
TARGET_MS_PER_SHAPE = 1.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def geomean(xs):
    xs = list(xs)
    return math.exp(sum(math.log(x) for x in xs) / len(xs))


def cpu_baseline(shapes, budget_s=15.0, min_s=10.0):
    """The FP64 oracle on the host cores over a bounded sample of the grid:
    shapes in increasing flop order, in repeated passes, until the time
    budget would be exceeded or, once every shape has run, at least `min_s`
    seconds are spent.  Each shape's rate is the median of its runs."""
    import numpy as np

    import oracle
    from paper_2507_15277_amd import datagen

    order = sorted(shapes, key=lambda s: s[0] * s[1] * s[2])
    runs, t_total, last_rate = {}, 0.0, 2e9
    operands = {}
    while True:
        stop = False
        for (M, N, K) in order:
            rate = float(np.median(runs[(M, N, K)])) if (M, N, K) in runs else last_rate
            if runs and t_total + 2.0 * M * N * K / rate > budget_s:
                stop = True
                break
            if (M, N, K) not in operands:
                operands[(M, N, K)] = datagen.gemm_operands(3, M, N, K)[:2]
            A, B = operands[(M, N, K)]
            t0 = time.perf_counter()
            oracle.ref_gemm(A, B)
            dt = time.perf_counter() - t0
            t_total += dt
            last_rate = 2.0 * M * N * K / dt
            runs.setdefault((M, N, K), []).append(last_rate)
            log(f"[cpu] oracle {M}x{N}x{K}: {last_rate / 1e9:.2f} GFLOP/s")
        if stop or (len(runs) == len(order) and t_total >= min_s):
            break
    done = [s for s in order if s in runs]
    n_runs = sorted({len(runs[s]) for s in done})
    return {"value": geomean(float(np.median(runs[s])) for s in done) / 1e12, "unit": "TFLOP/s",
            "cores": oracle.threads(), "kind": "oracle",
            "one_thread": cpu_one_thread(order),
            "sample": (f"{len(done)} of the 27 grid shapes, smallest flop count first "
                       f"({', '.join('x'.join(map(str, s)) for s in done)}), "
                       f"{n_runs[0] if n_runs[0] == n_runs[-1] else f'{n_runs[0]}-{n_runs[-1]}'} run(s) each (median per shape), "
                       f"{t_total:.1f} s total; FP64 triple loop with |A||B|, OpenMP over rows")}


_ONE_THREAD = r"""
import json, sys, time
import oracle
from paper_2507_15277_amd import datagen
out, spent = [], 0.0
for (M, N, K) in json.loads(sys.argv[1]):
    A, B, _ = datagen.gemm_operands(3, M, N, K)
    if out and spent + 2.0 * M * N * K / out[-1][1] > float(sys.argv[2]):
        break
    t0 = time.perf_counter()
    oracle.ref_gemm(A, B)
    dt = time.perf_counter() - t0
    spent += dt
    out.append(("x".join(map(str, (M, N, K))), 2.0 * M * N * K / dt))
print(json.dumps({"threads": oracle.threads(), "rates": out, "seconds": spent}))
"""


def cpu_one_thread(order, budget_s=4.0):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1,
    which touches no GPU) over the smallest shapes until `budget_s` is spent."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=ROOT)
    try:
        p = subprocess.run([sys.executable, "-c", _ONE_THREAD, json.dumps([list(s) for s in order]),
                            str(budget_s)], env=env, cwd=ROOT, capture_output=True, text=True, timeout=120)
        if p.returncode != 0:
            raise RuntimeError(p.stderr[-500:])
        r = json.loads(p.stdout.strip().splitlines()[-1])
    except (RuntimeError, ValueError, IndexError, subprocess.TimeoutExpired) as e:
        # A reported baseline only: its failure must not cost the bench line.
        log(f"[cpu] one-thread oracle run failed: {e}")
        return {"value": None, "unit": "TFLOP/s", "cores": 1, "sample": f"failed: {str(e)[-200:]}"}
    return {"value": geomean(x for _, x in r["rates"]) / 1e12, "unit": "TFLOP/s", "cores": r["threads"],
            "sample": f"{len(r['rates'])} smallest grid shapes ({', '.join(s for s, _ in r['rates'])}), "
                      f"one run each, {r['seconds']:.1f} s"}


def measured_traffic(kernel, k, khash, shapes):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None if there is none for this kernel source
    and the same shapes (the counters average over the kernel's launch mix)."""
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
    served = [x.strip() for x in next((v for key, v in vals.items() if key.startswith("shapes served")), "").split(",")]
    if served != list(shapes):
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
    ap.add_argument("--cold", action="store_true",
                    help="time each call alone after a 512 MB scrub write (operands from HBM)")
    ap.add_argument("--form", choices=tuple(FORMS), default="fp32",
                    help="precision form (fp32: the plain SGEMM metric)")
    args = ap.parse_args()
    form, fid = args.form, FORMS[args.form]
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2507_15277_amd import abi, datagen, tuned
    from paper_2507_15277_amd.abi import FORM_NAMES
    from paper_2507_15277_amd.portability import ACCURACY_TARGET, TABLE, matrix
    from paper_2507_15277_amd.tune import CFG_PRECISION, current_hashes, kernel_hash, load_rows, read_manifest

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    shapes = datagen.grid27()
    set_file = tuned.set_path(args.k, form)
    if not os.path.exists(set_file):
        raise SystemExit(f"{set_file} missing: run the tuner and portability selection first")
    k_loaded = abi.variant_set_load(set_file)
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    data = "uniform" if fid == 0 else "lognormal"
    rows = load_rows(TABLE, kernel_hash() if fid == 0 else current_hashes())
    t_table = matrix(rows, shapes, 0.0, data=data)
    precs = [prec for _, _, prec in sorted(read_manifest(with_prec=True))]
    if form == "mixed":
        # The mixed set is compared with the fastest variant of any form that
        # meets its accuracy target on the shape.
        err = matrix(rows, shapes, 0.0, nv=t_table.shape[0], data=data, field="err_norm")
        t_table[~(err <= ACCURACY_TARGET)] = np.inf
    else:
        of_form = np.array([prec == fid for prec in precs])
        t_table[~of_form[:t_table.shape[0]], :] = np.inf
    best_ids = [int(np.argmin(t_table[:, j])) for j in range(len(shapes))]

    # Inputs resident in HBM before timing.
    ops = []
    for (M, N, K) in shapes:
        if fid == 0:
            A, B, _ = datagen.gemm_operands(3, M, N, K)
        else:
            A = datagen.lognormal((CFG_PRECISION, M, N, K, datagen.OP_A), M, K)
            B = datagen.lognormal((CFG_PRECISION, M, N, K, datagen.OP_B), K, N)
        ops.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    torch.empty(M, N, dtype=torch.float32, device="cuda")))
    torch.cuda.synchronize()
    picks = [abi.variant_select_form(fid, *s) for s in shapes]
    reps = []
    for j, s in enumerate(shapes):
        est = float(t_table[picks[j], j]) if np.isfinite(t_table[picks[j], j]) else 1.0
        reps.append(max(1, min(1000, int(round(TARGET_MS_PER_SHAPE / est)))))

    # The C entry points are called straight through ctypes with the device
    # pointers and stream handle prepared once (the same calls the abi
    # wrappers make, without their per-call conversions); every call's status
    # is checked.
    L = abi.lib()
    h = stream.cuda_stream
    ptrs = [(a.data_ptr(), b.data_ptr(), c.data_ptr()) for a, b, c in ops]

    def run_step(vids, ev):
        bad = 0
        for j, (M, N, K) in enumerate(shapes):
            pa, pb, pc = ptrs[j]
            ev[j][0].record(stream)
            if vids is None and fid == 0:
                for _ in range(reps[j]):
                    bad |= L.sgemm(M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
            elif vids is None:
                for _ in range(reps[j]):
                    bad |= L.sgemm_form(fid, M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
            else:
                v = vids[j]
                for _ in range(reps[j]):
                    bad |= L.sgemm_variant(v, M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
            ev[j][1].record(stream)
        if bad:
            raise RuntimeError("sgemm failed: " + abi.last_error())

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

    COLD_CALLS = 8
    scrub = torch.empty(128 << 20, dtype=torch.float32, device="cuda") if args.cold else None

    def timed_cold(vids, steps, warmup):
        """Each call alone: a scrub write evicts the operands from the L2s and
        the memory-side cache, then the call runs between two HIP events."""
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(COLD_CALLS)] for _ in shapes]
        per = np.zeros(len(shapes))
        t0 = time.perf_counter()
        for step in range(warmup + steps):
            if step == warmup:
                t0 = time.perf_counter()   # wall time of the timed steps (scrub writes included)
            for j, (M, N, K) in enumerate(shapes):
                pa, pb, pc = ptrs[j]
                for c in range(COLD_CALLS):
                    scrub.fill_(float(c))
                    ev[j][c][0].record(stream)
                    if vids is None and fid == 0:
                        rc = L.sgemm(M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
                    elif vids is None:
                        rc = L.sgemm_form(fid, M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
                    else:
                        rc = L.sgemm_variant(vids[j], M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
                    ev[j][c][1].record(stream)
                    if rc:
                        raise RuntimeError("sgemm failed: " + abi.last_error())
            torch.cuda.synchronize()
            if step >= warmup:
                per += [np.median([a.elapsed_time(b) for a, b in ev[j]]) for j in range(len(shapes))]
        return per / steps, time.perf_counter() - t0

    if args.cold:
        timed = timed_cold                # noqa: F811 (the cold protocol replaces the warm one)
        reps = [COLD_CALLS] * len(shapes)

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

    # Per member of the set: its launches in a step, their algorithmic work
    # (2MNK flops; bytes 4(MK + KN + MN) with beta = 0, A and B read once and
    # C written once) and their HIP-event time measured in the timed region
    # above.  The dominant kernel is the member with the most measured time
    # in a step; every member with at least 10% of the step is reported too.
    share = {}
    for j, (M, N, K) in enumerate(shapes):
        v = picks[j]
        fl, tm, by, n = share.get(v, (0.0, 0.0, 0.0, 0))
        share[v] = (fl + reps[j] * 2.0 * M * N * K, tm + reps[j] * ms_shape[j],
                    by + reps[j] * 4.0 * (M * K + K * N + M * N), n + reps[j])
    step_ms = sum(tm for _, tm, _, _ in share.values())

    def member_roofline(v):
        fl, tm, by, launches = share[v]
        name = abi.variant_info(v).split()[1]
        mform = FORM_NAMES[precs[v]]      # the member's own form (they differ in the mixed set)
        served = ["x".join(map(str, s)) for j, s in enumerate(shapes) if picks[j] == v]
        if mform == "fp32" and fid == 0:
            achieved = fl / tm / 1e9
            r = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": achieved / FP32_MFMA_PEAK_TFLOPS,
                 "traffic": measured_traffic(name, args.k, kernel_hash(), served)}
        elif mform == "fp32":
            achieved = fl / tm / 1e9
            r = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": None, "form": mform}
        else:
            # MFMA work the form issues: its term products, each 2MNK on 16-bit MFMA.
            achieved = FORM_PRODUCTS[mform] * fl / tm / 1e9
            r = {"bound": "mfma", "achieved": achieved, "peak": MFMA16_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": achieved / MFMA16_PEAK_TFLOPS, "traffic": None,
                 "fp32_equivalent_tflops": fl / tm / 1e9, "mfma_products": FORM_PRODUCTS[mform], "form": mform}
        r.update({"kernel": name, "share_of_step": tm / step_ms, "launches_per_step": launches,
                  "flop_per_launch": fl / launches, "algorithmic_bytes_per_launch": by / launches,
                  "ms_per_launch": tm / launches, "shapes": served})
        return r

    dom = max(share, key=lambda v: share[v][1])
    roofline = member_roofline(dom)
    roofline["members_over_10pct"] = [
        {key: val for key, val in member_roofline(v).items() if key != "shapes"}
        for v in sorted(share, key=lambda v: -share[v][1]) if share[v][1] >= 0.1 * step_ms]

    metric = METRIC if fid == 0 else METRIC.replace("SGEMM", f"SGEMM ({form} form)", 1)
    workload = ("27-shape grid {256,1024,4096}^3 FP32 SGEMM, alpha=1 beta=0" if fid == 0 else
                f"27-shape grid {{256,1024,4096}}^3 SGEMM in the {form} form, lognormal operands, alpha=1 beta=0")
    if form == "mixed":
        metric = METRIC.replace("SGEMM", f"SGEMM (any form meeting normwise error <= {ACCURACY_TARGET:g})", 1)
        workload = (f"27-shape grid {{256,1024,4096}}^3 SGEMM, lognormal operands, alpha=1 beta=0, each shape in "
                    f"the form its mixed-set member uses (members chosen for normwise error <= {ACCURACY_TARGET:g})")
    out = {
        "metric": metric, "value": value, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if fid == 0 else form, "data": "synthetic",
        "pct_of_per_shape_best": 100.0 * frac,
        "config": {"workload": f"{workload}, dispatched over a k={k_loaded} portability-tuned variant set",
                   "k": k_loaded, "set_file": os.path.relpath(set_file, ROOT),
                   "launches_per_shape_per_step": reps,
                   "cache": "cold (512 MB scrub write before each call)" if args.cold else "warm",
                   "pct_of_best_uncapped": 100.0 * frac_raw,
                   "per_shape_tflops": {"x".join(map(str, s)): round(x, 3) for s, x in zip(shapes, tf)}},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and args.phase == "all" and fid == 0:
        out["cpu_baseline"] = cpu_baseline(shapes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
