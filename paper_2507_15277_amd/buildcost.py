"""Ahead-of-time build costs beside the run times they are paid for
(the analogues of the paper's Tables II and III, Sec. III-B).

Table II sets the median time to compile one kernel variant against the
median time of one run of a variant; Table III gives the average size of one
compiled variant.  Here both come from the compiled family: ``variants/build_stats.txt``
(hipcc seconds and code-object bytes per variant, written by
``build.build_variants``) and the execution-time table (FP32 rows of the
uniform workload).  The same two costs are summed over each committed set,
which is what a portable set saves against shipping the whole family.

    python -m paper_2507_15277_amd.buildcost [--out data/mi355x_buildcost.json]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics

from . import tuned
from .portability import TABLE, read_set
from .tune import current_hashes, load_rows, read_manifest

STATS = os.path.join(tuned.VARIANT_DIR, "build_stats.txt")


def read_stats(path=STATS):
    """{variant id: (name, compile seconds, code-object bytes)}."""
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        vid, name, secs, size = line.split()
        out[int(vid)] = (name, float(secs), int(size))
    return out


def report(stats, rows, sets):
    prec = {vid: p for vid, _, p in read_manifest(with_prec=True)}
    fp32 = [v for v in stats if prec.get(v) == 0]
    run_ms = [r["ms"] for r in rows if r["prec"] == 0 and r["status"] == "ok" and r["data"] == "uniform"]
    med_compile = statistics.median(stats[v][1] for v in fp32)
    med_run = statistics.median(run_ms)
    out = {
        "compile_note": "hipcc wall seconds per code object (device pass only), 8 compiles in parallel on 8 host cores",
        "table_ii": {"median_run_ms": med_run, "median_compile_ms": med_compile * 1e3,
                     "compile_over_run": med_compile * 1e3 / med_run,
                     "runs": len(run_ms), "variants": len(fp32)},
        "table_iii": {"fp32_mean_kb": statistics.mean(stats[v][2] for v in fp32) / 1024.0,
                      "all_mean_kb": statistics.mean(s[2] for s in stats.values()) / 1024.0,
                      "fp32_family_mb": sum(stats[v][2] for v in fp32) / 2.0 ** 20,
                      "all_family_mb": sum(s[2] for s in stats.values()) / 2.0 ** 20,
                      "all_family_compile_s": sum(s[1] for s in stats.values()),
                      "variants": len(stats)},
        "sets": {},
    }
    for label, ids in sets.items():
        out["sets"][label] = {"members": ids,
                              "kb": sum(stats[v][2] for v in ids) / 1024.0,
                              "compile_s": sum(stats[v][1] for v in ids)}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(TABLE), "mi355x_buildcost.json"))
    args = ap.parse_args(argv)
    stats = read_stats()
    rows = load_rows(TABLE, current_hashes())
    sets = {}
    for k in (1, 2, 4, 8):
        sets[f"fp32_k{k}"] = read_set(tuned.set_path(k))[0]
    for form in ("bf16x3", "bf16x6", "fp16s", "fp16x3"):
        sets[f"{form}_k4"] = read_set(tuned.set_path(4, form))[0]
    rep = report(stats, rows, sets)
    with open(args.out, "w") as f:
        json.dump(rep, f, indent=1)
    t2, t3 = rep["table_ii"], rep["table_iii"]
    print(f"median run {t2['median_run_ms']:.4f} ms, median compile {t2['median_compile_ms']:.0f} ms "
          f"({t2['compile_over_run']:.0f}x); mean code object {t3['fp32_mean_kb']:.1f} KB (FP32), "
          f"family {t3['all_family_mb']:.1f} MB / {t3['all_family_compile_s']:.0f} s")
    for label, s in rep["sets"].items():
        print(f"  {label}: {len(s['members'])} variants, {s['kb']:.0f} KB, {s['compile_s']:.1f} s")


if __name__ == "__main__":
    main()
