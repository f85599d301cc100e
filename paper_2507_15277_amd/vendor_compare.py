"""The vendor library's FP32 GEMM beside the k-variant set, on the 27-shape grid.

Times torch's FP32 matrix product on the device (rocBLAS / hipBLASLt
underneath; gfx950 has no reduced-precision FP32 MFMA, so it is a true FP32
SGEMM) and this library's dispatched ``sgemm`` with the same protocol as
``bench.py``: seeded uniform operands resident in HBM, per shape a loop of
back-to-back calls bracketed by HIP events, the median of six trials per
side, interleaved with the order alternating.
Context for the results, not part of the measured path.

With ``--dense16`` it times the vendor's dense FP16 and BF16 products
instead (torch.mm on 16-bit operands, FP32 accumulation inside the library)
on the same shapes: the 16-bit MFMA rate this device reaches in practice,
the ceiling against which the split-precision forms' MFMA work is read.

    python -m paper_2507_15277_amd.vendor_compare [--k 4] [--dense16] [--out vendor.json]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from . import abi, datagen, tuned

TARGET_MS = 1.0


def _time_loop(fn, reps, trials=5):
    import torch

    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
    return float(np.median(out))


def run(k=4, log=print):
    import torch

    torch.backends.cuda.matmul.allow_tf32 = False
    assert abi.variant_set_load(tuned.set_path(k)) == k
    L = abi.lib()
    stream = torch.cuda.current_stream()
    h = stream.cuda_stream
    rows = []
    for (M, N, K) in datagen.grid27():
        A, B, _ = datagen.gemm_operands(3, M, N, K)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        dC = torch.empty(M, N, device="cuda")
        dT = torch.empty(M, N, device="cuda")
        pa, pb, pc = dA.data_ptr(), dB.data_ptr(), dC.data_ptr()

        def ours():
            rc = L.sgemm(M, N, K, 1.0, pa, K, pb, N, 0.0, pc, N, h)
            if rc:
                raise RuntimeError(abi.last_error())

        def vendor():
            torch.mm(dA, dB, out=dT)

        t1 = _time_loop(vendor, 3, trials=1)
        reps = max(1, min(1000, int(round(TARGET_MS / max(t1, 1e-4)))))
        # Interleaved trials, the order alternating, so that neither side
        # always runs right after the other's heavy loop (clock and power
        # state); the median of each.
        tv, to = [], []
        for t in range(6):
            for which in ((vendor, ours) if t % 2 == 0 else (ours, vendor)):
                (tv if which is vendor else to).append(_time_loop(which, reps, trials=1))
        ms_v, ms_o = float(np.median(tv)), float(np.median(to))
        fl = 2.0 * M * N * K
        diff = float((dC - dT).abs().max())
        rows.append({"M": M, "N": N, "K": K, "tflops_set": fl / ms_o / 1e9, "tflops_vendor": fl / ms_v / 1e9,
                     "variant": abi.variant_select(M, N, K), "max_abs_diff": diff})
        log(f"[vendor] {M}x{N}x{K}: set {fl / ms_o / 1e9:7.1f} TFLOP/s, vendor {fl / ms_v / 1e9:7.1f} TFLOP/s "
            f"(x{ms_v / ms_o:.2f}), max |diff| {diff:.2e}")
    gm = lambda key: math.exp(sum(math.log(r[key]) for r in rows) / len(rows))  # noqa: E731
    rep = {"k": k, "shapes": rows, "geomean_tflops_set": gm("tflops_set"), "geomean_tflops_vendor": gm("tflops_vendor"),
           "geomean_speedup": math.exp(sum(math.log(r["tflops_set"] / r["tflops_vendor"]) for r in rows) / len(rows)),
           "vendor": f"torch {torch.__version__} torch.mm (FP32)"}
    log(f"[vendor] geomean: set {rep['geomean_tflops_set']:.1f} TFLOP/s, vendor {rep['geomean_tflops_vendor']:.1f} "
        f"TFLOP/s, speedup x{rep['geomean_speedup']:.2f}")
    return rep


def run_dense16(log=print):
    """The vendor's FP16 and BF16 matrix products on the 27 grid shapes
    (seeded normal operands, contiguous), TFLOP/s per shape and type."""
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    rows = []
    for (M, N, K) in datagen.grid27():
        fl = 2.0 * M * N * K
        row = {"M": M, "N": N, "K": K}
        for name, dt in (("fp16", torch.float16), ("bf16", torch.bfloat16)):
            a = torch.randn(M, K, device="cuda", generator=g).to(dt)
            b = torch.randn(K, N, device="cuda", generator=g).to(dt)
            c = torch.empty(M, N, device="cuda", dtype=dt)

            def vendor():
                torch.mm(a, b, out=c)

            t1 = _time_loop(vendor, 3, trials=1)
            reps = max(1, min(1000, int(round(TARGET_MS / max(t1, 1e-4)))))
            row[f"tflops_{name}"] = fl / _time_loop(vendor, reps, trials=5) / 1e9
        rows.append(row)
        log(f"[vendor16] {M}x{N}x{K}: fp16 {row['tflops_fp16']:7.1f} TFLOP/s, bf16 {row['tflops_bf16']:7.1f} TFLOP/s")
    gm = lambda key: math.exp(sum(math.log(r[key]) for r in rows) / len(rows))  # noqa: E731
    return {"shapes": rows, "geomean_tflops_fp16": gm("tflops_fp16"), "geomean_tflops_bf16": gm("tflops_bf16"),
            "vendor": f"torch {torch.__version__} torch.mm (FP16, BF16)"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--dense16", action="store_true", help="time the vendor's FP16 and BF16 products instead")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    rep = run_dense16(log) if args.dense16 else run(args.k, log=log)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
