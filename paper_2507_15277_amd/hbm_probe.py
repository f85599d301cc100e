"""Plain device-to-device copy of a known byte count.

Used only to calibrate hardware memory counters (FETCH_SIZE, WRITE_SIZE):
the copy reads and writes exactly ``--mib`` MiB each, so the counter value
per dispatch divided by that size is the scale factor applied to the GEMM
kernels' counter readings.

    python -m paper_2507_15277_amd.hbm_probe [--mib 1024] [--reps 3]
"""
from __future__ import annotations

import argparse
import json


def main(argv=None):
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    n = args.mib * 1024 * 1024 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(args.reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / args.reps
    print(json.dumps({"copy_mib": args.mib, "ms": ms,
                      "gbps_read_plus_write": 2 * args.mib * 1024 * 1024 / ms / 1e6}))


if __name__ == "__main__":
    main()
