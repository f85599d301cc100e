"""Run named variants on given shapes back to back (for profiler runs).

    python -m paper_2507_15277_amd.kernel_drive NAME:M:N:K:REPS [NAME:M:N:K:REPS ...]

Loads the compiled family, then for each argument launches variant NAME on
an M x N x K problem (uniform [-1, 1) operands on the device; lognormal for
the split-precision forms, their workload) REPS times after one warm-up
launch, and prints the mean time per launch from HIP events.
"""
from __future__ import annotations

import sys

from . import abi, tuned
from .tune import read_manifest


def main(argv=None):
    import torch

    argv = sys.argv[1:] if argv is None else argv
    abi.variant_manifest_load(tuned.VARIANT_DIR)
    ids = {name: (vid, prec) for vid, name, prec in read_manifest(with_prec=True)}
    stream = torch.cuda.current_stream()
    for arg in argv:
        name, M, N, K, reps = arg.split(":")
        M, N, K, reps = int(M), int(N), int(K), int(reps)
        vid, prec = ids[name]
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        if prec == 0:
            A = torch.rand(M, K, device="cuda", generator=g) * 2 - 1
            B = torch.rand(K, N, device="cuda", generator=g) * 2 - 1
        else:
            A = torch.randn(M, K, device="cuda", generator=g).mul_(2).exp_() * torch.sign(torch.randn(M, K, device="cuda", generator=g))
            B = torch.randn(K, N, device="cuda", generator=g).mul_(2).exp_() * torch.sign(torch.randn(K, N, device="cuda", generator=g))
        C = torch.empty(M, N, device="cuda")
        abi.sgemm_variant(vid, M, N, K, 1.0, A, K, B, N, 0.0, C, N, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            abi.sgemm_variant(vid, M, N, K, 1.0, A, K, B, N, 0.0, C, N, stream)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(f"{name} {M}x{N}x{K}: {ms * 1e3:.2f} us per launch, {2.0 * M * N * K / ms / 1e9:.1f} TFLOP/s", flush=True)


if __name__ == "__main__":
    main()
